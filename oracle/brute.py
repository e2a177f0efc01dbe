"""Brute-force LASSO by cyclic coordinate descent (TEST INFRASTRUCTURE).

An independent route to the minimiser of the LASSO (Eq. lasso) for tiny
problems: the complex operator Phi : R^N -> C^L (Eq. phi-discrete) is written
out as the real 2L x N matrix A = [Re Phi; Im Phi], and each coordinate is
minimised exactly in turn:
    x_j <- soft(x_j + a_j^T r / ||a_j||^2, lambda / ||a_j||^2),
with r = y - A x kept up to date.  Iterates until the relative duality gap is
below ``gap_tol``.  Shares nothing with the Frank-Wolfe route.  With
``positive`` the coordinates are kept non-negative (the positivity-constrained
LASSO of the positivity remarks in Sects. 4.1 and 5.1):
x_j <- max(0, x_j + (a_j^T r - lambda) / ||a_j||^2), and the dual point is
scaled by the largest positive correlation.
"""
from __future__ import annotations

import numpy as np

from .geometry import direction_cosines, n_term


def explicit_matrix(uv, npix: int, fov_rad: float) -> np.ndarray:
    """A = [Re Phi; Im Phi] (2L x N), column p = i*n + j; (L, 3) baselines
    add the w-term phase w (n - 1) of Eq. phi-plane."""
    uv = np.asarray(uv, np.float64)
    l = direction_cosines(npix, fov_rad)
    li = np.repeat(l, npix)
    mj = np.tile(l, npix)
    ph = np.outer(uv[:, 0], li) + np.outer(uv[:, 1], mj)
    if uv.shape[1] > 2:
        r2 = li ** 2 + mj ** 2
        ph += np.outer(uv[:, 2], -r2 / (1.0 + np.sqrt(1.0 - r2)))
    phi = np.exp(-2j * np.pi * ph) / n_term(npix, fov_rad).reshape(-1)[None, :]
    return np.concatenate([phi.real, phi.imag], axis=0)


def lasso_cd(A: np.ndarray, y: np.ndarray, lam: float, gap_tol: float = 1e-13,
             max_sweeps: int = 200000, positive: bool = False):
    """Cyclic coordinate descent for 1/2||y - Ax||^2 + lam ||x||_1 (x >= 0
    with ``positive``).

    Returns (x, objective, relative gap, sweeps)."""
    n = A.shape[1]
    x = np.zeros(n)
    r = y.astype(np.float64).copy()
    col2 = np.einsum("ij,ij->j", A, A)
    rel = np.inf
    obj = 0.5 * float(r @ r)
    for sweep in range(1, max_sweeps + 1):
        for j in range(n):
            if col2[j] == 0.0:
                continue
            zj = x[j] + float(A[:, j] @ r) / col2[j]
            if positive:
                xj = max(zj - lam / col2[j], 0.0)
            else:
                xj = np.sign(zj) * max(abs(zj) - lam / col2[j], 0.0)
            d = xj - x[j]
            if d != 0.0:
                r -= d * A[:, j]
                x[j] = xj
        if sweep % 10 == 0 or sweep == 1:
            obj = 0.5 * float(r @ r) + lam * float(np.abs(x).sum())
            corr = A.T @ r
            c = float(max(np.max(corr), 0.0)) if positive else float(np.max(np.abs(corr)))
            s = 1.0 if c <= lam else lam / c
            dual = s * float(y @ r) - 0.5 * s * s * float(r @ r)
            rel = (obj - dual) / obj if obj > 0 else 0.0
            if rel <= gap_tol:
                break
    obj = 0.5 * float(r @ r) + lam * float(np.abs(x).sum())
    return x, obj, rel, sweep
