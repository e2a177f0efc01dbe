"""Exact forward and adjoint measurement operators (TEST INFRASTRUCTURE; oracle).

Paper Sect. 2.2, Eq. phi-discrete (forward, "degridding"):
    V_k = sum_{i,j} I[i,j] / n(l_i, m_j) * exp(-j 2 pi (u_k l_i + v_k m_j)) * W
and Eq. adjoint-phi (adjoint, "gridding"):
    (Phi* h)[i,j] = Re{ sum_k h_k / n(l_i, m_j) * exp(+j 2 pi (u_k l_i + v_k m_j)) * W* }.
with the w-term of Sect. 2.1, Eq. phi-plane, W(l, m; w) = exp(-j 2 pi w (n - 1)).
Baselines come as (L, 2) arrays (u, v) for coplanar arrays, where W = 1 (the
coplanar remark of Sect. 2.1), or (L, 3) arrays (u, v, w).  Natural weighting:
every visibility has weight one (Sect. 2.1).

Both operators are evaluated as direct exponential sums in complex128, with
the phase u l + v m + w (n - 1) (n - 1 formed as -(l^2 + m^2) / (1 + n), free
of cancellation).  For coplanar arrays the full-image adjoint uses the
separability of exp(j2pi(u l + v m)) into exp(j2pi u l) exp(j2pi v m) and
evaluates the double sum as one complex matrix product per chunk of
visibilities; this is the same sum, only grouped, and a test checks it
against the per-pixel direct sum.  With w the sum is taken pixel block by
pixel block.
"""
from __future__ import annotations

import numpy as np

from .geometry import direction_cosines, n_term, pixel_coords

_CHUNK_ELEMS = 1 << 22  # bound on temporaries (complex128 elements)


def _as_uv(uv):
    uv = np.asarray(uv, dtype=np.float64)
    return uv[:, 0], uv[:, 1]


def _w_of(uv):
    """w per visibility, or None for (u, v) input or an all-zero w."""
    uv = np.asarray(uv, dtype=np.float64)
    if uv.shape[1] < 3 or not np.any(uv[:, 2]):
        return None
    return uv[:, 2]


def n_minus_one(l, m) -> np.ndarray:
    """n(l, m) - 1 = sqrt(1 - l^2 - m^2) - 1, as -(l^2 + m^2) / (1 + n)."""
    r2 = np.asarray(l) ** 2 + np.asarray(m) ** 2
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


def forward(uv, npix: int, fov_rad: float, pix, weight) -> np.ndarray:
    """V = Phi(x) for a sparse image x (pixel indices ``pix``, values ``weight``).

    Eq. phi-discrete restricted to the support of x.  Returns complex128 (L,).
    """
    u, v = _as_uv(uv)
    pix = np.asarray(pix, dtype=np.int64)
    weight = np.asarray(weight, dtype=np.float64)
    out = np.zeros(u.shape[0], dtype=np.complex128)
    if pix.size == 0:
        return out
    lp, mp, npp = pixel_coords(pix, npix, fov_rad)
    w = _w_of(uv)
    cp = n_minus_one(lp, mp)
    a = weight / npp
    step = max(1, _CHUNK_ELEMS // pix.size)
    for s in range(0, u.shape[0], step):
        ph = np.outer(u[s:s + step], lp) + np.outer(v[s:s + step], mp)
        if w is not None:
            ph += np.outer(w[s:s + step], cp)
        out[s:s + step] = np.exp(-2j * np.pi * ph) @ a
    return out


def forward_dense(uv, npix: int, fov_rad: float, image) -> np.ndarray:
    """Phi(I) for a dense n x n image (same definition, every pixel)."""
    image = np.asarray(image, dtype=np.float64).reshape(npix, npix)
    pix = np.flatnonzero(image)
    return forward(uv, npix, fov_rad, pix, image.reshape(-1)[pix])


def forward_images(uv, npix: int, fov_rad: float, images) -> np.ndarray:
    """Phi applied to k dense images at once: images (n^2, k) real, flat
    pixel p = i n + j; returns (L, k) complex128.  The definition of
    Eq. phi-discrete as one matrix product per chunk of visibilities."""
    u, v = _as_uv(uv)
    w = _w_of(uv)
    images = np.asarray(images, np.float64).reshape(npix * npix, -1)
    l = direction_cosines(npix, fov_rad)
    li = np.repeat(l, npix)
    mj = np.tile(l, npix)
    cij = n_minus_one(li, mj)
    inv_n = 1.0 / n_term(npix, fov_rad).reshape(-1)
    out = np.zeros((u.shape[0], images.shape[1]), dtype=np.complex128)
    step = max(1, _CHUNK_ELEMS // (npix * npix))
    for s in range(0, u.shape[0], step):
        ph = np.outer(u[s:s + step], li) + np.outer(v[s:s + step], mj)
        if w is not None:
            ph += np.outer(w[s:s + step], cij)
        e = np.exp(-2j * np.pi * ph)
        out[s:s + step] = (e * inv_n[None, :]) @ images
    return out


def adjoint(uv, npix: int, fov_rad: float, h) -> np.ndarray:
    """Phi* h as an (n, n) float64 image (Eq. adjoint-phi), all pixels."""
    if _w_of(uv) is not None:  # not separable: pixel block by pixel block
        pix = np.arange(npix * npix)
        return adjoint_pixels(uv, npix, fov_rad, h, pix).reshape(npix, npix)
    u, v = _as_uv(uv)
    h = np.asarray(h, dtype=np.complex128)
    l = direction_cosines(npix, fov_rad)
    acc = np.zeros((npix, npix), dtype=np.complex128)
    step = max(1, _CHUNK_ELEMS // npix)
    for s in range(0, u.shape[0], step):
        eu = np.exp(2j * np.pi * np.outer(u[s:s + step], l))   # [k, i]
        ev = np.exp(2j * np.pi * np.outer(v[s:s + step], l))   # [k, j]
        acc += (eu * h[s:s + step, None]).T @ ev
    return acc.real / n_term(npix, fov_rad)


def adjoint_pixels(uv, npix: int, fov_rad: float, h, pix) -> np.ndarray:
    """Phi* h evaluated only at the flat pixel indices ``pix`` (direct sum)."""
    u, v = _as_uv(uv)
    w = _w_of(uv)
    h = np.asarray(h, dtype=np.complex128)
    pix = np.asarray(pix, dtype=np.int64)
    lp, mp, npp = pixel_coords(pix, npix, fov_rad)
    cp = n_minus_one(lp, mp)
    out = np.zeros(pix.size, dtype=np.float64)
    bsz = max(1, min(pix.size, 1 << 14))  # pixel blocks bound the temporaries
    for b in range(0, pix.size, bsz):
        sl = slice(b, min(b + bsz, pix.size))
        step = max(1, _CHUNK_ELEMS // (sl.stop - sl.start))
        for s in range(0, u.shape[0], step):
            ph = np.outer(u[s:s + step], lp[sl]) + np.outer(v[s:s + step], mp[sl])
            if w is not None:
                ph += np.outer(w[s:s + step], cp[sl])
            out[sl] += (h[s:s + step] @ np.exp(2j * np.pi * ph)).real
    return out / npp


def restricted_adjoint(uv, npix: int, fov_rad: float, h, pix) -> np.ndarray:
    """Phi_S* h: the adjoint restricted to the active set S (Alg. 2, step 2
    works on images supported in S).  Identical to adjoint_pixels."""
    return adjoint_pixels(uv, npix, fov_rad, h, pix)


def psf(uv, dl: float, dm: float) -> float:
    """P(dl, dm) = sum_k cos(2 pi (u_k dl + v_k dm)): the dirty beam at a shift
    (Sect. 3, "Minor cycles"); for w = 0 the dirty image of a unit source at p
    equals P(l_q - l_p, m_q - m_p) / (n_p n_q) at pixel q."""
    u, v = _as_uv(uv)
    return float(np.sum(np.cos(2.0 * np.pi * (u * dl + v * dm))))


def dirty_image(uv, npix, fov_rad, vis) -> np.ndarray:
    """Dirty image Phi* V under natural weighting (Sect. 2.2)."""
    return adjoint(uv, npix, fov_rad, vis)


def lambda_max(dirty: np.ndarray) -> float:
    """lambda_max = || Phi* V ||_inf (Eq. lmax)."""
    return float(np.max(np.abs(dirty)))
