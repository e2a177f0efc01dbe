"""LASSO quantities and the Polyatomic Frank-Wolfe solver (TEST INFRASTRUCTURE).

Paper passages followed:
  * LASSO objective  P(x) = 1/2 ||V - Phi x||^2 + lambda ||x||_1   (Eq. lasso).
  * lambda_max = ||Phi* V||_inf (Eq. lmax); lambda = alpha lambda_max (Eq. lambda).
  * dual certificate mu = Phi*(V - Phi x) / lambda (Eq. dual_certif), with
    ||mu||_inf <= 1 and <mu, x> = ||x||_1 at a solution (Eqs. dual-saturation).
  * Polyatomic Frank-Wolfe of quality delta (Alg. 2):
        Delta = (1 - delta) ||Phi* V||_inf,  x_0 = 0, S_0 = {}
        for k = 0, 1, ...:
            eta_k = Phi*(V - Phi x_k)                      (dirty residual)
            I     = { j : |eta_k|_j >= ||eta_k||_inf - 2 Delta / (k + 2) }
            S     = S u I
            x     = argmin over supp(x) in S of the LASSO  (restricted solve)
            S     = supp(x)                                 (prune)
            stop if a criterion holds.
  * The restricted solve is an accelerated proximal gradient (APGD / FISTA,
    Sect. 4.4), stopped early with an accuracy that tightens over the FW
    iterations (Sect. 5.1, "The algorithmic steps").

Readings of points the paper leaves open (shared with the GPU path):
  * delta is a parameter (its value is never printed);
  * inner accuracy: the restricted solve stops when the relative duality
    gap of the restricted problem is <= tau_k = max(tau_min, tau_0 g_k),
    with g_k the relative duality gap of the full problem at the current
    iterate x_k (so the accuracy rises as the outer iteration converges),
    plus an iteration cap;
  * warm start: the previous weights, new atoms start at zero;
  * step size 1 / L_ip with L_ip the largest eigenvalue of the restricted
    normal matrix (computed exactly here);
  * relative improvement |P_k - P_{k-1}| / P_{k-1} with P_{-1} = P(0);
  * duality gap: primal P(x) minus the dual value D(nu) = Re<V, nu> - ||nu||^2/2
    at the rescaled residual nu = min(1, lambda / ||Phi* r||_inf) r;
  * ties in the exploration threshold are inclusive (">=", as printed).

Positivity (remarks on positivity in Sects. 4.1 and 5.1): with x >= 0 the
l1 term is lambda sum x, candidate atoms are placed only at the positive
maxima of the dirty residual, and the restricted solve keeps x >= 0.  Readings:
lambda_max = max(0, max_j (Phi* V)_j) (x = 0 is optimal exactly when
Phi* V <= lambda everywhere); the exploration threshold uses eta itself in
place of |eta| (and only eta > 0 qualifies); the proximal map is
max(0, z - t); the dual point is scaled by the largest positive correlation
max(0, max_j (Phi* r)_j), the one-sided dual constraint; the restricted gap
is tested only at extrapolated points inside x >= 0.

Synthesis dictionary (Sect. 4.3, Eq. lasso-synthesis): with ``dictionary``
(see dictionary.py) the atoms are the columns of Phi Psi, indexed s N + p;
eta is replaced by Psi* eta (one image per scale), lambda_max by
||Psi* Phi* V||_inf, and the restricted normal matrix is formed from the
atoms' visibility columns Phi(g_s centred on p).

The restricted problem is solved with the exact normal matrix
G_S = Re(Phi_S^H Phi_S) and b_S = Phi_S^* V, a different route from the GPU's
operator applications that computes the same mathematics.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import dictionary as dic
from .geometry import pixel_coords
from .operator import adjoint, forward, forward_images, n_minus_one

_CHUNK_ELEMS = 1 << 22


def soft(z: np.ndarray, t: float, positive: bool = False) -> np.ndarray:
    """Proximal map of t ||.||_1 (soft thresholding); of t ||.||_1 plus the
    indicator of x >= 0 with ``positive``."""
    if positive:
        return np.maximum(z - t, 0.0)
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def dual_scale_norm(g: np.ndarray, positive: bool = False) -> float:
    """The quantity the dual point is scaled by: ||g||_inf, or max(0, max g)
    for the one-sided constraint of the positive problem."""
    g = np.asarray(g)
    if g.size == 0:
        return 0.0
    return float(max(np.max(g), 0.0)) if positive else float(np.max(np.abs(g)))


def objective(vis, fit, weight, lam: float) -> float:
    """P(x) = 1/2 ||V - Phi x||^2 + lambda ||x||_1 (Eq. lasso)."""
    r = np.asarray(vis, np.complex128) - np.asarray(fit, np.complex128)
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.sum(np.abs(weight)))


def dual_gap(vis, resid, adj_resid_inf: float, primal: float, lam: float):
    """(gap, dual) for the rescaled-residual dual point."""
    vis = np.asarray(vis, np.complex128)
    resid = np.asarray(resid, np.complex128)
    s = 1.0 if adj_resid_inf <= lam else lam / adj_resid_inf
    nu = s * resid
    dual = float(np.vdot(vis, nu).real) - 0.5 * float(np.vdot(nu, nu).real)
    return primal - dual, dual


class GramCache:
    """Columns of G = Re(Phi^H Phi) for every pixel ever activated.

    G[p, q] = Re sum_k exp(+j2pi t_kp) exp(-j2pi t_kq) / (n_p n_q), with
    t_kp = u_k l_p + v_k m_p (+ w_k (n_p - 1) for (L, 3) baselines, the
    w-term of Eq. phi-plane).  Computed with complex128 matrix products over
    chunks of visibilities; only pairs involving new pixels are computed.
    """

    def __init__(self, uv, npix: int, fov_rad: float):
        self.uv = np.asarray(uv, np.float64)
        self.npix, self.fov = npix, fov_rad
        self.pix = np.zeros(0, np.int64)
        self.G = np.zeros((0, 0))

    def _phase(self, s, step, pix):
        """t_kp for visibilities s..s+step and pixels pix, and 1/n_p."""
        lp, mp, npp = pixel_coords(pix, self.npix, self.fov)
        uv = self.uv[s:s + step]
        ph = np.outer(uv[:, 0], lp) + np.outer(uv[:, 1], mp)
        if uv.shape[1] > 2:
            ph += np.outer(uv[:, 2], n_minus_one(lp, mp))
        return ph, npp

    def ensure(self, pix_new: np.ndarray):
        pix_new = np.setdiff1d(np.asarray(pix_new, np.int64), self.pix)
        if pix_new.size == 0:
            return
        old = self.pix
        allp = np.concatenate([old, pix_new])
        g_no = np.zeros((pix_new.size, old.size))
        g_nn = np.zeros((pix_new.size, pix_new.size))
        step = max(1, _CHUNK_ELEMS // max(1, allp.size))
        for s in range(0, self.uv.shape[0], step):
            ph_n, nn = self._phase(s, step, pix_new)
            en = np.exp(-2j * np.pi * ph_n) / nn
            g_nn += (en.conj().T @ en).real
            if old.size:
                ph_o, no = self._phase(s, step, old)
                eo = np.exp(-2j * np.pi * ph_o) / no
                g_no += (en.conj().T @ eo).real
        G = np.zeros((allp.size, allp.size))
        G[:old.size, :old.size] = self.G
        G[old.size:, :old.size] = g_no
        G[:old.size, old.size:] = g_no.T
        G[old.size:, old.size:] = g_nn
        order = np.argsort(allp)
        self.pix = allp[order]
        self.G = G[np.ix_(order, order)]

    def sub(self, pix: np.ndarray) -> np.ndarray:
        idx = np.searchsorted(self.pix, pix)
        return self.G[np.ix_(idx, idx)]


class DictGramCache:
    """G = Re(A_S^H A_S) for synthesis atoms, A_a = Phi(Psi e_a) computed by
    the exact forward over the element's (cropped) pixels; columns are kept
    per atom."""

    def __init__(self, uv, npix: int, fov_rad: float, dictionary):
        self.uv, self.npix, self.fov, self.dictionary = uv, npix, fov_rad, dictionary
        self.cols = {}

    def column(self, a: int) -> np.ndarray:
        if a not in self.cols:
            self.ensure([a])
        return self.cols[a]

    def ensure(self, atoms):
        new = sorted({int(a) for a in np.asarray(atoms, np.int64)} - set(self.cols))
        if not new:
            return
        W = np.zeros((self.npix * self.npix, len(new)))   # Psi e_a, one image per atom
        for c, a in enumerate(new):
            s, p = dic.split_atoms([a], self.npix)
            pix, val = dic.element_pixels(self.dictionary[int(s[0])], int(p[0]), self.npix)
            W[pix, c] = val
        cols = forward_images(self.uv, self.npix, self.fov, W)
        for c, a in enumerate(new):
            self.cols[a] = cols[:, c]

    def sub(self, atoms) -> np.ndarray:
        if len(atoms) == 0:
            return np.zeros((0, 0))
        C = np.stack([self.column(int(a)) for a in atoms], axis=1)
        return (C.conj().T @ C).real


def restricted_gap(G: np.ndarray, b: np.ndarray, vv: float, lam: float, y: np.ndarray,
                   positive: bool = False):
    """(P_S(y), gap) of the LASSO restricted to S at y, from the normal
    equations: ||V - Phi_S y||^2 = vv - 2 b.y + y.G.y, Re<V, r> = vv - b.y,
    Phi_S^* r = b - G y (vv = ||V||^2), with the rescaled-residual dual point."""
    gy = b - G @ y
    r2 = vv - 2.0 * float(b @ y) + float(y @ G @ y)
    vr = vv - float(b @ y)
    p = 0.5 * r2 + lam * float(np.sum(np.abs(y)))
    c = dual_scale_norm(gy, positive)
    s = 1.0 if c <= lam else lam / c
    return p, p - (s * vr - 0.5 * s * s * r2), gy


def fista_restricted(G: np.ndarray, b: np.ndarray, vv: float, lam: float, x0: np.ndarray,
                     tol: float, max_iter: int, lip: Optional[float] = None,
                     positive: bool = False):
    """argmin_x 1/2 x^T G x - b^T x + lam ||x||_1 by FISTA (Beck & Teboulle).

    Each step evaluates the gradient at the extrapolated point y, takes the
    proximal step x+ = soft(y + (b - G y)/L, lam/L) with L the largest
    eigenvalue of G, and updates the momentum t+ = (1 + sqrt(1 + 4 t^2))/2,
    y+ = x+ + ((t - 1)/t+)(x+ - x).  It stops, returning x+, when the relative
    duality gap of the restricted problem at y is <= tol (x+ is then at least
    as good as y) or after max_iter steps.  Returns (x, steps).  With
    ``positive`` the objective is +inf at an extrapolated y outside x >= 0, so
    the test is taken only at a y >= 0 (x+ is feasible in any case).
    """
    if lip is None:
        lip = float(np.linalg.eigvalsh(G)[-1]) if G.size else 1.0
    x = x0.astype(np.float64).copy()
    y = x.copy()
    t = 1.0
    it = 0
    for it in range(1, max_iter + 1):
        p, gap, gy = restricted_gap(G, b, vv, lam, y, positive)
        xn = soft(y + gy / lip, lam / lip, positive)
        if gap <= tol * p and not (positive and np.any(y < 0)):
            return xn, it
        tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        y = xn + ((t - 1.0) / tn) * (xn - x)
        x, t = xn, tn
    return x, it


@dataclasses.dataclass
class IterLog:
    k: int
    n_active: int
    n_new: int
    eta_inf: float
    objective: float
    rel_gap: float
    inner_iters: int


@dataclasses.dataclass
class SolveResult:
    pix: np.ndarray
    weight: np.ndarray
    objective: float
    rel_gap: float
    lam: float
    lambda_max: float
    iters: int
    converged: bool
    eta: np.ndarray          # final dirty residual Phi*(V - Phi x), (n, n); (S, n, n) = Psi* of it with a dictionary
    fit: np.ndarray          # Phi x, (L,)
    log: List[IterLog]

    @property
    def certificate(self) -> np.ndarray:
        return self.eta / self.lam


def pfw_solve(uv, npix: int, fov_rad: float, vis, *, alpha: float = 0.01,
              lam: Optional[float] = None, delta: float = 0.99,
              max_iter: int = 50, rel_obj_tol: float = 0.0,
              rel_gap_tol: float = 0.0, inner_tol0: float = 1e-1,
              inner_tol_min: float = 1e-8, inner_max_iter: int = 2000,
              dirty: Optional[np.ndarray] = None, positivity: bool = False,
              dictionary=None) -> SolveResult:
    """Polyatomic Frank-Wolfe for the point-source LASSO (Alg. 2).

    ``alpha`` sets lambda = alpha * lambda_max unless ``lam`` > 0 is given.
    Stops after the prune of iteration k when k + 1 = max_iter, or when the
    relative objective improvement is <= rel_obj_tol, or when the relative
    duality gap is <= rel_gap_tol (a tolerance <= 0 disables that test).
    """
    vis = np.asarray(vis, np.complex128)
    if dirty is None:
        dirty = adjoint(uv, npix, fov_rad, vis)
    if dictionary is not None:                      # Psi* Phi* V, one image per scale
        dirty = dic.analysis(dirty, dictionary)
    lmax = dual_scale_norm(dirty, positivity)
    if lam is None or lam <= 0:
        lam = alpha * lmax
    big_delta = (1.0 - delta) * lmax
    gram = (GramCache(uv, npix, fov_rad) if dictionary is None
            else DictGramCache(uv, npix, fov_rad, dictionary))
    b_all = dirty.reshape(-1)                       # Phi_S^* V = dirty image on S
    S = np.zeros(0, np.int64)
    x = np.zeros(0)
    eta = dirty.copy()
    vv = float(np.vdot(vis, vis).real)
    p_prev = 0.5 * vv                               # P(x_0 = 0)
    log: List[IterLog] = []
    fit = np.zeros_like(vis)
    gap0, _ = dual_gap(vis, vis, lmax, p_prev, lam)  # lmax is the scale at x = 0
    rel_gap = gap0 / p_prev if p_prev > 0 else 0.0
    converged = False
    k = 0
    for k in range(max_iter):
        a = (eta if positivity else np.abs(eta)).reshape(-1)
        tau = float(a.max()) - 2.0 * big_delta / (k + 2)
        new = np.flatnonzero((a >= tau) & (a > 0)) if positivity else np.flatnonzero(a >= tau)
        S_new = np.union1d(S, new)
        xw = np.zeros(S_new.size)
        if S.size:
            xw[np.searchsorted(S_new, S)] = x
        gram.ensure(S_new)
        G = gram.sub(S_new)
        tol = max(inner_tol_min, inner_tol0 * rel_gap)
        x, nin = fista_restricted(G, b_all[S_new], vv, lam, xw, tol, inner_max_iter,
                                  positive=positivity)
        keep = x != 0.0
        S, x = S_new[keep], x[keep]
        if dictionary is None:
            fit = forward(uv, npix, fov_rad, S, x)
        else:
            img = dic.synthesis(S, x, dictionary, npix).reshape(-1)
            nz = np.flatnonzero(img)
            fit = forward(uv, npix, fov_rad, nz, img[nz])
        resid = vis - fit
        eta = adjoint(uv, npix, fov_rad, resid)
        if dictionary is not None:
            eta = dic.analysis(eta, dictionary)
        p = objective(vis, fit, x, lam)
        gap, _ = dual_gap(vis, resid, dual_scale_norm(eta, positivity), p, lam)
        rel_gap = gap / p if p > 0 else 0.0
        rel_imp = abs(p - p_prev) / p_prev if p_prev > 0 else 0.0
        log.append(IterLog(k, int(S.size), int(new.size), float(a.max()), p, rel_gap, nin))
        p_prev = p
        if rel_obj_tol > 0 and rel_imp <= rel_obj_tol:
            converged = True
            break
        if rel_gap_tol > 0 and rel_gap <= rel_gap_tol:
            converged = True
            break
    p_final = objective(vis, fit, x, lam)
    return SolveResult(S, x, p_final, float(rel_gap), float(lam), lmax, k + 1,
                       converged, eta, fit, log)


def certificate(uv, npix, fov_rad, vis, pix, weight, lam: float) -> np.ndarray:
    """mu = Phi*(V - Phi x) / lambda (Eq. dual_certif) as an (n, n) image."""
    fit = forward(uv, npix, fov_rad, pix, weight)
    return adjoint(uv, npix, fov_rad, np.asarray(vis, np.complex128) - fit) / lam


def argmax_abs(img: np.ndarray):
    """(max |img|, lowest flat index attaining it)."""
    a = np.abs(np.asarray(img)).reshape(-1)
    m = a.max()
    return float(m), int(np.flatnonzero(a == m)[0])
