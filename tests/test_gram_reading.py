"""The Gram form of the restricted problem rests on an identity of the
coplanar measurement operator (Eqs. phi-discrete, adjoint-phi with w = 0):
Re(Phi_S^H Phi_S) has the entries psf(l_p - l_q, m_p - m_q) / (n_p n_q), psf
being the dirty beam of the uv coverage (Sect. 3, minor cycles, where it is
used without the 1/n factors as an approximation), so that the APGD gradient
Phi_S^*(V - Phi_S y) equals b - G y with b = Phi_S^* V, and the residual norm
is ||V||^2 - 2 y.b + y.G y.  Checked here on the oracle's operators (CPU)."""
import numpy as np

import sim
from oracle import geometry, operator


def _problem(n_atoms=14, seed=21):
    p = sim.config_c1()
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(p.npix ** 2, n_atoms, replace=False))
    return p, pix


def _columns(p, pix):
    """Phi_S as a dense (L, nS) matrix, one oracle forward per unit atom."""
    return np.stack([operator.forward(p.uv, p.npix, p.fov_rad, [q], [1.0]) for q in pix], axis=1)


def test_gram_entries_are_the_shifted_psf_over_n():
    p, pix = _problem()
    C = _columns(p, pix)
    G = np.real(C.conj().T @ C)
    l, m, nn = geometry.pixel_coords(pix, p.npix, p.fov_rad)
    Gf = np.array([[operator.psf(p.uv, l[a] - l[c], m[a] - m[c]) / (nn[a] * nn[c])
                    for c in range(pix.size)] for a in range(pix.size)])
    np.testing.assert_allclose(G, Gf, rtol=1e-10, atol=1e-10 * np.abs(G).max())
    # symmetric, and the diagonal is L / n_p^2 (every phase difference is zero)
    np.testing.assert_allclose(np.diag(G), p.nvis / nn ** 2, rtol=1e-12)


def test_gradient_and_residual_norm_in_gram_form():
    p, pix = _problem(seed=22)
    rng = np.random.default_rng(23)
    V = rng.normal(size=p.nvis) + 1j * rng.normal(size=p.nvis)
    y = rng.normal(size=pix.size)
    r = V - operator.forward(p.uv, p.npix, p.fov_rad, pix, y)
    g_op = operator.restricted_adjoint(p.uv, p.npix, p.fov_rad, r, pix)
    C = _columns(p, pix)
    G = np.real(C.conj().T @ C)
    b = operator.restricted_adjoint(p.uv, p.npix, p.fov_rad, V, pix)
    np.testing.assert_allclose(b - G @ y, g_op, rtol=1e-9, atol=1e-9 * np.abs(g_op).max())
    r2 = float(np.vdot(r, r).real)
    assert abs(float(np.vdot(V, V).real) - 2.0 * y @ b + y @ G @ y - r2) <= 1e-10 * r2
    # Re<V, r> = ||V||^2 - y.b (the other input of the duality gap)
    vr = float(np.vdot(V, r).real)
    assert abs(float(np.vdot(V, V).real) - y @ b - vr) <= 1e-10 * abs(vr)
