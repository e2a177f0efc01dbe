"""Pins for the oracle's multi-scale synthesis dictionary (Sect. 4.3, Eqs.
params-synthesis and lasso-synthesis; the Gaussian elements of Sect. 6.4).

Pinned against: the element's printed definition (unit l1 norm before the
scale bias, half-width 2 sigma, the Gaussian ratio of neighbouring taps),
scipy's 2-D convolution and correlation for Psi and Psi*, the adjoint
identity, the single point-source scale reducing to the plain LASSO, and an
independent coordinate-descent solve on the explicit matrix Phi Psi (whose
columns come from scipy's convolution of unit impulses)."""
import numpy as np
import pytest
from scipy.signal import convolve2d, correlate2d

from oracle import brute, dictionary as dic, operator, solver

TIGHT = dict(rel_gap_tol=1e-12, inner_tol0=1e-6, inner_tol_min=1e-15,
             inner_max_iter=50000, max_iter=300)


def test_gaussian_element():
    g0 = dic.gaussian_element(0.0, 1.0)
    assert g0.shape == (1, 1) and g0[0, 0] == 1.0
    for sigma, gamma in [(2.0, 1.2), (5.0, 1.44), (8.0, 1.728)]:
        g = dic.gaussian_element(sigma, gamma)
        h = int(2 * sigma)
        assert g.shape == (2 * h + 1, 2 * h + 1)
        assert abs(g.sum() - gamma) <= 1e-14 * gamma
        assert np.array_equal(g, g.T) and np.array_equal(g, g[::-1, ::-1])
        assert abs(g[h + 1, h] / g[h, h] - np.exp(-1 / sigma ** 2)) <= 1e-14
        assert abs(g[h + 2, h + 1] / g[h, h] - np.exp(-5 / sigma ** 2)) <= 1e-14
        assert np.unravel_index(np.argmax(g), g.shape) == (h, h)
    d = dic.gaussian_dictionary()
    assert [e.shape[0] for e in d] == [1, 9, 21, 33]
    assert np.allclose([e.sum() for e in d], [1.0, 1.2, 1.44, 1.728], rtol=1e-14)


def _sparse_theta(rng, S, n, k):
    atoms = np.sort(rng.choice(S * n * n, k, replace=False))
    return atoms, rng.normal(size=k)


def test_synthesis_is_cropped_convolution():
    rng = np.random.default_rng(1)
    n = 24
    d = dic.gaussian_dictionary((0.0, 2.0, 5.0))
    atoms, w = _sparse_theta(rng, 3, n, 40)
    got = dic.synthesis(atoms, w, d, n)
    want = np.zeros((n, n))
    for s in range(3):
        coef = np.zeros(n * n)
        sel = atoms // (n * n) == s
        coef[atoms[sel] % (n * n)] = w[sel]
        want += convolve2d(coef.reshape(n, n), d[s], mode="same")
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # an element on the border is cropped, not wrapped
    edge = dic.synthesis([0], [1.0], d[:2], n)
    assert abs(edge.sum() - d[0].sum()) <= 1e-15
    edge1 = dic.synthesis([n * n], [1.0], d[:2], n)
    assert abs(edge1.sum() - d[1][4:, 4:].sum()) <= 1e-14


def test_analysis_is_correlation_and_adjoint():
    rng = np.random.default_rng(2)
    n = 20
    d = dic.gaussian_dictionary((0.0, 1.0, 3.0), (1.0, 0.7, 2.0))
    img = rng.normal(size=(n, n))
    got = dic.analysis(img, d)
    for s in range(3):
        want = correlate2d(img, d[s], mode="same")
        assert np.max(np.abs(got[s] - want)) <= 1e-12 * np.max(np.abs(want))
    # <Psi theta, I> = <theta, Psi* I> over all S n^2 coefficients
    theta = rng.normal(size=3 * n * n)
    lhs = float(np.sum(dic.synthesis(np.arange(3 * n * n), theta, d, n) * img))
    rhs = float(theta @ got.reshape(-1))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def _problem(seed, L=150, n=12, fov=0.25):
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-10, 10, size=(L, 2))
    img = np.zeros((n, n))
    img[3:7, 4:9] = 1.0 + 0.3 * rng.normal(size=(4, 5))    # a diffuse patch
    img[9, 2] = 3.0                                         # and a point source
    pix = np.flatnonzero(img)
    V = operator.forward(uv, n, fov, pix, img.reshape(-1)[pix])
    V = V + 0.03 * np.max(np.abs(V)) * (rng.normal(size=L) + 1j * rng.normal(size=L))
    return uv, n, fov, V


def _psi_matrix(d, n):
    """Psi as an (n^2, S n^2) matrix from scipy's convolution of impulses."""
    cols = []
    for elem in d:
        for p in range(n * n):
            e = np.zeros(n * n)
            e[p] = 1.0
            cols.append(convolve2d(e.reshape(n, n), elem, mode="same").reshape(-1))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("positive", [False, True])
def test_dictionary_pfw_matches_coordinate_descent(positive):
    uv, n, fov, V = _problem(3)
    d = dic.gaussian_dictionary((0.0, 1.0, 2.0))
    res = solver.pfw_solve(uv, n, fov, V, alpha=0.05, delta=0.9, dictionary=d,
                           positivity=positive, **TIGHT)
    A = brute.explicit_matrix(uv, n, fov) @ _psi_matrix(d, n)
    y = np.concatenate([V.real, V.imag])
    lmax = np.max(A.T @ y) if positive else np.max(np.abs(A.T @ y))
    assert abs(res.lambda_max - lmax) <= 1e-12 * lmax
    x, obj, rel, _ = brute.lasso_cd(A, y, res.lam, positive=positive)
    assert rel <= 1e-12
    assert abs(res.objective - obj) <= 1e-9 * obj
    fit_cd = A @ x
    fit_fw = np.concatenate([res.fit.real, res.fit.imag])
    assert np.linalg.norm(fit_fw - fit_cd) <= 1e-5 * np.linalg.norm(fit_cd)
    # wide elements are used for the patch
    assert np.any(res.pix >= n * n)


def test_dictionary_kkt():
    """|mu| <= 1 over every scale, mu = sign(theta) on the support."""
    uv, n, fov, V = _problem(4, L=200, n=16)
    d = dic.gaussian_dictionary((0.0, 2.0, 3.0))
    res = solver.pfw_solve(uv, n, fov, V, alpha=0.05, delta=0.9, dictionary=d, **TIGHT)
    assert res.eta.shape == (3, n, n) and res.rel_gap <= 1e-12
    mu = res.certificate.reshape(-1)
    assert np.max(np.abs(mu)) <= 1 + 1e-6
    assert np.allclose(mu[res.pix], np.sign(res.weight), atol=1e-6, rtol=0)


def test_point_scale_reduces_to_the_plain_lasso():
    uv, n, fov, V = _problem(5)
    plain = solver.pfw_solve(uv, n, fov, V, alpha=0.05, delta=0.9, **TIGHT)
    one = solver.pfw_solve(uv, n, fov, V, alpha=0.05, delta=0.9,
                           dictionary=dic.gaussian_dictionary((0.0,), (1.0,)), **TIGHT)
    assert np.array_equal(plain.pix, one.pix)
    assert np.allclose(plain.weight, one.weight, rtol=1e-9, atol=0)
    assert abs(plain.objective - one.objective) <= 1e-12 * plain.objective


def test_dictionary_lambda_above_lambda_max_gives_zero():
    uv, n, fov, V = _problem(6)
    d = dic.gaussian_dictionary((0.0, 1.0, 2.0))
    res = solver.pfw_solve(uv, n, fov, V, alpha=1.0001, delta=0.9, max_iter=5,
                           rel_gap_tol=1e-12, dictionary=d)
    assert res.pix.size == 0 and res.converged
    want = np.max(np.abs(dic.analysis(operator.adjoint(uv, n, fov, V), d)))
    assert abs(res.lambda_max - want) <= 1e-14 * want
