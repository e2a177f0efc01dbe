"""Pins for the oracle's LASSO / Polyatomic Frank-Wolfe solver (T10-T16).

Pinned against: the closed-form LASSO solution of an orthogonal design,
the optimality conditions of the certificate (Eqs. dual-saturation1/2), the
alpha identity of Sect. 5.3, Hermitian doubling, the lambda >= lambda_max
case (Eq. lmax), an independent coordinate-descent solver, and the delta = 1
special case of Alg. 2.
"""
import numpy as np
import pytest

import sim
from oracle import brute, geometry, operator, solver

TIGHT = dict(rel_gap_tol=1e-12, inner_tol0=1e-6, inner_tol_min=1e-15,
             inner_max_iter=50000, max_iter=200)


def _problem(seed, L=160, n=8, fov=0.25, n_src=3, noise=0.05):
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-12, 12, size=(L, 2))
    pix = rng.choice(n * n, n_src, replace=False)
    amp = np.exp(rng.normal(size=n_src))
    V = operator.forward(uv, n, fov, pix, amp)
    V = V + noise * np.max(np.abs(V)) * (rng.normal(size=L) + 1j * rng.normal(size=L))
    return uv, n, fov, V


def test_soft_threshold():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    assert np.array_equal(solver.soft(z, 1.0), [-2.0, -0.0, 0.0, 0.0, 1.0])


def test_orthogonal_design_closed_form():
    """T10: uv on the DFT frequencies => x_p = soft((Phi*V)_p, lam) n_p^2 / n^2."""
    n, fov = 8, 0.3
    uv = sim.orthogonal_uv(n, fov)
    rng = np.random.default_rng(11)
    V = rng.normal(size=uv.shape[0]) + 1j * rng.normal(size=uv.shape[0])
    res = solver.pfw_solve(uv, n, fov, V, alpha=0.3, delta=0.5, **TIGHT)
    b = operator.adjoint(uv, n, fov, V).reshape(-1)
    nn = geometry.n_term(n, fov).reshape(-1)
    want = solver.soft(b, res.lam) * nn ** 2 / n ** 2
    got = np.zeros(n * n)
    got[res.pix] = res.weight
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))
    assert np.array_equal(res.pix, np.flatnonzero(want))


def test_brute_force_matches_orthogonal_closed_form():
    n, fov = 6, 0.3
    uv = sim.orthogonal_uv(n, fov)
    rng = np.random.default_rng(12)
    V = rng.normal(size=uv.shape[0]) + 1j * rng.normal(size=uv.shape[0])
    A = brute.explicit_matrix(uv, n, fov)
    y = np.concatenate([V.real, V.imag])
    b = operator.adjoint(uv, n, fov, V).reshape(-1)
    lam = 0.4 * np.max(np.abs(b))
    x, obj, rel, _ = brute.lasso_cd(A, y, lam)
    nn = geometry.n_term(n, fov).reshape(-1)
    assert np.allclose(x, solver.soft(b, lam) * nn ** 2 / n ** 2, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pfw_matches_coordinate_descent(seed):
    """T15: PFW and brute-force CD agree on objective (1e-9) and fit."""
    uv, n, fov, V = _problem(seed)
    res = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=0.9, **TIGHT)
    A = brute.explicit_matrix(uv, n, fov)
    y = np.concatenate([V.real, V.imag])
    x, obj, rel, _ = brute.lasso_cd(A, y, res.lam)
    assert abs(res.objective - obj) <= 1e-9 * obj
    fit_cd = A @ x
    fit_fw = np.concatenate([res.fit.real, res.fit.imag])
    assert np.linalg.norm(fit_fw - fit_cd) <= 1e-5 * np.linalg.norm(fit_cd)


def test_kkt_and_alpha_identity():
    """T11 + T12: ||mu||_inf <= 1 + 1e-6, mu = sign(x) on the support, and
    ||Phi*(V - Phi x)||_inf / ||Phi* V||_inf = alpha."""
    uv, n, fov, V = _problem(3, L=220, n=10)
    alpha = 0.08
    res = solver.pfw_solve(uv, n, fov, V, alpha=alpha, delta=0.9, **TIGHT)
    assert res.rel_gap <= 1e-12 and res.pix.size > 0
    mu = res.certificate.reshape(-1)
    assert np.max(np.abs(mu)) <= 1 + 1e-6
    assert np.allclose(mu[res.pix], np.sign(res.weight), atol=1e-6, rtol=0)
    # <mu, x> = ||x||_1 (Eq. dual-saturation1)
    assert abs(mu[res.pix] @ res.weight - np.abs(res.weight).sum()) <= 1e-6 * np.abs(res.weight).sum()
    assert abs(np.max(np.abs(res.eta)) / res.lambda_max - alpha) <= 1e-6 * alpha
    # certificate helper agrees with the solver's own final residual image
    mu2 = solver.certificate(uv, n, fov, V, res.pix, res.weight, res.lam)
    assert np.allclose(mu2.reshape(-1), mu, rtol=1e-10, atol=1e-10)


def test_hermitian_doubling():
    """T13: duplicating the conjugate half doubles P and lambda_max and keeps x."""
    uv, n, fov, V = _problem(4)
    r1 = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=0.9, **TIGHT)
    r2 = solver.pfw_solve(np.concatenate([uv, -uv]), n, fov, np.concatenate([V, V.conj()]),
                          alpha=0.1, delta=0.9, **TIGHT)
    assert abs(r2.lambda_max - 2 * r1.lambda_max) <= 1e-10 * r1.lambda_max
    assert abs(r2.objective - 2 * r1.objective) <= 1e-9 * r1.objective
    x1 = np.zeros(n * n); x1[r1.pix] = r1.weight
    x2 = np.zeros(n * n); x2[r2.pix] = r2.weight
    assert np.linalg.norm(x1 - x2) <= 1e-5 * np.linalg.norm(x1)


def test_lambda_above_lambda_max_gives_zero():
    """T14: alpha > 1 => empty support, P = ||V||^2/2, zero gap (Eq. lmax)."""
    uv, n, fov, V = _problem(5)
    res = solver.pfw_solve(uv, n, fov, V, alpha=1.0001, delta=0.9, max_iter=5,
                           rel_gap_tol=1e-12)
    assert res.pix.size == 0
    half = 0.5 * float(np.vdot(V, V).real)
    assert abs(res.objective - half) <= 1e-15 * half
    assert abs(res.rel_gap) <= 1e-14
    assert res.iters == 1 and res.converged


def test_delta_one_adds_only_the_argmax():
    """T16: delta = 1 => Delta = 0 => each exploration adds the argmax set."""
    uv, n, fov, V = _problem(6)
    dirty = operator.adjoint(uv, n, fov, V)
    res = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=1.0, max_iter=4)
    assert all(it.n_new == 1 for it in res.log)
    m, idx = solver.argmax_abs(dirty)
    # first iteration: the only atom is the dirty-image argmax
    r1 = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=1.0, max_iter=1)
    assert r1.pix.tolist() == [idx]


def test_exploration_band_size_grows_with_delta_gap():
    """Smaller delta admits at least as many candidates at k = 0."""
    uv, n, fov, V = _problem(7)
    a = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=0.99, max_iter=1)
    b = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=0.5, max_iter=1)
    assert b.log[0].n_new >= a.log[0].n_new


def test_objective_and_gap_helpers():
    uv, n, fov, V = _problem(8)
    p = solver.objective(V, np.zeros_like(V), np.zeros(0), 1.0)
    assert p == 0.5 * float(np.vdot(V, V).real)
    lmax = np.max(np.abs(operator.adjoint(uv, n, fov, V)))
    gap, dual = solver.dual_gap(V, V, lmax, p, lmax)
    assert abs(gap) <= 1e-12 * p


def test_stop_rules():
    uv, n, fov, V = _problem(9)
    r = solver.pfw_solve(uv, n, fov, V, alpha=0.05, delta=0.9, max_iter=3)
    assert r.iters == 3 and not r.converged
    r = solver.pfw_solve(uv, n, fov, V, alpha=0.05, delta=0.9, max_iter=100,
                         rel_obj_tol=1e-4)
    assert r.converged
    objs = [it.objective for it in r.log]
    assert abs(objs[-1] - objs[-2]) / objs[-2] <= 1e-4


# --- positivity (remarks on positivity in Sects. 4.1 and 5.1) ---------------

def _mixed_problem(seed, L=200, n=8, fov=0.25):
    """Sources of both signs, so that the positive solution differs from the
    unconstrained one and the dirty residual goes well below -lambda."""
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-12, 12, size=(L, 2))
    pix = rng.choice(n * n, 4, replace=False)
    amp = np.array([1.5, 1.0, -1.2, -0.8]) * np.exp(0.2 * rng.normal(size=4))
    V = operator.forward(uv, n, fov, pix, amp)
    V = V + 0.03 * np.max(np.abs(V)) * (rng.normal(size=L) + 1j * rng.normal(size=L))
    return uv, n, fov, V


def test_positive_prox():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    assert np.array_equal(solver.soft(z, 1.0, positive=True), [0.0, 0.0, 0.0, 0.0, 1.0])
    assert solver.dual_scale_norm(np.array([-5.0, 2.0]), positive=True) == 2.0
    assert solver.dual_scale_norm(np.array([-5.0, -2.0]), positive=True) == 0.0
    assert solver.dual_scale_norm(np.array([-5.0, 2.0])) == 5.0


def test_positive_cd_matches_bounded_quasi_newton():
    """The non-negative CD solver against scipy's L-BFGS-B on the smooth
    bound-constrained form (for x >= 0, lam ||x||_1 = lam sum x)."""
    from scipy.optimize import minimize
    uv, n, fov, V = _mixed_problem(31, L=120, n=6)
    A = brute.explicit_matrix(uv, n, fov)
    y = np.concatenate([V.real, V.imag])
    lam = 0.15 * float(np.max(A.T @ y))
    x, obj, rel, _ = brute.lasso_cd(A, y, lam, positive=True)
    assert np.all(x >= 0) and rel <= 1e-12

    def f(z):
        r = y - A @ z
        return 0.5 * r @ r + lam * z.sum(), -(A.T @ r) + lam

    q = minimize(f, np.zeros(A.shape[1]), jac=True, method="L-BFGS-B",
                 bounds=[(0, None)] * A.shape[1],
                 options=dict(ftol=1e-15, gtol=1e-12, maxiter=20000))
    assert abs(q.fun - obj) <= 1e-8 * obj
    assert np.linalg.norm(A @ q.x - A @ x) <= 1e-4 * np.linalg.norm(A @ x)


def test_positive_orthogonal_design_closed_form():
    """uv on the DFT frequencies => x_p = max((Phi*V)_p - lam, 0) n_p^2 / n^2
    (the one-sided threshold), for the PFW and the CD solvers alike."""
    n, fov = 8, 0.3
    uv = sim.orthogonal_uv(n, fov)
    rng = np.random.default_rng(13)
    V = rng.normal(size=uv.shape[0]) + 1j * rng.normal(size=uv.shape[0])
    b = operator.adjoint(uv, n, fov, V).reshape(-1)
    res = solver.pfw_solve(uv, n, fov, V, alpha=0.3, delta=0.5, positivity=True, **TIGHT)
    assert abs(res.lambda_max - np.max(b)) <= 1e-12 * np.max(b)
    nn = geometry.n_term(n, fov).reshape(-1)
    want = np.maximum(b - res.lam, 0.0) * nn ** 2 / n ** 2
    got = np.zeros(n * n)
    got[res.pix] = res.weight
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))
    assert np.array_equal(res.pix, np.flatnonzero(want))
    A = brute.explicit_matrix(uv, n, fov)
    x, _, _, _ = brute.lasso_cd(A, np.concatenate([V.real, V.imag]), res.lam, positive=True)
    assert np.allclose(x, want, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", [40, 41])
def test_positive_pfw_matches_coordinate_descent(seed):
    uv, n, fov, V = _mixed_problem(seed)
    res = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=0.9, positivity=True, **TIGHT)
    A = brute.explicit_matrix(uv, n, fov)
    y = np.concatenate([V.real, V.imag])
    x, obj, rel, _ = brute.lasso_cd(A, y, res.lam, positive=True)
    assert abs(res.objective - obj) <= 1e-9 * obj
    fit_cd = A @ x
    fit_fw = np.concatenate([res.fit.real, res.fit.imag])
    assert np.linalg.norm(fit_fw - fit_cd) <= 1e-5 * np.linalg.norm(fit_cd)
    # the constraint is active: the unconstrained optimum is lower
    free = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=0.9, lam=res.lam, **TIGHT)
    assert free.objective < res.objective * (1 - 1e-6)


def test_positive_one_sided_kkt():
    """x >= 0; mu <= 1 everywhere with mu = 1 on the support; mu is not
    bounded below (it goes below -1 at the negative sources); and
    max(eta) / lambda_max = alpha."""
    uv, n, fov, V = _mixed_problem(42, L=220, n=10)
    alpha = 0.08
    res = solver.pfw_solve(uv, n, fov, V, alpha=alpha, delta=0.9, positivity=True, **TIGHT)
    assert res.rel_gap <= 1e-12 and res.pix.size > 0
    assert np.all(res.weight > 0)
    mu = res.certificate.reshape(-1)
    assert np.max(mu) <= 1 + 1e-6
    assert np.allclose(mu[res.pix], 1.0, atol=1e-6, rtol=0)
    assert np.min(mu) < -1.0
    assert abs(np.max(res.eta) / res.lambda_max - alpha) <= 1e-6 * alpha


def test_positive_lambda_above_lambda_max_gives_zero():
    uv, n, fov, V = _mixed_problem(43)
    res = solver.pfw_solve(uv, n, fov, V, alpha=1.0001, delta=0.9, max_iter=5,
                           rel_gap_tol=1e-12, positivity=True)
    assert res.pix.size == 0 and res.converged
    dirty = operator.adjoint(uv, n, fov, V)
    assert abs(res.lambda_max - np.max(dirty)) <= 1e-14 * np.max(dirty)


def test_positive_exploration_takes_the_signed_maximum():
    """delta = 1 with positivity: the first atom is the argmax of the dirty
    image itself, even where its most negative value is larger in modulus."""
    rng = np.random.default_rng(44)
    n, fov, L = 8, 0.25, 160
    uv = rng.uniform(-12, 12, size=(L, 2))
    V = operator.forward(uv, n, fov, [10, 37], [0.6, -2.0])
    dirty = operator.adjoint(uv, n, fov, V).reshape(-1)
    assert -dirty.min() > dirty.max() > 0
    r1 = solver.pfw_solve(uv, n, fov, V, alpha=0.1, delta=1.0, max_iter=1, positivity=True)
    assert r1.pix.tolist() == [int(np.argmax(dirty))]
    assert r1.log[0].n_new == 1


def test_argmax_tie_rule_lowest_flat_index():
    """The certificate / dirty-image peak rule (reading R15): the largest
    |value| wins and, among exact ties, the lowest flat index; the sign does
    not break a tie.  Hand-built images whose answer is read off by eye."""
    img = np.zeros((4, 4))
    img[1, 1] = -3.0          # flat 5
    img[0, 2] = 2.9999999     # flat 2: smaller, earlier
    img[3, 0] = 3.0           # flat 12: ties with flat 5
    assert solver.argmax_abs(img) == (3.0, 5)
    img[0, 3] = 3.0           # flat 3 now ties too and comes first
    assert solver.argmax_abs(img) == (3.0, 3)
    assert solver.argmax_abs(np.zeros((8, 8))) == (0.0, 0)   # every pixel ties
    assert solver.argmax_abs(-np.ones(7)) == (1.0, 0)


def test_argmax_tie_of_a_zero_residual_certificate():
    """An exact tie reached through the operator: visibilities equal to the
    model's own forward leave a zero residual, so the certificate is zero
    everywhere and the peak is flat index 0."""
    uv, n, fov, _ = _problem(8)
    pix = np.array([3, n * n // 2 + 7])
    w = np.array([1.5, -0.25])
    V = operator.forward(uv, n, fov, pix, w)
    mu = solver.certificate(uv, n, fov, V, pix, w, lam=0.3)
    assert np.all(mu == 0.0)
    assert solver.argmax_abs(mu) == (0.0, 0)


def _problem_w(seed, L=160, n=8, fov=0.5, n_src=3, noise=0.05):
    """The same recipe with non-coplanar baselines: w as large as u and v, so
    that the w-term phase w (n - 1) reaches a sizeable fraction of a turn."""
    rng = np.random.default_rng(100 + seed)
    uvw = rng.uniform(-12, 12, size=(L, 3))
    uvw[:, 2] *= 4.0
    pix = rng.choice(n * n, n_src, replace=False)
    amp = np.exp(rng.normal(size=n_src))
    V = operator.forward(uvw, n, fov, pix, amp)
    V = V + noise * np.max(np.abs(V)) * (rng.normal(size=L) + 1j * rng.normal(size=L))
    return uvw, n, fov, V


def test_explicit_matrix_with_w_is_the_forward_operator():
    """The explicit 2L x N matrix reproduces the (pinned) oracle forward with
    w column by column, and differs from the coplanar matrix."""
    uvw, n, fov, _ = _problem_w(0)
    A = brute.explicit_matrix(uvw, n, fov)
    rng = np.random.default_rng(7)
    x = rng.normal(size=n * n)
    V = operator.forward(uvw, n, fov, np.arange(n * n), x)
    assert np.allclose(A @ x, np.concatenate([V.real, V.imag]), rtol=0, atol=1e-11 * np.abs(V).max())
    A0 = brute.explicit_matrix(uvw[:, :2], n, fov)
    assert np.linalg.norm(A - A0) > 0.1 * np.linalg.norm(A0)


@pytest.mark.parametrize("seed", [0, 1])
def test_pfw_matches_coordinate_descent_with_w(seed):
    """T15 with the w-term: the Frank-Wolfe route (Gram columns with the w
    phase) and coordinate descent on the explicit matrix agree."""
    uvw, n, fov, V = _problem_w(seed)
    res = solver.pfw_solve(uvw, n, fov, V, alpha=0.1, delta=0.9, **TIGHT)
    A = brute.explicit_matrix(uvw, n, fov)
    y = np.concatenate([V.real, V.imag])
    x, obj, rel, _ = brute.lasso_cd(A, y, res.lam)
    assert abs(res.objective - obj) <= 1e-9 * obj
    fit_fw = np.concatenate([res.fit.real, res.fit.imag])
    assert np.linalg.norm(fit_fw - A @ x) <= 1e-5 * np.linalg.norm(A @ x)
