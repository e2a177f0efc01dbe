"""GPU PolyCLEAN solve against the FP64 oracle's solve (Alg. 2).

LASSO minimisers may be non-unique, but the fit Phi x and the certificate are
unique (Sect. 4.2), so parity is asserted on the objective (1e-3 relative at
termination), the fit and the certificate (1e-4 relative L2 when both sides
are converged), and on the certificate peak: identical argmax for the dirty
image; at termination the GPU argmax must lie in the oracle's saturation set
{|mu| >= 1 - 1e-3} (the peak is a near-tie over the whole support there).
"""
import numpy as np
import pytest

import sim
from oracle import geometry, operator, solver
from tests.gpu_util import api, problem, rel_l2, say, to_dev, torch

pytestmark = pytest.mark.gpu


def _gpu_solve(p, vis, cap=65536, **kw):
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    cert = torch.empty((p.npix, p.npix), dtype=torch.float32, device="cuda")
    res = a.pc_polyclean_solve(plan, to_dev(vis), capacity=cap, cert=cert, want_certificate=1, **kw)
    return plan, res, cert.cpu().numpy().astype(np.float64)


def _oracle_solve(p, vis, **kw):
    return solver.pfw_solve(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128), **kw)


def _fit(p, pix, w):
    return operator.forward(p.uv, p.npix, p.fov_rad, pix, w)


# APGD and Lanczos in Gram form (default for direct sets up to 256 atoms),
# through the operators (gram_atoms < 0), and both within one solve (cap 8)
GRAM_MODES = [0, -1, 8]


@pytest.mark.parametrize("gram", GRAM_MODES)
def test_solve_c1_converged_matches_oracle(gram):
    """C1 run to a relative gap of 1e-5 on both sides (the FP32 residual floors the
    GPU gap near 5e-6): objective, fit, certificate."""
    say("solve c1 converged, gram_atoms", gram)
    p, vis = problem("c1")
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=300, rel_gap_tol=1e-5)
    plan, res, cert = _gpu_solve(p, vis, gram_atoms=gram, **kw)
    ref = _oracle_solve(p, vis, **kw)
    say("gpu", res["objective"], res["rel_gap"], res["iters"], res["natoms"],
        "oracle", ref.objective, ref.rel_gap, ref.iters, ref.pix.size)
    assert res["status"] == 0 and res["converged"] == 1
    assert abs(res["objective"] - ref.objective) <= 1e-3 * ref.objective
    assert abs(res["lambda_max"] - ref.lambda_max) <= 1e-4 * ref.lambda_max
    fit = _fit(p, res["pix"], res["weight"])
    assert rel_l2(fit, ref.fit) <= 1e-3
    assert rel_l2(cert, ref.certificate) <= 1e-3
    mu = np.abs(ref.certificate).reshape(-1)
    assert mu[res["cert_argmax"]] >= 1 - 1e-3
    # the objective the GPU reports is the objective of the x it returns
    p_or = solver.objective(vis.astype(np.complex128), fit, res["weight"], res["lambda"])
    assert abs(p_or - res["objective"]) <= 1e-5 * p_or
    # its certificate is the oracle's certificate of that x (T17, 1e-4)
    mu_x = solver.certificate(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128), res["pix"],
                              res["weight"], res["lambda"])
    assert rel_l2(cert, mu_x) <= 1e-4


def test_solve_c1_fifty_iterations():
    """The workload as specified: alpha 0.01, 50 FW iterations."""
    say("solve c1 50 iterations")
    p, vis = problem("c1")
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=50)
    plan, res, cert = _gpu_solve(p, vis, **kw)
    ref = _oracle_solve(p, vis, **kw)
    say("gpu", res["objective"], res["rel_gap"], res["iters"], "oracle", ref.objective, ref.rel_gap)
    assert res["iters"] <= 50
    assert abs(res["objective"] - ref.objective) <= 1e-3 * ref.objective
    mu = np.abs(ref.certificate).reshape(-1)
    assert mu[res["cert_argmax"]] >= 1 - 1e-3


@pytest.mark.parametrize("gram", GRAM_MODES)
def test_solve_c2_small_gap_stop(gram):
    say("solve c2_small, gram_atoms", gram)
    p, vis = problem("c2_small")
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=200, rel_gap_tol=1e-4)
    plan, res, cert = _gpu_solve(p, vis, gram_atoms=gram, **kw)
    ref = _oracle_solve(p, vis, **kw)
    say("gpu", res["objective"], res["rel_gap"], res["iters"], res["natoms"],
        "oracle", ref.objective, ref.rel_gap, ref.iters, ref.pix.size)
    assert res["converged"] == 1 and res["rel_gap"] <= 1e-4
    assert abs(res["objective"] - ref.objective) <= 1e-3 * ref.objective
    mu = np.abs(ref.certificate).reshape(-1)
    assert mu[res["cert_argmax"]] >= 1 - 1e-3
    assert res["cert_max"] <= 1 + 1e-3
    mu_x = solver.certificate(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128), res["pix"],
                              res["weight"], res["lambda"])
    assert rel_l2(cert, mu_x) <= 1e-4


def test_gram_form_follows_the_operator_form():
    """With the stopping rules off (12 FW iterations, at most 5 APGD steps
    each; the restricted gap test can still stop a step once the computed
    gap reaches zero) the Gram form and the operator form take the same
    trajectory up to FP32 operator rounding: equal objective to 1e-6."""
    say("gram vs operator form, fixed steps")
    p, vis = problem("c2_small")
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=12, rel_obj_tol=0.0, rel_gap_tol=0.0,
              inner_max_iter=5, inner_tol0=0.0, inner_tol_min=1e-300)
    _, rg, _ = _gpu_solve(p, vis, gram_atoms=0, **kw)
    _, ro, _ = _gpu_solve(p, vis, gram_atoms=-1, **kw)
    say("gram", rg["objective"], rg["inner_iters"], rg["natoms"],
        "operator", ro["objective"], ro["inner_iters"], ro["natoms"])
    assert rg["iters"] == ro["iters"] == 12
    assert 12 <= rg["inner_iters"] <= 12 * 5 and 12 <= ro["inner_iters"] <= 12 * 5
    assert abs(rg["objective"] - ro["objective"]) <= 1e-6 * ro["objective"]
    assert abs(rg["natoms"] - ro["natoms"]) <= 2


@pytest.mark.parametrize("name,grid_atoms", [("c1", 1), ("c1", 8), ("c2_small", 4)])
def test_solve_gridded_apgd_matches_oracle(name, grid_atoms):
    """Active sets above the crossover apply Phi_S and Phi_S* through the
    gridded operators (type 2 / type 1, pass B evaluated at the set) inside
    APGD and for the per-iteration residual.  Forced low here so that the
    whole solve runs that way; the result must still match the direct
    oracle."""
    say("solve gridded", name, grid_atoms)
    p, vis = problem(name)
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=300, rel_gap_tol=1e-4)
    plan, res, cert = _gpu_solve(p, vis, grid_atoms=grid_atoms, **kw)
    ref = _oracle_solve(p, vis, **kw)
    say("gpu", res["objective"], res["rel_gap"], res["iters"], res["natoms"],
        "oracle", ref.objective, ref.rel_gap, ref.iters, ref.pix.size)
    assert res["converged"] == 1 and res["rel_gap"] <= 1e-4
    assert abs(res["objective"] - ref.objective) <= 1e-3 * ref.objective
    fit = _fit(p, res["pix"], res["weight"])
    assert rel_l2(fit, ref.fit) <= 1e-2
    mu = np.abs(ref.certificate).reshape(-1)
    assert mu[res["cert_argmax"]] >= 1 - 1e-3
    assert res["cert_max"] <= 1 + 1e-3
    # the reported objective is that of the returned x (exact forward)
    p_or = solver.objective(vis.astype(np.complex128), fit, res["weight"], res["lambda"])
    assert abs(p_or - res["objective"]) <= 1e-4 * p_or


def test_gridded_solve_at_a_large_grid_matches_the_direct_solve():
    """A 4096^2 image (8192^2 fine grid: the pass-A buffer's 4-column blocks
    and the direct pass B at the set's rows and pixels), 30,000 random
    visibilities of 25 point sources: the solve with every restricted
    operator gridded (crossover 1) against the solve with direct sums only;
    objectives within 1e-3, and the gridded solve's reported objective equal
    to the oracle's evaluation of its returned x."""
    a = api()
    rng = np.random.default_rng(77)
    n, fov, L = 4096, 0.05, 30000
    d = fov / n
    uv = rng.uniform(-0.45 / d, 0.45 / d, size=(L, 2))
    pix = rng.choice(n * n, 25, replace=False)
    amp = rng.lognormal(size=25) * 10.0
    clean = operator.forward(uv, n, fov, pix, amp)
    vis = (clean + 0.05 * np.sqrt(np.mean(np.abs(clean) ** 2)) *
           (rng.normal(size=L) + 1j * rng.normal(size=L)) / np.sqrt(2)).astype(np.complex64)
    plan = a.pc_plan_create(uv, n, fov)
    assert plan.info["fine"] == 8192
    kw = dict(alpha=0.05, delta=0.99, max_iter=12, rel_gap_tol=1e-4, gram_atoms=-1, capacity=4096)
    dv = to_dev(vis)
    rg = a.pc_polyclean_solve(plan, dv, grid_atoms=1, **kw)
    rd = a.pc_polyclean_solve(plan, dv, grid_atoms=-1, **kw)
    say("gridded", rg["objective"], rg["iters"], rg["natoms"], "direct", rd["objective"],
        rd["iters"], rd["natoms"])
    assert abs(rg["objective"] - rd["objective"]) <= 1e-3 * rd["objective"]
    fit = operator.forward(uv, n, fov, rg["pix"], rg["weight"])
    p_or = solver.objective(vis.astype(np.complex128), fit, rg["weight"], rg["lambda"])
    assert abs(p_or - rg["objective"]) <= 1e-4 * p_or


def test_solve_orthogonal_design_closed_form():
    """uv on the DFT frequencies: x_p = soft((Phi* V)_p, lam) n_p^2 / n^2."""
    say("solve orthogonal")
    n, fov = 32, 0.3
    uv = sim.orthogonal_uv(n, fov)
    rng = np.random.default_rng(21)
    V = (rng.normal(size=uv.shape[0]) + 1j * rng.normal(size=uv.shape[0])).astype(np.complex64)
    a = api()
    plan = a.pc_plan_create(uv, n, fov)
    res = a.pc_polyclean_solve(plan, to_dev(V), alpha=0.5, delta=0.5, max_iter=100,
                               rel_gap_tol=1e-7)
    b = operator.adjoint(uv, n, fov, V.astype(np.complex128)).reshape(-1)
    nn = geometry.n_term(n, fov).reshape(-1)
    want = solver.soft(b, res["lambda"]) * nn ** 2 / n ** 2
    got = np.zeros(n * n)
    got[res["pix"]] = res["weight"]
    assert rel_l2(got, want) <= 1e-4
    assert set(res["pix"].tolist()) == set(np.flatnonzero(want).tolist())


def test_solve_lambda_above_lambda_max():
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    res = a.pc_polyclean_solve(plan, to_dev(vis), alpha=1.0001, delta=0.9, max_iter=5,
                               rel_gap_tol=1e-9)
    assert res["natoms"] == 0 and res["converged"] == 1 and res["iters"] == 1
    half = 0.5 * float(np.vdot(vis.astype(np.complex128), vis.astype(np.complex128)).real)
    assert abs(res["objective"] - half) <= 1e-6 * half


def test_step_api_equals_one_shot():
    import ctypes as C
    say("solver step api")
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    prm = a.solve_params(alpha=p.alpha, delta=p.delta, max_iter=20)
    one = a.pc_polyclean_solve(plan, to_dev(vis), params=prm)
    h = C.c_void_p()
    dv = to_dev(vis)
    stream = torch.cuda.current_stream().cuda_stream
    a.check(a.LIB.pc_solver_create(plan.handle, C.c_void_p(dv.data_ptr()), C.byref(prm),
                                   C.c_void_p(stream), C.byref(h)), "pc_solver_create")
    done = C.c_int32(0)
    steps = 0
    while not done.value:
        a.check(a.LIB.pc_solver_step(h, C.byref(done)), "pc_solver_step")
        steps += 1
    res = a.PcSolveResult()
    pix = np.zeros(65536, np.int32)
    w = np.zeros(65536)
    res.capacity = 65536
    res.pix = pix.ctypes.data_as(C.POINTER(C.c_int32))
    res.weight = w.ctypes.data_as(C.POINTER(C.c_double))
    a.check(a.LIB.pc_solver_result(h, C.byref(res)), "pc_solver_result")
    a.LIB.pc_solver_destroy(h)
    # the same algorithm through the same deterministic kernels (the gridding
    # adds every cell's terms in a fixed order, without atomics)
    assert steps == res.iters
    assert abs(res.objective - one["objective"]) <= 1e-6 * one["objective"]


def test_capacity_error_reports_required_size():
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    with pytest.raises(a.PolycleanError) as e:
        a.pc_polyclean_solve(plan, to_dev(vis), capacity=1, alpha=p.alpha, delta=p.delta,
                             max_iter=10)
    assert e.value.status == -4


def _mixed_sign_c1():
    """C1's array and sky with its second-brightest-listed source negated:
    the positive solution then differs widely from the unconstrained one and
    the certificate goes far below -1 there."""
    p, _ = problem("c1")
    amp = p.sky_amp.copy()
    amp[1] = -amp[1]
    vclean = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, amp)
    return p, sim.add_noise(vclean, p.noise, p.psnr_db).astype(np.complex64)


def _check_positive(p, vis, res, cert, ref, fit_tol=1e-3):
    assert res["converged"] == 1
    assert abs(res["objective"] - ref.objective) <= 1e-3 * ref.objective
    assert abs(res["lambda_max"] - ref.lambda_max) <= 1e-4 * ref.lambda_max
    assert np.all(res["weight"] > 0)
    fit = _fit(p, res["pix"], res["weight"])
    assert rel_l2(fit, ref.fit) <= fit_tol
    assert rel_l2(cert, ref.certificate) <= fit_tol
    # one-sided: max mu = 1 (to 1e-3), reached on the oracle's saturation set
    mu = ref.certificate.reshape(-1)
    assert res["cert_max"] <= 1 + 1e-3 and res["cert_max"] >= 1 - 1e-3
    assert mu[res["cert_argmax"]] >= 1 - 1e-3
    p_or = solver.objective(vis.astype(np.complex128), fit, res["weight"], res["lambda"])
    assert abs(p_or - res["objective"]) <= 1e-4 * p_or


@pytest.mark.parametrize("gram", [0, -1])
@pytest.mark.parametrize("mixed", [False, True])
def test_positive_solve_c1_matches_oracle(gram, mixed):
    """Positivity-constrained solve (remarks on positivity, Sects. 4.1 and
    5.1) against the oracle's, on C1's sky and on a mixed-sign sky."""
    say("positive solve c1, mixed", mixed, "gram_atoms", gram)
    p, vis = _mixed_sign_c1() if mixed else problem("c1")
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=300, rel_gap_tol=1e-5)
    plan, res, cert = _gpu_solve(p, vis, gram_atoms=gram, positivity=1, **kw)
    ref = _oracle_solve(p, vis, positivity=True, **kw)
    say("gpu", res["objective"], res["rel_gap"], res["iters"], res["natoms"],
        "oracle", ref.objective, ref.rel_gap, ref.iters, ref.pix.size)
    _check_positive(p, vis, res, cert, ref)
    # the constraint is active in both: mu < -1 somewhere, and the
    # unconstrained optimum is lower
    assert ref.certificate.min() < -1.0 and cert.min() < -1.0
    free = _oracle_solve(p, vis, lam=ref.lam, **kw)
    assert free.objective < ref.objective * (1 - 1e-4)


def test_positive_solve_gridded_apgd_matches_oracle():
    say("positive solve gridded")
    p, vis = _mixed_sign_c1()
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=300, rel_gap_tol=1e-4)
    plan, res, cert = _gpu_solve(p, vis, grid_atoms=8, positivity=1, **kw)
    ref = _oracle_solve(p, vis, positivity=True, **kw)
    say("gpu", res["objective"], res["rel_gap"], res["iters"], res["natoms"],
        "oracle", ref.objective, ref.rel_gap, ref.iters, ref.pix.size)
    _check_positive(p, vis, res, cert, ref, fit_tol=1e-2)


def test_positive_solve_orthogonal_closed_form():
    """uv on the DFT frequencies: x_p = max((Phi* V)_p - lam, 0) n_p^2 / n^2."""
    say("positive solve orthogonal")
    n, fov = 32, 0.3
    uv = sim.orthogonal_uv(n, fov)
    rng = np.random.default_rng(22)
    V = (rng.normal(size=uv.shape[0]) + 1j * rng.normal(size=uv.shape[0])).astype(np.complex64)
    a = api()
    plan = a.pc_plan_create(uv, n, fov)
    res = a.pc_polyclean_solve(plan, to_dev(V), alpha=0.5, delta=0.5, max_iter=100,
                               rel_gap_tol=1e-7, positivity=1)
    b = operator.adjoint(uv, n, fov, V.astype(np.complex128)).reshape(-1)
    assert abs(res["lambda_max"] - b.max()) <= 1e-4 * b.max()  # FP32 gridded adjoint
    nn = geometry.n_term(n, fov).reshape(-1)
    want = np.maximum(b - res["lambda"], 0.0) * nn ** 2 / n ** 2
    got = np.zeros(n * n)
    got[res["pix"]] = res["weight"]
    assert rel_l2(got, want) <= 1e-4
    assert set(res["pix"].tolist()) == set(np.flatnonzero(want).tolist())


def test_positive_flag_is_scoped_to_the_solve():
    """After a positive solve the plan's adjoint reports max |eta| again
    (visibilities negated, so that the dirty image's peak is negative)."""
    p, vis = problem("c1")
    vis = -vis
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    a.pc_polyclean_solve(plan, to_dev(vis), alpha=p.alpha, delta=p.delta, max_iter=3,
                         positivity=1)
    img, mx, am = a.pc_adjoint_grid(plan, to_dev(vis))
    dirty = np.abs(img.cpu().numpy()).reshape(-1)
    assert dirty.max() > 1.05 * img.cpu().numpy().max()  # the peak is negative here
    assert mx == float(dirty.max()) and am == int(np.argmax(dirty))


def _oracle_check_solution(p, vis, res, cert, positive=False):
    """The oracle's view of the GPU's returned x at full size: one exact
    adjoint of V - Phi x gives the certificate (compared over the whole image,
    relative L2 1e-4, T17) and the exact duality gap (rel gap <= 1e-3 bounds
    the objective within 1e-3 of the optimum); the GPU's reported objective is
    that of its x."""
    n = p.npix
    v128 = vis.astype(np.complex128)
    fit = operator.forward(p.uv, n, p.fov_rad, res["pix"], res["weight"])
    resid = v128 - fit
    eta = operator.adjoint(p.uv, n, p.fov_rad, resid)
    mu = eta / res["lambda"]
    err = rel_l2(cert, mu)
    p_or = solver.objective(v128, fit, res["weight"], res["lambda"])
    gap, _ = solver.dual_gap(v128, resid, solver.dual_scale_norm(eta, positive), p_or,
                             res["lambda"])
    say("oracle check: cert rel L2", err, "oracle rel gap", gap / p_or, "gpu rel gap",
        res["rel_gap"])
    assert err <= 1e-4
    assert gap / p_or <= 1e-3
    assert abs(p_or - res["objective"]) <= 1e-5 * p_or
    return mu


@pytest.mark.slow
def test_solve_full_c2_properties():
    """Full LOFAR-like solve: the gap stop fires, the certificate is at most
    one (to 1e-3), the alpha identity holds; the oracle's exact duality gap
    of the returned x is within 1e-3 and the GPU certificate equals the
    oracle's certificate of that x over the whole image (1e-4)."""
    say("solve full c2")
    p, vis = problem("c2")
    plan, res, cert = _gpu_solve(p, vis, alpha=p.alpha, delta=p.delta, max_iter=200,
                                 rel_gap_tol=1e-4)
    say("full c2", {k: res[k] for k in ("objective", "rel_gap", "iters", "natoms", "inner_iters",
                                         "seconds", "adjoint_seconds", "adjoint_calls")})
    assert res["converged"] == 1 and res["rel_gap"] <= 1e-4
    assert res["cert_max"] <= 1 + 1e-3
    assert abs(res["cert_max"] * res["lambda"] / res["lambda_max"] - p.alpha) <= 2e-3 * p.alpha
    mu = _oracle_check_solution(p, vis, res, cert)
    assert abs(mu.reshape(-1)[res["cert_argmax"]]) >= 1 - 1e-3


@pytest.mark.slow
def test_positive_solve_full_c2_properties():
    """Full LOFAR-like size with a third of the sources negated, so that the
    constraint is active: the gap stop fires, the weights are positive, the
    certificate is at most one with its maximum at lambda (the one-sided alpha
    identity) and well below -1 at the negated sources; the oracle's exact
    one-sided duality gap of the returned x is within 1e-3 and the whole
    certificate matches the oracle's (1e-4)."""
    say("positive solve full c2, mixed signs")
    p = sim.config_c2()
    amp = p.sky_amp * np.where(np.arange(p.sky_amp.size) % 3 == 1, -1.0, 1.0)
    vclean = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, amp)
    vis = sim.add_noise(vclean, p.noise, p.psnr_db).astype(np.complex64)
    plan, res, cert = _gpu_solve(p, vis, alpha=p.alpha, delta=p.delta, max_iter=2000,
                                 rel_gap_tol=1e-4, positivity=1)
    say("positive full c2", {k: res[k] for k in ("objective", "rel_gap", "iters", "natoms",
                                                  "inner_iters", "seconds")})
    assert res["converged"] == 1 and res["rel_gap"] <= 1e-4
    assert np.all(res["weight"] > 0)
    assert res["cert_max"] <= 1 + 1e-3 and cert.max() <= 1 + 1e-3
    assert abs(res["cert_max"] * res["lambda"] / res["lambda_max"] - p.alpha) <= 2e-3 * p.alpha
    assert cert.min() < -1.0
    mu = _oracle_check_solution(p, vis, res, cert, positive=True)
    assert mu.reshape(-1)[res["cert_argmax"]] >= 1 - 1e-3


def test_warm_start_from_the_solution_and_from_a_perturbed_point():
    """x0 (an interface option of the solve): from the converged solution the
    gap test passes at once (no FW iteration, same objective: the operators
    are deterministic); from a perturbed point (weights halved, stray atoms
    added) the solve reaches the oracle's objective."""
    say("warm start")
    p, vis = problem("c1")
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=300, rel_gap_tol=1e-5)
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    dv = to_dev(vis)
    cold = a.pc_polyclean_solve(plan, dv, **kw)
    warm = a.pc_polyclean_solve(plan, dv, x0=(cold["pix"], cold["weight"]), **kw)
    say("cold", cold["iters"], cold["objective"], "warm", warm["iters"], warm["objective"])
    assert warm["converged"] == 1 and warm["iters"] == 0
    assert warm["objective"] == cold["objective"] and warm["rel_gap"] == cold["rel_gap"]
    np.testing.assert_array_equal(warm["pix"], cold["pix"])
    assert warm["lambda_max"] == cold["lambda_max"]
    rng = np.random.default_rng(5)
    extra = np.setdiff1d(rng.choice(p.npix ** 2, 12, replace=False), cold["pix"])
    pix = np.concatenate([cold["pix"], extra])
    w = np.concatenate([0.5 * cold["weight"], rng.normal(size=extra.size)])
    pert = a.pc_polyclean_solve(plan, dv, x0=(pix, w), **kw)
    ref = _oracle_solve(p, vis, **kw)
    say("perturbed", pert["iters"], pert["objective"], "oracle", ref.objective)
    assert pert["converged"] == 1
    assert abs(pert["objective"] - ref.objective) <= 1e-3 * ref.objective
    # the stray atoms are pruned again (their weights end at zero or move)
    assert abs(pert["natoms"] - ref.pix.size) <= max(3, ref.pix.size // 10)


@pytest.mark.parametrize("case", ["range", "negative-index", "duplicate", "nan", "negative-positive"])
def test_warm_start_rejects_bad_atoms(case):
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    N = p.npix ** 2
    pix, w, extra = {"range": ([0, N], [1.0, 1.0], {}),
                     "negative-index": ([-1], [1.0], {}),
                     "duplicate": ([5, 5], [1.0, 2.0], {}),
                     "nan": ([5], [float("nan")], {}),
                     "negative-positive": ([5], [-1.0], {"positivity": 1})}[case]
    with pytest.raises(a.PolycleanError) as e:
        a.pc_polyclean_solve(plan, to_dev(vis), x0=(pix, w), max_iter=2, **extra)
    assert e.value.status == -1
