"""GPU synthesis-dictionary path (Sect. 4.3, Eq. lasso-synthesis; the Gaussian
elements of Sect. 6.4) against the FP64 oracle: the adjoint Psi* Phi* for
every scale, and the synthesis-form solve (objective, fit, certificate over
all scales, lambda_max = ||Psi* Phi* V||_inf), with and without positivity."""
import numpy as np
import pytest

import sim
from oracle import dictionary as dic, operator, solver
from tests.gpu_util import api, problem, ragged_problem, rel_l2, say, to_dev, torch

pytestmark = pytest.mark.gpu

PAPER = (list(dic.PAPER_SIGMAS), [1.2 ** s for s in range(4)])
STEEP = (list(dic.PAPER_SIGMAS), [2.0 ** s for s in range(4)])  # favours wide elements


def _diffuse(n=32):
    p = sim.config_diffuse(npix=n)
    vc = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, p.sky_amp)
    return p, sim.add_noise(vc, p.noise, p.psnr_db).astype(np.complex64)


def _case(name):
    if name == "ragged":
        uv, n, fov, h = ragged_problem()
        return uv, n, fov, h
    p, vis = _diffuse(32) if name == "diffuse32" else (_diffuse(64) if name == "diffuse64"
                                                      else problem(name))
    return p.uv, p.npix, p.fov_rad, vis


WIDE = ([0.0, 12.0, 16.0], [1.0, 1.5, 2.0])  # half-widths 24 and 32: the generic tile kernel


@pytest.mark.parametrize("name,scales", [("diffuse32", PAPER), ("diffuse64", PAPER),
                                         ("c1", PAPER), ("ragged", PAPER), ("c1", WIDE)],
                         ids=["diffuse32", "diffuse64", "c1", "ragged", "c1-wide"])
def test_adjoint_grid_ms_matches_oracle(name, scales):
    """Psi* Phi* h per scale (elements up to 65 x 65, cropped at the border
    of 32^2 to 128^2 images); maximum and its index over all scales."""
    say("adjoint ms", name, scales)
    uv, n, fov, h = _case(name)
    a = api()
    plan = a.pc_plan_create(uv, n, fov)
    img, mx, am = a.pc_adjoint_grid_ms(plan, to_dev(h), *scales)
    got = img.cpu().numpy().astype(np.float64)
    want = dic.analysis(operator.adjoint(uv, n, fov, h.astype(np.complex128)),
                        dic.gaussian_dictionary(*scales))
    errs = [rel_l2(got[s], want[s]) for s in range(len(scales[0]))]
    say("rel l2 per scale", errs)
    assert max(errs) <= 1e-4
    wmax = np.abs(want).max()
    assert abs(mx - wmax) <= 1e-4 * wmax
    assert abs(want.reshape(-1)[am]) >= (1 - 1e-4) * wmax
    assert abs(abs(got.reshape(-1)[am]) - mx) <= 1e-6 * mx


def _gpu_solve(p, vis, scales, **kw):
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    S = len(scales[0])
    cert = torch.empty((S, p.npix, p.npix), dtype=torch.float32, device="cuda")
    res = a.pc_polyclean_solve(plan, to_dev(vis), capacity=1 << 16, cert=cert,
                               want_certificate=1, scales=scales, **kw)
    return res, cert.cpu().numpy().astype(np.float64)


def _fit(p, d, atoms, w):
    img = dic.synthesis(atoms, w, d, p.npix).reshape(-1)
    nz = np.flatnonzero(img)
    return operator.forward(p.uv, p.npix, p.fov_rad, nz, img[nz])


@pytest.mark.parametrize("scales,positive", [(PAPER, False), (STEEP, False), (STEEP, True)],
                         ids=["paper", "steep", "steep-positive"])
def test_dictionary_solve_matches_oracle(scales, positive):
    say("dictionary solve", scales[1], "positive", positive)
    p, vis = _diffuse(32)
    d = dic.gaussian_dictionary(*scales)
    kw = dict(alpha=0.05, delta=0.99, max_iter=300, rel_gap_tol=1e-4)
    res, cert = _gpu_solve(p, vis, scales, positivity=int(positive), **kw)
    ref = solver.pfw_solve(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128), dictionary=d,
                           positivity=positive, **kw)
    N = p.npix ** 2
    say("gpu", res["objective"], res["rel_gap"], res["iters"], res["natoms"],
        np.bincount(res["pix"] // N, minlength=4),
        "oracle", ref.objective, ref.rel_gap, ref.iters, ref.pix.size,
        np.bincount(ref.pix // N, minlength=4))
    assert res["converged"] == 1 and ref.converged
    assert abs(res["lambda_max"] - ref.lambda_max) <= 1e-4 * ref.lambda_max
    assert abs(res["objective"] - ref.objective) <= 1e-3 * ref.objective
    assert np.all(res["pix"] < 4 * N) and np.any(res["pix"] >= N)  # wide elements used
    fit = _fit(p, d, res["pix"], res["weight"])
    # P(x) - P* >= 1/2 ||Phi Psi (x - x*)||^2 (the data term is 1-strongly
    # convex in the fit and 0 is a subgradient of P at x*), so each fit lies
    # within sqrt(2 gap) of the unique optimal fit; plus FP32 operator rounding
    bound = (np.sqrt(2 * res["rel_gap"] * res["objective"]) +
             np.sqrt(2 * ref.rel_gap * ref.objective) + 1e-4 * np.linalg.norm(ref.fit))
    say("fit distance", np.linalg.norm(fit - ref.fit), "bound", bound,
        "cert rel", rel_l2(cert, ref.certificate))
    assert np.linalg.norm(fit - ref.fit) <= bound
    assert rel_l2(cert, ref.certificate) <= 1e-2
    if positive:
        assert np.all(res["weight"] > 0)
        assert res["cert_max"] <= 1 + 1e-3 and cert.max() <= 1 + 1e-3
    else:
        assert res["cert_max"] <= 1 + 1e-3 and np.abs(cert).max() <= 1 + 1e-3
    # the reported objective is that of the returned coefficients
    p_or = solver.objective(vis.astype(np.complex128), fit, res["weight"], res["lambda"])
    assert abs(p_or - res["objective"]) <= 1e-4 * p_or
    # the certificate of the returned coefficients is the oracle's for them:
    # Psi* Phi* (V - Phi Psi x) / lambda over every scale (T17, 1e-4)
    eta = operator.adjoint(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128) - fit)
    mu_x = dic.analysis(eta, d) / res["lambda"]
    assert rel_l2(cert, mu_x) <= 1e-4


def test_point_scale_dictionary_equals_plain_solve():
    """One scale, sigma 0, gamma 1: the synthesis form is the plain LASSO
    (solved here through the gridded operators)."""
    p, vis = problem("c1")
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=300, rel_gap_tol=1e-5)
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    plain = a.pc_polyclean_solve(plan, to_dev(vis), **kw)
    one = a.pc_polyclean_solve(plan, to_dev(vis), scales=([0.0], [1.0]), **kw)
    say("plain", plain["objective"], plain["natoms"], "one scale", one["objective"], one["natoms"])
    assert abs(one["lambda_max"] - plain["lambda_max"]) <= 1e-6 * plain["lambda_max"]
    assert abs(one["objective"] - plain["objective"]) <= 1e-4 * plain["objective"]


@pytest.mark.parametrize("sig,gam", [([17.0], [1.0]), ([2.0], [0.0]), ([-1.0], [1.0]),
                                     ([0.0] * 9, [1.0] * 9)])
def test_dictionary_rejects_bad_scales(sig, gam):
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    with pytest.raises((a.PolycleanError, ValueError)):
        a.pc_polyclean_solve(plan, to_dev(vis), scales=(sig, gam), max_iter=2)
    if len(sig) <= 8:
        with pytest.raises(a.PolycleanError):
            a.pc_adjoint_grid_ms(plan, to_dev(vis), sig, gam)


def test_dictionary_lambda_above_lambda_max_gives_zero():
    p, vis = _diffuse(32)
    res, cert = _gpu_solve(p, vis, PAPER, alpha=1.0001, delta=0.9, max_iter=5,
                           rel_gap_tol=1e-9)
    want = np.abs(dic.analysis(operator.adjoint(p.uv, p.npix, p.fov_rad,
                                                 vis.astype(np.complex128)),
                               dic.gaussian_dictionary(*PAPER))).max()
    assert res["natoms"] == 0 and res["converged"] == 1 and res["iters"] == 1
    assert abs(res["lambda_max"] - want) <= 1e-4 * want
    half = 0.5 * float(np.vdot(vis.astype(np.complex128), vis.astype(np.complex128)).real)
    assert abs(res["objective"] - half) <= 1e-6 * half


def test_adjoint_grid_ms_eight_scales():
    """The largest dictionary the interface takes: eight scales (half-widths
    0 and 3 to 9, the register stencil for each)."""
    uv, n, fov, h = _case("diffuse64")
    sig, gam = [0.5 * s + (1.0 if s else 0.0) for s in range(8)], [1.1 ** s for s in range(8)]
    a = api()
    plan = a.pc_plan_create(uv, n, fov)
    img, mx, am = a.pc_adjoint_grid_ms(plan, to_dev(h), sig, gam)
    got = img.cpu().numpy().astype(np.float64)
    want = dic.analysis(operator.adjoint(uv, n, fov, h.astype(np.complex128)),
                        dic.gaussian_dictionary(sig, gam))
    assert max(rel_l2(got[s], want[s]) for s in range(8)) <= 1e-4
    assert abs(mx - np.abs(want).max()) <= 1e-4 * np.abs(want).max()


@pytest.mark.slow
def test_adjoint_grid_ms_full_c3_sampled():
    """Full precision-workload size (2,088,960 visibilities, 4096^2; the
    configuration the benchmark times): Psi* Phi* h at sampled outputs of
    every scale, each formed by the oracle from the exact adjoint over the
    element's window (a border sample exercises the cropping)."""
    p = sim.config_c3()
    pts = np.argsort(-p.sky_amp)[:20]
    vclean = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix[pts], p.sky_amp[pts])
    vis = sim.add_noise(vclean, p.noise, p.psnr_db).astype(np.complex64)
    n = p.npix
    a = api()
    plan = a.pc_plan_create(p.uv, n, p.fov_rad)
    say("adjoint ms full c3")
    img, mx, am = a.pc_adjoint_grid_ms(plan, to_dev(vis), *PAPER)
    d = dic.gaussian_dictionary(*PAPER)
    rng = np.random.default_rng(11)
    samples = [(0, int(q)) for q in rng.choice(n * n, 4, replace=False)]
    samples += [(1, int(q)) for q in rng.choice(n * n, 2, replace=False)]
    samples += [(2, int(rng.integers(n * n))), (3, 2 * n + 3)]  # sigma 8 near a corner
    if am // (n * n) <= 1:
        samples.append((int(am // (n * n)), int(am % (n * n))))
    v64 = vis.astype(np.complex128)
    got, want = [], []
    for s, q in samples:
        pix, val = dic.element_pixels(d[s], q, n)
        want.append(float(val @ operator.adjoint_pixels(p.uv, n, p.fov_rad, v64, pix)))
        got.append(float(img[s].reshape(-1)[q]))
    err = rel_l2(np.array(got), np.array(want))
    say("full c3 dictionary samples", len(samples), "rel L2", err)
    assert err <= 1e-4


def test_dictionary_warm_start_from_the_solution():
    """x0 holds synthesis atoms (s n^2 + p): from the converged solution the
    gap test passes at once with the same objective."""
    p, vis = _diffuse(32)
    kw = dict(alpha=0.05, delta=0.99, max_iter=300, rel_gap_tol=1e-4)
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    dv = to_dev(vis)
    cold = a.pc_polyclean_solve(plan, dv, scales=STEEP, **kw)
    assert cold["converged"] == 1 and np.any(cold["pix"] >= p.npix ** 2)
    warm = a.pc_polyclean_solve(plan, dv, scales=STEEP, x0=(cold["pix"], cold["weight"]), **kw)
    say("cold", cold["iters"], cold["objective"], "warm", warm["iters"], warm["objective"])
    assert warm["converged"] == 1 and warm["iters"] == 0
    assert abs(warm["objective"] - cold["objective"]) <= 1e-6 * cold["objective"]
    with pytest.raises(a.PolycleanError):  # an atom past the last scale
        a.pc_polyclean_solve(plan, dv, scales=STEEP, x0=([4 * p.npix ** 2], [1.0]), **kw)
