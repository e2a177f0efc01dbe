"""The allocation-free restricted gradient (pc_restricted_gradient_noalloc)
against pc_restricted_gradient: same inputs, bit-identical gradient and
residual, on two calls in a row (the second smaller), plus its size limit."""
import numpy as np
import pytest

from gpu_util import api, problem, ragged_problem, say, to_dev, torch

pytestmark = pytest.mark.gpu


def _atoms(p, na, seed):
    rng = np.random.default_rng(seed)
    pix = rng.choice(p.npix * p.npix, size=na, replace=False).astype(np.int32)
    w = rng.lognormal(size=na).astype(np.float32)
    return to_dev(pix), to_dev(w)


def _both(a, plan, dv, pix, w):
    g_ref, r_ref = a.pc_restricted_gradient(plan, dv, pix, w, want_resid=True)
    na = int(pix.numel())
    g = torch.full((na,), float("nan"), dtype=torch.float64, device="cuda")
    r = torch.full((plan.nvis,), float("nan"), dtype=torch.complex64, device="cuda")
    a.pc_restricted_gradient_noalloc(plan, dv, pix, w, g, r)
    torch.cuda.synchronize()
    return g.cpu().numpy(), r.cpu().numpy(), g_ref.cpu().numpy(), r_ref.cpu().numpy()


def test_noalloc_matches_restricted_gradient_two_calls():
    a = api()
    # first call: a larger plan and 300 atoms (forward, then restricted adjoint)
    p, vis = problem("c2_small")
    say("noalloc call 1: c2_small", p.nvis, "visibilities, 300 atoms")
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    dv = to_dev(vis)
    pix, w = _atoms(p, 300, 1)
    g, r, g_ref, r_ref = _both(a, plan, dv, pix, w)
    assert np.array_equal(g, g_ref)
    assert np.array_equal(r, r_ref)
    # second call: a smaller plan and 40 atoms (the one-pass kernel), on the
    # same scratch array
    p1, vis1 = problem("c1")
    say("noalloc call 2: c1", p1.nvis, "visibilities, 40 atoms")
    plan1 = a.pc_plan_create(p1.uv, p1.npix, p1.fov_rad)
    dv1 = to_dev(vis1)
    pix1, w1 = _atoms(p1, 40, 2)
    g1, r1, g1_ref, r1_ref = _both(a, plan1, dv1, pix1, w1)
    assert np.array_equal(g1, g1_ref)
    assert np.array_equal(r1, r1_ref)
    # without the residual output, and with no atoms (r = V)
    g2 = torch.empty(40, dtype=torch.float64, device="cuda")
    a.pc_restricted_gradient_noalloc(plan1, dv1, pix1, w1, g2)
    assert np.array_equal(g2.cpu().numpy(), g1_ref)
    r0 = torch.empty(p1.nvis, dtype=torch.complex64, device="cuda")
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    a.pc_restricted_gradient_noalloc(plan1, dv1, e, e.float(), e.double(), r0)
    assert np.array_equal(r0.cpu().numpy(), vis1)
    plan.close()
    plan1.close()


def test_noalloc_rejects_requests_beyond_its_scratch():
    a = api()
    uv, n, fov, h = ragged_problem(L=1237, n=1024, fov=0.3)
    say("noalloc limit: 1024^2 plan, 300000 atoms")
    plan = a.pc_plan_create(uv, n, fov)
    dv = to_dev(h)
    na = 300000  # 32 B per atom alone exceeds the 8 MiB array
    pix = torch.arange(na, dtype=torch.int32, device="cuda")
    w = torch.ones(na, dtype=torch.float32, device="cuda")
    g = torch.empty(na, dtype=torch.float64, device="cuda")
    with pytest.raises(a.PolycleanError) as ex:
        a.pc_restricted_gradient_noalloc(plan, dv, pix, w, g)
    assert ex.value.status == -5 and "scratch" in str(ex.value)
    # instrumentation on: refused (it would create events)
    a.pc_plan_profile(plan, True)
    with pytest.raises(a.PolycleanError) as ex:
        a.pc_restricted_gradient_noalloc(plan, dv, pix[:8], w[:8], g[:8])
    assert ex.value.status == -1
    a.pc_plan_profile(plan, False)
    plan.close()
