"""Device buffer pool behind plan and solver memory: a destroyed plan's
buffers are parked by size class and taken by the next plan of the same
shape (same results), a finished solve's arrays are parked too, and
pc_device_pool_trim frees what is parked (the count it returns is the
observable; the device's free memory is not, since the HIP runtime may keep
freed pages for itself)."""
import numpy as np
import pytest

from tests.gpu_util import api, problem, say, to_dev, torch

pytestmark = pytest.mark.gpu


def test_plan_buffers_are_reused_and_trimmed():
    a = api()
    p, vis = problem("c2_small")
    dv = to_dev(vis)
    img1 = torch.empty((p.npix, p.npix), dtype=torch.float32, device="cuda")
    img2 = torch.empty_like(img1)
    a.pc_device_pool_trim(0)
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    fp = plan.info["footprint"]
    assert fp == a.pc_plan_footprint(p.uv, p.npix, p.fov_rad)
    a.pc_adjoint_grid(plan, dv, img1)
    plan.close()  # its buffers are parked
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)  # and taken again
    left = a.pc_device_pool_trim(0)
    say("footprint", fp, "left in the pool after the second plan", left)
    assert left == 0
    a.pc_adjoint_grid(plan, dv, img2)
    torch.cuda.synchronize()
    assert torch.equal(img1, img2)
    plan.close()
    released = a.pc_device_pool_trim(0)
    assert released >= fp
    assert a.pc_device_pool_trim(0) == 0  # nothing left parked


def test_solver_arrays_return_to_the_pool():
    """A finished solve's arrays are parked (not freed) and an identical solve
    afterwards gives the same result."""
    a = api()
    p, vis = problem("c1")
    dv = to_dev(vis)
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=20)
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    a.pc_device_pool_trim(0)
    r1 = a.pc_polyclean_solve(plan, dv, **kw)
    parked = a.pc_device_pool_trim(0)
    say("solver arrays parked", parked)
    assert parked > 0
    r2 = a.pc_polyclean_solve(plan, dv, **kw)
    plan.close()
    assert r1["objective"] == r2["objective"] and np.array_equal(r1["pix"], r2["pix"])
    with pytest.raises(a.PolycleanError):
        a.pc_device_pool_trim(-1)
