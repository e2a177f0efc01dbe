"""Device buffer pool behind plan and solver memory: a destroyed plan's
buffers are reused by the next plan of the same shape (no new device memory,
same results), and pc_device_pool_trim frees them (the HIP runtime may keep
freed pages for itself, so the device's free memory is not asserted after
it)."""
import numpy as np
import pytest

from tests.gpu_util import api, problem, say, to_dev, torch

pytestmark = pytest.mark.gpu


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_plan_buffers_are_reused_and_trimmed():
    a = api()
    p, vis = problem("c2_small")
    dv = to_dev(vis)
    img1 = torch.empty((p.npix, p.npix), dtype=torch.float32, device="cuda")
    img2 = torch.empty_like(img1)
    # first use loads the kernels' code and the runtime's own state
    warm = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    a.pc_adjoint_grid(warm, dv, img1)
    warm.close()
    a.pc_device_pool_trim(0)
    free0 = _free()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    fp = plan.info["footprint"]
    assert fp == a.pc_plan_footprint(p.uv, p.npix, p.fov_rad)
    a.pc_adjoint_grid(plan, dv, img1)
    plan.close()
    free1 = _free()
    say("footprint", fp, "held after destroy", free0 - free1)
    assert free0 - free1 >= fp - (2 << 20)  # parked in the pool (2 MiB pages), not freed
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    free2 = _free()
    assert abs(free2 - free1) < (2 << 20)  # served from the pool
    a.pc_adjoint_grid(plan, dv, img2)
    torch.cuda.synchronize()
    assert torch.equal(img1, img2)
    plan.close()
    released = a.pc_device_pool_trim(0)
    free3 = _free()
    say("released", released, "free before / after", free0, free3)
    assert released >= fp
    assert a.pc_device_pool_trim(0) == 0  # nothing left parked


def test_solver_arrays_return_to_the_pool():
    """A finished solve's arrays are reused by the next identical solve; its
    result is unchanged."""
    a = api()
    p, vis = problem("c1")
    dv = to_dev(vis)
    kw = dict(alpha=p.alpha, delta=p.delta, max_iter=20)
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    r1 = a.pc_polyclean_solve(plan, dv, **kw)
    free1 = _free()
    r2 = a.pc_polyclean_solve(plan, dv, **kw)
    free2 = _free()
    plan.close()
    assert abs(free2 - free1) < (2 << 20)
    assert r1["objective"] == r2["objective"] and np.array_equal(r1["pix"], r2["pix"])
    with pytest.raises(a.PolycleanError):
        a.pc_device_pool_trim(-1)
