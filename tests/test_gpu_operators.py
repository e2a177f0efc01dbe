"""GPU parity of the measurement operators against the FP64 oracle.

Tolerance: 1e-4 relative L2 for every operator output (the accuracy target
for the operator), identical argmax of the dirty image (lowest index on ties).
"""
import numpy as np
import pytest

from oracle import operator, solver
from tests.gpu_util import api, problem, ragged_problem, rel_l2, say, to_dev, torch

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _adjoint_case(p_uv, n, fov, h, **kw):
    a = api()
    plan = a.pc_plan_create(p_uv, n, fov, **kw)
    img, mx, am = a.pc_adjoint_grid(plan, to_dev(h))
    torch.cuda.synchronize()
    return plan, img.cpu().numpy().astype(np.float64), mx, am


@pytest.mark.parametrize("name", ["c1", "c2_small", "c3_small"])
def test_adjoint_grid_dirty_image(name):
    say("adjoint_grid dirty", name)
    p, vis = problem(name)
    plan, img, mx, am = _adjoint_case(p.uv, p.npix, p.fov_rad, vis)
    want = operator.adjoint(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128))
    err = rel_l2(img, want)
    say(name, "rel L2", err, "info", plan.info)
    assert err <= TOL
    wmx, wam = solver.argmax_abs(want)
    assert am == wam
    assert abs(mx - wmx) <= TOL * wmx
    assert abs(mx - np.max(np.abs(img))) <= 1e-6 * mx


def test_adjoint_grid_split_tiles_present():
    p, vis = problem("c2_small")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    assert plan.info["n_partials"] > 0 and plan.info["wraps"] == 1


def test_adjoint_grid_partial_band():
    """Coverage confined to |u dl| < 0.2: the band is a sub-window of the fine
    grid (input pruning, no periodic wrap)."""
    say("adjoint_grid partial band")
    rng = np.random.default_rng(9)
    n, fov, L = 256, 0.03, 5003
    d = fov / n
    uv = rng.normal(0.0, 0.06 / d, size=(L, 2)).clip(-0.2 / d, 0.2 / d)
    h = (rng.normal(size=L) + 1j * rng.normal(size=L)).astype(np.complex64)
    plan, img, mx, am = _adjoint_case(uv, n, fov, h)
    assert plan.info["wraps"] == 0 and plan.info["band_nu"] < plan.info["fine"]
    want = operator.adjoint(uv, n, fov, h.astype(np.complex128))
    assert rel_l2(img, want) <= TOL
    assert am == solver.argmax_abs(want)[1]
    a = api()
    x = np.zeros((n, n), np.float32)
    pix = rng.choice(n * n, 500, replace=False)
    x.reshape(-1)[pix] = rng.normal(size=500)
    fx = a.pc_forward_grid(plan, to_dev(x)).cpu().numpy()
    wantf = operator.forward(uv, n, fov, pix, x.reshape(-1)[pix].astype(np.float64))
    assert rel_l2(fx, wantf) <= TOL


def test_adjoint_grid_ragged_random():
    say("adjoint_grid ragged")
    uv, n, fov, h = ragged_problem()
    plan, img, mx, am = _adjoint_case(uv, n, fov, h)
    want = operator.adjoint(uv, n, fov, h.astype(np.complex128))
    assert rel_l2(img, want) <= TOL
    assert am == solver.argmax_abs(want)[1]


def test_adjoint_grid_smallest_grid_and_single_vis():
    say("adjoint_grid n=16, L=1")
    uv = np.array([[3.7, -12.25]])
    h = np.array([1.5 - 0.25j], dtype=np.complex64)
    plan, img, mx, am = _adjoint_case(uv, 16, 0.2, h)
    want = operator.adjoint(uv, 16, 0.2, h.astype(np.complex128))
    assert rel_l2(img, want) <= TOL


@pytest.mark.parametrize("name", ["c1", "c2_small"])
def test_forward_sparse(name):
    say("forward_sparse", name)
    p, _ = problem(name)
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    amp32 = p.sky_amp.astype(np.float32)
    out = a.pc_forward_sparse(plan, to_dev(p.sky_pix.astype(np.int32)), to_dev(amp32))
    torch.cuda.synchronize()
    want = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, amp32.astype(np.float64))
    err = rel_l2(out.cpu().numpy(), want)
    say(name, "rel L2", err)
    assert err <= TOL


def test_forward_sparse_empty_and_centre():
    a = api()
    p, _ = problem("c1")
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    out = a.pc_forward_sparse(plan, to_dev(np.zeros(0, np.int32)), to_dev(np.zeros(0, np.float32)))
    assert torch.count_nonzero(out).item() == 0
    c = (p.npix // 2) * p.npix + p.npix // 2
    out = a.pc_forward_sparse(plan, to_dev(np.array([c], np.int32)), to_dev(np.array([2.5], np.float32)))
    o = out.cpu().numpy()
    assert np.allclose(o.real, 2.5, rtol=0, atol=1e-6) and np.allclose(o.imag, 0, atol=1e-6)


@pytest.mark.parametrize("name,natoms", [("c1", 1), ("c1", 2), ("c1", 3), ("c1", 7), ("c1", 33),
                                          ("c1", 64), ("c1", 65), ("c1", 300),
                                          ("c2_small", 1), ("c2_small", 300)])
def test_adjoint_sparse(name, natoms):
    """Every atoms-per-wave shape (1..64 and ragged last groups)."""
    say("adjoint_sparse", name, natoms)
    p, vis = problem(name)
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    rng = np.random.default_rng(3)
    pix = np.sort(rng.choice(p.npix ** 2, natoms, replace=False)).astype(np.int32)
    out = a.pc_adjoint_sparse(plan, to_dev(vis), to_dev(pix))
    torch.cuda.synchronize()
    want = operator.adjoint_pixels(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128), pix)
    err = rel_l2(out.cpu().numpy(), want)
    say(name, "rel L2", err)
    assert err <= TOL


@pytest.mark.parametrize("name,natoms", [("c1", 1), ("c1", 7), ("c1", 8), ("c1", 9), ("c1", 24),
                                          ("c1", 33), ("c1", 64), ("c1", 65), ("c1", 300),
                                          ("c2_small", 5), ("c2_small", 40), ("c2_small", 64),
                                          ("ragged", 13), ("c1", 0), ("c2", 40)])
def test_restricted_gradient(name, natoms):
    """Phi_S* (V - Phi_S x) and the residual against the oracle: the one-pass
    kernel at every atoms-per-pass size (8..64, padded groups), the two-pass
    path above 64 atoms, a visibility count that leaves a ragged last wave,
    the empty set (r = V), and the full LOFAR-like visibility set."""
    say("restricted_gradient", name, natoms)
    if name == "ragged":
        uv, n, fov, vis = ragged_problem()
    else:
        p, vis = problem(name)
        uv, n, fov = p.uv, p.npix, p.fov_rad
    a = api()
    plan = a.pc_plan_create(uv, n, fov)
    rng = np.random.default_rng(11)
    pix = np.sort(rng.choice(n * n, natoms, replace=False)).astype(np.int32)
    w = rng.normal(size=natoms).astype(np.float32) * float(np.abs(vis).mean())
    grad, resid = a.pc_restricted_gradient(plan, to_dev(vis), to_dev(pix), to_dev(w),
                                           want_resid=True)
    torch.cuda.synchronize()
    r_want = vis.astype(np.complex128) - operator.forward(uv, n, fov, pix, w.astype(np.float64))
    e_r = rel_l2(resid.cpu().numpy(), r_want)
    say(name, natoms, "residual rel L2", e_r)
    assert e_r <= TOL
    if natoms:
        g_want = operator.adjoint_pixels(uv, n, fov, r_want, pix)
        e_g = rel_l2(grad.cpu().numpy(), g_want)
        say(name, natoms, "gradient rel L2", e_g)
        assert e_g <= TOL
        # without the residual output the gradient is the same
        g2 = a.pc_restricted_gradient(plan, to_dev(vis), to_dev(pix), to_dev(w))
        torch.cuda.synchronize()
        assert torch.equal(g2, grad)


@pytest.mark.parametrize("name", ["c1", "c3_small"])
def test_forward_grid_dense(name):
    say("forward_grid", name)
    p, _ = problem(name)
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    rng = np.random.default_rng(4)
    img = np.zeros((p.npix, p.npix), np.float32)
    pix = rng.choice(p.npix ** 2, min(4000, p.npix ** 2 // 4), replace=False)
    img.reshape(-1)[pix] = rng.normal(size=pix.size).astype(np.float32)
    out = a.pc_forward_grid(plan, to_dev(img))
    torch.cuda.synchronize()
    want = operator.forward(p.uv, p.npix, p.fov_rad, pix, img.reshape(-1)[pix].astype(np.float64))
    err = rel_l2(out.cpu().numpy(), want)
    say(name, "rel L2", err)
    assert err <= TOL


@pytest.mark.parametrize("n", [16, 32, 64, 256, 1024, 2048, 4096, 8192])
def test_forward_grid_every_first_radix(n):
    """The gridded forward on fine grids of 32 to 16384 cells, which start
    their FFTs with every first-stage radix (2, 4, 8, 16) applied while
    loading: random uv filling the band, an image set at the centre, the
    corners, the edges and random pixels, against the oracle's exact sum at
    every visibility."""
    say("forward_grid sizes", n)
    a = api()
    rng = np.random.default_rng(100 + n)
    fov = 0.02 if n <= 1024 else 0.05
    d = fov / n
    L = 20000
    uv = rng.uniform(-0.49 / d, 0.49 / d, size=(L, 2))
    c = n // 2
    pix = np.unique(np.concatenate([
        [c * n + c, 0, n - 1, (n - 1) * n, n * n - 1, c, c * n, (n - 1) * n + c, c * n + n - 1],
        rng.choice(n * n, min(48, n * n // 4), replace=False)]))
    img = np.zeros(n * n, np.float32)
    img[pix] = rng.normal(size=pix.size).astype(np.float32)
    plan = a.pc_plan_create(uv, n, fov)
    assert plan.info["fine"] == 2 * n
    out = a.pc_forward_grid(plan, to_dev(img.reshape(n, n)))
    torch.cuda.synchronize()
    want = operator.forward(uv, n, fov, pix, img[pix].astype(np.float64))
    err = rel_l2(out.cpu().numpy(), want)
    say(n, "rel L2", err)
    assert err <= TOL


def _rows_case(n, L=20000, seed=0):
    rng = np.random.default_rng(700 + n + seed)
    fov = 0.02 if n <= 1024 else 0.05
    d = fov / n
    uv = rng.uniform(-0.49 / d, 0.49 / d, size=(L, 2))
    h = (rng.normal(size=L) + 1j * rng.normal(size=L)).astype(np.complex64)
    return rng, uv, fov, h


@pytest.mark.parametrize("n", [64, 512, 1024, 4096, 8192])
def test_forward_grid_rows_equals_full(n):
    """The row-restricted gridded forward of an image that is zero outside the
    mask's rows equals the full gridded forward bit for bit (it skips only
    transforms of zero rows), at fine grids with one and with several rows
    per pass-B workgroup, including the first and last rows."""
    say("forward_grid_rows", n)
    a = api()
    rng, uv, fov, _ = _rows_case(n)
    plan = a.pc_plan_create(uv, n, fov)
    rows = np.unique(np.concatenate([[0, n - 1, n // 2], rng.choice(n, min(40, n // 2), replace=False)]))
    img = np.zeros((n, n), np.float32)
    for r in rows:
        cols = rng.choice(n, 3, replace=False)
        img[r, cols] = rng.normal(size=3).astype(np.float32)
    full = a.pc_forward_grid(plan, to_dev(img))
    part = a.pc_forward_grid_rows(plan, to_dev(img), a.row_mask(n, rows))
    torch.cuda.synchronize()
    assert torch.equal(full, part)
    # a mask with more rows than the image uses gives the same result
    extra = np.union1d(rows, rng.choice(n, 5, replace=False))
    part2 = a.pc_forward_grid_rows(plan, to_dev(img), a.row_mask(n, extra))
    torch.cuda.synchronize()
    assert torch.equal(full, part2)


@pytest.mark.parametrize("n", [64, 512, 1024, 4096, 8192])
def test_adjoint_grid_rows_equals_full(n):
    """The row-restricted gridded adjoint writes exactly the mask's rows of
    the full adjoint's image (bit for bit) and leaves every other row as it
    was; an empty mask writes nothing."""
    say("adjoint_grid_rows", n)
    a = api()
    rng, uv, fov, h = _rows_case(n, seed=1)
    plan = a.pc_plan_create(uv, n, fov)
    full, _, _ = a.pc_adjoint_grid(plan, to_dev(h))
    rows = np.unique(np.concatenate([[0, n - 1], rng.choice(n, min(40, n // 2), replace=False)]))
    sentinel = 12345.0
    img = torch.full((n, n), sentinel, dtype=torch.float32, device="cuda")
    a.pc_adjoint_grid_rows(plan, to_dev(h), a.row_mask(n, rows), img)
    torch.cuda.synchronize()
    sel = torch.from_numpy(rows).cuda()
    assert torch.equal(img[sel], full[sel])
    other = np.setdiff1d(np.arange(n), rows)
    assert bool((img[torch.from_numpy(other).cuda()] == sentinel).all())
    before = img.clone()
    a.pc_adjoint_grid_rows(plan, to_dev(h), a.row_mask(n, []), img)
    torch.cuda.synchronize()
    assert torch.equal(img, before)


def test_grid_rows_reject_bad_masks():
    """A mask of the wrong length is refused by the binding; a set bit past
    npix (npix = 16: one word, bits 16..31 past the image) by the library."""
    a = api()
    _, uv, fov, h = _rows_case(16, L=500)
    plan = a.pc_plan_create(uv, 16, fov)
    img = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        a.pc_adjoint_grid_rows(plan, to_dev(h), np.zeros(2, np.uint32), img)
    m = a.row_mask(16, [3, 15])
    a.pc_adjoint_grid_rows(plan, to_dev(h), m, img)
    m[0] |= np.uint32(1) << np.uint32(20)
    with pytest.raises(a.PolycleanError) as e:
        a.pc_forward_grid_rows(plan, img, m)
    assert e.value.status == -1
    with pytest.raises(ValueError):
        a.row_mask(16, [16])


@pytest.mark.parametrize("n", [64, 512, 1024, 4096, 8192])
def test_restricted_gradient_grid_matches_direct(n):
    """The gridded restricted gradient (interpolation, pass A over the band
    rows, pass B evaluated at the set's rows and pixels) against the direct
    sums, at fine grids of 128 to 16384 cells (both layouts of the pass-A
    buffer): atoms in caller order, several on one row, a repeated pixel, the
    image corners and edges; gradient and residual within 1e-4 relative L2."""
    say("restricted gradient grid", n)
    a = api()
    rng, uv, fov, h = _rows_case(n, seed=2)
    plan = a.pc_plan_create(uv, n, fov)
    c = n // 2
    pix = np.concatenate([rng.choice(n * n, 40, replace=False),
                          [c * n + c, c * n + c + 3, c * n + 7, 0, n * n - 1, (n - 1) * n, n - 1,
                           c * n + c]])
    rng.shuffle(pix)
    w = rng.normal(size=pix.size).astype(np.float32)
    dv, dp, dw = to_dev(h), to_dev(pix.astype(np.int32)), to_dev(w)
    gd, rd = a.pc_restricted_gradient(plan, dv, dp, dw, want_resid=True)
    gg, rg = a.pc_restricted_gradient_grid(plan, dv, dp, dw, want_resid=True)
    torch.cuda.synchronize()
    eg = rel_l2(gg.cpu().numpy(), gd.cpu().numpy())
    er = rel_l2(rg.cpu().numpy(), rd.cpu().numpy())
    say(n, "gradient rel L2", eg, "residual rel L2", er)
    assert eg <= TOL and er <= TOL
    # the repeated pixel gets one value, the same as the direct sums give it
    q = np.flatnonzero(pix == c * n + c)
    assert gg[q[0]].item() == gg[q[1]].item()


def test_restricted_gradient_grid_small_against_oracle_and_edges():
    """At the plain workload: the gridded gradient against the oracle's exact
    Phi_S* (V - Phi_S x); no atoms gives r = V; a pixel out of range is
    refused (-1)."""
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    w = p.sky_amp.astype(np.float32)
    g, r = a.pc_restricted_gradient_grid(plan, to_dev(vis), to_dev(p.sky_pix.astype(np.int32)),
                                         to_dev(w), want_resid=True)
    torch.cuda.synchronize()
    v128 = vis.astype(np.complex128)
    r_want = v128 - operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, w.astype(np.float64))
    g_want = operator.adjoint_pixels(p.uv, p.npix, p.fov_rad, r_want, p.sky_pix)
    assert rel_l2(r.cpu().numpy(), r_want) <= TOL
    assert rel_l2(g.cpu().numpy(), g_want) <= TOL
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    _, r0 = a.pc_restricted_gradient_grid(plan, to_dev(vis), empty,
                                          torch.zeros(0, device="cuda"), want_resid=True)
    torch.cuda.synchronize()
    assert torch.equal(r0, to_dev(vis))
    bad = to_dev(np.array([3, p.npix * p.npix], np.int32))
    with pytest.raises(a.PolycleanError) as e:
        a.pc_restricted_gradient_grid(plan, to_dev(vis), bad, to_dev(np.ones(2, np.float32)))
    assert e.value.status == -1


def test_dot_product_gridded_pair():
    """<Phi_grid x, h> = <x, Phi*_grid h> up to the gridding error."""
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(p.npix, p.npix)).astype(np.float32)
    h = (rng.normal(size=p.nvis) + 1j * rng.normal(size=p.nvis)).astype(np.complex64)
    fx = a.pc_forward_grid(plan, to_dev(x)).cpu().numpy().astype(np.complex128)
    ah, _, _ = a.pc_adjoint_grid(plan, to_dev(h), want_max=False)
    lhs = float(np.vdot(h.astype(np.complex128), fx).real)
    rhs = float(np.sum(x.astype(np.float64) * ah.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-4 * (abs(lhs) + abs(rhs))


def test_dual_certificate_fixed_x():
    say("dual_certificate c2_small")
    p, vis = problem("c2_small")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    amp = (0.8 * p.sky_amp).astype(np.float32)
    lam = 0.05 * 1000.0
    cert, mx, am = a.pc_dual_certificate(plan, to_dev(vis), to_dev(p.sky_pix.astype(np.int32)),
                                         to_dev(amp), lam)
    torch.cuda.synchronize()
    want = solver.certificate(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128), p.sky_pix,
                              amp.astype(np.float64), lam)
    err = rel_l2(cert.cpu().numpy(), want)
    say("rel L2", err)
    assert err <= TOL
    assert am == solver.argmax_abs(want)[1]


def test_fp64_twin():
    say("fp64 twin c1")
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad, nufft_eps=1e-12, precision=a.PC_PREC_FP64)
    v128 = vis.astype(np.complex128)
    img, mx, am = a.pc_adjoint_grid_f64(plan, to_dev(v128))
    want = operator.adjoint(p.uv, p.npix, p.fov_rad, v128)
    err = rel_l2(img.cpu().numpy(), want)
    say("fp64 adjoint rel L2", err)
    assert err <= 1e-9
    out = a.pc_forward_sparse_f64(plan, to_dev(p.sky_pix.astype(np.int32)), to_dev(p.sky_amp))
    wantf = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, p.sky_amp)
    errf = rel_l2(out.cpu().numpy(), wantf)
    say("fp64 forward rel L2", errf)
    assert errf <= 1e-12


def test_precision_mismatch_rejected():
    p, vis = problem("c1")
    a = api()
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    with pytest.raises(a.PolycleanError) as e:
        a.pc_adjoint_grid_f64(plan, to_dev(vis.astype(np.complex128)))
    assert e.value.status == -1


@pytest.mark.slow
@pytest.mark.slow
def test_adjoint_grid_full_c2_whole_image():
    """Full LOFAR-like size (424,800 visibilities, 1024^2): the whole dirty
    image against the oracle's exact adjoint (Eq. adjoint-phi), relative L2
    within 1e-4, the same argmax (lowest index on ties) and maximum."""
    say("adjoint_grid full c2, whole image")
    p, vis = problem("c2")
    plan, img, mx, am = _adjoint_case(p.uv, p.npix, p.fov_rad, vis)
    want = operator.adjoint(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128))
    err = rel_l2(img, want)
    wmx, wam = solver.argmax_abs(want)
    say("full c2 whole image rel L2", err, "argmax", am, wam, "info", plan.info)
    assert err <= TOL
    assert am == wam
    assert abs(mx - wmx) <= TOL * wmx


def test_fused_maximum_tie_rule_on_a_flat_image():
    """Every pixel ties when the visibilities are zero: the fused maximum key
    reports 0 at flat index 0, the oracle's rule on the same input (lowest
    index wins; pinned on the CPU)."""
    say("fused max key, all-zero visibilities")
    p, vis = problem("c2_small")
    z = np.zeros_like(vis)
    plan, img, mx, am = _adjoint_case(p.uv, p.npix, p.fov_rad, z)
    assert np.all(img == 0.0)
    want = operator.adjoint(p.uv[:64], p.npix, p.fov_rad, z[:64].astype(np.complex128))
    assert solver.argmax_abs(want) == (0.0, 0)
    assert (mx, am) == (0.0, 0)


def test_adjoint_grid_batch_equals_single():
    """Shared launches over plans of different grid and visibility sizes give
    every plan's own gridded adjoint bit for bit, and the same maxima."""
    a = api()
    cases = []
    for name in ("c1", "c2_small", "c3_small"):
        p, vis = problem(name)
        cases.append((a.pc_plan_create(p.uv, p.npix, p.fov_rad), to_dev(vis)))
    uv, n, fov, h = ragged_problem()
    cases.append((a.pc_plan_create(uv, n, fov), to_dev(h)))
    plans = [c[0] for c in cases]
    vis = [c[1] for c in cases]
    say("batched adjoint over", [p.npix for p in plans])
    singles = []
    for pl, v in cases:
        img = torch.empty((pl.npix, pl.npix), dtype=torch.float32, device="cuda")
        _, mx, am = a.pc_adjoint_grid(pl, v, img)
        singles.append((img, mx, am))
    for rep in range(2):  # the second call reuses the launch tables
        imgs, mxs, ams = a.pc_adjoint_grid_batch(plans, vis)
        torch.cuda.synchronize()
        for (img, mx, am), bi, bm, ba in zip(singles, imgs, mxs, ams):
            assert torch.equal(img, bi)
            assert mx == bm and am == ba
    # a single-plan batch and an empty batch
    imgs, mxs, ams = a.pc_adjoint_grid_batch(plans[:1], vis[:1])
    assert torch.equal(imgs[0], singles[0][0])
    assert a.pc_adjoint_grid_batch([], [])[0] == []


def test_adjoint_grid_batch_rejects_bad_input():
    a = api()
    p, vis = problem("c1")
    plan = a.pc_plan_create(p.uv, p.npix, p.fov_rad)
    dv = to_dev(vis)
    with pytest.raises(a.PolycleanError):
        a.pc_adjoint_grid_batch([plan, plan], [dv, dv])  # the same plan twice
    plan64 = a.pc_plan_create(p.uv, p.npix, p.fov_rad, precision=a.PC_PREC_FP64)
    with pytest.raises(a.PolycleanError):
        a.pc_adjoint_grid_batch([plan64], [dv], images=[torch.empty((p.npix, p.npix),
                                                                    device="cuda")])


@pytest.mark.slow
def test_adjoint_grid_c5_large_all_visibilities_sampled():
    """The memory-pressure large job at its full size (8,372,224 visibilities,
    8192^2 image, 16384^2 fine grid, FP32 only), the launch configuration the
    benchmark times: the input is the generator's complex-normal draw plus
    four point sources by the oracle's exact forward; the GPU image against
    the oracle's exact sum at 160 sampled pixels, the centre and its
    neighbours, the four sources and the GPU argmax (relative L2 1e-4)."""
    import sim as _sim
    a = api()
    p = _sim.config_c5_large()
    rng = np.random.default_rng(51)
    n = p.npix
    src = np.array([(n // 2) * n + n // 2 + 3, 1234 * n + 4321, 6000 * n + 777, 77 * n + 8000])
    amp = np.array([40.0, -25.0, 30.0, 20.0])
    h = (p.noise + operator.forward(p.uv, n, p.fov_rad, src, amp)).astype(np.complex64)
    say("adjoint c5 large, all visibilities", p.uv.shape[0], n)
    plan = a.pc_plan_create(p.uv, n, p.fov_rad)
    assert plan.info["fine"] == 16384 and plan.nvis == 8372224
    img, mx, am = a.pc_adjoint_grid(plan, to_dev(h))
    c = n // 2
    pix = np.unique(np.concatenate([rng.choice(n * n, 160, replace=False), src,
                                    [c * n + c, c * n + c + 1, (c + 1) * n + c, am]]))
    want = operator.adjoint_pixels(p.uv, n, p.fov_rad, h.astype(np.complex128), pix)
    got = img.reshape(-1)[torch.from_numpy(pix).cuda()].double().cpu().numpy()
    err = rel_l2(got, want)
    say("c5 large rel L2 at", pix.size, "samples", err, "info", plan.info)
    assert err <= TOL
    # the reported maximum is the image's, and it is the largest sampled value
    assert abs(mx - float(img.abs().max())) <= 1e-6 * mx
    assert abs(float(img.reshape(-1)[am].abs()) - mx) <= 1e-6 * mx
    assert np.max(np.abs(want)) <= abs(want[np.searchsorted(pix, am)]) * (1 + TOL)
