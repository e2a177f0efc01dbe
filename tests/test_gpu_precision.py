"""Per-stage precision report at the fine-resolution workload (2.1 M
visibilities, 4096^2 grid): every FP32 stage against its FP64 GPU twin over
the whole output, and both against the FP64 oracle on seeded samples.

Stages: gridded adjoint (spread + pruned FFT + correction), direct sparse
forward, restricted adjoint, dual certificate, and the type-2 (gridded)
forward.  The FP32 stages must stay within the 1e-4 relative-L2 operator
tolerance of the twin; the twin's direct sums must match the oracle to
rounding, and its gridded stages to the gridding accuracy (1e-5 requested).
"""
import functools
import json

import numpy as np
import pytest

import sim
from oracle import operator
from tests.gpu_util import api, rel_l2, say, to_dev, torch

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-4          # FP32 operator outputs vs the FP64 twin / the oracle
TWIN_DIRECT = 1e-9  # FP64 direct sums vs the oracle (summation order only)
TWIN_GRID = 2e-5    # FP64 gridded stages vs the oracle (gridding error)


@functools.lru_cache(maxsize=None)
def c3():
    """The workload's geometry and sky; the visibilities hold the 20
    brightest point sources (oracle forward) plus 15 dB noise, so that the
    oracle can synthesise them in seconds."""
    p = sim.config_c3()
    pts = np.argsort(-p.sky_amp)[:20]
    vclean = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix[pts], p.sky_amp[pts])
    vis = sim.add_noise(vclean, p.noise, p.psnr_db)
    return p, vis.astype(np.complex64)


def _plans(p):
    a = api()
    return (a.pc_plan_create(p.uv, p.npix, p.fov_rad),
            a.pc_plan_create(p.uv, p.npix, p.fov_rad, precision=a.PC_PREC_FP64))


REPORT = {}


def _record(stage, **kw):
    REPORT[stage] = kw
    say(stage, json.dumps(kw))


def test_gridded_adjoint_precision():
    a = api()
    p, vis = c3()
    f32, f64 = _plans(p)
    n = p.npix
    img32 = torch.empty((n, n), dtype=torch.float32, device="cuda")
    img64 = torch.empty((n, n), dtype=torch.float64, device="cuda")
    _, mx32, am32 = a.pc_adjoint_grid(f32, to_dev(vis), img32)
    _, mx64, am64 = a.pc_adjoint_grid_f64(f64, to_dev(vis.astype(np.complex128)), img64)
    e_twin = float(torch.linalg.norm(img32.double() - img64) / torch.linalg.norm(img64))
    rng = np.random.default_rng(31)
    c = n // 2
    centre = [(c + di) * n + (c + dj) for di in range(-4, 4) for dj in range(-4, 4)]
    pix = np.unique(np.concatenate([rng.choice(n * n, 63, replace=False), centre, [am64]]))
    ref = operator.adjoint_pixels(p.uv, n, p.fov_rad, vis.astype(np.complex128), pix)
    s32 = img32.reshape(-1)[torch.from_numpy(pix).cuda()].double().cpu().numpy()
    s64 = img64.reshape(-1)[torch.from_numpy(pix).cuda()].cpu().numpy()
    _record("gridded_adjoint", fp32_vs_twin_rel_l2=e_twin,
            twin_vs_oracle_rel_l2=rel_l2(s64, ref), fp32_vs_oracle_rel_l2=rel_l2(s32, ref),
            samples=int(pix.size), argmax_fp32=int(am32), argmax_twin=int(am64),
            max_fp32=mx32, max_twin=mx64)
    assert e_twin <= TOL
    assert rel_l2(s64, ref) <= TWIN_GRID and rel_l2(s32, ref) <= TOL
    assert am32 == am64 and abs(mx32 - mx64) <= 1e-5 * mx64


def test_direct_forward_precision():
    a = api()
    p, _ = c3()
    f32, f64 = _plans(p)
    w = p.sky_amp
    pix = to_dev(p.sky_pix.astype(np.int32))
    v32 = a.pc_forward_sparse(f32, pix, to_dev(w.astype(np.float32)))
    v64 = a.pc_forward_sparse_f64(f64, pix, to_dev(w))
    e_twin = float(torch.linalg.norm(v32.to(torch.complex128) - v64) / torch.linalg.norm(v64))
    rng = np.random.default_rng(32)
    ks = np.sort(rng.choice(p.nvis, 4096, replace=False))
    ref = operator.forward(p.uv[ks], p.npix, p.fov_rad, p.sky_pix, w)
    kd = torch.from_numpy(ks).cuda()
    s32 = v32[kd].cpu().numpy().astype(np.complex128)
    s64 = v64[kd].cpu().numpy()
    # the FP32 path rounds the weights to FP32 first: compare it with the
    # oracle of the same rounded weights
    ref32 = operator.forward(p.uv[ks], p.npix, p.fov_rad, p.sky_pix,
                             w.astype(np.float32).astype(np.float64))
    _record("direct_forward", atoms=int(w.size), fp32_vs_twin_rel_l2=e_twin,
            twin_vs_oracle_rel_l2=rel_l2(s64, ref), fp32_vs_oracle_rel_l2=rel_l2(s32, ref32),
            samples=int(ks.size))
    assert e_twin <= TOL
    assert rel_l2(s64, ref) <= TWIN_DIRECT and rel_l2(s32, ref32) <= TOL


def test_restricted_adjoint_precision():
    a = api()
    p, vis = c3()
    f32, f64 = _plans(p)
    pix = p.sky_pix.astype(np.int32)
    g32 = a.pc_adjoint_sparse(f32, to_dev(vis), to_dev(pix)).cpu().numpy()
    g64 = a.pc_adjoint_sparse_f64(f64, to_dev(vis.astype(np.complex128)), to_dev(pix)).cpu().numpy()
    rng = np.random.default_rng(33)
    sel = np.sort(rng.choice(pix.size, 48, replace=False))
    ref = operator.adjoint_pixels(p.uv, p.npix, p.fov_rad, vis.astype(np.complex128), pix[sel])
    _record("restricted_adjoint", atoms=int(pix.size), fp32_vs_twin_rel_l2=rel_l2(g32, g64),
            twin_vs_oracle_rel_l2=rel_l2(g64[sel], ref), fp32_vs_oracle_rel_l2=rel_l2(g32[sel], ref),
            samples=int(sel.size))
    assert rel_l2(g32, g64) <= TOL
    assert rel_l2(g64[sel], ref) <= TWIN_DIRECT and rel_l2(g32[sel], ref) <= TOL


def test_certificate_and_type2_precision():
    a = api()
    p, vis = c3()
    f32, f64 = _plans(p)
    n = p.npix
    # certificate of a sparse image near the data: the 300 point sources
    pts = np.argsort(-p.sky_amp)[:300]
    pix = to_dev(p.sky_pix[pts].astype(np.int32))
    w = p.sky_amp[pts]
    dv32, dv64 = to_dev(vis), to_dev(vis.astype(np.complex128))
    lam = 0.05 * a.pc_adjoint_grid(f32, dv32, torch.empty((n, n), device="cuda"))[1]
    c32, m32, am32 = a.pc_dual_certificate(f32, dv32, pix, to_dev(w.astype(np.float32)), lam)
    c64, m64, am64 = a.pc_dual_certificate_f64(f64, dv64, pix, to_dev(w), lam)
    e_cert = float(torch.linalg.norm(c32.double() - c64) / torch.linalg.norm(c64))
    # type-2 forward of a dense image against the twin's exact direct forward
    rng = np.random.default_rng(34)
    q = rng.choice(n * n, 20000, replace=False).astype(np.int32)
    wq = rng.normal(size=q.size)
    img = torch.zeros(n * n, dtype=torch.float32, device="cuda")
    img[torch.from_numpy(q.astype(np.int64)).cuda()] = torch.from_numpy(wq.astype(np.float32)).cuda()
    vg = a.pc_forward_grid(f32, img.reshape(n, n))
    vx = a.pc_forward_sparse_f64(f64, to_dev(q), to_dev(wq.astype(np.float32).astype(np.float64)))
    e_t2 = float(torch.linalg.norm(vg.to(torch.complex128) - vx) / torch.linalg.norm(vx))
    _record("certificate", fp32_vs_twin_rel_l2=e_cert, max_fp32=m32, max_twin=m64,
            argmax_fp32=int(am32), argmax_twin=int(am64))
    _record("type2_forward", atoms=int(q.size), fp32_vs_twin_exact_rel_l2=e_t2)
    assert e_cert <= TOL and abs(m32 - m64) <= 1e-4 * m64
    assert e_t2 <= TOL
