"""Why the direct DFTs form and reduce their phases in FP64 (CPU-only, an
arithmetic argument on the fine-resolution geometry).

The phase of visibility k and atom p is t = u_k l_p + v_k m_p turns.  At the
4096^2 / 40 km workload |t| reaches hundreds of turns, so an FP32 product
keeps only ~5e-5 turn of absolute resolution: the per-term error of the
exponential then exceeds the 1e-4 operator tolerance.  Forming t in FP64,
subtracting the nearest integer and only then rounding to FP32 leaves an
error of at most half an FP32 ulp of a number in [-1/2, 1/2] (3e-8 turn).
"""
import numpy as np

import sim
from oracle import geometry


def _phases(n_pairs=200000, seed=7):
    p = sim.config_c3()
    rng = np.random.default_rng(seed)
    k = rng.integers(0, p.nvis, n_pairs)
    pix = rng.integers(0, p.npix * p.npix, n_pairs)
    dl = geometry.pixel_step(p.npix, p.fov_rad)
    a = (pix // p.npix - p.npix // 2).astype(np.float64)
    b = (pix % p.npix - p.npix // 2).astype(np.float64)
    A = p.uv[k, 0] * dl
    B = p.uv[k, 1] * dl
    return A, B, a, b


def _reduce(t):
    return t - np.rint(t)


def test_fp32_phase_formation_breaks_the_tolerance():
    A, B, a, b = _phases()
    t64 = A * a + B * b
    assert np.abs(t64).max() > 100.0  # hundreds of turns at this geometry
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    t32 = (A32 * a.astype(np.float32) + B32 * b.astype(np.float32)).astype(np.float64)
    err = np.abs(_reduce(t32 - t64))
    # the exponential's error is 2 pi |dt|: far above 1e-4 somewhere
    assert 2 * np.pi * err.max() > 1e-4


def test_fp64_formation_then_fp32_meets_it():
    A, B, a, b = _phases()
    t64 = np.fma(A, a, B * b) if hasattr(np, "fma") else A * a + B * b
    r = _reduce(t64)
    assert np.abs(r).max() <= 0.5
    r32 = r.astype(np.float32).astype(np.float64)
    err = np.abs(r32 - r)
    assert err.max() <= 2.0 ** -25  # half an ulp of [1/4, 1/2]
    # and the per-term error of exp(2 pi i t) is then ~2e-7
    e = np.abs(np.exp(2j * np.pi * r32) - np.exp(2j * np.pi * r))
    assert e.max() <= 2e-7
