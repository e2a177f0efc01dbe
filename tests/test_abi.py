"""Boundary tests that need no GPU: the library loads, exports every symbol
include/polyclean.h declares, and rejects bad arguments on the host before any
device work (pc_plan_footprint runs entirely on the host)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import sim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polyclean.h")


def _lib():
    from paper_2406_01342_amd import _lib
    return _lib


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^PC_API\s+[^;]*?\b(pc_[a-z0-9_]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("pc_adjoint_grid", "pc_forward_sparse", "pc_dual_certificate",
                 "pc_polyclean_solve", "pc_plan_create", "pc_plan_destroy", "pc_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib().LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    assert set(declared_symbols()) <= set(_lib().SIGNATURES)


def _fp(uv, n=64, fov=0.05, **kw):
    from paper_2406_01342_amd import api
    return api.pc_plan_footprint(uv, n, fov, **kw)


def _status(fn):
    from paper_2406_01342_amd import api
    with pytest.raises(api.PolycleanError) as e:
        fn()
    return e.value.status


UV = np.random.default_rng(0).uniform(-100, 100, size=(500, 2))


@pytest.mark.parametrize("kw,status", [
    (dict(n=63), -1), (dict(n=8), -1), (dict(n=16384), -1), (dict(fov=0.0), -1),
    (dict(fov=-1.0), -1), (dict(fov=float("nan")), -1), (dict(fov=2.0), -1),
    (dict(upsamp=1.5), -5), (dict(precision=7), -1), (dict(uv_units=3), -1),
    (dict(uv_units=1, freq_hz=0.0), -1),
])
def test_footprint_rejects_bad_geometry(kw, status):
    assert _status(lambda: _fp(UV, **kw)) == status


def test_rejects_nonfinite_and_sizes_w_planes():
    bad = UV.copy()
    bad[17, 1] = np.inf
    assert _status(lambda: _fp(bad)) == -1
    w = np.zeros(len(UV))
    w[3] = np.nan
    assert _status(lambda: _fp(UV, w=w)) == -1
    flat = _fp(UV, w=np.zeros(len(UV)))
    assert flat == _fp(UV)  # an all-zero w is a coplanar plan
    w[3] = 100.0
    # a non-coplanar plan adds w, one plane's weighted values and the quadrature
    assert _fp(UV, w=w) >= flat + len(UV) * 16
    # w-stacking is an FP32 path
    from paper_2406_01342_amd import api
    assert _status(lambda: _fp(UV, w=w, precision=api.PC_PREC_FP64)) == -5


def test_rejects_empty():
    assert _status(lambda: _fp(np.zeros((0, 2)))) == -1


def test_last_error_message_is_thread_local_text():
    from paper_2406_01342_amd import api
    with pytest.raises(api.PolycleanError) as e:
        _fp(UV, n=63)
    assert "npix" in str(e.value)


def test_footprint_scales_with_problem():
    small = sim.config_c1()
    f1 = _fp(small.uv, small.npix, small.fov_rad)
    p2 = sim.config_c2(n_snap=24, npix=256)
    f2 = _fp(p2.uv, p2.npix, p2.fov_rad)
    assert 0 < f1 < f2
    # FP64 twin needs more memory
    assert _fp(small.uv, small.npix, small.fov_rad, precision=1) > f1


def test_metres_conversion_matches_wavelengths():
    lam = 299792458.0 / 150e6
    f1 = _fp(UV * lam, uv_units=1, freq_hz=150e6)
    f2 = _fp(UV)
    assert f1 == f2


def test_solve_params_marshalling():
    """The binding's solve parameters on the host: defaults from the library,
    the dictionary's scales and the warm start laid out as the header states,
    and malformed inputs refused before any call."""
    from paper_2406_01342_amd import api
    p = api.solve_params()
    assert (p.alpha, p.delta, p.max_iter, p.inner_max_iter) == (0.01, 0.99, 50, 2000)
    assert p.n_scales == 0 and p.x0_n == 0 and p.positivity == 0
    sig, gam = [0.0, 2.0, 5.0, 8.0], [1.2 ** s for s in range(4)]
    atoms, w = np.array([3, 70000, 9], np.int64), np.array([1.0, 0.5, -2.0])
    p = api.solve_params(scales=(sig, gam), x0=(atoms, w), positivity=1, lam=3.0)
    assert p.n_scales == 4 and list(p.scale_sigma)[:4] == sig and list(p.scale_gamma)[:4] == gam
    assert p.x0_n == 3 and [p.x0_pix[i] for i in range(3)] == [3, 70000, 9]
    assert [p.x0_w[i] for i in range(3)] == [1.0, 0.5, -2.0]
    assert p.positivity == 1 and p.lambda_ == 3.0
    with pytest.raises(ValueError):
        api.solve_params(scales=([0.0, 1.0], [1.0]))
    with pytest.raises(ValueError):
        api.solve_params(scales=([0.0] * 9, [1.0] * 9))
    with pytest.raises(ValueError):
        api.solve_params(x0=([1, 2], [1.0]))
    with pytest.raises(KeyError):
        api.solve_params(no_such_field=1)
