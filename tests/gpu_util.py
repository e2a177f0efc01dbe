"""Shared helpers for the GPU parity tests (inputs come from sim + oracle)."""
import functools
import sys

import numpy as np
import pytest

import sim
from oracle import operator

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def api():
    need_gpu()
    from paper_2406_01342_amd import api as a
    return a


def say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@functools.lru_cache(maxsize=None)
def problem(name: str):
    """Named test problems built from the workload recipes, with their noisy
    visibilities synthesised by the oracle's exact forward operator."""
    if name == "c1":
        p = sim.config_c1()
    elif name == "c2":
        p = sim.config_c2()
    elif name == "c2_small":
        p = sim.config_c2(n_snap=24, npix=256)
    elif name == "c3_small":
        p = sim.config_c3(n_snap=8, npix=512, n_ant=64, with_blobs=False)
    elif name == "c4_0":
        p = sim.config_c4_request(0)
    elif name == "c2w":  # non-coplanar variants: uv holds (u, v, w)
        p = sim.config_c2(keep_w=True)
    elif name == "c2w_small":
        p = sim.config_c2(n_snap=24, npix=256, keep_w=True)
    elif name == "c2w_128":
        p = sim.config_c2(n_snap=4, npix=128, n_src=10, keep_w=True)
    elif name == "c2w_64":
        p = sim.config_c2(n_snap=4, npix=64, n_src=10, keep_w=True)
    else:
        raise KeyError(name)
    vclean = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, p.sky_amp)
    vis = sim.add_noise(vclean, p.noise, p.psnr_db)
    vis64 = vis.astype(np.complex64)
    return p, vis64


def ragged_problem(L=1237, n=64, fov=0.02, seed=5):
    rng = np.random.default_rng(seed)
    d = fov / n
    uv = rng.uniform(-0.49 / d, 0.49 / d, size=(L, 2))
    h = (rng.normal(size=L) + 1j * rng.normal(size=L)).astype(np.complex64)
    return uv, n, fov, h


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
