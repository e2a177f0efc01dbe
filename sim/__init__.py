"""Seeded synthetic inputs for the PolyCLEAN measurement-operator workloads.

This module produces *inputs only*: antenna layouts, Earth-rotation (u, v)
coverage, sky models (pixel indices and amplitudes, optionally an extended
image) and raw complex-normal noise draws.  It holds none of the method's
arithmetic: no forward or adjoint operator, no solver.  Turning a sky into
visibilities is done by the caller (the FP64 oracle in tests, the library's
own forward operator in benchmarks); the noise draw and its scaling rule are
returned separately so both sides use the exact same numbers.

Conventions (paper, Sect. 2.1 "Forward operator" and Sect. 2.2):
  * (u, v, w) are baseline coordinates in wavelengths; the arrays here are
    coplanar (w = 0), the narrow-field / coplanar remark of Sect. 2.1, except
    the non-coplanar variant of the LOFAR-like recipe, which keeps w.
  * One Hermitian half is generated: baselines i < j, no autocorrelations.
  * Noise is white complex Gaussian (Sect. 2.1 "Noise model"); its standard
    deviation is set from a peak signal-to-noise ratio as
    sigma = max_k |V_clean_k| * 10**(-psnr/20), with real and imaginary parts
    each N(0, sigma^2/2).  The paper only names the PSNR (Sect. 6.1), so the
    definition of sigma is this module's reading.

Random streams: numpy.random.default_rng([cfg_id, job_id, stream]) with
stream 0 = layout, 1 = sky, 2 = noise, 3 = request arrivals.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C_LIGHT = 299_792_458.0  # m/s
DEG = math.pi / 180.0

STREAM_LAYOUT, STREAM_SKY, STREAM_NOISE, STREAM_ARRIVAL = 0, 1, 2, 3


def rng_for(cfg_id: int, job_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(cfg_id), int(job_id), int(stream)])


# ----------------------------------------------------------------------------
# Antenna layouts: local East/North positions in metres (Up = 0).
# ----------------------------------------------------------------------------
def layout_disk(rng: np.random.Generator, n_ant: int, radius_m: float) -> np.ndarray:
    """Positions uniform over a disk of the given radius."""
    r = radius_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * math.pi * rng.random(n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def layout_core_ring(rng: np.random.Generator, n_core: int, core_sigma_m: float,
                     n_ring: int, r_in_m: float, r_out_m: float) -> np.ndarray:
    """Gaussian core plus stations uniform (in area) over an annulus."""
    core = rng.normal(0.0, core_sigma_m, size=(n_core, 2))
    r = np.sqrt(rng.uniform(r_in_m ** 2, r_out_m ** 2, size=n_ring))
    th = 2.0 * math.pi * rng.random(n_ring)
    ring = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    return np.concatenate([core, ring], axis=0)


def layout_core_arms(rng: np.random.Generator, n_ant: int, core_frac: float,
                     core_sigma_m: float, r_min_m: float, r_max_m: float,
                     n_arms: int = 3) -> np.ndarray:
    """SKA-low-like layout: Gaussian core plus log-radial spiral arms."""
    n_core = int(round(n_ant * core_frac))
    n_arm = n_ant - n_core
    core = rng.normal(0.0, core_sigma_m, size=(n_core, 2))
    arm_id = rng.integers(0, n_arms, size=n_arm)
    r = np.exp(rng.uniform(math.log(r_min_m), math.log(r_max_m), size=n_arm))
    th = (2.0 * math.pi * arm_id / n_arms + 0.35 * np.log(r / r_min_m)
          + rng.normal(0.0, 0.04, size=n_arm))
    arms = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    return np.concatenate([core, arms], axis=0)


# ----------------------------------------------------------------------------
# Earth-rotation synthesis (standard equatorial relations; coplanar array).
# ----------------------------------------------------------------------------
def earth_rotation_uv(pos_en: np.ndarray, freq_hz: float, n_snap: int,
                      duration_h: float, dec_rad: float,
                      lat_rad: float = -26.7 * DEG, keep_w: bool = False) -> np.ndarray:
    """(u, v) in wavelengths for all baselines i<j and snapshots.

    Returns an array of shape (n_snap * n_bl, 2), time-major (all baselines of
    snapshot 0, then snapshot 1, ...), which is the order a correlator writes.
    Hour angles are symmetric about transit.  w is discarded (set to 0), or
    kept as a third column with ``keep_w`` (the non-coplanar case).
    """
    e, nth = pos_en[:, 0], pos_en[:, 1]
    # local (E, N, U=0) -> equatorial (X, Y, Z)
    X = -math.sin(lat_rad) * nth
    Y = e
    Z = math.cos(lat_rad) * nth
    i, j = np.triu_indices(len(e), k=1)
    bx, by, bz = X[j] - X[i], Y[j] - Y[i], Z[j] - Z[i]
    lam = C_LIGHT / freq_hz
    if n_snap == 1:
        hs = np.zeros(1)
    else:
        hs = (np.arange(n_snap) - (n_snap - 1) / 2.0) * (duration_h / (n_snap - 1))
    h = hs * (15.0 * DEG)  # hours -> radians
    sh, ch = np.sin(h)[:, None], np.cos(h)[:, None]
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    u = sh * bx[None, :] + ch * by[None, :]
    v = -sd * ch * bx[None, :] + sd * sh * by[None, :] + cd * bz[None, :]
    cols = [u.reshape(-1) / lam, v.reshape(-1) / lam]
    if keep_w:
        w = cd * ch * bx[None, :] - cd * sh * by[None, :] + sd * bz[None, :]
        cols.append(w.reshape(-1) / lam)
    return np.stack(cols, axis=1)


# ----------------------------------------------------------------------------
# Sky models.
# ----------------------------------------------------------------------------
def point_sky(rng: np.random.Generator, npix: int, n_src: int):
    """Distinct on-grid pixels (flat index p = i*n + j) and log-normal amplitudes."""
    pix = np.sort(rng.choice(npix * npix, size=n_src, replace=False)).astype(np.int64)
    amp = np.exp(rng.normal(0.0, 1.0, size=n_src))
    return pix, amp


def blob_sky(rng: np.random.Generator, npix: int, n_blob: int, sig_lo: float,
             sig_hi: float):
    """Elliptical Gaussian blobs as a sparse list of (pixel, value) pairs.

    Each blob has a log-normal peak, axis sigmas drawn in [sig_lo, sig_hi]
    pixels, a random axis ratio and orientation, truncated at 3 sigma.
    Overlapping blobs add.
    """
    acc = {}
    for _ in range(n_blob):
        s1 = rng.uniform(sig_lo, sig_hi)
        s2 = s1 * rng.uniform(0.3, 1.0)
        ang = rng.uniform(0.0, math.pi)
        peak = math.exp(rng.normal(0.0, 1.0)) * 0.05
        ci = rng.integers(npix // 8, npix - npix // 8)
        cj = rng.integers(npix // 8, npix - npix // 8)
        rad = int(math.ceil(3.0 * s1))
        di, dj = np.meshgrid(np.arange(-rad, rad + 1), np.arange(-rad, rad + 1), indexing="ij")
        ca, sa = math.cos(ang), math.sin(ang)
        x = ca * di + sa * dj
        y = -sa * di + ca * dj
        q = (x / s1) ** 2 + (y / s2) ** 2
        keep = q <= 9.0
        ii = (ci + di[keep]) % npix
        jj = (cj + dj[keep]) % npix
        val = peak * np.exp(-0.5 * q[keep])
        for p, a in zip((ii * npix + jj).tolist(), val.tolist()):
            acc[p] = acc.get(p, 0.0) + a
    pix = np.array(sorted(acc), dtype=np.int64)
    amp = np.array([acc[p] for p in pix.tolist()], dtype=np.float64)
    return pix, amp


def merge_sparse(pix_a, amp_a, pix_b, amp_b):
    allp = np.concatenate([pix_a, pix_b])
    alla = np.concatenate([amp_a, amp_b])
    up, inv = np.unique(allp, return_inverse=True)
    out = np.zeros(len(up))
    np.add.at(out, inv, alla)
    return up.astype(np.int64), out


def complex_normal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit-power circular complex normal draws: Re, Im ~ N(0, 1/2)."""
    z = rng.normal(0.0, math.sqrt(0.5), size=(n, 2))
    return z[:, 0] + 1j * z[:, 1]


def add_noise(v_clean: np.ndarray, z: np.ndarray, psnr_db: float) -> np.ndarray:
    """V = V_clean + sigma z with sigma = max|V_clean| * 10^(-PSNR/20)."""
    sigma = float(np.max(np.abs(v_clean))) * 10.0 ** (-psnr_db / 20.0)
    return v_clean + sigma * z


# ----------------------------------------------------------------------------
# Workload recipes.
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """One imaging problem: geometry, sky truth and the noise draw."""
    name: str
    uv: np.ndarray            # (L, 2) float64, wavelengths, caller order
    npix: int
    fov_rad: float
    freq_hz: float
    sky_pix: np.ndarray       # (S,) int64 flat pixel indices p = i*n + j
    sky_amp: np.ndarray       # (S,) float64 Jy/pixel
    noise: np.ndarray         # (L,) complex128 unit-power draws
    psnr_db: float
    alpha: float
    delta: float
    max_iter: int
    rel_obj_tol: float
    rel_gap_tol: float

    @property
    def nvis(self) -> int:
        return int(self.uv.shape[0])


def _problem(name, cfg_id, job_id, pos, freq, n_snap, dur_h, dec, npix, fov_deg,
             sky, psnr, alpha, delta, max_iter, rel_obj_tol, rel_gap_tol,
             keep_w: bool = False) -> Problem:
    uv = earth_rotation_uv(pos, freq, n_snap, dur_h, dec, keep_w=keep_w)
    pix, amp = sky
    noise = complex_normal(rng_for(cfg_id, job_id, STREAM_NOISE), uv.shape[0])
    return Problem(name, uv, npix, fov_deg * DEG, freq, pix, amp, noise, psnr,
                   alpha, delta, max_iter, rel_obj_tol, rel_gap_tol)


def config_c1(job_id: int = 0) -> Problem:
    """Plain: 32 antennas in a 2 km-diameter disk, 8 snapshots over 1 h at
    dec -45 deg, 128^2 grid, FOV 2 deg, 20 on-grid sources, 20 dB, alpha 0.01,
    50 FW iterations."""
    pos = layout_disk(rng_for(1, job_id, STREAM_LAYOUT), 32, 1000.0)
    sky = point_sky(rng_for(1, job_id, STREAM_SKY), 128, 20)
    return _problem("C1", 1, job_id, pos, 150e6, 8, 1.0, -45 * DEG, 128, 2.0, sky,
                    20.0, 0.01, 0.99, 50, 0.0, 0.0)


def config_c2(job_id: int = 0, n_snap: int = 240, npix: int = 1024,
              n_core: int = 48, n_ring: int = 12, n_src: int = 150,
              keep_w: bool = False) -> Problem:
    """LOFAR-like: 48 Gaussian-core (300 m) + 12 ring (1-10 km) stations, 240
    snapshots over 4 h, 1024^2 grid, FOV 4 deg, 150 sources, 20 dB, alpha 0.05,
    stop at relative dual gap 1e-4.  Smaller variants keep the recipe;
    ``keep_w`` keeps the baselines' w (the non-coplanar variant, uv then has
    three columns)."""
    pos = layout_core_ring(rng_for(2, job_id, STREAM_LAYOUT), n_core, 300.0, n_ring,
                           1000.0, 10000.0)
    sky = point_sky(rng_for(2, job_id, STREAM_SKY), npix, n_src)
    return _problem("C2W" if keep_w else "C2", 2, job_id, pos, 150e6, n_snap, 4.0, -45 * DEG,
                    npix, 4.0, sky, 20.0, 0.05, 0.95, 500, 0.0, 1e-4, keep_w=keep_w)


def config_c3(job_id: int = 0, n_snap: int = 64, npix: int = 4096, n_ant: int = 256,
              with_blobs: bool = True) -> Problem:
    """Precision: 256 SKA-low-like stations (40 km max baseline), 64 snapshots,
    4096^2 grid, FOV 3 deg, 300 points + 10 elliptical Gaussian blobs, 15 dB."""
    pos = layout_core_arms(rng_for(3, job_id, STREAM_LAYOUT), n_ant, 0.5, 500.0,
                           1000.0, 20000.0)
    srng = rng_for(3, job_id, STREAM_SKY)
    pix, amp = point_sky(srng, npix, 300)
    if with_blobs:
        bp, ba = blob_sky(srng, npix, 10, 2.0, 20.0)
        pix, amp = merge_sparse(pix, amp, bp, ba)
    return _problem("C3", 3, job_id, pos, 150e6, n_snap, 4.0, -45 * DEG, npix, 3.0,
                    (pix, amp), 15.0, 0.05, 0.95, 200, 1e-4, 0.0)


def config_c5_large(job_id: int = 0, n_ant: int = 512, n_snap: int = 16) -> Problem:
    """Memory-pressure large job: 512 C3-like stations, 16 snapshots x 4
    channels (120-180 MHz) stacked, 8192^2 grid, FOV 3 deg."""
    pos = layout_core_arms(rng_for(5, job_id, STREAM_LAYOUT), n_ant, 0.5, 500.0,
                           1000.0, 20000.0)
    uv = np.concatenate([earth_rotation_uv(pos, f, n_snap, 4.0, -45 * DEG)
                         for f in (120e6, 140e6, 160e6, 180e6)], axis=0)
    pix, amp = point_sky(rng_for(5, job_id, STREAM_SKY), 8192, 200)
    noise = complex_normal(rng_for(5, job_id, STREAM_NOISE), uv.shape[0])
    return Problem("C5L", uv, 8192, 3.0 * DEG, 150e6, pix, amp, noise, 20.0, 0.05,
                   0.95, 200, 1e-4, 0.0)


def config_diffuse(job_id: int = 0, npix: int = 64, n_ant: int = 32, n_snap: int = 8,
                   n_blob: int = 0, n_src: int = 4, sig_lo: float = 0.0,
                   sig_hi: float = 0.0) -> Problem:
    """Diffuse emission for the synthesis dictionary (the setting of Sect. 6.4,
    scaled down): a 5 km-diameter disk of n_ant antennas, n_snap snapshots over
    4 h at dec -45 deg, npix^2 pixels of about 0.8 nominal resolutions
    (FOV 1.2 deg at 64^2), elliptical Gaussian blobs with peaks ten times
    those of the precision sky (n_blob of them, axis sigmas sig_lo to sig_hi
    pixels; by default max(3, npix^2 / 2048) blobs of npix/16 to npix/8
    pixels) plus n_src points, 20 dB, alpha 0.02, delta 0.99, stop on a
    relative improvement of 1e-5."""
    pos = layout_disk(rng_for(7, job_id, STREAM_LAYOUT), n_ant, 2500.0)
    srng = rng_for(7, job_id, STREAM_SKY)
    n_blob = n_blob or max(3, npix * npix // 2048)
    bp, ba = blob_sky(srng, npix, n_blob, sig_lo or npix / 16, sig_hi or npix / 8)
    pp, pa = point_sky(srng, npix, n_src)
    return _problem("DIFFUSE", 7, job_id, pos, 150e6, n_snap, 4.0, -45 * DEG, npix,
                    1.2 * npix / 64, merge_sparse(pp, pa, bp, 10.0 * ba), 20.0, 0.02, 0.99,
                    300, 1e-5, 0.0)


def config_c5_small(job_id: int = 0) -> Problem:
    """Memory-pressure small job: 64 antennas, 25 snapshots, 512^2, FOV 2 deg."""
    pos = layout_disk(rng_for(6, job_id, STREAM_LAYOUT), 64, 2500.0)
    sky = point_sky(rng_for(6, job_id, STREAM_SKY), 512, 50)
    return _problem("C5S", 6, job_id, pos, 150e6, 25, 2.0, -45 * DEG, 512, 2.0, sky,
                    20.0, 0.05, 0.95, 200, 1e-4, 0.0)


@dataclasses.dataclass
class Request:
    job_id: int
    arrival_s: float
    problem: Problem


def config_c4_request(job_id: int) -> Problem:
    """One serving request: n in {256,512,1024,2048}, L log-uniform in
    [1e4, 5e5], A uniform in [32,128] antennas with T = round(L/(A(A-1)/2))
    snapshots, FOV 2 deg, array radius chosen so that the pixel is about half
    the nominal resolution 1/(3 B0) (Sect. 6.1), 5-200 sources, 20 dB."""
    r = rng_for(4, job_id, STREAM_LAYOUT)
    npix = int(r.choice([256, 512, 1024, 2048]))
    L_target = math.exp(r.uniform(math.log(1e4), math.log(5e5)))
    n_ant = int(r.integers(32, 129))
    n_bl = n_ant * (n_ant - 1) // 2
    n_snap = max(1, int(round(L_target / n_bl)))
    fov = 2.0 * DEG
    b0 = npix / (6.0 * fov)               # wavelengths, SRF = 2
    lam = C_LIGHT / 150e6
    pos = layout_disk(r, n_ant, 0.5 * b0 * lam)
    srng = rng_for(4, job_id, STREAM_SKY)
    n_src = int(srng.integers(5, 201))
    sky = point_sky(srng, npix, n_src)
    return _problem("C4", 4, job_id, pos, 150e6, n_snap, 4.0, -45 * DEG, npix, 2.0,
                    sky, 20.0, 0.05, 0.95, 100, 1e-4, 0.0)


def poisson_arrivals(n_req: int, rate_per_s: float, seed_job: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process; rate <= 0 puts all at t = 0."""
    if rate_per_s <= 0:
        return np.zeros(n_req)
    gaps = rng_for(4, seed_job, STREAM_ARRIVAL).exponential(1.0 / rate_per_s, size=n_req)
    return np.cumsum(gaps) - gaps[0]


def c4_requests(n_req: int, rate_per_s: float) -> List[Request]:
    t = poisson_arrivals(n_req, rate_per_s)
    return [Request(k, float(t[k]), config_c4_request(k)) for k in range(n_req)]


def orthogonal_uv(npix: int, fov_rad: float, rows: Optional[np.ndarray] = None):
    """(u, v) exactly on the n x n DFT frequencies u = p/(n dl), p in
    [-n/2, n/2): the sampling for which the normal operator is diagonal.
    ``rows`` optionally restricts to a subset of frequency indices (flat)."""
    d = fov_rad / npix
    p = np.arange(-npix // 2, npix // 2)
    uu, vv = np.meshgrid(p / (npix * d), p / (npix * d), indexing="ij")
    uv = np.stack([uu.reshape(-1), vv.reshape(-1)], axis=1)
    if rows is not None:
        uv = uv[rows]
    return uv
