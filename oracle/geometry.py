"""Pixel grid and direction cosines (TEST INFRASTRUCTURE; oracle only).

Paper Sect. 2.2: the field of view is discretised with a uniform n x n grid
(l_i, m_j); a pixel of the image I[i, j] sits at (l_i, m_j).  Sect. 2.1 defines
n(l, m) = sqrt(1 - l^2 - m^2).

Readings where the paper is silent:
  * pixel step: dl = FOV / n, used directly as the direction-cosine step
    (Tables 1, 2 and A.1 print pixel sizes equal to FOV / n);
  * centring for even n: l_i = (i - n/2) dl, so pixel (n/2, n/2) is the phase
    centre;
  * axis order: row-major image, i (slow axis) <-> l <-> u, j <-> m <-> v.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299_792_458.0


def wavelengths(uv_m: np.ndarray, freq_hz: float) -> np.ndarray:
    """Baseline coordinates in metres -> wavelengths (Sect. 2.1: baselines are
    given in units of the observed wavelength)."""
    return np.asarray(uv_m, dtype=np.float64) * (freq_hz / C_LIGHT)


def pixel_step(npix: int, fov_rad: float) -> float:
    return float(fov_rad) / int(npix)


def direction_cosines(npix: int, fov_rad: float) -> np.ndarray:
    """l_i (= m_i) for i = 0..n-1: (i - n/2) * FOV/n."""
    d = pixel_step(npix, fov_rad)
    return (np.arange(npix, dtype=np.float64) - npix // 2) * d


def n_term(npix: int, fov_rad: float) -> np.ndarray:
    """n(l_i, m_j) = sqrt(1 - l_i^2 - m_j^2) as an (n, n) array (Sect. 2.1)."""
    l = direction_cosines(npix, fov_rad)
    r2 = l[:, None] ** 2 + l[None, :] ** 2
    if np.any(r2 >= 1.0):
        raise ValueError("field of view reaches the horizon")
    return np.sqrt(1.0 - r2)


def pixel_coords(pix: np.ndarray, npix: int, fov_rad: float):
    """Flat index p = i*n + j -> (l_i, m_j, n_ij)."""
    pix = np.asarray(pix, dtype=np.int64)
    i, j = pix // npix, pix % npix
    l = direction_cosines(npix, fov_rad)
    li, mj = l[i], l[j]
    return li, mj, np.sqrt(1.0 - li * li - mj * mj)


def nominal_resolution(uvw: np.ndarray) -> float:
    """delta l_0 = 1 / (3 B0) radians with B0 the largest baseline norm in
    wavelengths (Sect. 6.1, "Resolution of the images")."""
    b0 = float(np.max(np.linalg.norm(np.asarray(uvw, dtype=np.float64), axis=1)))
    return 1.0 / (3.0 * b0)


def rad_to_arcsec(x: float) -> float:
    return x * 180.0 / math.pi * 3600.0
