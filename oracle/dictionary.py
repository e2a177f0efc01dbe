"""Multi-scale synthesis dictionary (TEST INFRASTRUCTURE; oracle).

Sect. 4.3 (synthesis form, Eqs. params-synthesis and lasso-synthesis): the
image is I = Psi theta, and the LASSO is solved for the coefficients theta,
with lambda_max = ||Psi* Phi* V||_inf.  The dictionary the paper uses for
diffuse emission (Sect. 6.4, reconstruction methods) has one Gaussian
element per scale: g_s = gamma_s g~_s with

    g~_s[a, b] = exp(-(a^2 + b^2) / sigma_s^2) / G_s  for |a|, |b| <= 2 sigma_s,

G_s making ||g~_s||_1 = 1; sigma_s = 0 is a single pixel (point sources).
The paper's values are sigma = (0, 2, 5, 8) and gamma_s = 1.2^s.

Readings (shared with the GPU path):
  * coefficient (s, p) puts g_s centred on pixel p = i n + j; a runs along
    the image rows (i), b along the columns (j); flat atom index s N + p with
    N = n^2;
  * element pixels falling outside the n x n image are dropped (the
    synthesis crops), so Psi* is the correlation with g_s of the image
    extended by zeros;
  * the half-width is floor(2 sigma_s) (2 sigma_s itself for the paper's
    integer scales).

Synthesis is written as an explicit loop over the non-zero coefficients;
analysis (Psi*) as a sum over element offsets of shifted copies of the
zero-padded image.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

PAPER_SIGMAS = (0.0, 2.0, 5.0, 8.0)
PAPER_GAMMA_RATIO = 1.2


def half_width(sigma: float) -> int:
    return int(math.floor(2.0 * float(sigma) + 1e-12))


def gaussian_element(sigma: float, gamma: float = 1.0) -> np.ndarray:
    """g_s = gamma g~_s as a (2h + 1) x (2h + 1) array, centre at [h, h]."""
    h = half_width(sigma)
    if h == 0:
        return np.full((1, 1), float(gamma))
    a = np.arange(-h, h + 1, dtype=np.float64)
    e = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / float(sigma) ** 2)
    return float(gamma) * e / e.sum()


def gaussian_dictionary(sigmas: Sequence[float] = PAPER_SIGMAS,
                        gammas: Sequence[float] = None) -> List[np.ndarray]:
    """The elements for the given scales; gamma_s = 1.2^s unless given."""
    if gammas is None:
        gammas = [PAPER_GAMMA_RATIO ** s for s in range(len(sigmas))]
    return [gaussian_element(s, g) for s, g in zip(sigmas, gammas)]


def split_atoms(atoms, npix: int):
    """Flat atom indices s N + p -> (scale s, pixel p)."""
    atoms = np.asarray(atoms, np.int64)
    N = npix * npix
    return atoms // N, atoms % N


def element_pixels(elem: np.ndarray, p: int, npix: int):
    """(pixel indices, values) of an element centred on pixel p, cropped."""
    h = elem.shape[0] // 2
    i0, j0 = divmod(int(p), npix)
    pix, val = [], []
    for a in range(-h, h + 1):
        i = i0 + a
        if i < 0 or i >= npix:
            continue
        for b in range(-h, h + 1):
            j = j0 + b
            if j < 0 or j >= npix:
                continue
            pix.append(i * npix + j)
            val.append(elem[a + h, b + h])
    return np.array(pix, np.int64), np.array(val, np.float64)


def synthesis(atoms, weights, dictionary: Sequence[np.ndarray], npix: int) -> np.ndarray:
    """I = Psi theta (Eq. params-synthesis) for a sparse theta, as (n, n)."""
    img = np.zeros(npix * npix)
    s_idx, p_idx = split_atoms(atoms, npix)
    for s, p, w in zip(s_idx, p_idx, np.asarray(weights, np.float64)):
        pix, val = element_pixels(dictionary[int(s)], int(p), npix)
        img[pix] += w * val
    return img.reshape(npix, npix)


def analysis(image: np.ndarray, dictionary: Sequence[np.ndarray]) -> np.ndarray:
    """Psi* I as an (S, n, n) array: (Psi* I)_s[i, j] =
    sum_{a, b} g_s[a, b] I[i + a, j + b], I extended by zeros."""
    image = np.asarray(image, np.float64)
    n = image.shape[0]
    out = np.zeros((len(dictionary), n, n))
    for s, elem in enumerate(dictionary):
        h = elem.shape[0] // 2
        padded = np.zeros((n + 2 * h, n + 2 * h))
        padded[h:h + n, h:h + n] = image
        for a in range(-h, h + 1):
            for b in range(-h, h + 1):
                out[s] += elem[a + h, b + h] * padded[h + a:h + a + n, h + b:h + b + n]
    return out
