"""Pins for the oracle's forward and adjoint operators (T3-T7).

Each pin is fixed by mathematics independent of the oracle's own code path:
closed forms of the forward sum, the adjoint identity <Phi x, h> = <x, Phi* h>
(which ties the GEMM-factorised adjoint to the direct forward), the per-pixel
direct sum, and the shifted-PSF identity of the dirty image of one source.
"""
import math

import numpy as np
import pytest

import sim
from oracle import geometry, operator


def _small(seed=0, L=300, n=16, fov=0.2):
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-40, 40, size=(L, 2))
    return uv, n, fov, rng


def test_forward_phase_centre_source_is_constant():
    """T3: a source at the phase centre (l = m = 0, n = 1) gives V_k = a."""
    uv, n, fov, _ = _small()
    p = (n // 2) * n + n // 2
    V = operator.forward(uv, n, fov, [p], [2.5])
    assert np.allclose(V, 2.5, rtol=1e-15, atol=0)


def test_forward_single_source_closed_form():
    """T4: V_k = a / n_p * exp(-2 pi j (u_k l_p + v_k m_p))."""
    uv, n, fov, _ = _small(1)
    i, j = 3, 12
    d = fov / n
    lp, mp = (i - n // 2) * d, (j - n // 2) * d
    npp = math.sqrt(1 - lp * lp - mp * mp)
    want = 1.7 / npp * np.exp(-2j * math.pi * (uv[:, 0] * lp + uv[:, 1] * mp))
    got = operator.forward(uv, n, fov, [i * n + j], [1.7])
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_forward_is_linear_in_atoms():
    uv, n, fov, rng = _small(2)
    pix = rng.choice(n * n, 7, replace=False)
    w = rng.normal(size=7)
    full = operator.forward(uv, n, fov, pix, w)
    parts = sum(operator.forward(uv, n, fov, [p], [a]) for p, a in zip(pix, w))
    assert np.allclose(full, parts, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adjoint_dot_product(seed):
    """T5: <Phi x, h>_R = <x, Phi* h> to 1e-12 (dense x, random h)."""
    uv, n, fov, rng = _small(seed, L=257, n=18, fov=0.3)
    x = rng.normal(size=(n, n))
    h = rng.normal(size=uv.shape[0]) + 1j * rng.normal(size=uv.shape[0])
    lhs = float(np.vdot(h, operator.forward_dense(uv, n, fov, x)).real)
    rhs = float(np.sum(x * operator.adjoint(uv, n, fov, h)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def test_adjoint_factorised_equals_direct_sum():
    """T6: the separable matrix-product adjoint equals the per-pixel sum."""
    uv, n, fov, rng = _small(3, L=211, n=12, fov=0.25)
    h = rng.normal(size=uv.shape[0]) + 1j * rng.normal(size=uv.shape[0])
    full = operator.adjoint(uv, n, fov, h)
    pix = np.arange(n * n)
    direct = operator.adjoint_pixels(uv, n, fov, h, pix).reshape(n, n)
    assert np.max(np.abs(full - direct)) <= 1e-13 * np.max(np.abs(direct))


def test_adjoint_per_pixel_brute_loop():
    """T6 (tiny): a pure-Python double loop over k for two pixels."""
    uv, n, fov, rng = _small(4, L=40, n=8, fov=0.2)
    h = rng.normal(size=40) + 1j * rng.normal(size=40)
    full = operator.adjoint(uv, n, fov, h)
    d = fov / n
    for (i, j) in ((0, 0), (5, 2)):
        l, m = (i - n // 2) * d, (j - n // 2) * d
        acc = 0.0
        for k in range(40):
            acc += (h[k] * complex(math.cos(2 * math.pi * (uv[k, 0] * l + uv[k, 1] * m)),
                                   math.sin(2 * math.pi * (uv[k, 0] * l + uv[k, 1] * m)))).real
        assert abs(full[i, j] - acc / math.sqrt(1 - l * l - m * m)) <= 1e-12 * abs(acc)


def test_dirty_image_of_one_source_is_shifted_psf():
    """T7: (Phi* Phi delta_p)[q] n_q n_p = P(l_q - l_p, m_q - m_p), w = 0."""
    uv, n, fov, _ = _small(5, L=180, n=10, fov=0.2)
    p_i, p_j = 2, 7
    img = operator.adjoint(uv, n, fov, operator.forward(uv, n, fov, [p_i * n + p_j], [1.0]))
    l = geometry.direction_cosines(n, fov)
    nn = geometry.n_term(n, fov)
    for (q_i, q_j) in ((2, 7), (0, 0), (9, 3), (5, 5)):
        want = operator.psf(uv, l[q_i] - l[p_i], l[q_j] - l[p_j])
        got = img[q_i, q_j] * nn[q_i, q_j] * nn[p_i, p_j]
        assert abs(got - want) <= 1e-12 * uv.shape[0]


def test_peak_of_psf_is_L():
    uv, n, fov, _ = _small(6)
    assert operator.psf(uv, 0.0, 0.0) == uv.shape[0]


def test_hermitian_half_doubles_adjoint():
    """Appending the conjugate half (-u, -v, conj V) doubles Phi* V."""
    uv, n, fov, rng = _small(7, L=90, n=8, fov=0.2)
    h = rng.normal(size=90) + 1j * rng.normal(size=90)
    a1 = operator.adjoint(uv, n, fov, h)
    a2 = operator.adjoint(np.concatenate([uv, -uv]), n, fov, np.concatenate([h, h.conj()]))
    assert np.allclose(a2, 2 * a1, rtol=1e-12, atol=1e-12)


def test_orthogonal_design_normal_operator_is_diagonal():
    """With uv on the n x n DFT frequencies, Phi* Phi = n^2 diag(1/n_p^2)."""
    n, fov = 8, 0.3
    uv = sim.orthogonal_uv(n, fov)
    nn = geometry.n_term(n, fov).reshape(-1)
    for p in (0, 9, 36, 63):
        col = operator.adjoint(uv, n, fov, operator.forward(uv, n, fov, [p], [1.0])).reshape(-1)
        want = np.zeros(n * n)
        want[p] = n * n / nn[p] ** 2
        assert np.max(np.abs(col - want)) <= 1e-10 * n * n


def test_restricted_adjoint_matches_full_on_support():
    uv, n, fov, rng = _small(8, L=120, n=16)
    h = rng.normal(size=120) + 1j * rng.normal(size=120)
    pix = np.array([0, 17, 100, 255])
    full = operator.adjoint(uv, n, fov, h).reshape(-1)
    assert np.allclose(operator.restricted_adjoint(uv, n, fov, h, pix), full[pix],
                       rtol=1e-12, atol=1e-12)


def test_forward_images_equals_forward_per_image():
    """The batched dense forward is the sparse forward applied column by column."""
    rng = np.random.default_rng(77)
    n, fov, L = 12, 0.2, 90
    uv = rng.uniform(-8, 8, size=(L, 2))
    imgs = rng.normal(size=(n * n, 3))
    got = operator.forward_images(uv, n, fov, imgs)
    for c in range(3):
        want = operator.forward(uv, n, fov, np.arange(n * n), imgs[:, c])
        assert np.max(np.abs(got[:, c] - want)) <= 1e-12 * np.max(np.abs(want))


# --- the w-term (Sect. 2.1, Eq. phi-plane: W(l, m; w) = exp(-j 2 pi w (n - 1))) ---

def _small_w(seed=0, L=300, n=16, fov=0.6):
    rng = np.random.default_rng(seed)
    uvw = rng.uniform(-40, 40, size=(L, 3))
    return uvw, n, fov, rng


def test_w_phase_centre_source_is_constant():
    """At the phase centre n = 1, so W = 1 whatever w: V_k = a."""
    uvw, n, fov, _ = _small_w()
    p = (n // 2) * n + n // 2
    V = operator.forward(uvw, n, fov, [p], [2.5])
    assert np.allclose(V, 2.5, rtol=1e-15, atol=0)


def test_w_forward_is_the_spherical_phase_in_any_frame():
    """Eq. phi-sphere referred to the phase centre r0 = (0, 0, 1): a source at
    direction r = (l, m, n) gives V_k = (a / n) exp(-j 2 pi <r - r0, p_k>),
    p_k = (u, v, w).  The inner product is evaluated here on 3-vectors rotated
    into a random orthonormal frame (it is rotation invariant), a route
    independent of the oracle's tangent-plane formula."""
    uvw, n, fov, rng = _small_w(1)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    for (i, j) in ((2, 13), (11, 4), (0, 0)):
        d = fov / n
        l, m = (i - n // 2) * d, (j - n // 2) * d
        nn = math.sqrt(1 - l * l - m * m)
        r = q @ np.array([l, m, nn])
        r0 = q @ np.array([0.0, 0.0, 1.0])
        pk = uvw @ q.T
        want = 0.8 / nn * np.exp(-2j * math.pi * (pk @ (r - r0)))
        got = operator.forward(uvw, n, fov, [i * n + j], [0.8])
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("seed", [0, 1])
def test_w_adjoint_dot_product(seed):
    """<Phi x, h>_R = <x, Phi* h> with the w-term (dense x, random h)."""
    uvw, n, fov, rng = _small_w(seed, L=211, n=14, fov=0.8)
    x = rng.normal(size=(n, n))
    h = rng.normal(size=uvw.shape[0]) + 1j * rng.normal(size=uvw.shape[0])
    lhs = float(np.vdot(h, operator.forward_dense(uvw, n, fov, x)).real)
    rhs = float(np.sum(x * operator.adjoint(uvw, n, fov, h)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def test_w_direct_adjoint_reduces_to_the_coplanar_one():
    """A negligible w sends the adjoint through the per-pixel direct sum; it
    must equal the separable (pinned) coplanar evaluation."""
    uvw, n, fov, rng = _small_w(3, L=250, n=12, fov=0.5)
    h = rng.normal(size=uvw.shape[0]) + 1j * rng.normal(size=uvw.shape[0])
    tiny = uvw.copy()
    tiny[:, 2] = 1e-300
    a = operator.adjoint(tiny, n, fov, h)
    b = operator.adjoint(uvw[:, :2], n, fov, h)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_w_dirty_image_at_the_source_pixel():
    """Phi* Phi delta_p at p itself: every phase cancels, so the value is
    L / n_p^2 whatever the w of the visibilities."""
    uvw, n, fov, _ = _small_w(4)
    for p in (5, 3 * n + 9, n * n - 1):
        V = operator.forward(uvw, n, fov, [p], [1.0])
        img = operator.adjoint_pixels(uvw, n, fov, V, [p])
        _, _, npp = geometry.pixel_coords(np.array([p]), n, fov)
        assert abs(img[0] - uvw.shape[0] / npp[0] ** 2) <= 1e-12 * uvw.shape[0]


def test_generator_w_keeps_the_baseline_length():
    """Earth rotation only rotates a baseline: u^2 + v^2 + w^2 is the squared
    baseline length in wavelengths at every snapshot."""
    p = sim.config_c2(n_snap=5, npix=64, keep_w=True)
    nbl = 60 * 59 // 2
    b2 = (p.uv ** 2).sum(axis=1).reshape(5, nbl)
    assert np.allclose(b2, b2[0][None, :], rtol=1e-12)
    assert np.max(np.abs(p.uv[:, 2])) > 100.0
