"""Pins for the oracle's geometry against the printed tables (T1, T2)."""
import json
import math
import os

import numpy as np

from oracle import geometry

GOLD = os.path.join(os.path.dirname(__file__), "golden", "resolution_tables.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def test_table2_pixel_sizes_are_fov_over_n():
    """Table 2's SRF columns equal FOV/n with n from Table A.1 (FOV 5 deg)."""
    g = _gold()
    fov = g["fov_deg_dataset_I"] * math.pi / 180
    t2 = g["table2_resolution_arcsec"]["rows"]
    ta = g["tableA1_pix_per_side"]["rows"]
    for r2, ra in zip(t2, ta):
        assert r2[0] == ra[0]
        for col in (2, 3, 4):
            arcsec = geometry.rad_to_arcsec(geometry.pixel_step(ra[col], fov))
            assert abs(arcsec - r2[col]) <= 0.05 + 1e-9, (r2, ra, col, arcsec)


def test_table1_resolutions():
    g = _gold()["table1"]
    for key in ("dataset_II", "dataset_III"):
        d = g[key]
        used = geometry.rad_to_arcsec(geometry.pixel_step(d["npix"], d["fov_deg"] * math.pi / 180))
        assert abs(used - d["used_arcsec"]) <= 0.05 + 1e-9
        b0 = d["longest_baseline_wavelengths"]
        nom = geometry.rad_to_arcsec(geometry.nominal_resolution(np.array([[b0, 0.0, 0.0]])))
        assert abs(nom - d["nominal_arcsec"]) <= 0.05 + 1e-9


def test_nominal_resolution_dataset_I_endpoints():
    """Table 1's longest baselines (195 and 3241 wavelengths, printed to the
    unit) bracket Table 2's nominal resolutions at r_max 0.3 km and 6 km."""
    g = _gold()
    lo, hi = g["table1"]["dataset_I_longest_baseline_wavelengths"]
    t2 = g["table2_resolution_arcsec"]["rows"]
    for b0, printed in ((lo, t2[0][1]), (hi, t2[-1][1])):
        r_hi = geometry.rad_to_arcsec(1.0 / (3.0 * (b0 - 0.5)))
        r_lo = geometry.rad_to_arcsec(1.0 / (3.0 * (b0 + 0.5)))
        assert r_lo - 0.05 <= printed <= r_hi + 0.05


def test_super_resolution_factor_dataset_II():
    g = _gold()
    d = g["table1"]["dataset_II"]
    nom = geometry.nominal_resolution(np.array([[d["longest_baseline_wavelengths"], 0.0, 0.0]]))
    used = geometry.pixel_step(d["npix"], d["fov_deg"] * math.pi / 180)
    assert abs(nom / used - g["dataset_II_super_resolution_factor"]) <= 0.005


def test_nominal_resolution_uses_3d_norm():
    uvw = np.array([[3.0, 4.0, 0.0], [1.0, 1.0, 1.0], [0.0, 0.0, -2.0]])
    assert geometry.nominal_resolution(uvw) == 1.0 / 15.0


def test_direction_cosines_centring():
    l = geometry.direction_cosines(8, 0.08)
    assert np.allclose(l, (np.arange(8) - 4) * 0.01, rtol=0, atol=1e-17)
    assert l[4] == 0.0
    nn = geometry.n_term(8, 0.08)
    assert nn[4, 4] == 1.0
    assert np.isclose(nn[0, 0], math.sqrt(1 - 2 * 0.04 ** 2), rtol=1e-15)
    assert np.isclose(nn[0, 4], math.sqrt(1 - 0.04 ** 2), rtol=1e-15)


def test_wavelength_conversion():
    uv = geometry.wavelengths(np.array([[299.792458, -599.584916]]), 1e6)
    assert np.allclose(uv, [[1.0, -2.0]], rtol=1e-15)
