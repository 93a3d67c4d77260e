"""CPU tests of the focal-spot analysis that bench.py applies to the Table I workload:
peak intensity I_E = c E^2 / 2 and the FWHM / eccentricity of the focal spot, on a synthetic
field with a known elliptical Gaussian intensity."""
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def synthetic(n=81, half=2.0e-6, fx=0.8e-6, fy=0.5e-6, peak_field=3.0e12, t_peak=5):
    s = np.linspace(-half, half, n)
    yy, xx = np.meshgrid(s, s, indexing="ij")
    # intensity exp(-4 ln2 (x^2/fx^2 + y^2/fy^2)): field amplitude is its square root
    amp = peak_field * np.exp(-2.0 * math.log(2.0) * (xx ** 2 / fx ** 2 + yy ** 2 / fy ** 2))
    n_t = 11
    Et = np.zeros((n_t, n * n, 3), np.complex64)
    Bt = np.zeros_like(Et)
    for t in range(n_t):
        scale = math.exp(-((t - t_peak) / 3.0) ** 2)
        Et[t, :, 0] = 0.5 * scale * amp.ravel()       # physical field 2 Re E
        Bt[t, :, 2] = 0.25 * scale * amp.ravel()
    return Et, Bt, n, half


def test_focal_spot_recovers_a_known_ellipse():
    Et, Bt, n, half = synthetic()
    r = bench.focal_spot(Et, Bt, n, half)
    assert r["time_index"] == 5
    assert abs(r["peak_x_m"]) < 1e-12 and abs(r["peak_y_m"]) < 1e-12
    expect_I = 0.5 * bench.C_LIGHT * 3.0e12 ** 2 * 1e-4
    assert math.isclose(r["peak_intensity_W_cm2"], expect_I, rel_tol=1e-5)
    assert math.isclose(r["fwhm_x_m"], 0.8e-6, rel_tol=0.02)
    assert math.isclose(r["fwhm_y_m"], 0.5e-6, rel_tol=0.02)
    assert math.isclose(r["eccentricity"], math.sqrt(1 - (0.5 / 0.8) ** 2), rel_tol=0.03)
    assert math.isclose(r["max_Bz_over_max_Ex"], 0.5, rel_tol=1e-6)
    assert r["max_Ez_over_max_Ex"] == 0.0


def test_fwhm_is_none_when_the_profile_does_not_fall_to_half():
    cut = np.array([0.9, 0.95, 1.0, 0.95, 0.9])
    assert bench._fwhm(cut, 2, 1.0) is None
    cut = np.array([0.0, 0.5, 1.0, 0.5, 0.0])
    assert math.isclose(bench._fwhm(cut, 2, 1.0), 2.0)
