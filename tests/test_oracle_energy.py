"""Energy normalisation of the incident spectrum (Sec. III-B) in the oracle,
pinned by closed forms, the discrete total-energy identity and the values
Table I and Fig. 1 print for the super-Gaussian pulse."""
import json
import math
import os

import numpy as np
import pytest

import workloads

K = 2 * math.pi
C = workloads.C_LIGHT
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_fig1.json")


def _fwhm(x, y):
    """Full width at half maximum of a single-peaked sampled curve (linear interpolation)."""
    y = np.asarray(y, float) / np.max(y)
    i0 = int(np.argmax(y))
    lo = i0
    while y[lo] > 0.5:
        lo -= 1
    hi = i0
    while y[hi] > 0.5:
        hi += 1
    xl = x[lo] + (0.5 - y[lo]) / (y[lo + 1] - y[lo]) * (x[lo + 1] - x[lo])
    xr = x[hi - 1] + (0.5 - y[hi - 1]) / (y[hi] - y[hi - 1]) * (x[hi] - x[hi - 1])
    return xr - xl


def test_power_closed_forms(orc):
    f, a = 20.0, 25.0
    m = orc.mirror(f, a, 60, 32)
    ks = [K, 1.3 * K]
    Ei, Bi = orc.incident_tables(m, ks, orc.PLANE)
    np.testing.assert_allclose(orc.incident_power(m, Ei, Bi), 4 * math.pi * math.pi * a * a, rtol=1e-13)
    for w0 in (8.0, 25.0, 60.0):          # from nearly unclipped to strongly clipped
        lit = 4 * math.pi * (math.pi * w0 * w0 / 2) * (1 - math.exp(-2 * a * a / (w0 * w0)))
        for pol in (0.0, 0.4, math.pi / 2):
            Ei, Bi = orc.incident_tables(m, ks, orc.GAUSSIAN, w0, pol=pol)
            np.testing.assert_allclose(orc.incident_power(m, Ei, Bi), lit, rtol=1e-12)
    w0 = 5.0
    Ei, Bi = orc.incident_tables(m, ks, orc.GAUSSIAN_CONSISTENT, w0)
    ex = [4 * math.pi * (math.pi * w0 * w0 / 2) * (1 + 1 / (k * w0) ** 2) for k in ks]
    np.testing.assert_allclose(orc.incident_power(m, Ei, Bi), ex, rtol=1e-12)


def test_power_is_quadratic_in_the_spectrum(orc):
    m = orc.mirror(20.0, 25.0, 30, 16)
    ks = np.array([K, 1.1 * K, 1.2 * K])
    amp = np.array([0.5 + 0.2j, 2.0, -1j])
    E1, B1 = orc.incident_tables(m, ks, orc.GAUSSIAN_CONSISTENT, 6.0)
    E2, B2 = orc.incident_tables(m, ks, orc.GAUSSIAN_CONSISTENT, 6.0, spectrum=amp)
    np.testing.assert_allclose(orc.incident_power(m, E2, B2), orc.incident_power(m, E1, B1) * np.abs(amp) ** 2,
                               rtol=1e-13)


def test_energy_amplitudes_meet_the_total_energy(orc):
    w = workloads.table1(n_k=12, n_nodes=24).subset(obs_idx=[0])
    m = orc.mirror(w.f, w.a, w.n_r, w.n_phi)
    Ei, Bi = orc.incident_tables(m, w.k, orc.GAUSSIAN, w.w0)
    P = orc.incident_power(m, Ei, Bi)
    eps, e_tot = w.meta["eps"], w.meta["e_tot"]
    amp = orc.energy_amplitudes(P, eps, e_tot, w.dk)
    E2, B2 = orc.incident_tables(m, w.k, orc.GAUSSIAN, w.w0, spectrum=amp)
    P2 = orc.incident_power(m, E2, B2)
    assert abs(P2.sum() * w.dk / e_tot - 1) < 1e-13            # the discrete total-energy condition
    np.testing.assert_allclose(P2 / P2.max(), eps / eps.max(), rtol=1e-12)   # the spectral shape


def test_table1_spectrum_and_pulse_match_fig1(orc):
    g = json.load(open(GOLDEN))
    T, F = g["table1"], g["fig1"]
    lam_c, dlam, order = T["lambda_c_nm"] * 1e-9, T["delta_lambda_nm"] * 1e-9, T["order_n"]
    # spectral FWHM of the power spectrum (printed to two figures)
    k, eps, _ = workloads.super_gaussian_power(20001, lam_c, dlam, order)
    lam = 2 * math.pi / k
    assert abs(_fwhm(lam[::-1], eps[::-1]) * 1e9 - F["spectral_fwhm_nm"]) < 2.5
    # main-pulse duration from the energy-normalised components (Fig. 1 sampling: 100 samples)
    k, eps, dk = workloads.super_gaussian_power(F["frequency_samples"], lam_c, dlam, order)
    amp = orc.energy_amplitudes(np.ones_like(eps), eps, T["E_tot_J"], dk)
    t = np.linspace(-40e-15, 40e-15, 4001) * C
    Et = orc.time_transform(k, dk, t, amp[:, None])[:, 0]
    dur = _fwhm(t / C * 1e15, np.abs(Et))
    assert abs(dur / F["main_pulse_fwhm_fs"] - 1) < 0.05, dur
    # the plain power spectrum used as the amplitude (a plausible slip) misses it
    Et2 = orc.time_transform(k, dk, t, eps[:, None].astype(complex))[:, 0]
    assert abs(_fwhm(t / C * 1e15, np.abs(Et2)) / F["main_pulse_fwhm_fs"] - 1) > 0.05
