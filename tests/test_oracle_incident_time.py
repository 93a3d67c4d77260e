"""Pins of the oracle's incident-beam generator and of its semi-discrete transform.

Incident beams (Sec. III-A, collimated beam travelling along -z):
  * the plane wave is an exact Maxwell field: curl E = ik B, curl B = -ik E;
  * the curl-consistent Gaussian satisfies div E = div B = 0 and
    curl B = -ik E exactly, and curl E = ik B up to O(1/(k w0)^2);
  * the literal Gaussian equals the plane wave on the axis.

Time reconstruction (Sec. III-B, eq. impl.semiDiscreteFFT):
  F(t) = sum_n F_n e^{-i k_n t} dk.
  * one sample is a pure carrier;
  * a flat spectrum on a uniform grid sums to the Dirichlet kernel
    e^{-i k_0 t} dk (1 - e^{-i N dk t}) / (1 - e^{-i dk t});
  * the sum is periodic with period 2 pi / dk (up to the carrier phase);
  * a Gaussian spectrum sampled to +-6 sigma reproduces the continuous
    transform sqrt(2 pi) sigma e^{-i k_c t} e^{-sigma^2 t^2 / 2}.
"""
import math

import numpy as np
import pytest

import workloads

K = 2 * math.pi


def _fd(orc, kind, p0, h, w0=3.0, pol=0.3):
    pts = [p0]
    for ax in range(3):
        for s in (-2, -1, 1, 2):
            d = np.zeros(3)
            d[ax] = s * h
            pts.append(p0 + d)
    E, B = orc.incident(kind, np.array(pts), K, w0, pol)
    dE = np.zeros((3, 3), complex)
    dB = np.zeros((3, 3), complex)
    for ax in range(3):
        sl = slice(1 + 4 * ax, 5 + 4 * ax)
        for D, F in ((dE, E), (dB, B)):
            fm2, fm1, fp1, fp2 = F[sl]
            D[ax] = (fm2 - 8 * fm1 + 8 * fp1 - fp2) / (12 * h)
    return E[0], B[0], dE, dB


def _curl(d):
    return np.array([d[1, 2] - d[2, 1], d[2, 0] - d[0, 2], d[0, 1] - d[1, 0]])


def test_plane_wave_is_maxwell(orc):
    E, B, dE, dB = _fd(orc, orc.PLANE, np.array([0.2, -0.4, 0.7]), 1e-3)
    assert np.abs(_curl(dE) - 1j * K * B).max() < 1e-8
    assert np.abs(_curl(dB) + 1j * K * E).max() < 1e-8
    np.testing.assert_allclose(E, [math.cos(0.3) * np.exp(-1j * K * 0.7), math.sin(0.3) * np.exp(-1j * K * 0.7), 0],
                               atol=1e-15)


def test_consistent_gaussian_divergence_free_and_curl_b(orc):
    for p0 in [np.array([0.2, -0.4, 0.7]), np.array([1.5, 2.0, -0.3])]:
        E, B, dE, dB = _fd(orc, orc.GAUSSIAN_CONSISTENT, p0, 1e-3)
        s = K * max(np.abs(E).max(), 1e-3)
        assert abs(np.trace(dE)) / s < 1e-8
        assert abs(np.trace(dB)) / s < 1e-8
        assert np.abs(_curl(dB) + 1j * K * E).max() / s < 1e-8
        # curl E - ik B is the paraxial residual, O(1/(k w0)^2) relative
        r = np.abs(_curl(dE) - 1j * K * B).max() / s
        assert 1e-6 < r < 10 / (K * 3.0) ** 2


def test_literal_gaussian_on_axis_equals_plane_wave(orc):
    pts = np.array([[0.0, 0.0, -3.1], [0.0, 0.0, 2.0]])
    Eg, Bg = orc.incident(orc.GAUSSIAN, pts, K, 5.0)
    Ep, Bp = orc.incident(orc.PLANE, pts, K)
    np.testing.assert_allclose(Eg, Ep, atol=1e-15)
    np.testing.assert_allclose(Bg, Bp, atol=1e-15)
    np.testing.assert_allclose(Bp[:, 1], -Ep[:, 0], atol=0)


def test_time_single_frequency_is_carrier(orc):
    k0, dk = 7.3, 0.25
    t = np.linspace(-3, 3, 11)
    F = np.array([[1.5 - 0.5j, 2.0j]])
    Ft = orc.time_transform([k0], dk, t, F)
    expect = F[0][None, :] * np.exp(-1j * k0 * t)[:, None] * dk
    np.testing.assert_allclose(Ft, expect, rtol=1e-15, atol=1e-15)


def test_time_flat_spectrum_dirichlet_kernel(orc):
    n, k0, dk = 37, 5.0, 0.125
    k = k0 + dk * np.arange(n)
    t = np.linspace(-20.0, 20.0, 81) + 1e-3
    Ft = orc.time_transform(k, dk, t, np.ones((n, 1)))[:, 0]
    z = np.exp(-1j * dk * t)
    expect = np.exp(-1j * k0 * t) * dk * (1 - z ** n) / (1 - z)
    np.testing.assert_allclose(Ft, expect, rtol=1e-13, atol=1e-14)


def test_time_periodicity(orc):
    rng = np.random.default_rng(3)
    n, k0, dk = 16, 4.0, 0.5
    k = k0 + dk * np.arange(n)
    F = rng.normal(size=(n, 4)) + 1j * rng.normal(size=(n, 4))
    T = 2 * math.pi / dk
    t = np.array([0.3, 1.7])
    a = orc.time_transform(k, dk, t, F)
    b = orc.time_transform(k, dk, t + T, F)
    np.testing.assert_allclose(b, a * np.exp(-1j * k0 * T), rtol=1e-13, atol=1e-13)


def test_time_gaussian_pulse(orc):
    k, amp, dk = workloads.gaussian_spectrum(129, n_sigma=6.0)
    sigma = 2.0 * math.sqrt(math.log(2.0)) / workloads.TAU_FWHM / workloads.C_LIGHT
    kc = 2 * math.pi / workloads.LAMBDA0
    t = np.linspace(-3.0 / sigma, 3.0 / sigma, 25)
    Ft = orc.time_transform(k, dk, t, amp[:, None])[:, 0]
    expect = math.sqrt(2 * math.pi) * sigma * np.exp(-1j * kc * t) * np.exp(-(sigma * t) ** 2 / 2)
    # truncation at 6 sigma and the (exponentially small) aliasing are < 1e-7 relative
    assert np.abs(Ft - expect).max() / abs(expect).max() < 1e-7


def test_time_large_phase_is_exact(orc):
    """k t up to 2e7 rad: one sample at k = 2 pi (as a double, 2 pi + eps with eps = sin(k)) gives
    F(t) = e^{-i k t} = e^{-i (eps t + 2 pi t)}; for t an integer plus a quarter that is
    -i e^{-i eps t} exactly.  A phase rounded to a 64-bit mantissa would be off by ~5e-13 rad here."""
    k = K
    eps = math.sin(k)                    # k - 2 pi, to ~1e-48
    t = np.array([1e5, 1e6 + 0.25, 3e6 + 0.5, 3e6 + 0.75])
    F = orc.time_transform([k], 1.0, t, np.ones((1, 1), complex))[:, 0]
    turn = np.array([1.0, -1j, -1.0, 1j])   # e^{-2 pi i t} for the fractional parts 0, 1/4, 1/2, 3/4
    ref = turn * np.exp(-1j * eps * t)
    assert np.abs(F - ref).max() < 1e-15, np.abs(F - ref)


def test_time_focus_closed_form_pulse(orc):
    """The focus closed form of a plane wave (P1) under a Gaussian spectral amplitude A(k),
    transformed to time by the oracle's chain (reflected field, then the semi-discrete sum), equals
    the direct sum of the closed form: E_x(t) = dk sum_n E_ref(k_n) A(k_n) e^{-i k_n t}."""
    f, a = 20.0, 25.0
    U = a * a / (4 * f)
    ks = K * (1 + 0.05 * np.linspace(-3, 3, 25))
    dk = ks[1] - ks[0]
    A = np.exp(-((ks - K) / (0.05 * K)) ** 2 / 2)
    m = orc.mirror(f, a, 80, 32)
    Ei, Bi = orc.incident_tables(m, ks, orc.PLANE, spectrum=A)
    E, B = orc.reflected_field(m, ks, Ei, Bi, np.zeros((1, 3)))
    t = 2 * f + np.linspace(-30, 30, 13)
    Et = orc.time_transform(ks, dk, t, E)[:, 0]
    Bt = orc.time_transform(ks, dk, t, B)[:, 0]
    ph = np.exp(2j * ks * f)
    ex = ph * (2j * ks * f * U / (f + U) + U * (U - 2 * f) / (f + U) ** 2 - 2j * f * U / (ks * (f + U) ** 3))
    by = ph * (2j * ks * f * U / (f + U) - U * (U + 2 * f) / (f + U) ** 2)
    tw = np.exp(-1j * np.outer(t, ks)) * dk
    ref_x, ref_y = tw @ (ex * A), tw @ (by * A)
    scale = np.abs(ref_x).max()
    assert np.abs(Et[:, 0] - ref_x).max() < 1e-12 * scale
    assert np.abs(Bt[:, 1] - ref_y).max() < 1e-12 * scale
    assert np.abs(Et[:, 1:]).max() < 1e-12 * scale
