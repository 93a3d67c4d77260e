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
