"""The oracle's Maxwell-residual and energy diagnostics (Sec. IV-A), pinned by
exact solutions of Maxwell's equations (plane wave, oscillating dipole, a
plane-wave pulse), fields that violate them, and a closed-form energy."""
import math

import numpy as np

import workloads

K = 2 * math.pi


def plane_wave(pts, k, flip_b=False):
    """E = x e^{ikz}, B = y e^{ikz}: curl E = ik B, curl B = -ik E (e^{-ikt})."""
    ph = np.exp(1j * k * pts[:, 2])
    E = np.zeros((pts.shape[0], 3), complex)
    B = np.zeros_like(E)
    E[:, 0] = ph
    B[:, 1] = -ph if flip_b else ph
    return E, B


def dipole(pts, k):
    """Fields of an oscillating electric dipole p = z at the origin (c = 1, e^{-ikt})."""
    r = np.linalg.norm(pts, axis=1)[:, None]
    n = pts / r
    p = np.array([0.0, 0.0, 1.0])
    g = np.exp(1j * k * r) / (4 * math.pi)
    nxp = np.cross(n, p)
    E = g * (k * k * np.cross(nxp, n) / r + (3 * n * (n @ p)[:, None] - p) * (1 / r ** 3 - 1j * k / r ** 2))
    B = g * k * k * nxp / r * (1 - 1 / (1j * k * r))
    return E, B


def test_stencil_layout(orc):
    s = orc.stencil(np.array([[1.0, 2.0, 3.0]]), 0.5).reshape(13, 3)
    assert np.array_equal(s[0], [1, 2, 3])
    assert np.array_equal(s[1:5, 0], [0.0, 0.5, 1.5, 2.0]) and np.all(s[1:5, 1:] == [2, 3])
    assert np.array_equal(s[9:13, 2], [2.0, 2.5, 3.5, 4.0]) and np.all(s[9:13, :2] == [1, 2])


def test_residual_freq_vanishes_for_exact_fields(orc):
    h = 0.01
    pts = np.array([[0.3, -0.2, 0.1], [1.0, 0.5, -0.7], [-0.4, 0.9, 1.3]])
    st = orc.stencil(pts, h)
    ks = [K, 1.5 * K]
    for field in (plane_wave, dipole):
        E = np.stack([field(st, k)[0] for k in ks])
        B = np.stack([field(st, k)[1] for k in ks])
        ef = orc.maxwell_residual_freq(ks, E, B, len(pts), h)
        assert ef.shape == (2, 3) and ef.max() < 2e-5, (field.__name__, ef.max())   # (kh)^4 at kh ~ 0.1
    # a field that breaks Maxwell's equations: B of the wrong sign
    E, B = plane_wave(st, K, flip_b=True)
    ef = orc.maxwell_residual_freq([K], E[None], B[None], len(pts), h)
    assert ef.min() > 1.0
    # and a dipole whose B is the transverse part only is caught too
    E, B = dipole(st, K)
    ef = orc.maxwell_residual_freq([K], E[None], (B * 1.01)[None], len(pts), h)
    assert ef.max() > 1e-3


def test_residual_freq_converges_at_fourth_order(orc):
    pts = np.array([[0.6, 0.4, 0.5]])
    errs = []
    for h in (0.08, 0.04):
        st = orc.stencil(pts, h)
        E, B = dipole(st, K)
        errs.append(orc.maxwell_residual_freq([K], E[None], B[None], 1, h).max())
    assert 12 < errs[0] / errs[1] < 20     # 2^4 = 16


def test_residual_of_the_reflected_field(orc):
    # the paper's check: Maxwell's equations near focus; curl-consistent beam ~ FD error, literal beam ~ 1e-2
    m = orc.mirror(20.0, 40.0, 80, 64)
    pts = np.array([[0.3, 0.2, 0.1], [-0.5, 0.1, 0.4]])
    h = 0.01
    st = orc.stencil(pts, h)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 20.0)
    E, B = orc.reflected_field(m, [K], Ei, Bi, st)
    assert orc.maxwell_residual_freq([K], E, B, 2, h).max() < 5e-6
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN, 20.0)
    E, B = orc.reflected_field(m, [K], Ei, Bi, st)
    assert orc.maxwell_residual_freq([K], E, B, 2, h).max() > 1e-3


def test_residual_time_vanishes_for_a_plane_wave_pulse(orc):
    k0, n = K, 21
    ks = k0 + 0.05 * k0 * np.linspace(-1, 1, n)
    dk = ks[1] - ks[0]
    amp = np.exp(-np.linspace(-2, 2, n) ** 2)
    pts = np.array([[0.1, 0.2, 0.0], [0.0, 0.0, 0.3], [-0.2, 0.1, -0.1]])
    h, dt = 0.01, 0.007     # unequal steps: the space and time difference errors do not cancel
    st = orc.stencil(pts, h)
    E = np.stack([a * plane_wave(st, k)[0] for a, k in zip(amp, ks)])
    B = np.stack([a * plane_wave(st, k)[1] for a, k in zip(amp, ks)])
    t = np.array([-0.5, 0.0, 0.25])
    et = orc.maxwell_residual_time(ks, dk, t, dt, E, B, len(pts), h)
    assert et.shape == (3, 3) and et.max() < 2e-5
    E2 = np.stack([a * plane_wave(st, k, flip_b=True)[0] for a, k in zip(amp, ks)])
    B2 = np.stack([a * plane_wave(st, k, flip_b=True)[1] for a, k in zip(amp, ks)])
    assert orc.maxwell_residual_time(ks, dk, t, dt, E2, B2, len(pts), h).max() > 1.0


def test_field_energy_closed_form(orc):
    # one frequency, F = x e^{ikz} (E) and y e^{ikz} (B), dk = 1: physical E = 2 cos(k (z - t)) x, so the
    # energy density 1/2 (E^2 + B^2) = 4 cos^2; sampling whole wavelengths uniformly sums cos^2 to N/2
    n_per, n_waves = 7, 3
    z = np.arange(n_per * n_waves) / n_per
    pts = np.stack([np.zeros_like(z), np.zeros_like(z), z], axis=1)
    E, B = plane_wave(pts, K)
    dV = 0.37
    W = orc.field_energy([K], 1.0, np.array([0.0, 0.13, 0.5]), E[None], B[None], dV)
    np.testing.assert_allclose(W, 2.0 * dV * len(z), rtol=1e-13)
    # and the time transform of a broadband pulse conserves the sum over a periodic box only on average
    assert np.all(np.isfinite(W))
