"""Pins of the oracle's Laguerre-Gauss incident beams (Sec. III-A uses the Laguerre-Gauss modes of
the paraxial wave equation as the expansion basis of linearly and radially polarised beams).

The mode u_{p,l} = C (sqrt(2) r / w0)^|l| L_p^|l|(2 r^2 / w0^2) exp(-r^2 / w0^2) e^{i l phi} carried
along -z is checked against what fixes it independently of the oracle's own formula:

* the generalized Laguerre polynomial against scipy's (a library routine);
* LG_00 is the oracle's literal Gaussian (pinned by the focus closed form) times sqrt(2/pi)/w0;
* the power through the aperture against its closed form: for p = 0 the regularized lower
  incomplete gamma function P(|l| + 1, 2 a^2 / w0^2), for any p the term-by-term integral of the
  squared Laguerre polynomial against e^{-t} (scipy's incomplete gamma), and 4 pi (unit power) for
  every mode over an aperture that holds the whole beam;
* orthogonality: modes of different l carry no cross power on the trapezoid rule, modes of the
  same l and different p none on the whole plane;
* the radially polarised beam is the combination of LG_{0,1} and LG_{0,-1} in x and y polarisation.
"""
import math

import numpy as np
import pytest
from scipy import special

K = 2 * math.pi


def aperture_power_closed_form(p, l, w0, a):
    """4 pi int_0^a |u_{p,l}|^2 2 pi r dr: with t = 2 r^2 / w0^2 the integrand is
    C^2 (pi w0^2 / 2) t^|l| L_p^|l|(t)^2 e^{-t}, integrated monomial by monomial."""
    al = abs(l)
    c2 = 2 * math.factorial(p) / (math.pi * math.factorial(p + al)) / w0 ** 2
    poly = special.genlaguerre(p, al) ** 2          # coefficients of L^2, highest power first
    T = 2 * a * a / (w0 * w0)
    total = 0.0
    for power, coef in enumerate(poly.coeffs[::-1]):
        s = al + power + 1
        total += coef * special.gammainc(s, T) * special.gamma(s)
    return 4 * math.pi * c2 * (math.pi * w0 * w0 / 2) * total


def test_laguerre_polynomial_against_scipy(orc):
    w0 = 1.7
    r = np.linspace(0.0, 3.0 * w0, 13)[1:]
    pts = np.stack([r, 0 * r, 0 * r], axis=-1)          # phi = 0, z = 0: E_x = u
    for p, l in [(0, 0), (1, 0), (2, 1), (3, 2), (5, 3), (4, -2)]:
        E, _ = orc.incident_lg([(p, l, 1.0, 0.0)], pts, K, w0)
        t = 2 * r * r / (w0 * w0)
        rest = np.sqrt(2 * math.factorial(p) / (math.pi * math.factorial(p + abs(l)))) / w0 * \
            (np.sqrt(t)) ** abs(l) * np.exp(-t / 2)
        lag = E[:, 0].real / rest
        ref = special.eval_genlaguerre(p, abs(l), t)
        assert np.abs(lag - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), (p, l)
        assert np.abs(E[:, 0].imag).max() < 1e-15 * np.abs(E[:, 0]).max()   # phi = 0: e^{i l phi} = 1


def test_lg00_is_the_gaussian(orc):
    w0 = 2.5
    pts = np.random.default_rng(3).uniform(-6, 6, size=(40, 3))
    E, B = orc.incident_lg([(0, 0, 1.0, 0.0)], pts, 1.3 * K, w0, amp=0.7 - 0.2j)
    Eg, Bg = orc.incident(orc.GAUSSIAN, pts, 1.3 * K, w0, amp=0.7 - 0.2j)
    c = math.sqrt(2 / math.pi) / w0
    assert np.abs(E - c * Eg).max() < 1e-15 * np.abs(Eg).max()
    assert np.abs(B - c * Bg).max() < 1e-15 * np.abs(Bg).max()
    # y polarisation is the Gaussian turned by 90 degrees
    E, B = orc.incident_lg([(0, 0, 0.0, 1.0)], pts, K, w0)
    Eg, Bg = orc.incident(orc.GAUSSIAN, pts, K, w0, pol=math.pi / 2)
    assert np.abs(E - c * Eg).max() < 1e-15 * np.abs(Eg).max()
    assert np.abs(B - c * Bg).max() < 1e-15 * np.abs(Bg).max()


@pytest.mark.parametrize("p,l", [(0, 0), (0, 1), (0, -3), (1, 0), (2, 1), (3, -2)])
def test_aperture_power_closed_form(orc, p, l):
    w0, a = 6.0, 9.0                                   # clipped: the aperture cuts the beam
    m = orc.mirror(20.0, a, 120, 64)
    Ei, Bi = orc.incident_lg_tables(m, [K, 1.2 * K], [(p, l, 1.0, 0.0)], w0)
    P = orc.incident_power(m, Ei, Bi)
    ex = aperture_power_closed_form(p, l, w0, a)
    assert np.abs(P / ex - 1).max() < 1e-12, (P, ex)
    if p == 0:   # the regularized incomplete gamma function, written out
        T = 2 * a * a / (w0 * w0)
        ex0 = 4 * math.pi * (1 - math.exp(-T) * sum(T ** j / math.factorial(j) for j in range(abs(l) + 1)))
        assert abs(ex / ex0 - 1) < 1e-13
    # an aperture that holds the whole beam: unit power per mode (the normalisation)
    m = orc.mirror(20.0, 7 * w0, 200, 64)
    Ei, Bi = orc.incident_lg_tables(m, [K], [(p, l, 0.6, 0.8j)], w0)
    assert abs(orc.incident_power(m, Ei, Bi)[0] / (4 * math.pi) - 1) < 1e-12


def test_orthogonality_through_the_power(orc):
    w0 = 6.0
    m = orc.mirror(20.0, 9.0, 80, 32)
    one = lambda modes: orc.incident_power(m, *orc.incident_lg_tables(m, [K], modes, w0))[0]  # noqa: E731
    # different l: exactly orthogonal on the trapezoid rule in phi (|l1 - l2| < n_phi), any aperture
    for m1, m2 in [((0, 1, 1.0, 0.0), (0, -1, 1.0, 0.0)), ((1, 2, 0.3, 0.0), (2, 0, 0.0, 0.5j)),
                   ((0, 0, 1.0, 0.0), (0, 3, 0.7, 0.0))]:
        assert abs(one([m1, m2]) - one([m1]) - one([m2])) < 1e-13 * one([m1, m2])
    # same l, different p: orthogonal on the whole plane, so with a = 7 w0 to exp(-98)
    m = orc.mirror(20.0, 7 * w0, 200, 32)
    for m1, m2 in [((0, 1, 1.0, 0.0), (2, 1, 1.0, 0.0)), ((1, 0, 1.0, 0.0), (3, 0, 0.0, -1.0))]:
        assert abs(one([m1, m2]) - one([m1]) - one([m2])) < 1e-12 * one([m1, m2])
        assert abs(one([m1, m2]) / (4 * math.pi) - 2) < 1e-12
    # x and y polarisation of the same mode do not interfere
    assert abs(one([(1, 1, 1.0, 1.0j)]) / (4 * math.pi) - 2) < 1e-12


def test_radial_beam_is_lg01_combination(orc):
    """(x, y) e^{-r^2/w0^2} / w0 = r^ (r / w0) e^{-r^2/w0^2}: x = r (e^{i phi} + e^{-i phi}) / 2 and
    y = r (e^{i phi} - e^{-i phi}) / 2i, so the radial beam is (LG_{0,1} + LG_{0,-1}) / (2 sqrt 2 C_{0,1})
    in x polarisation plus (LG_{0,1} - LG_{0,-1}) / (2i sqrt 2 C_{0,1}) in y polarisation."""
    w0 = 3.0
    c01 = math.sqrt(2 / math.pi) / w0
    al = 1 / (2 * math.sqrt(2) * c01)
    modes = [(0, 1, al, -1j * al), (0, -1, al, 1j * al)]
    pts = np.random.default_rng(8).uniform(-7, 7, size=(50, 3))
    E, B = orc.incident_lg(modes, pts, 1.1 * K, w0, amp=1.5 + 0.5j)
    Er, Br = orc.incident(orc.RADIAL, pts, 1.1 * K, w0, amp=1.5 + 0.5j)
    assert np.abs(E - Er).max() < 1e-14 * np.abs(Er).max()
    assert np.abs(B - Br).max() < 1e-14 * np.abs(Br).max()
