"""Closed-form pins of the oracle's reflected field (Sec. II, eq. stratton-chu-poa-og).

Plane-wave incidence E_inc = x e^{-ikz}, B_inc = -y e^{-ikz} (c = 1).

P1 -- paraboloid, field at the focus.  With r' = 0, R = |r_s| = f + r^2/4f and
R - z_s = 2f for every mirror point, so every phase is e^{2ikf}.  Writing
U = a^2/4f and integrating the three terms of the Stokes form over the
paraboloid analytically (the r-integrals are elementary; the logarithms of the
surface terms cancel):

  E_x = e^{2ikf} [ 2ikfU/(f+U) + U(U-2f)/(f+U)^2 - 2ifU/(k(f+U)^3) ]
  B_y = e^{2ikf} [ 2ikfU/(f+U) - U(U+2f)/(f+U)^2 ],  all other components 0.

  The last term of E_x comes from the rim line integral alone.  For f >> a the
  leading term is i k a^2/(2f) e^{2ikf}, the Fresnel focal amplitude.

P2 -- flat disk z = 0 of radius a, field on the axis at height z' (R_a = sqrt(a^2+z'^2)):

  E_x(0,0,z') = e^{ikR_a} - e^{ikz'} - (a^2/(2R_a^2)) (1 + i/(kR_a)) e^{ikR_a}.

  As a -> infinity this tends to -e^{ikz'}, the wave reflected by an infinite
  perfect conductor whose normal points toward the incoming beam.

Both closed forms are exact for the continuous integrals; the Gauss-Legendre x
trapezoid sums reach them to rounding because the integrands are smooth
(polynomial-times-exponential in r, trigonometric polynomials in phi).
"""
import math

import mpmath
import numpy as np
import pytest


def cis(*factors):
    """exp(i * prod(factors)) with the (large) phase formed and reduced in 50-digit arithmetic."""
    with mpmath.workdps(50):
        x = mpmath.mpf(1)
        for v in factors:
            x *= mpmath.mpf(v)
        return complex(mpmath.cos(x)) + 1j * complex(mpmath.sin(x))


def p1_closed_form(f, a, k):
    U = a * a / (4 * f)
    ph = cis(2, k, f)
    ex = ph * (2j * k * f * U / (f + U) + U * (U - 2 * f) / (f + U) ** 2 - 2j * f * U / (k * (f + U) ** 3))
    by = ph * (2j * k * f * U / (f + U) - U * (U + 2 * f) / (f + U) ** 2)
    return ex, by


# In SI units (k ~ 8e6 / m) each node coordinate, rounded to double, sits up to
# ~1e-17 m off the ideal paraboloid: ~5e-11 rad of phase per node, ~1e-13 after
# averaging over the nodes.  The closed form assumes the exact surface.
@pytest.mark.parametrize("f,a,tol", [(20.0, 40.0, 2e-14), (20.0, 25.0, 2e-14), (5.0, 15.0, 2e-14),
                                     (0.1, 0.075, 1e-12)])
def test_p1_focus_closed_form(orc, f, a, tol):
    # several wavenumbers in one call also pins the [n_k][n_obs][3] output layout
    lam = 1.0 if f > 1 else 800e-9
    ks = 2 * math.pi / lam * np.array([1.0, 1.07, 0.93])
    nr = 200 if f > 1 else 160
    m = orc.mirror(f, a, nr, 64)
    Ei, Bi = orc.incident_tables(m, ks, orc.PLANE)
    obs = np.zeros((2, 3))
    E, B = orc.reflected_field(m, ks, Ei, Bi, obs)
    for i, k in enumerate(ks):
        ex, by = p1_closed_form(f, a, k)
        for o in range(2):
            assert abs(E[i, o, 0] - ex) / abs(ex) < tol
            assert abs(B[i, o, 1] - by) / abs(by) < tol
            assert max(abs(E[i, o, 1]), abs(E[i, o, 2]), abs(B[i, o, 0]), abs(B[i, o, 2])) < 1e-12 * abs(ex)


def test_p1_line_term_is_the_rim_piece(orc):
    f, a, k = 20.0, 40.0, 2 * math.pi
    m = orc.mirror(f, a, 200, 64)
    Ei, Bi = orc.incident_tables(m, [k], orc.PLANE)
    E0, B0 = orc.reflected_field(m, [k], Ei, Bi, np.zeros((1, 3)), line_term=False)
    U = a * a / (4 * f)
    line = -cis(2, k, f) * (2 * f * U / (f + U) ** 2) * (1 + 1j / (k * (f + U)))
    ex, by = p1_closed_form(f, a, k)
    assert abs((ex - E0[0, 0, 0]) - line) / abs(line) < 1e-12
    assert abs(B0[0, 0, 1] - by) / abs(by) < 2e-14   # B has no line term


def test_p1_large_f_fresnel_limit(orc):
    a, k = 50.0, 2 * math.pi
    for f in [2000.0, 20000.0]:
        m = orc.mirror(f, a, 60, 32)
        Ei, Bi = orc.incident_tables(m, [k], orc.PLANE)
        E, _ = orc.reflected_field(m, [k], Ei, Bi, np.zeros((1, 3)))
        fres = 1j * k * a * a / (2 * f) * cis(2, k, f)
        # relative correction is O(a^2/f^2) + O(1/kf)
        assert abs(E[0, 0, 0] / fres - 1) < 2 * (a * a / (f * f)) + 2 / (k * f)


@pytest.mark.parametrize("zp", [0.5, 2.5, 7.0])
def test_p2_flat_disk_on_axis(orc, zp):
    a, k = 10.0, 2 * math.pi
    m = orc.mirror(1.0, a, 200, 32, kind=orc.FLAT)
    Ei, Bi = orc.incident_tables(m, [k], orc.PLANE)
    E, B = orc.reflected_field(m, [k], Ei, Bi, np.array([[0.0, 0.0, zp]]))
    Ra = math.hypot(a, zp)
    ex = cis(k, Ra) - cis(k, zp) - (a * a / (2 * Ra * Ra)) * (1 + 1j / (k * Ra)) * cis(k, Ra)
    assert abs(E[0, 0, 0] - ex) < 1e-12
    assert max(abs(E[0, 0, 1]), abs(E[0, 0, 2])) < 1e-12


def test_flat_mirror_reflects_gaussian_as_pec(orc):
    # A flat mirror much wider than a collimated Gaussian (waist w0 at the mirror)
    # reflects it like an infinite perfect conductor whose normal points toward the
    # incoming beam: on the axis the paraxial result is
    #   E_x = B_y = -e^{ikz'} / (1 + i z'/z_R),  z_R = k w0^2 / 2,
    # up to O(1/(k w0)^2) and the edge wave ~ G(a)/2 (here ~1e-4).
    a, k, w0 = 80.0, 2 * math.pi, 20.0
    zR = k * w0 * w0 / 2
    m = orc.mirror(1.0, a, 400, 16, kind=orc.FLAT)
    Ei, Bi = orc.incident_tables(m, [k], orc.GAUSSIAN, w0)
    for zp in [1.3, 40.0]:
        E, B = orc.reflected_field(m, [k], Ei, Bi, np.array([[0.0, 0.0, zp]]))
        ex = -cis(k, zp) / (1 + 1j * zp / zR)
        assert abs(E[0, 0, 0] - ex) < 5e-4
        assert abs(B[0, 0, 1] - ex) < 5e-4
