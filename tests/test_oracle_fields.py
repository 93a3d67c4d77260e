"""Pins of the oracle's reflected field that hold at any observation point.

* Stokes-converted form (eq. stratton-chu-poa-og) == double-gradient form
  (eq. stratton-chu-poa): the two are equal by Stokes' theorem whenever the
  incident field obeys curl B = -ik E on the mirror (plane wave; curl-consistent
  Gaussian), and only with the rim line integral included.
* Maxwell's equations in the frequency domain (the residual e_f of Sec. IV-A),
  by 4th-order central finite differences.  curl E = ik B holds for ANY
  incident tables (the Stokes-form E differs from a curl-free field only by
  gradient terms), so it also pins the relative sign/scale of E and B.
* Mirror symmetries of an x-polarised, axisymmetric beam on the paraboloid.
* Paraxial (large f) limit: a Gaussian focused by an ideal thin focusing
  element with the waist at the mirror (ABCD / complex beam parameter).
* Refinement: the integrands are smooth and periodic in phi, so the
  Gauss-Legendre x trapezoid sums converge exponentially (Sec. III-C-1).
* Energy: the time-averaged Poynting flux of the reflected field through
  planes before and after the focus is the same, and equals the incident power
  intercepted by the aperture (Sec. IV-A, energy conservation check).
"""
import math

import numpy as np
import pytest

import workloads

K = 2 * math.pi


def _fd_stencil(p0, h):
    pts = [p0]
    for ax in range(3):
        for s in (-2, -1, 1, 2):
            d = np.zeros(3)
            d[ax] = s * h
            pts.append(p0 + d)
    return np.array(pts)


def _jacobian(F, h):
    """d[ax][comp] from the 13-point stencil values F[13][3] (4th order)."""
    d = np.zeros((3, 3), complex)
    for ax in range(3):
        fm2, fm1, fp1, fp2 = F[1 + 4 * ax: 5 + 4 * ax]
        d[ax] = (fm2 - 8 * fm1 + 8 * fp1 - fp2) / (12 * h)
    return d


def _curl(d):
    return np.array([d[1, 2] - d[2, 1], d[2, 0] - d[0, 2], d[0, 1] - d[1, 0]])


@pytest.mark.parametrize("kind", ["plane", "consistent"])
def test_stokes_form_equals_double_gradient_form(orc, kind):
    m = orc.mirror(20.0, 40.0, 200, 64)
    if kind == "plane":
        Ei, Bi = orc.incident_tables(m, [K], orc.PLANE)
        tol, line_size = 2e-14, 1e-3
    else:
        # the beam is down to e^{-4} at the rim, so the line term is smaller
        Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 20.0)
        tol, line_size = 1e-12, 5e-5
    obs = np.array([[0.3, 0.2, 0.1], [1.0, -0.5, 0.7], [-1.5, 1.1, -0.9]])
    E, _ = orc.reflected_field(m, [K], Ei, Bi, obs)
    E_noline, _ = orc.reflected_field(m, [K], Ei, Bi, obs, line_term=False)
    Edg = orc.reflected_field_dgrad(m, [K], Bi, obs)
    scale = np.abs(Edg).max()
    assert np.abs(E - Edg).max() / scale < tol
    # the rim line integral is essential: without it the forms differ visibly
    assert np.abs(E_noline - Edg).max() / scale > line_size


def test_maxwell_curl_e_is_ikb_for_arbitrary_tables(orc):
    # random (unphysical) tables: only curl E = ik B and div B = 0 must survive
    m = orc.mirror(20.0, 40.0, 60, 32)
    Ei, Bi = workloads.random_incident_tables(1, m.n_tot, seed=7)
    h = 0.01
    for p0 in [np.array([0.3, 0.2, 0.1]), np.array([-1.2, 0.8, 0.5])]:
        E, B = orc.reflected_field(m, [K], Ei, Bi, _fd_stencil(p0, h))
        dE, dB = _jacobian(E[0], h), _jacobian(B[0], h)
        s = K * max(np.abs(E[0, 0]).max(), np.abs(B[0, 0]).max())
        assert np.abs(_curl(dE) - 1j * K * B[0, 0]).max() / s < 2e-6
        assert abs(np.trace(dB)) / s < 2e-6


@pytest.mark.parametrize("p0", [(0.3, 0.2, 0.1), (1.0, -0.7, 0.5)])
def test_maxwell_all_four_with_curl_consistent_beam(orc, p0):
    m = orc.mirror(20.0, 40.0, 120, 96)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 20.0)
    h = 0.01
    E, B = orc.reflected_field(m, [K], Ei, Bi, _fd_stencil(np.array(p0), h))
    dE, dB = _jacobian(E[0], h), _jacobian(B[0], h)
    s = K * np.abs(E[0, 0]).max()
    assert np.abs(_curl(dE) - 1j * K * B[0, 0]).max() / s < 1e-6
    assert np.abs(_curl(dB) + 1j * K * E[0, 0]).max() / s < 1e-6
    assert abs(np.trace(dE)) / s < 1e-6
    assert abs(np.trace(dB)) / s < 1e-6


def test_literal_beam_breaks_only_the_source_free_equations(orc):
    # E_x = G e^{-ikz}, B = -y G e^{-ikz} is not a Maxwell field (O(1/k w0));
    # curl E = ik B still holds exactly, div E and curl B + ik E do not.
    m = orc.mirror(20.0, 40.0, 120, 96)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN, 20.0)
    h = 0.01
    E, B = orc.reflected_field(m, [K], Ei, Bi, _fd_stencil(np.array([0.3, 0.2, 0.1]), h))
    dE, dB = _jacobian(E[0], h), _jacobian(B[0], h)
    s = K * np.abs(E[0, 0]).max()
    assert np.abs(_curl(dE) - 1j * K * B[0, 0]).max() / s < 1e-6
    assert abs(np.trace(dE)) / s > 1e-3


def test_mirror_symmetries_x_polarised(orc):
    m = orc.mirror(20.0, 40.0, 100, 64)
    Ei, Bi = orc.incident_tables(m, [K, 1.1 * K], orc.GAUSSIAN, 20.0)
    p = np.array([[0.7, 0.4, 0.3], [1.3, -0.2, -0.5]])
    E, B = orc.reflected_field(m, [K, 1.1 * K], Ei, Bi, p)

    def flip(q, ax):
        q = q.copy()
        q[:, ax] *= -1
        return q

    Ex, Bx = orc.reflected_field(m, [K, 1.1 * K], Ei, Bi, flip(p, 0))
    Ey, By = orc.reflected_field(m, [K, 1.1 * K], Ei, Bi, flip(p, 1))
    sE, sB = np.abs(E).max(), np.abs(B).max()
    # x -> -x: Ex, By, Bz even; Ey, Ez, Bx odd.   y -> -y: Ex, Ez, By even; Ey, Bx, Bz odd.
    assert np.abs(Ex - E * np.array([1, -1, -1])).max() / sE < 1e-14
    assert np.abs(Bx - B * np.array([-1, 1, 1])).max() / sB < 1e-14
    assert np.abs(Ey - E * np.array([1, -1, 1])).max() / sE < 1e-14
    assert np.abs(By - B * np.array([-1, 1, -1])).max() / sB < 1e-14
    # a 90 degree rotation maps the x-polarised solution onto the y-polarised one
    Ei2, Bi2 = orc.incident_tables(m, [K, 1.1 * K], orc.GAUSSIAN, 20.0, pol=math.pi / 2)
    rot = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    E2, B2 = orc.reflected_field(m, [K, 1.1 * K], Ei2, Bi2, p @ rot.T)
    assert np.abs(E2 - E @ rot.T).max() / sE < 1e-14
    assert np.abs(B2 - B @ rot.T).max() / sB < 1e-14


@pytest.mark.parametrize("f,bound", [(2000.0, 3e-3), (8000.0, 4e-4)])
def test_paraxial_limit(orc, f, bound):
    # Literal Gaussian, waist w0 at the mirror, reflected by a long-focus paraboloid.
    # Near the focus, E_x ~ B_y ~ -e^{ikf} (q_m/q) exp(ik rho'^2/(2q)) e^{ik(f+z')},
    # q_m = -f / (1 - i f/z_R), z_R = k w0^2 / 2, q = q_m + f + z'.
    w0 = 100.0
    a = 3 * w0
    m = orc.mirror(f, a, 200, 64)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN, w0)
    zR = K * w0 * w0 / 2
    qm = -f / (1 - 1j * f / zR)
    obs = np.array([[0, 0, 0], [3, 0, 0], [0, 3, 0], [2, 2, 0], [0, 0, 50], [0, 0, -50], [2, 0, 30]], float)
    E, B = orc.reflected_field(m, [K], Ei, Bi, obs)
    q = qm + f + obs[:, 2]
    rho2 = obs[:, 0] ** 2 + obs[:, 1] ** 2
    ex = -np.exp(1j * K * f) * (qm / q) * np.exp(1j * K * rho2 / (2 * q)) * np.exp(1j * K * (f + obs[:, 2]))
    sc = np.abs(ex).max()
    assert np.abs(E[0, :, 0] - ex).max() / sc < bound
    assert np.abs(B[0, :, 1] - ex).max() / sc < bound
    # the focal amplitude is i (k w0^2 / 2f) e^{2ikf}
    assert abs(E[0, 0, 0] / (1j * zR / f * np.exp(2j * K * f)) - 1) < bound


def test_refinement_exponential_convergence(orc):
    wl = workloads.mono()
    sub = wl.subset(obs_idx=np.arange(0, 1024, 37))
    Eref, Bref = orc.solve(sub.with_nodes(400, 400))
    E200, B200 = orc.solve(sub)
    sE = np.abs(Eref).max()
    assert np.abs(E200 - Eref).max() / sE < 1e-12
    assert np.abs(B200 - Bref).max() / np.abs(Bref).max() < 1e-12
    # and the error really falls off: 24 radial nodes are far from converged
    E24, _ = orc.solve(sub.with_nodes(24, 24))
    assert np.abs(E24 - Eref).max() / sE > 1e-6


def test_flux_conservation_through_focus(orc):
    # NA ~ 0.66 mirror (rim at z = -17.2); planes z = -3 and z = +3 bound a
    # source-free slab around the focus.
    f, a, w0 = 20.0, 15.0, 6.0
    m = orc.mirror(f, a, 120, 64)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, w0)
    L, n = 6.0, 49
    h = 2 * L / (n - 1)
    flux = []
    for z in (-3.0, 3.0):
        E, B = orc.reflected_field(m, [K], Ei, Bi, workloads.focal_plane(L, n, z))
        Sz = 0.5 * np.real(E[0, :, 0] * np.conj(B[0, :, 1]) - E[0, :, 1] * np.conj(B[0, :, 0]))
        flux.append(Sz.sum() * h * h)
    p_inc = math.pi * w0 * w0 / 4 * (1 - math.exp(-2 * a * a / (w0 * w0)))
    assert abs(flux[0] - flux[1]) / p_inc < 2e-6
    assert abs(flux[1] / p_inc - 1) < 1e-5
