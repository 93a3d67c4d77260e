"""General mirror surfaces in the oracle (a surface given by its quadrature),
pinned by the built-in paraboloid, the Stokes / double-gradient identity on an
off-axis segment, additivity over pieces with their boundaries, the flat-disk
closed form and the aperture power."""
import math

import numpy as np

import workloads

K = 2 * math.pi


def _as_surface(orc, m):
    dl = m.tan * m.wgt[m.n_surf:, None]
    return orc.surface(m.pos[:m.n_surf], m.nrm[:m.n_surf] * m.wgt[:m.n_surf, None], m.pos[m.n_surf:],
                       m.nrm[m.n_surf:], dl)


def test_built_in_paraboloid_as_a_general_surface(orc):
    m = orc.mirror(20.0, 40.0, 40, 32)
    s = _as_surface(orc, m)
    obs = np.array([[0.3, 0.2, 0.1], [-1.0, 0.5, -0.7]])
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 20.0)
    E1, B1 = orc.reflected_field(m, [K], Ei, Bi, obs)
    E2, B2 = orc.reflected_field(s, [K], Ei, Bi, obs)
    assert np.abs(E1 - E2).max() < 1e-13 * np.abs(E1).max()
    assert np.abs(B1 - B2).max() < 1e-13 * np.abs(B1).max()
    np.testing.assert_allclose(orc.incident_power(s, Ei, Bi), orc.incident_power(m, Ei, Bi), rtol=1e-14)


def test_off_axis_segment_stokes_equals_double_gradient(orc):
    f, cx, rad = 20.0, 30.0, 12.0
    s = orc.surface(*workloads.oap_segment(f, cx, rad, 60, 64))
    obs = np.array([[0.3, 0.2, 0.1], [-0.5, 0.4, 0.7], [0.0, 0.0, 0.0]])
    # the identity needs fields that obey Maxwell's equations on the mirror: the plane wave and the
    # curl-consistent Gaussian (here centred on the axis, off the segment's centre)
    for kind, w0 in ((orc.PLANE, np.inf), (orc.GAUSSIAN_CONSISTENT, 25.0)):
        Ei, Bi = orc.incident_tables(s, [K], kind, w0)
        E, _ = orc.reflected_field(s, [K], Ei, Bi, obs)
        Edg = orc.reflected_field_dgrad(s, [K], Bi, obs)
        assert np.abs(E - Edg).max() < 1e-9 * np.abs(Edg).max(), kind
        E0, _ = orc.reflected_field(s, [K], Ei, Bi, obs, line_term=False)
        assert np.abs(E0 - Edg).max() > 1e-4 * np.abs(Edg).max()      # the boundary term matters


def test_pieces_add_up_with_their_boundaries(orc):
    f, a1, a2 = 20.0, 18.0, 40.0
    whole = orc.mirror(f, a2, 80, 64)
    disk = orc.mirror(f, a1, 60, 64)
    ring = orc.surface(*workloads.paraboloid_annulus(f, a1, a2, 60, 64))
    obs = np.array([[0.3, 0.2, 0.1], [-0.5, 0.4, 0.7]])
    out = []
    for m in (whole, disk, ring):
        Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 15.0)
        out.append(orc.reflected_field(m, [K], Ei, Bi, obs))
    for c in range(2):   # E and B
        s = out[1][c] + out[2][c]
        assert np.abs(s - out[0][c]).max() < 1e-9 * np.abs(out[0][c]).max()


def test_flat_disk_closed_form_through_a_general_surface(orc):
    a, zp = 10.0, 2.5
    m = orc.mirror(1.0, a, 200, 16, kind=orc.FLAT)
    s = _as_surface(orc, m)
    Ei, Bi = orc.incident_tables(s, [K], orc.PLANE)
    E, _ = orc.reflected_field(s, [K], Ei, Bi, np.array([[0.0, 0.0, zp]]))
    Ra = math.hypot(a, zp)
    cis = lambda x: complex(math.cos(x), math.sin(x))
    ex = cis(K * Ra) - cis(K * zp) - (a * a / (2 * Ra * Ra)) * (1 + 1j / (K * Ra)) * cis(K * Ra)
    assert abs(E[0, 0, 0] - ex) < 1e-9


def test_off_axis_aperture_power(orc):
    f, cx, rad = 20.0, 30.0, 12.0
    s = orc.surface(*workloads.oap_segment(f, cx, rad, 40, 48))
    Ei, Bi = workloads.shifted_gaussian_fields(s.pos, [K, 2 * K], np.inf, cx)
    np.testing.assert_allclose(orc.incident_power(s, Ei, Bi), 4 * math.pi * math.pi * rad * rad, rtol=1e-13)
    w0 = 3.0
    Ei, Bi = workloads.shifted_gaussian_fields(s.pos, [K], w0, cx)
    ex = 4 * math.pi * (math.pi * w0 * w0 / 2) * (1 - math.exp(-2 * rad * rad / (w0 * w0)))
    np.testing.assert_allclose(orc.incident_power(s, Ei, Bi), ex, rtol=1e-12)
