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


# ---------------------------------------------------------------- ellipsoidal cap (Sec. III-C-1)
# The ellipsoid z^2/c^2 + r^2/a^2 = 1 (a^2 = 2 f c: the vertex curvature of the paraboloid of focal
# length f), lower cap, lower focus moved to the origin.  For it the zeroth-order phase
# k(|r_s| - z) of the folded tables varies over the mirror (Sec. III-C-1), where it is 2kf on the
# paraboloid.

def test_ellipsoid_cap_geometry():
    f, c, rm = 20.0, 60.0, 30.0
    xyz, ndS, rx, rn, dl = workloads.ellipsoid_cap(f, c, rm, 40, 32)
    a2 = 2 * f * c
    e = math.sqrt(c * c - a2)
    r2 = xyz[:, 0] ** 2 + xyz[:, 1] ** 2
    assert np.abs((xyz[:, 2] - e) ** 2 / (c * c) + r2 / a2 - 1).max() < 1e-14
    # focal property: a ray from the upper focus (0, 0, 2e) reflected at any node heads for the origin
    nh = ndS / np.linalg.norm(ndS, axis=1, keepdims=True)
    d = xyz - np.array([0.0, 0.0, 2 * e])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    refl = d - 2 * np.einsum("ij,ij->i", d, nh)[:, None] * nh
    to_focus = -xyz / np.linalg.norm(xyz, axis=1, keepdims=True)
    assert np.abs(refl - to_focus).max() < 1e-13
    # normals point toward the focus side, the projected quadrature covers the aperture disk
    assert np.all(np.einsum("ij,ij->i", ndS, -xyz) > 0)
    assert abs(ndS[:, 2].sum() / (math.pi * rm * rm) - 1) < 1e-13
    # the rim: on the edge circle, dl tangent to the surface, total length 2 pi r_max, counter-clockwise
    assert np.abs(np.hypot(rx[:, 0], rx[:, 1]) - rm).max() < 1e-13
    assert np.abs(np.einsum("ij,ij->i", dl, rn)).max() < 1e-13
    assert abs(np.linalg.norm(dl, axis=1).sum() / (2 * math.pi * rm) - 1) < 1e-13
    assert np.all(np.cross(rx, dl)[:, 2] > 0)


def test_ellipsoid_stokes_equals_double_gradient(orc):
    s = orc.surface(*workloads.ellipsoid_cap(20.0, 60.0, 30.0, 60, 64))
    obs = np.array([[0.3, 0.2, 0.1], [-0.5, 0.4, 0.7], [0.0, 0.0, 0.0]])
    for kind, w0 in ((orc.PLANE, np.inf), (orc.GAUSSIAN_CONSISTENT, 15.0)):
        Ei, Bi = orc.incident_tables(s, [K], kind, w0)
        E, _ = orc.reflected_field(s, [K], Ei, Bi, obs)
        Edg = orc.reflected_field_dgrad(s, [K], Bi, obs)
        assert np.abs(E - Edg).max() < 1e-12 * np.abs(Edg).max(), kind
        E0, _ = orc.reflected_field(s, [K], Ei, Bi, obs, line_term=False)
        assert np.abs(E0 - Edg).max() > 1e-4 * np.abs(Edg).max()


def test_ellipsoid_tends_to_the_paraboloid(orc):
    """As c grows the cap approaches the paraboloid of focal length f; the focal field follows
    linearly in 1/c (the vertex-to-focus distance is f + f^2 / 2c + ...)."""
    f, rm, w0 = 20.0, 30.0, 15.0
    obs = np.array([[0.3, 0.2, 0.1], [0.0, 0.0, 0.0]])
    m = orc.mirror(f, rm, 60, 48)
    Ep, _ = orc.reflected_field(m, [K], *orc.incident_tables(m, [K], orc.GAUSSIAN, w0), obs)
    diffs = []
    for c in (1e5, 1e6):
        s = orc.surface(*workloads.ellipsoid_cap(f, c, rm, 60, 48))
        E, _ = orc.reflected_field(s, [K], *orc.incident_tables(s, [K], orc.GAUSSIAN, w0), obs)
        diffs.append(np.abs(E - Ep).max() / np.abs(Ep).max())
    assert diffs[1] < 3e-3 and abs(diffs[0] / diffs[1] - 10) < 0.05, diffs


def test_ellipsoid_folded_tables_oscillate(orc):
    """f = 200, c = 600, aperture 300 (wavelength 1): k(|r_s| - z) spans over 300 rad across the cap
    where the paraboloid keeps 2kf exactly, so the radial quadrature must resolve some fifty periods:
    100 Gauss-Legendre nodes in r leave an O(1) error that 200 and 300 nodes remove."""
    f, c, rm, w0 = 200.0, 600.0, 300.0, 150.0
    obs = np.array([[0.3, 0.2, 0.1], [0.0, 0.0, 0.0]])
    xyz = workloads.ellipsoid_cap(f, c, rm, 300, 8)[0]
    ph = K * (np.linalg.norm(xyz, axis=1) - xyz[:, 2])
    assert ph.max() - ph.min() > 300
    m = orc.mirror(f, rm, 300, 8)
    php = K * (np.linalg.norm(m.pos[: m.n_surf], axis=1) - m.pos[: m.n_surf, 2])
    assert np.abs(php - 2 * K * f).max() < 1e-9 * 2 * K * f
    out = {}
    for n in (100, 200, 300):
        s = orc.surface(*workloads.ellipsoid_cap(f, c, rm, n, 64))
        out[n], _ = orc.reflected_field(s, [K], *orc.incident_tables(s, [K], orc.GAUSSIAN, w0), obs)
    scale = np.abs(out[300]).max()
    assert np.abs(out[100] - out[300]).max() > 0.1 * scale
    assert np.abs(out[200] - out[300]).max() < 1e-10 * scale
