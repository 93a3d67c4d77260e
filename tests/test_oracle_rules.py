"""Pins for the oracle's quadrature rule and mirror discretisation (Sec. III-C).

The Gauss-Legendre rule is checked against scipy's independent implementation
and against its defining exactness property; the mirror nodes, normals and
weights against the closed-form geometry of the paraboloid z = r^2/4f - f.
"""
import math

import numpy as np
import pytest
import scipy.special


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 200, 400, 800])
def test_gauss_legendre_matches_scipy(orc, n):
    x, w = orc.gauss_legendre(n)
    xs, ws = scipy.special.roots_legendre(n)
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, xs, rtol=0, atol=4e-16)
    # scipy's weights carry ~1e-11 (n=200) .. ~3e-9 (n=800) relative error;
    # the exactness test below is the sharp check.
    np.testing.assert_allclose(w, ws, rtol=1e-8)


@pytest.mark.parametrize("n", [1, 5, 33, 200, 800])
def test_gauss_legendre_exact_to_degree_2n_minus_1(orc, n):
    x, w = orc.gauss_legendre(n)
    assert abs(w.sum() - 2.0) < 4e-15
    # sum_i w_i P_j(x_i) = 0 for 1 <= j <= 2n-1 (P_j by Bonnet's recurrence)
    p0, p1 = np.ones_like(x), x.copy()
    worst = abs(np.dot(w, p1))
    for m in range(1, 2 * n - 1):
        p0, p1 = p1, ((2 * m + 1) * x * p1 - m * p0) / (m + 1)
        worst = max(worst, abs(np.dot(w, p1)))
    assert worst < 2e-15
    # degree 2n is NOT integrated exactly (the rule really has n nodes)
    p2n = ((2 * (2 * n - 1) + 1) * x * p1 - (2 * n - 1) * p0) / (2 * n)
    assert abs(np.dot(w, p2n)) > 1e-3


def test_mirror_geometry_paraboloid(orc):
    f, a, nr, nphi = 0.1, 0.075, 40, 48
    m = orc.mirror(f, a, nr, nphi)
    pos, nrm = m.pos, m.nrm
    r = np.hypot(pos[:, 0], pos[:, 1])
    # every node lies on the paraboloid, and the rim row at r = a
    np.testing.assert_allclose(pos[:, 2], r * r / (4 * f) - f, rtol=0, atol=1e-16)
    np.testing.assert_allclose(r[m.n_surf:], a, rtol=1e-15)
    # focal property: distance to the focus = distance to the directrix z = -2f
    np.testing.assert_allclose(np.linalg.norm(pos, axis=1), pos[:, 2] + 2 * f, rtol=2e-16 * 8)
    # unnormalised normal = (d r_s/dr x d r_s/dphi) / r, by finite differences of the parametrisation
    x, _ = orc.gauss_legendre(nr)
    ri = a * (1 + x) / 2
    for q in [0, 7, nphi * 13 + 5, nphi * (nr - 1) + nphi - 1]:
        i, j = divmod(q, nphi)
        phi = 2 * math.pi * j / nphi
        h = 1e-6

        def rs(rr, pp):
            return np.array([rr * math.cos(pp), rr * math.sin(pp), rr * rr / (4 * f) - f])

        dr = (rs(ri[i] + h, phi) - rs(ri[i] - h, phi)) / (2 * h)
        dp = (rs(ri[i], phi + h) - rs(ri[i], phi - h)) / (2 * h)
        np.testing.assert_allclose(nrm[q], np.cross(dr, dp) / ri[i], rtol=1e-8, atol=1e-9)
    # the normal points away from the mirror toward the focus (+z at the vertex)
    assert np.all(nrm[:, 2] > 0)
    assert np.all(np.einsum("ij,ij->i", nrm, -pos) > 0)
    # rim tangent = d r_s / dphi at r = a
    j = np.arange(nphi)
    phi = 2 * np.pi * j / nphi
    np.testing.assert_allclose(m.tan, np.stack([-a * np.sin(phi), a * np.cos(phi), 0 * phi], -1), atol=1e-16)


def test_mirror_weights_integrate_closed_forms(orc):
    f, a = 0.05, 0.15
    m = orc.mirror(f, a, 120, 64)
    W, nrm = m.wgt[: m.n_surf], m.nrm[: m.n_surf]
    # sum W = int r dr dphi = pi a^2 ; sum W n~ = (0, 0, pi a^2)
    assert abs(W.sum() / (math.pi * a * a) - 1) < 1e-14
    np.testing.assert_allclose((W[:, None] * nrm).sum(0), [0, 0, math.pi * a * a], atol=1e-15)
    # curved area of the paraboloid: 2 pi (4 f^2 / 3) [ (1 + a^2/4f^2)^{3/2} - 1 ]
    area = 2 * math.pi * (4 * f * f / 3) * ((1 + a * a / (4 * f * f)) ** 1.5 - 1)
    got = np.sum(W * np.linalg.norm(nrm, axis=1))
    assert abs(got / area - 1) < 1e-13
    # trapezoid rule in phi: exact for cos(m phi) with m < n_phi, aliases at m = n_phi
    phi = np.arctan2(m.pos[: m.n_surf, 1], m.pos[: m.n_surf, 0])
    for mm in [1, 5, 63]:
        assert abs(np.sum(W * np.cos(mm * phi))) < 1e-15
    assert abs(np.sum(W * np.cos(64 * phi)) / (math.pi * a * a) - 1) < 1e-12
    # rim weights are the trapezoid step
    np.testing.assert_allclose(m.wgt[m.n_surf:], 2 * math.pi / 64, rtol=1e-16)


def test_mirror_rejects_bad_parameters(orc):
    with pytest.raises(ValueError):
        orc.mirror(0.0, 1.0, 10, 10)
    with pytest.raises(ValueError):
        orc.mirror(1.0, -1.0, 10, 10)
    with pytest.raises(ValueError):
        orc.mirror(1.0, 1.0, 0, 10)
