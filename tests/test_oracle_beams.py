"""The oracle's cylindrical vector beams (radially and azimuthally polarised,
Sec. IV-A) pinned by closed-form aperture power, Maxwell's equations for the
curl-consistent variants and the symmetries of the reflected field."""
import math

import numpy as np
import pytest

K = 2 * math.pi


def _fd_jac(F, h):
    d = np.zeros((3, 3), complex)
    for ax in range(3):
        fm2, fm1, fp1, fp2 = F[1 + 4 * ax: 5 + 4 * ax]
        d[ax] = (fm2 - 8 * fm1 + 8 * fp1 - fp2) / (12 * h)
    return d


def _curl(d):
    return np.array([d[1, 2] - d[2, 1], d[2, 0] - d[0, 2], d[0, 1] - d[1, 0]])


@pytest.mark.parametrize("kind_name", ["RADIAL", "RADIAL_CONSISTENT", "AZIMUTHAL", "AZIMUTHAL_CONSISTENT"])
def test_cylindrical_beam_power_closed_form(orc, kind_name):
    kind = getattr(orc, kind_name)
    a = 25.0
    m = orc.mirror(20.0, a, 60, 32)
    for w0 in (6.0, 15.0, 30.0):
        Ei, Bi = orc.incident_tables(m, [K, 1.4 * K], kind, w0)
        b = 2 * a * a / (w0 * w0)
        ex = math.pi ** 2 * w0 * w0 * (1 - math.exp(-b) * (1 + b))
        np.testing.assert_allclose(orc.incident_power(m, Ei, Bi), ex, rtol=1e-12)


def test_consistent_cylindrical_beams_obey_maxwell(orc):
    h, w0 = 1e-3, 3.0
    for p0 in (np.array([0.7, -0.4, 0.3]), np.array([2.1, 1.3, -1.0])):
        pts = [p0]
        for ax in range(3):
            for s in (-2, -1, 1, 2):
                d = np.zeros(3)
                d[ax] = s * h
                pts.append(p0 + d)
        pts = np.array(pts)
        for kind in (orc.RADIAL_CONSISTENT, orc.AZIMUTHAL_CONSISTENT):
            E, B = orc.incident(kind, pts, K, w0)
            dE, dB = _fd_jac(E, h), _fd_jac(B, h)
            s = K * max(np.abs(E[0]).max(), np.abs(B[0]).max())
            if kind == orc.RADIAL_CONSISTENT:
                assert abs(np.trace(dE)) / s < 1e-9                              # div E = 0
                assert np.abs(_curl(dB) + 1j * K * E[0]).max() / s < 1e-9        # curl B = -ik E
            else:
                assert abs(np.trace(dB)) / s < 1e-9                              # div B = 0
                assert np.abs(_curl(dE) - 1j * K * B[0]).max() / s < 1e-9        # curl E = ik B
        # the literal variants miss the longitudinal term at order 1/(k w0)
        E, B = orc.incident(orc.RADIAL, pts, K, w0)
        assert np.abs(_curl(_fd_jac(B, h)) + 1j * K * E[0]).max() / (K * np.abs(E[0]).max()) > 1e-3


def test_transverse_part_and_literal_relation(orc):
    pts = np.array([[0.3, -0.8, 0.1], [1.5, 0.2, -0.4]])
    for lit, con in ((orc.RADIAL, orc.RADIAL_CONSISTENT), (orc.AZIMUTHAL, orc.AZIMUTHAL_CONSISTENT)):
        El, Bl = orc.incident(lit, pts, K, 2.0)
        Ec, Bc = orc.incident(con, pts, K, 2.0)
        np.testing.assert_array_equal(El[:, :2], Ec[:, :2])
        np.testing.assert_array_equal(Bl[:, :2], Bc[:, :2])
        np.testing.assert_allclose(Bl, np.cross(np.array([0, 0, -1.0]), El), atol=1e-15)   # B = (-z) x E
    E, B = orc.incident(orc.RADIAL, pts, K, 2.0)
    r = np.hypot(pts[:, 0], pts[:, 1])
    # radial: E parallel to (x, y), |E| = r/w0 exp(-r^2/w0^2) / w0 ... / w0 normalisation: r exp(-r^2/w0^2) / w0
    np.testing.assert_allclose(np.abs(E[:, 0] * pts[:, 1] - E[:, 1] * pts[:, 0]), 0, atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(np.abs(E), axis=1), r * np.exp(-r * r / 4.0) / 2.0, rtol=1e-14)


def test_reflected_cylindrical_fields_are_tm_and_te(orc):
    # radial polarisation reflects as a TM field (B azimuthal, B_z = 0), azimuthal as TE (E_z = 0);
    # on the axis the transverse E (radial) resp. transverse B (azimuthal) vanishes
    m = orc.mirror(20.0, 40.0, 60, 64)
    pts = np.array([[0.4, 0.0, 0.1], [0.0, -0.7, 0.3], [0.5, 0.5, -0.2], [0.0, 0.0, 0.0], [0.0, 0.0, 0.6]])
    for kind, zero_field in ((orc.RADIAL_CONSISTENT, "B"), (orc.AZIMUTHAL_CONSISTENT, "E")):
        Ei, Bi = orc.incident_tables(m, [K], kind, 20.0)
        E, B = orc.reflected_field(m, [K], Ei, Bi, pts)
        F, G = (B, E) if zero_field == "B" else (E, B)
        s = max(np.abs(E).max(), np.abs(B).max())
        assert np.abs(F[0, :, 2]).max() < 1e-11 * s              # B_z (TM) or E_z (TE) vanishes
        assert np.abs(G[0, 3:, :2]).max() < 1e-11 * s            # transverse part of the other on the axis
        assert np.abs(F[0, 3:, :]).max() < 1e-11 * s             # the azimuthal field vanishes on the axis
        assert np.abs(G[0, 3, 2]) > 1e-2 * s                     # a strong longitudinal field at the focus


def _tie(m, Ei, Bi):
    """Per surface node: J = n x B and rho = n . E over the frequencies; returns the residual of J
    off one real direction u, and of rho off gamma * (u . J) with one real gamma for all frequencies,
    each relative to the node's largest |J| and |J| + |rho|."""
    ns = m.n_surf
    n = m.nrm[:ns]
    J = np.cross(n[None], Bi[:, :ns])                        # [k, q, 3]
    rho = np.einsum("qc,kqc->kq", n, Ei[:, :ns])
    kb = np.argmax(np.linalg.norm(J, axis=-1), axis=0)        # per node, the k of the largest |J|
    Jb = J[kb, np.arange(ns)]
    part = np.where(np.linalg.norm(Jb.real, axis=-1) >= np.linalg.norm(Jb.imag, axis=-1), 0, 1)
    u = np.where(part[:, None] == 0, Jb.real, Jb.imag)
    u /= np.linalg.norm(u, axis=-1, keepdims=True)
    c = np.einsum("qc,kqc->kq", u, J)
    scale = np.linalg.norm(J, axis=-1).max(axis=0)
    res_J = (np.linalg.norm(J - u[None] * c[..., None], axis=-1).max(axis=0) / scale).max()
    cb = c[kb, np.arange(ns)]
    gamma = (rho[kb, np.arange(ns)] / cb).real
    scale_r = (np.abs(rho) + np.abs(c)).max(axis=0)
    res_rho = (np.abs(rho - gamma[None] * c).max(axis=0) / scale_r).max()
    return res_J, res_rho


@pytest.mark.parametrize("kind_name,tied", [("GAUSSIAN", True), ("PLANE", True), ("RADIAL", True),
                                            ("AZIMUTHAL", True), ("AZIMUTHAL_CONSISTENT", True),
                                            ("RADIAL_CONSISTENT", False)])
def test_charge_tied_to_the_current(orc, kind_name, tied):
    """The tied-charge layout of the split kernels rests on a property of the incident fields: where
    the current n x B keeps one real direction u with amplitude c at every frequency, n . E = gamma c
    with gamma real and the same for all frequencies, for every beam without a longitudinal E
    (B = -z x E: both carry one complex amplitude; on the paraboloid n . E of the azimuthal beams
    vanishes, gamma = 0).  The curl-consistent radial beam's E_z = i c' g turns n . E against n x B by
    an amount that changes with k, so its current factors and its charge does not tie."""
    kind = getattr(orc, kind_name)
    m = orc.mirror(20.0, 25.0, 30, 24)
    spec = np.array([1.0, 0.3 - 0.8j, -0.6 + 0.2j])
    Ei, Bi = orc.incident_tables(m, [K, 1.3 * K, 1.7 * K], kind, 12.0, 0.4, spec)
    res_J, res_rho = _tie(m, Ei, Bi)
    assert res_J < 1e-13
    if tied:
        assert res_rho < 1e-13
    else:
        assert res_rho > 1e-4
