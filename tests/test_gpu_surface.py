"""GPU parity of general mirror surfaces (sc_set_surface) against the oracle:
an off-axis paraboloid segment lit by an off-axis beam, an annulus with two
boundary curves, and the built-in paraboloid handed over as a general surface."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08146_amd import Context
    c = Context(0)
    yield c
    c.close()


def _surface_problem(ctx, surf, k, E, B, obs):
    from paper_1609_08146_amd import Problem
    p = Problem(ctx)
    p.set_surface(*surf)
    p.set_frequencies(k)
    p.set_incident(E, B)
    p.set_observation(obs)
    return p


def test_off_axis_segment_matches_oracle(ctx, orc):
    base = workloads.broadband(n_k=6, n_nodes=40)
    f, cx, rad, w0 = base.f, 0.1, 0.04, 0.03
    surf = workloads.oap_segment(f, cx, rad, 80, 96)
    m = orc.surface(*surf)
    obs = base.obs[::53]
    E_in, B_in = workloads.shifted_gaussian_fields(m.pos, base.k, w0, cx, base.spectrum)
    Eo, Bo = orc.reflected_field(m, base.k, E_in, B_in, obs)
    p = _surface_problem(ctx, surf, base.k, E_in, B_in, obs)
    assert p.num_nodes() == (80 * 96, 96)
    np.testing.assert_allclose(p.incident_power(), orc.incident_power(m, E_in, B_in), rtol=1e-12)
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        E, B = p.evaluate(prec)
        err = max(rel_l2(E, Eo), rel_l2(B, Bo))
        print(f"off-axis segment {prec}: {err:.2e}")
        assert err < tol
    p.close()


def test_annulus_with_two_boundaries_matches_oracle(ctx, orc):
    K = 2 * np.pi
    surf = workloads.paraboloid_annulus(20.0, 18.0, 40.0, 50, 64)
    m = orc.surface(*surf)
    Ei, Bi = orc.incident_tables(m, [K, 1.1 * K], orc.GAUSSIAN_CONSISTENT, 15.0)
    obs = workloads.focal_plane(2.0, 9)
    Eo, Bo = orc.reflected_field(m, [K, 1.1 * K], Ei, Bi, obs)
    p = _surface_problem(ctx, surf, [K, 1.1 * K], Ei, Bi, obs)
    E, B = p.evaluate("fp64")
    err = max(rel_l2(E, Eo), rel_l2(B, Bo))
    print(f"annulus fp64: {err:.2e}")
    assert err < 1e-12
    p.close()


def test_built_in_mirror_as_general_surface(ctx):
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.broadband(n_k=4, n_nodes=50).subset(obs_idx=np.arange(0, 4160, 71))
    p1 = problem_from_workload(ctx, w)
    xyz, nrm, wgt = p1.get_nodes()
    ns, nr = p1.num_nodes()
    rim = xyz[ns:]
    dl = np.stack([-rim[:, 1], rim[:, 0], np.zeros(nr)], axis=1) * (2 * np.pi / nr)
    from paper_1609_08146_amd import Problem
    p2 = Problem(ctx)
    p2.set_surface(xyz[:ns], nrm[:ns] * wgt[:ns, None], rim, nrm[ns:], dl)
    p2.set_frequencies(w.k)
    p2.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
    p2.set_observation(w.obs)
    np.testing.assert_allclose(p2.incident_power(), p1.incident_power(), rtol=1e-14)
    for prec in ("fp64", "fp32_split"):
        E1, B1 = p1.evaluate(prec)
        E2, B2 = p2.evaluate(prec)
        assert max(rel_l2(E2, E1), rel_l2(B2, B1)) < (1e-13 if prec == "fp64" else 1e-6), prec
    p1.close()
    p2.close()


def test_surface_rejections(ctx):
    from paper_1609_08146_amd import Problem, ScError
    from paper_1609_08146_amd._abi import SC_E_INVAL
    p = Problem(ctx)
    good = workloads.oap_segment(0.1, 0.1, 0.04, 4, 8)
    bad_xyz = good[0].copy()
    bad_xyz[3, 1] = np.nan
    zero_n = good[3].copy()
    zero_n[2] = 0.0
    for args in ((bad_xyz,) + good[1:], good[:3] + (zero_n,) + good[4:]):
        with pytest.raises(ScError) as e:
            p.set_surface(*args)
        assert e.value.status == SC_E_INVAL
    with pytest.raises(ValueError):
        p.set_surface(good[0], good[1][:-1])
    p.set_surface(good[0], good[1])          # no boundary: surface terms only
    assert p.num_nodes() == (32, 0)
    p.close()


def test_ellipsoid_cap_matches_oracle(ctx, orc):
    """A non-parabolic mirror (Sec. III-C-1): the ellipsoidal cap z^2/c^2 + r^2/(2fc) = 1 (f = 200,
    c = 600, aperture radius 300, wavelength 1) lit by the built-in Gaussian, whose folded tables
    turn through some 50 periods over the cap, at a mesh that resolves them (240 Gauss-Legendre
    nodes in r): aperture power, FP64 and FP32-split against the oracle."""
    from paper_1609_08146_amd import Problem
    K = 2 * np.pi
    f, c, rm, w0 = 200.0, 600.0, 300.0, 150.0
    surf = workloads.ellipsoid_cap(f, c, rm, 240, 64)
    m = orc.surface(*surf)
    ks = np.array([K, 1.05 * K])
    obs = workloads.random_points(40, 2.0, seed=17)
    Ei, Bi = orc.incident_tables(m, ks, orc.GAUSSIAN, w0)
    Eo, Bo = orc.reflected_field(m, ks, Ei, Bi, obs)
    p = Problem(ctx)
    p.set_surface(*surf)
    p.set_frequencies(ks)
    p.set_incident_beam("linear", w0, 0.0, None, False)
    p.set_observation(obs)
    np.testing.assert_allclose(p.incident_power(), orc.incident_power(m, Ei, Bi), rtol=1e-12)
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        E, B = p.evaluate(prec)
        err = max(rel_l2(E, Eo), rel_l2(B, Bo))
        peak = max(np.abs(Eo).max(), np.abs(Bo).max())
        worst = max(np.abs(E - Eo).max(), np.abs(B - Bo).max()) / peak
        print(f"ellipsoidal cap {prec}: relative L2 {err:.2e}, largest error over the peak {worst:.2e}")
        assert err < tol
    p.close()
