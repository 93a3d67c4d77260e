"""GPU tests of the incident-power and energy-normalisation entry points
(Sec. III-B) against the oracle, through the C ABI."""
from dataclasses import replace

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


def test_incident_power_matches_oracle(ctx, orc):
    from paper_1609_08146_amd import problem_from_workload
    base = workloads.broadband(n_k=5, n_nodes=64)
    m = orc.mirror(base.f, base.a, base.n_r, base.n_phi)
    for w0, pol, consistent in ((0.05, 0.0, 0), (0.03, 0.7, 0), (0.02, 0.3, 1), (np.inf, 0.0, 0)):
        w = replace(base, w0=w0, pol=pol, consistent=consistent,
                    spectrum=base.spectrum * np.exp(1j * np.arange(base.n_k)))
        p = problem_from_workload(ctx, w)
        kind = orc.PLANE if not np.isfinite(w0) else (orc.GAUSSIAN_CONSISTENT if consistent else orc.GAUSSIAN)
        Ei, Bi = orc.incident_tables(m, w.k, kind, w0, pol, w.spectrum)
        Po = orc.incident_power(m, Ei, Bi)
        P = p.incident_power()
        print(f"w0={w0} pol={pol} consistent={consistent}: max rel {np.max(np.abs(P / Po - 1)):.1e}")
        assert np.max(np.abs(P / Po - 1)) < 1e-13
        # user-supplied fields: power from the uploaded tables
        Er, Br = workloads.random_incident_tables(base.n_k, m.n_tot, seed=7)
        p.set_incident(Er, Br)
        np.testing.assert_allclose(p.incident_power(), orc.incident_power(m, Er, Br), rtol=1e-12)
        p.close()


def test_normalised_table1_field_matches_oracle(ctx, orc):
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.table1(n_k=6, n_nodes=80).subset(obs_idx=np.arange(0, 4160, 61))
    eps, e_tot = w.meta["eps"], w.meta["e_tot"]
    p = problem_from_workload(ctx, w)
    p.normalize_energy(eps, e_tot, w.dk)
    target = eps * e_tot / (eps.sum() * w.dk)
    np.testing.assert_allclose(p.incident_power(), target, rtol=1e-13)
    m = orc.mirror(w.f, w.a, w.n_r, w.n_phi)
    Ei, Bi = orc.incident_tables(m, w.k, orc.GAUSSIAN, w.w0)
    amp = orc.energy_amplitudes(orc.incident_power(m, Ei, Bi), eps, e_tot, w.dk)
    Ei, Bi = orc.incident_tables(m, w.k, orc.GAUSSIAN, w.w0, spectrum=amp)
    Eo, Bo = orc.reflected_field(m, w.k, Ei, Bi, w.obs)
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        E, B = p.evaluate(prec)
        err = max(rel_l2(E, Eo), rel_l2(B, Bo))
        print(f"{prec}: {err:.2e}")
        assert err < tol, prec
    # normalising again to the same spectrum changes nothing but rounding
    p.normalize_energy(target, 0.0, 0.0)
    E2, _ = p.evaluate("fp64")
    assert rel_l2(E2, Eo) < 1e-12
    p.close()


def test_scale_spectrum_equals_setting_the_chirped_spectrum(ctx):
    from paper_1609_08146_amd import Problem, problem_from_workload
    w = workloads.broadband(n_k=8, n_nodes=60).subset(obs_idx=np.arange(0, 4160, 37))
    kc = w.k.mean()
    chirp = 0.7 * np.exp(2e-12j * (w.k - kc) ** 2)
    p1 = problem_from_workload(ctx, w)
    p1.scale_spectrum(chirp)
    p2 = problem_from_workload(ctx, replace(w, spectrum=w.spectrum * chirp))
    np.testing.assert_allclose(p1.incident_power(), p2.incident_power(), rtol=1e-13)
    E1, B1 = p1.evaluate("fp64")
    E2, B2 = p2.evaluate("fp64")
    assert max(rel_l2(E1, E2), rel_l2(B1, B2)) < 1e-14
    # FP32-only table storage: the FP32 tables are scaled in place
    p3 = Problem(ctx)
    p3.set_mirror(w.f, w.a, w.n_r, w.n_phi)
    p3.set_frequencies(w.k)
    p3.set_table_storage(False)
    p3.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
    p3.set_observation(w.obs)
    p3.scale_spectrum(chirp)
    E3, B3 = p3.evaluate("fp32_split")
    assert max(rel_l2(E3, E2), rel_l2(B3, B2)) < 1e-5
    for p in (p1, p2, p3):
        p.close()


def test_energy_error_paths(ctx):
    from paper_1609_08146_amd import Problem, ScError
    from paper_1609_08146_amd._abi import SC_E_INVAL, SC_E_STATE
    w = workloads.broadband(n_k=4, n_nodes=32)
    p = Problem(ctx)
    p.set_mirror(w.f, w.a, w.n_r, w.n_phi)
    p.set_frequencies(w.k)
    for call in (lambda: p.normalize_energy(np.ones(4)), lambda: p.incident_power(),
                 lambda: p.scale_spectrum(np.ones(4))):
        with pytest.raises(ScError) as e:
            call()
        assert e.value.status == SC_E_STATE
    p.set_incident_gaussian(w.w0, 0.0, np.array([1.0, 0.0, 1.0, 1.0]), False)
    P = p.incident_power()
    assert P[1] == 0.0 and np.all(P[[0, 2, 3]] > 0)
    bad = [
        (np.array([1.0, 0.0, -1.0, 1.0]), 0.0, 0.0),       # negative power
        (np.array([1.0, 0.0, np.nan, 1.0]), 0.0, 0.0),     # not finite
        (np.array([1.0, 0.0, 1.0, 1.0]), 5.0, 0.0),        # e_tot without dk
        (np.array([1.0, 1.0, 1.0, 1.0]), 0.0, 0.0),        # energy asked of a component with no power
        (np.zeros(4), 5.0, 1.0),                           # nothing to normalise
    ]
    for eps, e_tot, dk in bad:
        with pytest.raises(ScError) as e:
            p.normalize_energy(eps, e_tot, dk)
        assert e.value.status == SC_E_INVAL, (eps, e_tot, dk)
    np.testing.assert_array_equal(p.incident_power(), P)   # failed calls change nothing
    p.normalize_energy(np.array([2.0, 0.0, 1.0, 3.0]))      # zero power, zero energy: allowed
    np.testing.assert_allclose(p.incident_power(), [2.0, 0.0, 1.0, 3.0], rtol=1e-14)
    with pytest.raises(ScError) as e:
        p.scale_spectrum(np.array([1, np.inf, 1, 1], complex))
    assert e.value.status == SC_E_INVAL
    with pytest.raises(ValueError):
        p.normalize_energy(np.ones(3))
    p.close()


def test_table1_focal_spot_matches_the_paper(ctx):
    """The Table I workload (energy-normalised to 150 J, FP32-split) against the focal-spot figures
    the paper prints in Sec. IV-B: peak electric intensity, eccentricity of the focal spot, and the
    size of the longitudinal magnetic field (tests/golden/table1_focal_spot.json)."""
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    from paper_1609_08146_amd import problem_from_workload
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "table1_focal_spot.json")))
    w = workloads.table1()
    lam = workloads.TABLE1["lam_c"]
    p = problem_from_workload(ctx, w)
    p.normalize_energy(w.meta["eps"], w.meta["e_tot"], w.dk)
    p.evaluate("fp32_split", keep_on_device=True)
    t = 2 * w.f + np.arange(-128, 129) * (lam / 32)
    Et, Bt = p.to_time_at(w.dk, t)
    p.close()
    r = bench.focal_spot(Et, Bt, 64, 2.0 * lam)
    print({k: r[k] for k in ("peak_intensity_W_cm2", "eccentricity", "max_Bz_over_max_Ex", "fwhm_x_m",
                             "fwhm_y_m")})
    assert abs(r["peak_intensity_W_cm2"] / gold["peak_electric_intensity_W_cm2"] - 1.0) < 0.3
    assert abs(r["eccentricity"] - gold["focal_spot_eccentricity"]) < 0.05
    assert r["fwhm_x_m"] > r["fwhm_y_m"]          # major axis along the polarisation
    assert abs(r["max_Bz_over_max_Ex"] - gold["max_Bz_over_max_Ex"]) < 0.1
