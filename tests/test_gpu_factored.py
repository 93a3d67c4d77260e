"""GPU: the factored current of the split form (Jt = u s with a real direction u per node).

The factored and the general FP32 split paths compute the same sums with a
different sequence of FP32 operations, so both are held to the oracle at the
split tolerance (1e-5 relative L2 per field) and to each other at 2e-6.

Which incident fields factor is fixed by the physics, so the detection is
tested against it: the surface current n x B (n = (-x/2f, -y/2f, 1) on the
paraboloid) must keep one real direction per node at every frequency.  It
does for the literal linearly polarised beam and the plane wave (B along a
fixed transverse axis, any spectrum), for both radially polarised variants
(B = (y, -x, 0) g is transverse; only E gains the longitudinal term) and for
both azimuthally polarised ones: B = (x, y, c) g gives
n x B = (1 + c/2f) (-y, x, 0) g, azimuthal whatever the longitudinal c.
The curl-consistent linear beam does not: its B_z = -2iy/(k w0^2) psi adds
(-y c/2f, x c/2f, 0) to n x (0, -1, 0) psi = (1, 0, x/2f) psi, a direction
that changes with k.  Random tables have no structure either.

The charge is tied to the factored current (rho_t = -i beta s / k, beta real per
node) when n.E carries the amplitude of n x B: for every factoring beam with no
longitudinal E.  The radially polarised curl-consistent beam has E_z = i c g,
which turns n.E by 90 degrees against n x B, so it keeps the factored layout
without the tie; the azimuthally polarised ones have n.E = 0 on the paraboloid
(E = (-y, x, 0) g against n = (-x/2f, -y/2f, 1)), tied with beta = 0.  The tied
layout computes the charge term from s, so it is held to the oracle and to the
other two layouts at the same tolerances.
"""
from dataclasses import replace

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


# table layout -> sc_set_factoring arguments (enable, tie_charge)
LAYOUTS = {"tied": (True, True), "factored": (True, False), "general": (False, True)}


def set_layout(p, name):
    p.set_factoring(*LAYOUTS[name])


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08146_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("beam,consistent,w0,layout", [
    (0, 0, 0.05, "tied"), (0, 0, np.inf, "tied"), (0, 1, 0.05, "general"),
    (1, 0, 0.05, "tied"), (1, 1, 0.05, "factored"), (2, 0, 0.05, "tied"), (2, 1, 0.05, "tied")])
def test_which_fields_factor(ctx, beam, consistent, w0, layout):
    from paper_1609_08146_amd import Problem
    rng = np.random.default_rng(11)
    k = 7.854e6 * np.array([0.8, 1.0, 1.25])
    spec = rng.normal(size=3) + 1j * rng.normal(size=3)     # any complex spectrum keeps the direction
    p = Problem(ctx)
    p.set_mirror(0.1, 0.075, 24, 16)
    p.set_frequencies(k)
    p.set_incident_beam(beam, w0, 0.3 if beam == 0 else 0.0, spec, bool(consistent))
    p.set_observation(np.zeros((1, 3)))
    expect = layout != "general"
    assert p.factored is expect and p.layout_for("fp32_split") == layout
    # the beams that factor at all do so to rounding, below the FP64 form's tolerance too
    assert p.factored_for("fp64") is expect and p.factored_for("fp32") is False
    assert p.layout_for("fp64") == layout and p.layout_for("fp32") == "general"
    p.set_factoring(False)
    assert p.factored is False and p.factored_for("fp64") is False
    p.set_factoring(True, tie_charge=False)
    assert p.layout_for("fp32_split") == ("factored" if expect else "general")
    p.set_factoring(True)
    assert p.factored is expect and p.layout_for("fp64") == layout
    p.close()


def test_random_tables_do_not_factor(ctx):
    from paper_1609_08146_amd import Problem
    p = Problem(ctx)
    p.set_mirror(20.0, 40.0, 12, 8)
    p.set_frequencies([6.0, 7.0])
    Ei, Bi = workloads.random_incident_tables(2, 13 * 8, seed=3)
    p.set_incident(Ei, Bi)
    assert p.factored is False and p.factored_for("fp64") is False
    p.close()


@pytest.mark.parametrize("name", ["broadband", "stress"])
def test_factored_and_general_match_the_oracle(ctx, orc, name):
    from paper_1609_08146_amd import problem_from_workload
    if name == "broadband":
        w = workloads.broadband(n_k=128, n_nodes=120)
        sub = w.subset(obs_idx=np.arange(0, w.n_obs, 29), k_idx=np.arange(0, 128, 21))
    else:                                   # kR up to 1.6e6 rad
        w = workloads.stress(n_k=64, n_nodes=200)
        sub = w.subset(obs_idx=np.arange(0, w.n_obs, 1023), k_idx=[0, 31, 63])
    Eo, Bo = orc.solve(sub)
    p = problem_from_workload(ctx, sub)
    res = {}
    for layout in LAYOUTS:
        set_layout(p, layout)
        assert p.layout_for("fp32_split") == layout
        res[layout] = p.evaluate("fp32_split")
    errs = {k: max(rel_l2(E, Eo), rel_l2(B, Bo)) for k, (E, B) in res.items()}
    for a, b in [("tied", "general"), ("factored", "general"), ("tied", "factored")]:
        errs[f"{a}-{b}"] = max(rel_l2(res[a][0], res[b][0]), rel_l2(res[a][1], res[b][1]))
    print(name, {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["tied"] < 1e-5 and errs["factored"] < 1e-5 and errs["general"] < 1e-5
    assert errs["tied-general"] < 2e-6 and errs["factored-general"] < 2e-6 and errs["tied-factored"] < 2e-6
    p.close()


@pytest.mark.parametrize("beam,consistent", [(1, 0), (1, 1), (2, 0), (2, 1)])
def test_factored_cylindrical_beams_match_the_oracle(ctx, orc, beam, consistent):
    from paper_1609_08146_amd import problem_from_workload
    kind = {(1, 0): orc.RADIAL, (1, 1): orc.RADIAL_CONSISTENT, (2, 0): orc.AZIMUTHAL,
            (2, 1): orc.AZIMUTHAL_CONSISTENT}[(beam, consistent)]
    w = replace(workloads.broadband(n_k=6, n_nodes=90).subset(obs_idx=np.arange(0, 4160, 41)),
                beam=beam, consistent=consistent, w0=0.03)
    m = orc.mirror(w.f, w.a, w.n_r, w.n_phi)
    Ei, Bi = orc.incident_tables(m, w.k, kind, w.w0, 0.0, w.spectrum)
    Eo, Bo = orc.reflected_field(m, w.k, Ei, Bi, w.obs)
    p = problem_from_workload(ctx, w)
    assert p.layout_for("fp32_split") == ("factored" if (beam, consistent) == (1, 1) else "tied")
    for layout in ("tied", "factored"):
        set_layout(p, layout)
        E, B = p.evaluate("fp32_split")
        err = max(rel_l2(E, Eo), rel_l2(B, Bo))
        print(f"beam {beam} consistent {consistent} {p.layout_for('fp32_split')}: {err:.2e}")
        assert err < 1e-5
    p.close()


def test_factored_launch_shapes_and_batch_bitwise(ctx):
    """Launch shape never changes the bits of either path, and one persistent launch may mix
    factored and general problems: each keeps the bits it has alone."""
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.broadband(n_k=5, n_nodes=64)
    p = problem_from_workload(ctx, w)
    # with one point 400 wavelengths out, the phase takes the fractional-turn path
    far = np.concatenate([w.obs, [[0.0, 0.0, 400 * workloads.LAMBDA0]]])
    for obs in (w.obs, far):
        p.set_observation(obs)
        for layout in LAYOUTS:
            set_layout(p, layout)
            assert p.layout_for("fp32_split") == layout
            ref = None
            for opl, fpb in [(1, 1), (2, 1), (1, 2), (2, 2), (1, 4)]:
                for wpb in (1, 4):
                    p.set_launch(obs_per_lane=opl, freq_per_lane=fpb, waves_per_block=wpb, chunk=1024)
                    E, B = p.evaluate("fp32_split")
                    if ref is None:
                        ref = (E, B)
                    else:
                        assert np.array_equal(E, ref[0]) and np.array_equal(B, ref[1]), \
                            (len(obs), layout, opl, fpb, wpb)
    p.close()
    ws = workloads.sweep(6)
    ws = [w.with_nodes(min(w.n_r, 80), min(w.n_phi, 48)).subset(k_idx=np.arange(min(w.n_k, 3))) for w in ws]
    ws[1] = replace(ws[1], consistent=1)          # does not factor
    probs = [problem_from_workload(ctx, w) for w in ws]
    probs[2].set_factoring(False)                 # factors, but forced onto the general tables
    set_layout(probs[3], "factored")              # ties, but forced onto the factored layout alone
    assert [q.layout_for("fp32_split") for q in probs] == ["tied", "general", "general", "factored", "tied",
                                                           "tied"]
    alone = [q.evaluate("fp32_split") for q in probs]
    ctx.evaluate_batch(probs, "fp32_split")
    for q, (E, B) in zip(probs, alone):
        Eb, Bb = q.result()
        assert np.array_equal(E, Eb) and np.array_equal(B, Bb)
    for q in probs:
        q.close()


def test_spectrum_scaling_on_fp32_only_factored_tables(ctx, orc):
    """With the FP64 tables released, a spectral phase (chirp) and amplitude scale the factored
    FP32 tables in place; the field equals that of the scaled spectrum set directly."""
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.broadband(n_k=8, n_nodes=80).subset(obs_idx=np.arange(0, 4160, 37))
    phase = 40.0 * ((w.k - w.k.mean()) / (w.k.max() - w.k.min())) ** 2
    fac = 0.5 * np.exp(1j * phase)
    q = problem_from_workload(ctx, w)
    q.set_table_storage(False)
    q.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
    assert q.factored
    q.scale_spectrum(fac)
    E1, B1 = q.evaluate("fp32_split")
    w2 = replace(w, spectrum=w.spectrum * fac)
    Eo, Bo = orc.solve(w2)
    err = max(rel_l2(E1, Eo), rel_l2(B1, Bo))
    print(f"scaled factored FP32-only tables vs oracle: {err:.2e}")
    assert err < 1e-5
    q.close()


@pytest.mark.parametrize("name", ["broadband", "stress"])
def test_fp64_factored_and_general_match_the_oracle(ctx, orc, name):
    """The FP64 form on the factored tables: the oracle's tolerance for FP64 (1e-12 relative L2
    per field), and within 1e-13 of the FP64 form on the general tables."""
    from paper_1609_08146_amd import problem_from_workload
    if name == "broadband":
        w = workloads.broadband(n_k=128, n_nodes=120)
        sub = w.subset(obs_idx=np.arange(0, w.n_obs, 29), k_idx=np.arange(0, 128, 21))
    else:                                   # kR up to 1.6e6 rad
        w = workloads.stress(n_k=64, n_nodes=200)
        sub = w.subset(obs_idx=np.arange(0, w.n_obs, 1023), k_idx=[0, 31, 63])
    Eo, Bo = orc.solve(sub)
    p = problem_from_workload(ctx, sub)
    res = {}
    for layout in LAYOUTS:
        set_layout(p, layout)
        assert p.layout_for("fp64") == layout
        res[layout] = p.evaluate("fp64")
    errs = {k: max(rel_l2(E, Eo), rel_l2(B, Bo)) for k, (E, B) in res.items()}
    for a, b in [("tied", "general"), ("factored", "general"), ("tied", "factored")]:
        errs[f"{a}-{b}"] = max(rel_l2(res[a][0], res[b][0]), rel_l2(res[a][1], res[b][1]))
    print(name, {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["tied"] < 1e-12 and errs["factored"] < 1e-12 and errs["general"] < 1e-12
    assert errs["tied-general"] < 1e-13 and errs["factored-general"] < 1e-13 and errs["tied-factored"] < 1e-13
    p.close()


def test_fp64_factored_launch_shapes_batch_and_rescaling(ctx, orc):
    """FP64 on the factored tables: launch shapes keep the bits, a batch mixing factored and
    general FP64 problems keeps each problem's bits, and a spectral factor applied after the
    factored FP64 tables were built rebuilds them (the field equals the oracle's for the scaled
    spectrum)."""
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.broadband(n_k=5, n_nodes=64)
    p = problem_from_workload(ctx, w)
    for layout in LAYOUTS:                        # every layout takes the near-focus series here
        set_layout(p, layout)
        assert p.layout_for("fp64") == layout
        ref = None
        for opl, fpb in [(1, 1), (2, 1), (1, 2), (2, 2), (1, 4)]:
            p.set_launch(obs_per_lane=opl, freq_per_lane=fpb, waves_per_block=2, chunk=1024)
            E, B = p.evaluate("fp64")
            if ref is None:
                ref = (E, B)
            else:
                assert np.array_equal(E, ref[0]) and np.array_equal(B, ref[1]), (layout, opl, fpb)
    p.close()

    ws = workloads.sweep(4)
    ws = [w.with_nodes(min(w.n_r, 60), min(w.n_phi, 40)).subset(k_idx=np.arange(min(w.n_k, 2))) for w in ws]
    ws[1] = replace(ws[1], consistent=1)          # does not factor
    probs = [problem_from_workload(ctx, w) for w in ws]
    set_layout(probs[2], "factored")
    assert [q.layout_for("fp64") for q in probs] == ["tied", "general", "factored", "tied"]
    alone = [q.evaluate("fp64") for q in probs]
    ctx.evaluate_batch(probs, "fp64")
    for q, (E, B) in zip(probs, alone):
        Eb, Bb = q.result()
        assert np.array_equal(E, Eb) and np.array_equal(B, Bb)
    for q in probs:
        q.close()

    w = workloads.broadband(n_k=6, n_nodes=70).subset(obs_idx=np.arange(0, 4160, 53))
    fac = 0.7 * np.exp(1j * np.linspace(0.0, 3.0, w.n_k))
    q = problem_from_workload(ctx, w)
    q.evaluate("fp64")                            # builds the factored FP64 tables
    q.scale_spectrum(fac)
    assert q.factored_for("fp64")
    E1, B1 = q.evaluate("fp64")
    Eo, Bo = orc.solve(replace(w, spectrum=w.spectrum * fac))
    err = max(rel_l2(E1, Eo), rel_l2(B1, Bo))
    print(f"rescaled factored FP64 tables vs oracle: {err:.2e}")
    assert err < 1e-12
    q.close()


def test_releasing_the_fp64_tables_releases_their_factored_copy(ctx):
    """Dropping the FP64 tables (sc_set_table_storage(p, 0)) after an FP64 evaluation built the
    factored FP64 records frees those too: FP64 evaluation is refused, the split form still runs
    on its factored FP32 tables, and the device footprint shrinks by both FP64 layouts less the
    FP32 general tables the release casts (64 + 32 - 32 B per (k, node), 64 B per node)."""
    from paper_1609_08146_amd import problem_from_workload, ScError
    w = workloads.broadband(n_k=6, n_nodes=60).subset(obs_idx=np.arange(0, 4160, 97))
    p = problem_from_workload(ctx, w)
    E32, B32 = p.evaluate("fp32_split")
    p.evaluate("fp64")
    before = p.device_bytes()
    n_tot = (w.n_r + 1) * w.n_phi
    p.set_table_storage(False)
    after = p.device_bytes()
    assert before - after >= w.n_k * n_tot * 64 + n_tot * 64   # 32 B per (k, node) less if kept
    assert not p.factored_for("fp64") and p.factored
    with pytest.raises(ScError):
        p.evaluate("fp64")
    E, B = p.evaluate("fp32_split")
    assert np.array_equal(E, E32) and np.array_equal(B, B32)
    p.close()


def test_current_that_factors_only_at_the_split_tolerance(ctx, orc):
    """Tables whose current turns by ~3e-12 of its size from node direction u (a Gaussian beam's
    B plus a small random field, set through sc_set_incident) pass the split form's factoring
    test (1e-10) but not the FP64 form's (1e-14): FP32-split takes the factored tables, FP64 the
    general ones, and each stays within its tolerance of the oracle on the same tables."""
    from paper_1609_08146_amd import Problem
    f, a, nr, nphi = 20.0, 40.0, 40, 24
    ks = np.array([2 * np.pi, 2.3 * np.pi])
    m = orc.mirror(f, a, nr, nphi)
    Ei, Bi = orc.incident_tables(m, ks, orc.GAUSSIAN, 20.0)
    rng = np.random.default_rng(21)
    noise = rng.normal(size=Bi.shape) + 1j * rng.normal(size=Bi.shape)
    Bi = Bi + 3e-12 * np.abs(Bi).max(axis=-1, keepdims=True) * noise
    obs = workloads.random_points(64, 2.0, seed=4)
    Eo, Bo = orc.reflected_field(m, ks, Ei, Bi, obs)
    p = Problem(ctx)
    p.set_mirror(f, a, nr, nphi)
    p.set_frequencies(ks)
    p.set_incident(Ei, Bi)
    p.set_observation(obs)
    assert p.factored and not p.factored_for("fp64")
    E32, B32 = p.evaluate("fp32_split")
    E64, B64 = p.evaluate("fp64")
    e32 = max(rel_l2(E32, Eo), rel_l2(B32, Bo))
    e64 = max(rel_l2(E64, Eo), rel_l2(B64, Bo))
    print(f"split (factored) {e32:.2e}, fp64 (general) {e64:.2e}")
    assert e32 < 1e-5 and e64 < 1e-12
    p.close()


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_delta_by_series_and_by_division(ctx, orc, layout):
    """delta = |r_s - r'| - |r_s| comes from its series when every point lies within 4e-4 |r_s|
    (here f = 0.1 m, points within 4 wavelengths), else from the division.  One point 100
    wavelengths out switches the series off while the phase still skips the fractional turn
    (121 turns), so the two problems differ in delta alone.  Both match the oracle on the near
    points, and each other to FP32 rounding, on either table layout."""
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.broadband(n_k=6, n_nodes=60)
    near = w.obs[::41]
    far = np.array([[0.0, 0.0, 100 * workloads.LAMBDA0]])
    sub = replace(w, obs=near)
    Eo, Bo = orc.solve(sub)
    p = problem_from_workload(ctx, sub)
    set_layout(p, layout)
    assert p.layout_for("fp32_split") == layout
    Es, Bs = p.evaluate("fp32_split")
    p.set_observation(np.concatenate([near, far]))
    Ed, Bd = p.evaluate("fp32_split")
    Ed, Bd = Ed[:, : len(near)], Bd[:, : len(near)]
    errs = dict(series=max(rel_l2(Es, Eo), rel_l2(Bs, Bo)), division=max(rel_l2(Ed, Eo), rel_l2(Bd, Bo)),
                between=max(rel_l2(Es, Ed), rel_l2(Bs, Bd)))
    print(layout, {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["series"] < 1e-5 and errs["division"] < 1e-5
    assert errs["between"] < 2e-6
    assert not np.array_equal(Es, Ed)          # the two paths really differ in rounding
    p.close()


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_fp64_delta_by_series_and_by_division(ctx, orc, layout):
    """The FP64 form near the focus: delta and 1/|R| by their series (host points within 4e-4 |r_s|)
    against the division and the square root (the same points handed over in device memory take
    the general forms), on either table layout.  Both within 1e-12 of the oracle and within 1e-13 of
    each other."""
    import torch
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.broadband(n_k=6, n_nodes=60)
    near = w.obs[::41]
    sub = replace(w, obs=near)
    Eo, Bo = orc.solve(sub)
    p = problem_from_workload(ctx, sub)
    set_layout(p, layout)
    assert p.layout_for("fp64") == layout
    Es, Bs = p.evaluate("fp64")
    p.set_observation(torch.tensor(near, dtype=torch.float64, device="cuda"))
    Ed, Bd = p.evaluate("fp64")
    errs = dict(series=max(rel_l2(Es, Eo), rel_l2(Bs, Bo)), division=max(rel_l2(Ed, Eo), rel_l2(Bd, Bo)),
                between=max(rel_l2(Es, Ed), rel_l2(Bs, Bd)))
    print(layout, {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["series"] < 1e-12 and errs["division"] < 1e-12
    assert errs["between"] < 1e-13
    assert not np.array_equal(Es, Ed)          # the two paths really differ in rounding
    p.close()
