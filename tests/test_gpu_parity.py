"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (relative L2 per field, over all observation points, frequencies
and components, E and B separately):
  * SC_FP64        <= 1e-12
  * SC_FP32_SPLIT  <= 1e-5
Sizes are chosen so the oracle finishes in seconds while the GPU path still
spans several node chunks, several observation blocks and ragged tails.
"""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K = 2 * math.pi


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


def make_problem(ctx, f, a, n_r, n_phi, k, obs, launch=None):
    from paper_1609_08146_amd import Problem
    p = Problem(ctx)
    p.set_mirror(f, a, n_r, n_phi)
    p.set_frequencies(k)
    p.set_observation(obs)
    if launch:
        p.set_launch(**launch)
    return p


def test_nodes_match_oracle(ctx, orc):
    # Independent implementations of the same rule: both round quad-precision
    # Gauss-Legendre roots and evaluate the phi nodes with libm's sincos, and
    # the device forms the node records with IEEE products and quotients, so
    # the node sets are bitwise equal.  (A 1-ulp node difference moves a phase
    # by ~1e-10 rad at k ~ 1e7 / m, which is visible at the FP64 tolerance.)
    for (f, a, nr, nphi) in [(20.0, 40.0, 200, 200), (0.1, 0.075, 60, 60), (0.1, 0.075, 37, 24),
                             (0.05, 0.15, 801, 16)]:
        p = make_problem(ctx, f, a, nr, nphi, [K], np.zeros((1, 3)))
        xyz, nrm, w = p.get_nodes()
        m = orc.mirror(f, a, nr, nphi)
        for name, g, o in (("xyz", xyz, m.pos), ("normal", nrm, m.nrm), ("weight", w, m.wgt)):
            n_diff = int(np.count_nonzero(g != o))
            print(f"{name}: {n_diff} of {g.size} entries differ")
            assert n_diff == 0, name
        p.close()


@pytest.mark.parametrize("launch", [dict(chunk=256), dict(chunk=4096)])
def test_fp64_random_tables(ctx, orc, launch):
    # arbitrary tables exercise the quadrature as a linear map of E_inc, B_inc
    f, a, nr, nphi = 20.0, 40.0, 37, 24
    ks = np.array([K, 1.3 * K, 0.7 * K])
    obs = workloads.random_points(200, 2.5, seed=5)
    m = orc.mirror(f, a, nr, nphi)
    Ei, Bi = workloads.random_incident_tables(len(ks), m.n_tot, seed=9)
    Eo, Bo = orc.reflected_field(m, ks, Ei, Bi, obs)
    p = make_problem(ctx, f, a, nr, nphi, ks, obs, launch)
    p.set_incident(Ei, Bi)
    E, B = p.evaluate("fp64")
    assert rel_l2(E, Eo) < 1e-12
    assert rel_l2(B, Bo) < 1e-12
    p.close()


def test_fp64_gaussian_mono(ctx, orc):
    w = workloads.mono()
    sub = w.subset(obs_idx=np.arange(0, 1024, 5))   # 205 points: ragged vs the 128-point blocks
    Eo, Bo = orc.solve(sub)
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, sub)
    p.set_launch(chunk=2048)                         # 40200 nodes -> 20 chunks, ragged last chunk
    E, B = p.evaluate("fp64")
    assert rel_l2(E, Eo) < 1e-12
    assert rel_l2(B, Bo) < 1e-12
    p.close()


def test_fp64_and_split_broadband_subset(ctx, orc):
    w = workloads.broadband(n_k=128, n_nodes=120)
    sub = w.subset(obs_idx=np.arange(0, w.n_obs, 29), k_idx=np.arange(0, 128, 21))
    Eo, Bo = orc.solve(sub)
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, sub)
    E, B = p.evaluate("fp64")
    assert rel_l2(E, Eo) < 1e-12
    assert rel_l2(B, Bo) < 1e-12
    E, B = p.evaluate("fp32_split")
    assert E.dtype == np.complex64
    assert rel_l2(E, Eo) < 1e-5
    assert rel_l2(B, Bo) < 1e-5
    p.close()


def test_fp32_split_stress_geometry(ctx, orc):
    # deep dish, kR up to 1.6e6 rad: the split form keeps FP32 accuracy, the naive form does not
    w = workloads.stress(n_k=64, n_nodes=200)
    sub = w.subset(obs_idx=np.arange(0, w.n_obs, 1023), k_idx=[0, 31, 63])
    Eo, Bo = orc.solve(sub)
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, sub)
    E, B = p.evaluate("fp32_split")
    err_split = max(rel_l2(E, Eo), rel_l2(B, Bo))
    E, B = p.evaluate("fp32")
    err_naive = max(rel_l2(E, Eo), rel_l2(B, Bo))
    E, B = p.evaluate("fp64")
    err_64 = max(rel_l2(E, Eo), rel_l2(B, Bo))
    print(f"stress: fp64 {err_64:.2e}  fp32_split {err_split:.2e}  fp32 naive {err_naive:.2e}")
    assert err_64 < 1e-12
    assert err_split < 1e-5
    assert err_naive > 100 * err_split
    p.close()


def test_full_size_stress_sampled(ctx, orc):
    """The precision workload at full size (800 x 800 nodes, 128 x 128 points, 64 frequencies,
    6.7e11 evaluations) in the default launch: sampled outputs against the oracle, and the whole
    grid of the split form against the GPU FP64 form."""
    w = workloads.stress()
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, w)
    E, B = p.evaluate("fp32_split")
    rng = np.random.default_rng(3)
    oi = np.sort(rng.choice(w.n_obs, 6, replace=False))
    ki = np.array([0, 21, 42, 63])
    Eo, Bo = orc.solve(w.subset(obs_idx=oi, k_idx=ki))
    err = max(rel_l2(E[ki][:, oi], Eo), rel_l2(B[ki][:, oi], Bo))
    E64, B64 = p.evaluate("fp64")
    err64 = max(rel_l2(E64[ki][:, oi], Eo), rel_l2(B64[ki][:, oi], Bo))
    whole = max(rel_l2(E, E64), rel_l2(B, B64))
    print(f"stress full size: split vs oracle {err:.2e}, fp64 vs oracle {err64:.2e}, split vs fp64 {whole:.2e}")
    assert err < 1e-5 and err64 < 1e-12 and whole < 1e-5
    p.close()


def test_full_size_sweep_batch_sampled(ctx, orc):
    """Sweep instances at their full sizes in one persistent launch; sampled outputs per instance."""
    from paper_1609_08146_amd import problem_from_workload
    ws = workloads.sweep(24)
    probs = [problem_from_workload(ctx, w) for w in ws]
    ctx.evaluate_batch(probs, "fp32_split")
    rng = np.random.default_rng(9)
    worst = 0.0
    for w, p in zip(ws, probs):
        E, B = p.result()
        # like the relative L2 norm over a whole output, the sample holds the strong focal field:
        # the point nearest the focus and the carrier, plus two random points and one random frequency
        # (a lone point 4 wavelengths out at a band-edge frequency can be 1e-4 of the peak)
        focus = int(np.argmin(np.linalg.norm(w.obs, axis=1)))
        oi = np.unique(np.concatenate([[focus], rng.choice(w.n_obs, 2, replace=False)]))
        ki = np.unique([w.n_k // 2, int(rng.integers(w.n_k))])
        Eo, Bo = orc.solve(w.subset(obs_idx=oi, k_idx=ki))
        err = max(rel_l2(E[ki][:, oi], Eo), rel_l2(B[ki][:, oi], Bo))
        worst = max(worst, err)
        assert err < 1e-5, (w.name, err)
        p.close()
    print(f"sweep full size, 24 instances in one launch: worst sampled relative L2 {worst:.2e}")


def test_time_transform(ctx, orc):
    w = workloads.broadband(n_k=32, n_nodes=60)
    sub = w.subset(obs_idx=np.arange(0, w.n_obs, 97))
    Eo, Bo = orc.solve(sub)
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, sub)
    t = w.t[::5]
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        E, B = p.evaluate(prec)
        Et, Bt = p.to_time_at(w.dk, t)
        # 1) the spectrum, 2) the transform kernel on the GPU's own spectrum, 3) end to end
        e_spec = max(rel_l2(E, Eo), rel_l2(B, Bo))
        Etg = orc.time_transform(sub.k, w.dk, t, E.astype(np.complex128))
        Btg = orc.time_transform(sub.k, w.dk, t, B.astype(np.complex128))
        e_tr = max(rel_l2(Et, Etg), rel_l2(Bt, Btg))
        Eto = orc.time_transform(sub.k, w.dk, t, Eo)
        Bto = orc.time_transform(sub.k, w.dk, t, Bo)
        e_all = max(rel_l2(Et, Eto), rel_l2(Bt, Bto))
        print(f"{prec}: spectrum {e_spec:.2e}, transform {e_tr:.2e}, end to end {e_all:.2e}")
        assert e_spec < tol, prec
        # both sides form k t (~1.6e6 rad) beyond double precision: the device in double-double, the
        # oracle in quad precision
        assert e_tr < (1e-13 if prec == "fp64" else 1e-6), prec
        assert e_all < tol, prec
    p.close()


def test_uniform_time_grid_form(ctx):
    """sc_to_time takes the uniform time grid t0 + m dt and the step (k_last - k_first) / (n_k - 1) of
    the uniform frequency grid as its weight: it gives sc_to_time_at's bits on the same times with
    that weight, and refuses a frequency grid that is not uniform."""
    from paper_1609_08146_amd import ScError, problem_from_workload
    from paper_1609_08146_amd._abi import SC_E_INVAL
    w = workloads.broadband(n_k=16, n_nodes=40).subset(obs_idx=np.arange(0, 4160, 211))
    p = problem_from_workload(ctx, w)
    dk = (w.k[-1] - w.k[0]) / (len(w.k) - 1)
    for prec in ("fp64", "fp32_split"):
        p.evaluate(prec)
        t0, dt = float(w.t[96]), float(w.t[1] - w.t[0])      # 64 samples across the pulse
        Et, Bt = p.to_time(t0, dt, 64)
        Ea, Ba = p.to_time_at(dk, t0 + np.arange(64) * dt)
        assert Et.shape == (64, w.n_obs, 3)
        assert np.array_equal(Et, Ea) and np.array_equal(Bt, Ba), prec
    p.close()
    q = make_problem(ctx, 20.0, 40.0, 20, 16, [K, 1.1 * K, 1.3 * K], np.zeros((2, 3)) + 0.1)
    q.set_incident_gaussian(20.0)
    q.evaluate("fp64")
    with pytest.raises(ScError) as e:
        q.to_time(0.0, 0.1, 8)
    assert e.value.status == SC_E_INVAL
    q.close()


def test_launch_shape_does_not_change_bits(ctx):
    # 5 frequencies: frequency blocks of 2 and 4 leave a ragged last block
    w = workloads.broadband(n_k=5, n_nodes=64)
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, w)
    ref = {}
    shapes = [(1, 1), (2, 1), (1, 2), (2, 2), (1, 4)]
    for opl, fpb in shapes:
        for wpb in (1, 2, 4):
            for bpc in (0, 1):
                p.set_launch(obs_per_lane=opl, freq_per_lane=fpb, waves_per_block=wpb, chunk=1024,
                             blocks_per_cu=bpc)
                for prec in ("fp32_split", "fp64", "fp32"):
                    E, B = p.evaluate(prec)
                    if prec not in ref:
                        ref[prec] = (E, B)
                    else:
                        assert np.array_equal(E, ref[prec][0]) and np.array_equal(B, ref[prec][1]), \
                            (prec, opl, fpb, wpb, bpc)
    p.close()


def test_autotune_chunk_sets_the_bits_and_its_cache_round_trips(ctx, orc, tmp_path):
    """The tuner searches kernel shapes, then the chunk.  The tuned launch (from the context's cache)
    gives exactly the bits of an explicit launch with the tuned chunk, stays within the tolerance
    of the oracle, and its cache file loads back into a fresh context and rejects junk."""
    from paper_1609_08146_amd import Context, ScError, problem_from_workload
    w = workloads.broadband(n_k=6, n_nodes=96).subset(obs_idx=np.arange(0, 4160, 13))
    Eo, Bo = orc.solve(w)
    p = problem_from_workload(ctx, w)
    best = p.autotune("fp32_split", budget_ms=20000)
    assert best["obs_per_lane"] in (1, 2) and best["freq_per_lane"] in (1, 2, 4)
    assert best["waves_per_block"] in (1, 2, 4) and best["blocks_per_cu"] in (0, 1, 2)
    assert best["chunk"] in (512, 1024, 2048, 4096, 8192, 16384)
    assert p.launch("fp32_split") == best
    E1, B1 = p.evaluate("fp32_split")        # resolved from the context's tuning cache
    assert max(rel_l2(E1, Eo), rel_l2(B1, Bo)) < 1e-5
    q = problem_from_workload(ctx, w)
    q.set_launch(chunk=best["chunk"])         # the library's kernel shape, the tuned chunk
    E2, B2 = q.evaluate("fp32_split")
    assert np.array_equal(E1, E2) and np.array_equal(B1, B2)
    q.close()
    path = tmp_path / "tune.txt"
    ctx.autotune_save(str(path))
    rows = [ln.split() for ln in path.read_text().splitlines() if not ln.startswith("#")]
    assert any([int(x) for x in r[5:]] == [best["obs_per_lane"], best["waves_per_block"], best["chunk"],
                                          best["blocks_per_cu"], best["freq_per_lane"]] for r in rows)
    ctx2 = Context(0)
    try:
        ctx2.autotune_load(str(path))
        p2 = problem_from_workload(ctx2, w)
        E3, B3 = p2.evaluate("fp32_split")
        assert np.array_equal(E1, E3) and np.array_equal(B1, B3)
        p2.close()
        bad = tmp_path / "bad.txt"
        bad.write_text("1 2 3\n")
        with pytest.raises(ScError):
            ctx2.autotune_load(str(bad))
        bad.write_text("1 1 8 2 17 3 4 4096 0 2\n")     # 3 observation points per lane: not a kernel shape
        with pytest.raises(ScError):
            ctx2.autotune_load(str(bad))
    finally:
        ctx2.close()
    p.close()


def test_batch_autotune_and_batch_launch(ctx):
    """The batch tuner times batched launches on the batch and keeps the winner as the context's batch
    launch; every problem of a tuned batch equals its alone result at the batch's chunk (or its own),
    and clearing the batch launch brings back the default launch's bits."""
    from paper_1609_08146_amd import problem_from_workload
    ws = workloads.sweep(6)
    ws = [w.with_nodes(min(w.n_r, 90), min(w.n_phi, 64)).subset(k_idx=np.arange(min(w.n_k, 5))) for w in ws]
    probs = [problem_from_workload(ctx, w) for w in ws]
    default = [p.evaluate("fp32_split") for p in probs]
    best = ctx.autotune_batch(probs, "fp32_split", budget_ms=15000)
    assert best["chunk"] in (0, 1024, 2048, 4096, 8192, 16384)
    ctx.evaluate_batch(probs, "fp32_split")
    for w, p, (E0, B0) in zip(ws, probs, default):
        Eb, Bb = p.result()
        if best["chunk"]:
            q = problem_from_workload(ctx, w)
            q.set_launch(chunk=best["chunk"])
            Ea, Ba = q.evaluate("fp32_split")
            q.close()
        else:
            Ea, Ba = E0, B0
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
        assert rel_l2(Eb, E0) < 1e-5
    ctx.set_batch_launch("fp32_split", reset=True)
    ctx.evaluate_batch(probs, "fp32_split")
    for p, (E0, B0) in zip(probs, default):
        Eb, Bb = p.result()
        assert np.array_equal(E0, Eb) and np.array_equal(B0, Bb)
    for p in probs:
        p.close()


def test_batch_equals_alone_bitwise(ctx):
    from paper_1609_08146_amd import problem_from_workload
    ws = workloads.sweep(5)
    ws = [w.with_nodes(min(w.n_r, 80), min(w.n_phi, 48)).subset(k_idx=np.arange(min(w.n_k, 3))) for w in ws]
    probs = [problem_from_workload(ctx, w) for w in ws]
    alone = [p.evaluate("fp32_split") for p in probs]
    ctx.evaluate_batch(probs, "fp32_split")
    for p, (E, B) in zip(probs, alone):
        Eb, Bb = p.result()
        assert np.array_equal(E, Eb) and np.array_equal(B, Bb)
    from paper_1609_08146_amd import ScError
    from paper_1609_08146_amd._abi import SC_E_INVAL
    with pytest.raises(ScError) as e:              # one problem twice would share its partial sums
        ctx.evaluate_batch([probs[0], probs[1], probs[0]], "fp32_split")
    assert e.value.status == SC_E_INVAL
    Eb, Bb = probs[0].result()                     # the rejected call left the earlier result alone
    assert np.array_equal(alone[0][0], Eb)
    for p in probs:
        p.close()


def test_batch_keeps_partials_within_the_cap(ctx):
    """A batch whose split-K partials at the default chunk would exceed max(2 x 16 B x frequencies x
    nodes, 8 GiB) raises the chunk of the problems that fix none (here 10.3 GB at 2048 nodes ->
    4096); a problem with its own chunk keeps it, and each result equals the alone result at the
    chunk the batch used."""
    from paper_1609_08146_amd import Problem
    big = Problem(ctx)
    big.set_mirror(20.0, 40.0, 320, 320)                    # 102 720 nodes
    big.set_frequencies(np.linspace(2 * np.pi, 3 * np.pi, 256))
    big.set_incident_gaussian(20.0)
    big.set_observation(workloads.random_points(16384, 2.0, seed=21))
    small = Problem(ctx)
    small.set_launch(chunk=1024)
    small.set_mirror(20.0, 40.0, 40, 32)
    small.set_frequencies([2 * np.pi])
    small.set_incident_gaussian(20.0)
    small.set_observation(workloads.random_points(100, 2.0, seed=22))
    ctx.evaluate_batch([big, small], "fp32_split")
    assert big.timing()["chunk"] == 4096 and small.timing()["chunk"] == 1024
    Eb, Bb = big.result()
    Es, Bs = small.result()
    big.set_launch(chunk=4096)
    E, B = big.evaluate("fp32_split")
    assert big.timing()["chunk"] == 4096
    assert np.array_equal(E, Eb) and np.array_equal(B, Bb)
    E, B = small.evaluate("fp32_split")
    assert np.array_equal(E, Es) and np.array_equal(B, Bs)
    big.close()
    small.close()


def test_error_paths(ctx):
    from paper_1609_08146_amd import Problem, ScError
    from paper_1609_08146_amd._abi import SC_E_INVAL, SC_E_STATE
    p = Problem(ctx)
    with pytest.raises(ScError) as e:
        p.evaluate("fp64")
    assert e.value.status == SC_E_STATE
    with pytest.raises(ScError) as e:
        p.set_mirror(-1.0, 1.0, 10, 10)
    assert e.value.status == SC_E_INVAL
    with pytest.raises(ScError) as e:
        p.set_frequencies([1.0, -2.0])
    assert e.value.status == SC_E_INVAL
    p.set_mirror(1.0, 1.0, 8, 8)
    with pytest.raises(ScError) as e:
        p.set_incident_gaussian(1.0)          # no frequencies yet
    assert e.value.status == SC_E_STATE
    with pytest.raises(ScError) as e:
        p.set_launch(obs_per_lane=3)
    assert e.value.status == SC_E_INVAL
    # buffers the library would read or write through raw pointers are checked before the call
    import torch
    p.set_frequencies([1.0, 2.0])
    n_tot = sum(p.num_nodes())
    with pytest.raises(ValueError):
        p.set_incident(np.zeros((2, n_tot - 1, 3), complex), np.zeros((2, n_tot - 1, 3), complex))
    p.set_incident_gaussian(1.0)
    p.set_observation(np.zeros((5, 3)) + 0.1)
    small = torch.empty((2, 4, 3), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        p.evaluate("fp32_split", out=(small, small))
    wrong = torch.empty((2, 5, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(TypeError):
        p.evaluate("fp32_split", out=(wrong, wrong))
    with pytest.raises(TypeError):
        p.set_observation(torch.zeros((5, 3), dtype=torch.float32, device="cuda"))
    good = torch.empty((2, 5, 3), dtype=torch.complex64, device="cuda")
    p.evaluate("fp32_split", out=(good, good))
    with pytest.raises(ValueError):
        p.to_time_at(1.0, np.zeros(3), out=(good, good))       # 3 times x 5 points do not fit 2 x 5
    p.close()


def test_full_size_broadband_sampled(ctx, orc):
    """The bench configuration itself (400x400 nodes, 4160 points, all 128 frequencies, default
    launch, factored current): sampled (point, frequency) outputs against the oracle, the focus
    among them, and the whole grid of the split form against the GPU FP64 form."""
    w = workloads.broadband()
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, w)
    assert p.factored and p.factored_for("fp64")
    E, B = p.evaluate("fp32_split")
    rng = np.random.default_rng(1)
    focus = int(np.argmin(np.linalg.norm(w.obs, axis=1)))
    oi = np.unique(np.concatenate([[focus], rng.choice(w.n_obs, 11, replace=False)]))
    ki = np.array([0, 31, 64, 77, 127])
    Eo, Bo = orc.solve(w.subset(obs_idx=oi, k_idx=ki))
    err = max(rel_l2(E[ki][:, oi], Eo), rel_l2(B[ki][:, oi], Bo))
    E64, B64 = p.evaluate("fp64")
    err64 = max(rel_l2(E64[ki][:, oi], Eo), rel_l2(B64[ki][:, oi], Bo))
    whole = max(rel_l2(E, E64), rel_l2(B, B64))
    print(f"broadband full size: split vs oracle {err:.2e}, fp64 vs oracle {err64:.2e}, split vs fp64 {whole:.2e}")
    assert err < 1e-5 and err64 < 1e-12 and whole < 1e-5
    p.close()


def test_fp32_only_table_storage(ctx):
    from paper_1609_08146_amd import ScError, problem_from_workload
    from paper_1609_08146_amd._abi import SC_E_STATE
    w = workloads.broadband(n_k=3, n_nodes=80).subset(obs_idx=np.arange(0, 4160, 13))
    p = problem_from_workload(ctx, w)
    E0, B0 = p.evaluate("fp32_split")
    N0, _ = p.evaluate("fp32")
    full = p.device_bytes()
    p.set_table_storage(False)          # cast now, release the FP64 tables
    E1, B1 = p.evaluate("fp32_split")
    assert np.array_equal(E0, E1) and np.array_equal(B0, B1)
    with pytest.raises(ScError) as e:
        p.evaluate("fp64")
    assert e.value.status == SC_E_STATE
    assert p.device_bytes() < full
    p.close()
    # the same from the start: tables built, cast and released inside set_incident
    q = problem_from_workload(ctx, w)
    q.set_table_storage(False)
    q.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
    E2, B2 = q.evaluate("fp32_split")
    assert np.array_equal(E0, E2) and np.array_equal(B0, B2)
    N2, _ = q.evaluate("fp32")          # naive tables derived from the FP32 split tables
    assert rel_l2(N2, N0) < 1e-6
    q.close()


def test_phase_with_and_without_the_fractional_turn(ctx, orc):
    """The split phase goes to the hardware sin/cos as is when every point of a problem keeps
    |k delta| / 2 pi below 250 turns, else through its fractional part.  Points near the focus alone
    take the first path; the same points with one far point (|r'| = 300 wavelengths) take the
    second.  Both match the oracle, and each other to FP32 rounding."""
    from paper_1609_08146_amd import Problem
    f, a, nr, nphi = 20.0, 40.0, 48, 32
    near = workloads.random_points(150, 2.5, seed=21)
    far = np.array([[0.0, 0.0, 300.0]])
    m = orc.mirror(f, a, nr, nphi)
    Ei, Bi = workloads.random_incident_tables(1, m.n_tot, seed=4)
    res = {}
    for name, pts in (("near", near), ("near+far", np.concatenate([near, far]))):
        p = Problem(ctx)
        p.set_mirror(f, a, nr, nphi)
        p.set_frequencies([K])
        p.set_incident(Ei, Bi)
        p.set_observation(pts)
        res[name] = p.evaluate("fp32_split")
        p.close()
    Eo, Bo = orc.reflected_field(m, np.array([K]), Ei, Bi, near)
    En, Bn = res["near"]
    Ef, Bf = res["near+far"]
    Ef, Bf = Ef[:, : len(near)], Bf[:, : len(near)]
    errs = dict(raw=max(rel_l2(En, Eo), rel_l2(Bn, Bo)), fract=max(rel_l2(Ef, Eo), rel_l2(Bf, Bo)),
                between=max(rel_l2(En, Ef), rel_l2(Bn, Bf)))
    print({k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["raw"] < 1e-5 and errs["fract"] < 1e-5
    assert errs["between"] < 2e-6
    assert not np.array_equal(En, Ef)          # the two paths really differ in rounding


def test_split_form_away_from_the_focus(ctx, orc):
    """Points 50 to 300 wavelengths from the focus (in the diverging reflected beam of the
    monochromatic mirror).  The split form rounds to FP32 the observation point, the node
    coordinates, the product r_s . r' behind delta and the phase k delta itself, each an error of
    about k |r'| 2^-24 rad per term, so its error grows linearly with |r'|: at each distance it must
    stay below 8 k |r'| 2^-24 relative (1.5e-4 at 50 wavelengths, 9e-4 at 300).  The FP64
    form, at k |r'| 2^-53, stays within 1e-12."""
    from paper_1609_08146_amd import Problem
    f, a, nr, nphi = 20.0, 40.0, 96, 64
    m = orc.mirror(f, a, nr, nphi)
    Ei, Bi = orc.incident_tables(m, np.array([K]), orc.GAUSSIAN, 20.0)
    th = np.radians([0.0, 20.0, 40.0])
    dirs = np.stack([np.sin(th), 0.0 * th, np.cos(th)], axis=-1)
    for d in (50.0, 100.0, 200.0, 300.0):
        pts = d * dirs
        Eo, Bo = orc.reflected_field(m, np.array([K]), Ei, Bi, pts)
        p = Problem(ctx)
        p.set_mirror(f, a, nr, nphi)
        p.set_frequencies([K])
        p.set_incident(Ei, Bi)
        p.set_observation(pts)
        E32, B32 = p.evaluate("fp32_split")
        E64, B64 = p.evaluate("fp64")
        p.close()
        e32 = max(rel_l2(E32, Eo), rel_l2(B32, Bo))
        e64 = max(rel_l2(E64, Eo), rel_l2(B64, Bo))
        bound = 8 * K * d * 2.0 ** -24
        print(f"|r'| = {d:5.0f} wavelengths: fp32_split {e32:.1e} (bound {bound:.1e}), fp64 {e64:.1e}")
        assert e32 < bound and e64 < 1e-12
