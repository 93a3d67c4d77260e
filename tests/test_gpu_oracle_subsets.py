"""GPU parity on the deterministic oracle subsets of the four workloads (Sec. IV-A numerical checks):

  * mono (200 x 200 nodes, 32 x 32 focal-plane points, one frequency): every output, FP64 and
    FP32-split;
  * broadband (the bench workload, 400 x 400 nodes, all 128 frequencies, default launch): every
    64th observation point (the grid column through the focal spot) x all 128 frequencies;
  * stress (800 x 800 nodes, kR up to 1.6e6 rad): 64 points x 8 frequencies, with the naive FP32
    form far off;
  * sweep: all 256 uneven instances in ONE persistent launch with FP32-only table storage and the
    batch chunk of 16384 nodes, 16 points (the one nearest the focus among them) x up to 4
    frequencies per instance.

Every comparison is element by element against the CPU oracle: relative L2 per field (the
tolerance: 1e-12 FP64, 1e-5 FP32-split) and, per output component, the largest error divided by
the peak |F| of the field, under the same bound.  The per-component e_rel of the paper (largest
error over the component's own peak) is printed for the record.
"""
import numpy as np
import pytest

import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = {"fp64": 1e-12, "fp32_split": 1e-5}
COMPONENTS = ("x", "y", "z")


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def compare(E, B, Eo, Bo, tol, label, quiet=False):
    """Relative L2 per field and per-component maxima; returns the worst figure against `tol`."""
    worst = 0.0
    rows = []
    for name, F, Fo in (("E", E, Eo), ("B", B, Bo)):
        F, Fo = np.asarray(F, np.complex128), np.asarray(Fo)
        peak = float(np.max(np.linalg.norm(Fo, axis=-1)))
        r = rel_l2(F, Fo)
        worst = max(worst, r)
        for c, ax in enumerate(COMPONENTS):
            err = float(np.max(np.abs(F[..., c] - Fo[..., c])))
            own = float(np.max(np.abs(Fo[..., c])))
            worst = max(worst, err / peak)
            rows.append(f"{name}_{ax} {err / peak:.1e} [e_rel {err / own if own > 0 else 0.0:.1e}]")
        rows.append(f"{name} relL2 {r:.1e}")
    if not quiet:
        print(f"{label}: " + ", ".join(rows))
    assert worst < tol, (label, worst, rows)
    return worst


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08146_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_mono_in_full(ctx, orc):
    """The monochromatic workload in full: all 1024 points, FP64 and FP32-split."""
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.mono()
    Eo, Bo = orc.solve(w)
    p = problem_from_workload(ctx, w)
    for prec in ("fp64", "fp32_split"):
        E, B = p.evaluate(prec)
        compare(E, B, Eo, Bo, TOL[prec], f"mono {prec}")
    p.close()


def test_broadband_every_64th_point_all_frequencies(ctx, orc):
    """The bench workload in the default launch: every 64th observation point from the 33rd on
    (the grid column nearest x = 0 through the focal spot, and one axial point; 65 points) x all
    128 frequencies x all 160 400 nodes against the oracle, both forms."""
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.broadband()
    p = problem_from_workload(ctx, w)
    launch = p.launch("fp32_split")
    assert launch["obs_per_lane"] == 1 and launch["blocks_per_cu"] == 0   # the library default
    oi = np.arange(32, w.n_obs, 64)
    Eo, Bo = orc.solve(w.subset(obs_idx=oi))
    for prec in ("fp32_split", "fp64"):
        E, B = p.evaluate(prec)
        compare(E[:, oi], B[:, oi], Eo, Bo, TOL[prec], f"broadband 1/64 points x 128 freq {prec}")
    p.close()


def test_stress_64_points_8_frequencies(ctx, orc):
    """The precision workload at full size: 64 points x 8 frequencies against the oracle; the naive
    FP32 form (whole kR per pair in FP32) is far outside the tolerance."""
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.stress()
    oi = np.linspace(0, w.n_obs - 1, 64).round().astype(int)
    ki = np.arange(0, 64, 8)
    sub = w.subset(obs_idx=oi, k_idx=ki)
    Eo, Bo = orc.solve(sub)
    p = problem_from_workload(ctx, w)
    worst = {}
    for prec in ("fp64", "fp32_split"):
        E, B = p.evaluate(prec)
        worst[prec] = compare(E[ki][:, oi], B[ki][:, oi], Eo, Bo, TOL[prec], f"stress 64 x 8 {prec}")
    E, B = p.evaluate("fp32")
    naive = max(rel_l2(E[ki][:, oi], Eo), rel_l2(B[ki][:, oi], Bo))
    print(f"stress 64 x 8 naive fp32: relL2 {naive:.1e}")
    assert naive > 1e3 * worst["fp32_split"]
    p.close()


def test_sweep_all_instances_in_one_launch(ctx, orc):
    """All 256 sweep instances in one persistent launch (FP32-only tables, chunk 16384, the batch
    bench's set-up), then per instance 16 points x up to 4 frequencies against the oracle."""
    from paper_1609_08146_amd import Problem
    ws = workloads.sweep(256)
    probs = []
    for w in ws:
        p = Problem(ctx)
        p.set_table_storage(False)
        p.set_launch(chunk=16384)
        p.set_mirror(w.f, w.a, w.n_r, w.n_phi)
        p.set_frequencies(w.k)
        p.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
        p.set_observation(w.obs)
        probs.append(p)
    ctx.evaluate_batch(probs, "fp32_split")
    worst = 0.0
    for i, (w, p) in enumerate(zip(ws, probs)):
        E, B = p.result()
        p.close()
        focus = int(np.argmin(np.linalg.norm(w.obs, axis=1)))
        oi = np.unique(np.concatenate([[focus], np.linspace(0, w.n_obs - 1, 15).round().astype(int)]))
        ki = np.unique(np.linspace(0, w.n_k - 1, min(4, w.n_k)).round().astype(int))
        Eo, Bo = orc.solve(w.subset(obs_idx=oi, k_idx=ki))
        worst = max(worst, compare(E[ki][:, oi], B[ki][:, oi], Eo, Bo, TOL["fp32_split"], f"sweep {i} {w.name}",
                                   quiet=True))
    print(f"sweep, 256 instances in one launch: worst relative L2 or per-component maximum {worst:.1e}")
