"""Benchmark of the Stratton-Chu mirror-focusing hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--shard S] [--precision fp32_split]

One step is one pass of the whole path over the broadband workload (800 nm,
10 fs Gaussian spectrum, f = 0.1 m, aperture radius 0.075 m, w0 = 0.05 m,
400 x 400 mirror nodes, 64 x 64 focal-plane points over +-4 lambda0 plus 64
axial points): mirror node tables, incident / current tables for every
frequency, the surface quadrature for every (point, frequency), the split-K
reduction, and the transform to 256 time samples, over all 128 frequencies
(8.5e10 integrand evaluations).  ``--shard S`` keeps every S-th frequency.

Prints one JSON line.  `value` is integrand evaluations per second
(observation points x frequencies x surface nodes) of the whole step;
`roofline` reports the quadrature kernel against the FP32 vector ALU peak,
with its duration measured by HIP events on the library's stream;
`cpu_baseline` is the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# Algorithmic work of the split form, counted from the kernel source (FMA = 2
# flops; the transcendental instructions rsq, rcp, sin, cos are not counted).
# General tables:
#   per (node, point) geometry:  R, |R|^2, R, r_s.r', delta                 18
#   per (node, point, frequency): phase 2, g 2, (ik - 1/R)/R 2, h 6,
#                                 E += Jt g 24, rho_t h 6, E += .. R 12,
#                                 Jt h 18, B += (Jt h) x R 24              96
# Factored current Jt = u s (a real direction u per node):
#   per (node, point):            geometry 18, 1/R^2 1, v = u/R 3,
#                                 e = R/R^2 3, w = u x e 9                 34
#   per (node, point, frequency): phase 2, A = s Z 6, C = rho_t Z 6,
#                                 A m, C m (m = ik - 1/R) 12, E += v A 12,
#                                 E += (C m) e 12, B += (A m) w 12         62
# The same with the charge tied to the current (rho_t = -i beta s / k) and s
# in polar form (|s|, arg s / 2 pi), its phase added to the sine's argument:
#   per (node, point):            the factored 34, e' = beta e 3           37
#   per (node, point, frequency): phase 2, A = |s| (cos, sin) 2,
#                                 q = 1/(kR) 1, M = A (i - q) 4, E += v A 12,
#                                 E += e' (-i M) 12, B += M w 12           45
#   (the FP64 form keeps s as a complex number: A = s Z 6,                 49)
# The kernel shares the per-(node, point) work among the frequencies of a
# lane (freq_per_lane of the launch, read back from the library for every
# figure below).  Where the observation points lie within 4e-4 |r_s|
# of the focus, the kernel forms delta and 1/|R| by short series instead of a
# reciprocal and a square root (5 more flops per (node, point), not counted:
# the constant stays the formula's).
FLOPS = {"general": (18, 96), "factored": (34, 62), "tied": (37, 45)}   # (per node and point, per frequency)
FLOPS_FP64 = {**FLOPS, "tied": (37, 49)}


def flops_per_eval(layout: str, freq_per_lane: int, fp64: bool = False) -> float:
    """Algorithmic flops per evaluation of a table layout ("general", "factored", "tied")."""
    geom, freq = (FLOPS_FP64 if fp64 else FLOPS)[layout]
    return freq + geom / freq_per_lane


# MI355X vector peaks: 256 CU x 4 SIMD x 2.4 GHz x (32 FP32 | 16 FP64) lanes x 2 (FMA)
PEAK_FP32 = 256 * 4 * 32 * 2 * 2.4e9 / 1e12   # 157.3 TFLOP/s
PEAK_FP64 = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6 TFLOP/s


# HBM traffic of the quadrature kernel, from the committed rocprofv3 counter
# summary; reported only while the kernel sources are the ones it was taken on.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_quad_broadband_hbm_traffic.md")
KERNEL_SOURCES = ["paper_1609_08146_amd/csrc/sc_quad.hip", "paper_1609_08146_amd/csrc/sc_device.h",
                  "paper_1609_08146_amd/csrc/sc_quadjob.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Calibrated HBM bytes per quadrature launch, or None if the kernel changed since the counters."""
    try:
        fields = {}
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                key, sep, val = line.strip().partition(":")
                if sep and key in ("kernel_source_sha256", "traffic_bytes_per_launch"):
                    fields[key] = val.strip()
        if fields.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def progress(msg: str):
    """One line per finished phase on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shard", type=int, default=1,
                    help="take every S-th frequency (S > 1 models one GPU's share under frequency sharding)")
    ap.add_argument("--precision", default="fp32_split", choices=["fp32_split", "fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--general-tables", action="store_true",
                    help="step, batch: never use the factored current (time the general-table layout)")
    ap.add_argument("--no-tie", action="store_true",
                    help="step, batch: the factored current without the tied charge (time that layout)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0, help="target CPU time of the oracle sample")
    ap.add_argument("--mode", default="step",
                    choices=["step", "batch", "serve", "copy", "table1", "valu", "convergence", "refine"],
                    help="step: the hot path on the broadband workload (default); batch: the seeded sweep of "
                         "uneven instances in one persistent launch; serve: a Poisson request stream; "
                         "table1: the Table I workload with energy normalisation and diagnostics; "
                         "valu: issue cost of the kernel's vector instructions; "
                         "convergence: e_rel per component under mesh refinement (Sec. IV-A); "
                         "refine: e_rel under refinement on the paraboloid and an ellipsoidal cap (Sec. III-C-1)")
    ap.add_argument("--instances", type=int, default=256, help="batch: instances of the sweep")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of arrivals")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: HBM admission budget")
    ap.add_argument("--quantum-ms", type=float, default=20.0, help="serve: device time per scheduling quantum")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="step: seconds of the request stream timed after the steps for the latency figures (0: none)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="step: arrivals per second of that stream")
    ap.add_argument("--serve-seconds-low", type=float, default=20.0,
                    help="step: seconds of a second stream at a sustainable rate (0: none)")
    ap.add_argument("--serve-rate-low", type=float, default=20.0, help="step: arrivals per second of that stream")
    ap.add_argument("--no-batch", action="store_true", help="step: skip the 256-instance batch")
    return ap.parse_args()


def shard_workload(shard: int):
    full = workloads.broadband()
    if shard <= 1:
        return full, "all 128 frequencies"
    kidx = np.arange(0, full.n_k, shard)
    desc = f"frequency shard 1/{shard} ({len(kidx)} of 128, every {shard}th)"
    return full.subset(k_idx=kidx, name="broadband-shard"), desc


def run_step(p, w, precision):
    """One pass of the whole path on problem object `p`: mirror nodes, frequencies, incident and
    current tables, observation points, quadrature, reduction and time transform are all rebuilt
    from the workload's parameters (the object only keeps its device allocations between steps)."""
    p.set_mirror(w.f, w.a, w.n_r, w.n_phi)
    p.set_frequencies(w.k)
    p.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
    p.set_observation(w.obs)
    p.evaluate(precision, keep_on_device=True)
    p.to_time_at(w.dk, w.t, out=_time_out(w, precision))
    return p


_TIME_BUF = {}


def _time_out(w, precision):
    import torch
    key = (w.n_obs, len(w.t), precision)
    if key not in _TIME_BUF:
        dt = torch.complex128 if precision == "fp64" else torch.complex64
        _TIME_BUF[key] = (torch.empty((len(w.t), w.n_obs, 3), dtype=dt, device="cuda"),
                          torch.empty((len(w.t), w.n_obs, 3), dtype=dt, device="cuda"))
    return _TIME_BUF[key]


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s):
    import oracle
    oracle.build()
    threads = oracle.max_threads()
    # calibrate on a small sample (long enough that thread start-up does not dominate), then size
    # the sample to ~target_s of work; thread counts are passed explicitly (the setting persists)
    n_probe = max(threads, 16)
    probe = w.subset(obs_idx=np.linspace(0, w.n_obs - 1, n_probe).astype(int), k_idx=np.arange(min(4, w.n_k)))
    t0 = time.perf_counter()
    oracle.solve(probe, threads=threads)
    rate = probe.evals / (time.perf_counter() - t0)
    n_obs = int(max(threads, min(w.n_obs, target_s * rate / (w.n_k * w.n_nodes))))
    idx = np.linspace(0, w.n_obs - 1, n_obs).astype(int)
    sample = w.subset(obs_idx=idx)
    t0 = time.perf_counter()
    oracle.solve(sample, threads=threads)
    dt = time.perf_counter() - t0
    # one thread, for comparison with the paper's per-core rate (Sec. III-C-3): 2 points x 4 frequencies
    one = w.subset(obs_idx=np.linspace(0, w.n_obs - 1, 2).astype(int), k_idx=np.arange(min(4, w.n_k)))
    t0 = time.perf_counter()
    oracle.solve(one, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": sample.evals / dt, "unit": "integrand evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_obs} evenly spaced observation points x all {w.n_k} shard frequencies x "
                      f"{w.n_nodes} surface nodes (+ rim), FP64 with long-double phase, {dt:.1f} s",
            "cpu_model": _cpu_model(),
            "single_thread_value": one.evals / dt1,
            "single_thread_sample": f"2 observation points x {one.n_k} frequencies x {w.n_nodes} surface nodes, "
                                    f"one thread, {dt1:.1f} s"}


def batch_run(n_instances: int = 256, general: bool = False, tune: bool = True, tune_budget_ms: float = 20000.0,
              tie: bool = True):
    """All instances of the seeded sweep in ONE persistent launch (FP32 split, FP32-only tables),
    timed with the library's batch launch and, when `tune`, again after sc_autotune_batch has tuned
    the launch on every 16th instance.  Returns a dict of both runs."""
    import torch
    from paper_1609_08146_amd import Context, Problem
    ws = workloads.sweep(n_instances)
    ctx = Context(0)
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    probs = []
    for w in ws:
        p = Problem(ctx)
        p.set_table_storage(False)
        p.set_factoring(not general, tie_charge=tie)
        p.set_mirror(w.f, w.a, w.n_r, w.n_phi)
        p.set_frequencies(w.k)
        p.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
        p.set_observation(w.obs)
        probs.append(p)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    evals = sum(w.evals for w in ws)
    layouts = [p.layout_for("fp32_split") for p in probs]
    layout_evals = {lay: sum(w.evals for w, l in zip(ws, layouts) if l == lay) for lay in FLOPS}

    def partial_bytes():
        # split-K partials: 12 reals per (chunk, frequency, padded point), at the chunk each problem used
        return sum(4 * 12 * -(-(w.n_r + 1) * w.n_phi // p.timing()["chunk"]) * w.n_k * (-(-w.n_obs // 128) * 128)
                   for w, p in zip(ws, probs))

    def timed(label, launch):
        ctx.evaluate_batch(probs, "fp32_split")          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.evaluate_batch(probs, "fp32_split")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        quad_ms = probs[0].timing()["quad_ms"]
        fpl = launch["freq_per_lane"]
        flops = sum(flops_per_eval(lay, fpl) * n for lay, n in layout_evals.items())
        return {"label": label, "value": evals / dt, "seconds": dt, "quad_ms": quad_ms,
                "quad_evals_per_s": evals / (quad_ms * 1e-3), "launch": launch,
                "tflops": flops / (quad_ms * 1e-3) / 1e12,
                "frac_fp32_peak": flops / (quad_ms * 1e-3) / 1e12 / PEAK_FP32,
                "chunks_used": sorted({p.timing()["chunk"] for p in probs}),
                "partial_bytes": partial_bytes()}

    # the library's batch launch: the shape of the layout carrying most evaluations, each problem's chunk
    fact_major = 2 * (layout_evals["factored"] + layout_evals["tied"]) > evals
    lib = {"obs_per_lane": 1, "freq_per_lane": 4 if fact_major else 2, "waves_per_block": 4, "chunk": 0,
           "blocks_per_cu": 0}
    runs = [timed("library launch", lib)]
    if tune:
        t0 = time.perf_counter()
        best = ctx.autotune_batch(probs[::16], "fp32_split", budget_ms=tune_budget_ms)
        tune_s = time.perf_counter() - t0
        r = timed("tuned launch", best)
        r["tune_seconds"] = tune_s
        r["tuned_on"] = f"every 16th instance ({len(probs[::16])} of {len(probs)})"
        runs.append(r)
        ctx.set_batch_launch("fp32_split", reset=True)
    out = {"instances": len(ws), "evals": evals, "setup_s": setup,
           "instances_by_layout": {lay: layouts.count(lay) for lay in FLOPS}, "precision": "fp32_split",
           "tables": "general" if general else ("factored where the current allows, the charge tied where it is"
                                                if tie else "factored where the current allows"), "runs": runs}
    for p in probs:
        p.close()
    ctx.close()
    return out


def bench_batch(args):
    """--mode batch: the 256-instance sweep in one persistent launch, library and tuned launch."""
    out = batch_run(args.instances, args.general_tables, tie=not args.no_tie)
    best = max(out["runs"], key=lambda r: r["value"])
    print(json.dumps({"metric": "integrand evals/s, seeded sweep of uneven instances in one persistent launch",
                      "value": best["value"], "unit": "integrand evals/s", "n_gpus": 1, **out}), flush=True)


def bench_serve(args):
    """--mode serve: one JSON line for a serving run (see serve_run)."""
    print(json.dumps(serve_run(args.rate, args.duration, args.budget_gb, args.quantum_ms)), flush=True)


def serve_run(rate: float, duration: float, budget_gb: float = 200.0, quantum_ms: float = 20.0) -> dict:
    """Poisson stream of sweep-like requests through the serving loop; p50/p99 latency and throughput.

    One thread submits at the drawn arrival times, another collects results in submission order as
    they complete (as a client would), so finished requests do not pile up in host memory.  When the
    arrivals end, in-flight work gets a bounded drain and requests that never started are cancelled.
    Latency is the server's own submit-to-result-on-host time."""
    import threading
    import torch
    from paper_1609_08146_amd import Context, ScError, Server
    from paper_1609_08146_amd._abi import SC_E_TIMEOUT
    torch.cuda.init()
    times, draw = workloads.serving_arrivals(rate, duration)
    ctx = Context(0, use_torch_stream=False)
    srv = Server(ctx, hbm_budget=int(budget_gb * 1e9), max_running=64, quantum_ms=quantum_ms)
    tickets = []
    lock = threading.Lock()
    submitted_all = threading.Event()
    drain_deadline = []
    lat, evals_done = [], [0]
    start = time.perf_counter()

    def submitter():
        for i, ta in enumerate(times):
            now = time.perf_counter() - start
            if ta > now:
                time.sleep(ta - now)
            w = draw(i)
            try:
                tk = srv.submit(w, "fp32_split", t=w.t, dk=w.dk)
                with lock:
                    tickets.append(tk)
            except ScError:
                pass
        submitted_all.set()

    def collector():
        i = 0
        while True:
            with lock:
                tk = tickets[i] if i < len(tickets) else None
            if tk is None:
                if submitted_all.is_set():
                    with lock:
                        if i >= len(tickets):
                            return
                    continue
                time.sleep(0.002)
                continue
            while True:
                rem_ms = 250.0
                if drain_deadline:
                    rem_ms = min(rem_ms, (drain_deadline[0] - time.perf_counter()) * 1e3)
                    if rem_ms <= 0:
                        try:
                            srv.cancel(tk)      # never admitted: drop it; admitted ones finish in close()
                        except ScError:
                            pass
                        break
                try:
                    _, _, _, _, st = srv.wait(tk, timeout_ms=rem_ms)
                    lat.append(st["total_ms"])
                    evals_done[0] += st["evals"]
                    break
                except ScError as e:
                    if e.status != SC_E_TIMEOUT:
                        break
            i += 1

    th_s = threading.Thread(target=submitter)
    th_c = threading.Thread(target=collector)
    th_s.start()
    th_c.start()
    th_s.join()
    drain_deadline.append(time.perf_counter() + max(10.0, 0.25 * duration))
    th_c.join()
    elapsed = time.perf_counter() - start
    s = srv.stats()
    srv.close()
    ctx.close()
    lat = np.array(lat) if lat else np.array([np.nan])
    return {
        "metric": "serving: p50/p99 request latency and integrand evals/s",
        "rate_hz": rate, "duration_s": duration, "arrivals": len(times),
        "completed": int(s["completed"]), "cancelled": int(s["cancelled"]), "rejected": int(s["rejected"]),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "evals_per_s": s["evals_done"] / elapsed, "elapsed_s": elapsed, "launches": int(s["launches"]),
        "launched_evals_per_s": s["evals_launched"] / elapsed,
        "quanta_evals_per_device_s": s["evals_launched"] / max(s["quad_ms"] * 1e-3, 1e-9),
        "device_busy_frac": s["quad_ms"] * 1e-3 / elapsed,
        "prep_ms_per_request": s["prep_ms"] / max(1, int(s["admitted"])),
        "hbm_budget_gb": budget_gb, "quantum_ms": quantum_ms}


C_LIGHT = 299792458.0   # m/s


def _fwhm(cut: np.ndarray, i: int, dx: float):
    """Full width at half maximum of a sampled profile around its sample i (linear interpolation of
    the two half-maximum crossings); None if the profile does not fall to half within the samples."""
    half = 0.5 * cut[i]
    edges = []
    for step in (-1, 1):
        j = i
        while 0 <= j + step < len(cut) and cut[j + step] >= half:
            j += step
        if not 0 <= j + step < len(cut):
            return None
        a, b = cut[j], cut[j + step]
        edges.append((j + step * (a - half) / (a - b)) * dx)
    return float(edges[1] - edges[0])


def focal_spot(Et: np.ndarray, Bt: np.ndarray, n: int, half_width: float):
    """Peak electric intensity I_E = (1/2) c E^2 of Sec. IV-B and the shape of the focal spot.

    Et, Bt: time samples [n_t][n_points][3] of the analytic field on an n x n focal-plane grid over
    +-half_width (x fastest; the physical field is 2 Re).  The field is in Lorentz-Heaviside units
    (sqrt(J/m^3), lengths in m), so c E^2 / 2 is W/m^2.  At the time sample and point of the largest
    intensity: the intensity, the FWHM of the intensity along x and y through that point, the
    eccentricity sqrt(1 - (minor/major)^2) of those widths; and the largest longitudinal components
    relative to the largest E_x over all samples (max |E_z| / max |E_x|, max |B_z| / max |E_x|)."""
    E = 2.0 * np.real(Et[:, : n * n])
    B = 2.0 * np.real(Bt[:, : n * n])
    inten = 0.5 * C_LIGHT * np.sum(E * E, axis=-1)
    ti, oi = np.unravel_index(int(np.argmax(inten)), inten.shape)
    grid = inten[ti].reshape(n, n)          # [y][x]
    iy, ix = divmod(int(oi), n)
    dx = 2.0 * half_width / (n - 1)
    fx, fy = _fwhm(grid[iy, :], ix, dx), _fwhm(grid[:, ix], iy, dx)
    ecc = None
    if fx and fy:
        lo, hi = min(fx, fy), max(fx, fy)
        ecc = float(np.sqrt(1.0 - (lo / hi) ** 2))
    return {"peak_intensity_W_cm2": float(inten[ti, oi]) * 1e-4, "time_index": int(ti),
            "peak_x_m": (ix - (n - 1) / 2) * dx, "peak_y_m": (iy - (n - 1) / 2) * dx,
            "fwhm_x_m": fx, "fwhm_y_m": fy, "eccentricity": ecc,
            "max_Ez_over_max_Ex": float(np.max(np.abs(E[..., 2])) / np.max(np.abs(E[..., 0]))),
            "max_Bz_over_max_Ex": float(np.max(np.abs(B[..., 2])) / np.max(np.abs(E[..., 0])))}


def bench_table1(args):
    """The Table I workload end to end with the diagnostics of Sec. IV-A: energy-normalised
    super-Gaussian spectrum (100 samples, 150 J), 400 x 400 nodes, focal plane + axis, time
    transform; then Maxwell residuals on 13-point stencils around a focal-region grid and the
    field energy of a focal volume.  Reports rates and per-phase times."""
    import torch
    from paper_1609_08146_amd import Context, problem_from_workload, stencil_points
    torch.cuda.init()
    w = workloads.table1()
    lam = workloads.TABLE1["lam_c"]
    ctx = Context(0)
    ctx.set_profiling(True)
    prec = args.precision
    out = {"metric": "Table I workload: whole-path evaluations/s and diagnostics", "precision": prec,
           "n_freq": w.n_k, "n_nodes": w.n_nodes}
    for rep in range(2):                       # the first pass warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = problem_from_workload(ctx, w)
        p.normalize_energy(w.meta["eps"], w.meta["e_tot"], w.dk)
        p.evaluate(prec, keep_on_device=True)
        Et, Bt = _time_out(w, prec)
        p.to_time_at(w.dk, w.t, out=(Et, Bt))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tm = p.timing()
        if rep == 1:
            # the 256-sample window resolves the envelope, not the carrier: for the instantaneous
            # intensity, sample +-4 periods about the focal arrival 2f every lambda_c / 32
            t_fine = 2 * w.f + np.arange(-128, 129) * (lam / 32)
            Ef, Bf = p.to_time_at(w.dk, t_fine)
        p.close()
    out["path"] = {"evals": w.evals, "seconds": dt, "evals_per_s": w.evals / dt,
                   "phases_ms": {k: tm[k] for k in ("prep_ms", "quad_ms", "reduce_ms", "time_ms")}}
    # peak electric intensity and focal-spot ellipticity at the time of the largest intensity (Sec. IV-B)
    out["focal_spot"] = focal_spot(Ef, Bf, 64, 2.0 * lam)
    out["focal_spot"]["time_offset_m"] = float(t_fine[out["focal_spot"]["time_index"]] - 2 * w.f)
    # Maxwell residuals (Fig. 5 methodology): 8 x 8 x 8 points over +-2 lambda_c, h = lambda_c / 20
    g = np.linspace(-2 * lam, 2 * lam, 8)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    h = lam / 20
    st = stencil_points(pts, h)
    wd = workloads.Workload(name="table1-stencil", f=w.f, a=w.a, n_r=w.n_r, n_phi=w.n_phi, k=w.k,
                            spectrum=w.spectrum, obs=st, w0=w.w0, t=w.t, dk=w.dk, meta=w.meta)
    p = problem_from_workload(ctx, wd)
    p.normalize_energy(w.meta["eps"], w.meta["e_tot"], w.dk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.evaluate(prec, keep_on_device=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ef = p.maxwell_residual_freq(len(pts), h)
    t2 = time.perf_counter()
    tt = 2 * w.f + np.linspace(-10, 10, 9) * lam
    et = p.maxwell_residual_time(len(pts), h, tt, lam / 20, w.dk)
    t3 = time.perf_counter()
    out["maxwell"] = {"points": len(pts), "stencil_evals": wd.evals, "evaluate_s": t1 - t0,
                      "residual_freq_ms": (t2 - t1) * 1e3, "residual_time_ms": (t3 - t2) * 1e3,
                      "mean_e_f": float(ef.mean()), "mean_e_t": float(et.mean())}
    p.close()
    # field energy of a focal volume of 24 lambda_c per side at the focal arrival t = 2f, cells of
    # (lambda_c / 3)^3 (Sec. IV-A: it should hold the 150 J that the normalisation put on the mirror)
    g = np.arange(-36, 37) * (lam / 3)
    vol = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    wv = workloads.Workload(name="table1-volume", f=w.f, a=w.a, n_r=w.n_r, n_phi=w.n_phi, k=w.k,
                            spectrum=w.spectrum, obs=vol, w0=w.w0, t=w.t, dk=w.dk, meta=w.meta)
    p = problem_from_workload(ctx, wv)
    p.normalize_energy(w.meta["eps"], w.meta["e_tot"], w.dk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.evaluate(prec, keep_on_device=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    W = p.field_energy(np.array([2 * w.f]), w.dk, float(lam / 3) ** 3)
    t2 = time.perf_counter()
    out["energy"] = {"points": len(vol), "evals": wv.evals, "evaluate_s": t1 - t0, "energy_ms": (t2 - t1) * 1e3,
                     "W_focus_J": float(W[0]), "E_tot_J": w.meta["e_tot"]}
    p.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_convergence(args):
    """The convergence study of Sec. IV-A with the GPU path: the radially polarised beam on the
    Table I mirror at the central wavelength, focal-region points, N x N nodes for growing N; per
    component, e_rel = max |F_ref - F_N| / max |F_ref| against the finest mesh (FP64 form), with the
    paper's average cell area <A>_N = dtheta dr^2 (N+1)^2 / (2N) as the mesh measure."""
    import torch
    from paper_1609_08146_amd import Context, Problem
    torch.cuda.init()
    T = workloads.TABLE1
    lam = T["lam_c"]
    k = np.array([2 * np.pi / lam])
    g = np.linspace(-lam, lam, 16)
    plane = workloads.focal_plane(lam, 16)
    obs = np.concatenate([plane, np.stack([0 * g, 0 * g, 2 * g], axis=-1)])
    ctx = Context(0)

    def field(n):
        p = Problem(ctx)
        p.set_mirror(T["f"], T["r_max"], n, n)
        p.set_frequencies(k)
        p.set_incident_beam("radial", T["w0"], 0.0, None, True)
        p.set_observation(obs)
        E, B = p.evaluate("fp64")
        p.close()
        return np.concatenate([E[0], B[0]], axis=-1)       # [n_obs][6]

    ns = [8, 12, 16, 20, 25, 30, 40, 50, 100, 200, 400]
    ref = field(1200)
    names = ["E_x", "E_y", "E_z", "B_x", "B_y", "B_z"]
    rows = []
    for n in ns:
        F = field(n)
        dr, dth = T["r_max"] / n, 2 * np.pi / n
        cell = np.sqrt(dth * dr * dr * (n + 1) ** 2 / (2 * n))
        peak = np.max(np.abs(ref), axis=0)
        err = np.max(np.abs(F - ref), axis=0)
        # a component that vanishes by symmetry (B_z of the radial beam) has no relative error
        live = peak > 1e-9 * peak.max()
        rows.append({"n": n, "cell_over_lambda": cell / lam,
                     "e_rel": {c: (float(err[i] / peak[i]) if live[i] else None) for i, c in enumerate(names)}})
    ctx.close()
    print(json.dumps({"metric": "convergence of the FP64 field under refinement (Sec. IV-A)",
                      "beam": "radially polarised, curl-consistent", "reference_n": 1200, "rows": rows}),
          flush=True)


def bench_refine(args):
    """Mesh refinement on a non-parabolic mirror (Sec. III-C-1): the paraboloid of focal length f
    and the ellipsoidal cap of the same aperture whose vertex curvature matches it
    (workloads.ellipsoid_cap), lit by the same literal Gaussian, wavelength 1, N x N nodes for
    growing N.  Per surface and form, e_rel = max |F_N - F_ref| / max |F_ref| over the focal-plane
    and axial points and the six components, against the FP64 field at the finest N.  The folded
    tables of the paraboloid are smooth (k(|r_s| - z) = 2kf); the cap's turn through some fifty
    periods, which the radial rule must resolve."""
    import torch
    from paper_1609_08146_amd import Context, Problem
    torch.cuda.init()
    f, c, rm, w0 = 200.0, 600.0, 300.0, 150.0
    k = np.array([2 * np.pi])
    g = np.linspace(-2.0, 2.0, 16)
    obs = np.concatenate([workloads.focal_plane(2.0, 16), np.stack([0 * g, 0 * g, g], axis=-1)])
    ctx = Context(0)

    def field(surface, n, prec):
        p = Problem(ctx)
        if surface == "paraboloid":
            p.set_mirror(f, rm, n, n)
        else:
            p.set_surface(*workloads.ellipsoid_cap(f, c, rm, n, n))
        p.set_frequencies(k)
        p.set_incident_beam("linear", w0, 0.0, None, False)
        p.set_observation(obs)
        E, B = p.evaluate(prec)
        p.close()
        return np.concatenate([E[0], B[0]], axis=-1).astype(np.complex128)

    ns = [8, 12, 16, 24, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 512]
    rows = {}
    for surface in ("paraboloid", "ellipsoid"):
        ref = field(surface, 1024, "fp64")
        peak = np.abs(ref).max()
        rows[surface] = [{"n": n, **{prec: float(np.abs(field(surface, n, prec) - ref).max() / peak)
                                     for prec in ("fp64", "fp32_split")}} for n in ns]
    first = {s: next((r["n"] for r in rows[s] if r["fp64"] < 1e-6), None) for s in rows}
    xyz = workloads.ellipsoid_cap(f, c, rm, 512, 4)[0]
    ph = 2 * np.pi * (np.linalg.norm(xyz, axis=1) - xyz[:, 2])
    ctx.close()
    print(json.dumps({"metric": "e_rel under mesh refinement, paraboloid vs ellipsoidal cap (Sec. III-C-1)",
                      "geometry": {"f": f, "c": c, "r_max": rm, "w0": w0, "wavelength": 1.0,
                                   "ellipsoid_table_phase_span_rad": float(ph.max() - ph.min())},
                      "reference_n": 1024, "rows": rows, "first_n_below_1e-6_fp64": first}), flush=True)


def bench_valu(args):
    """Issue cost of the vector instructions of the quadrature kernel: a separate microbenchmark
    (not part of the library), compiled here on demand for gfx950 and run once."""
    import subprocess
    import tempfile
    from paper_1609_08146_amd import build as b
    src = os.path.join(ROOT, "paper_1609_08146_amd", "csrc", "valu_rates.hip")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "valu_rates")
        res = subprocess.run([b.hipcc(), *b.HIP_FLAGS, src, "-o", exe], capture_output=True, text=True)
        if res.returncode != 0:
            raise SystemExit(f"hipcc failed on valu_rates.hip: {res.stderr}")
        res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if res.returncode != 0:
        raise SystemExit(f"valu_rates failed ({res.returncode}): {res.stderr}")
    out = json.loads(res.stdout)
    out["metric"] = "gfx950 vector instruction issue cost"
    print(json.dumps(out), flush=True)


def bench_copy(args):
    """A plain device copy of known size (calibrates the HBM byte counters)."""
    import torch
    n = 1 << 28   # 2^28 floats = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                      "copies": 3}), flush=True)


def main():
    args = parse()
    if args.mode == "copy":
        return bench_copy(args)
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "table1":
        return bench_table1(args)
    if args.mode == "valu":
        return bench_valu(args)
    if args.mode == "convergence":
        return bench_convergence(args)
    if args.mode == "refine":
        return bench_refine(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the frequency-sharded multi-GPU "
                                   "design is described but not built, so --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1609_08146_amd import Context, Problem

    torch.cuda.init()
    w, shard_desc = shard_workload(args.shard)
    ctx = Context(0)
    ctx.set_profiling(True)

    p = Problem(ctx)
    p.set_factoring(not args.general_tables, tie_charge=not args.no_tie)
    for _ in range(args.warmup):
        run_step(p, w, args.precision)
    torch.cuda.synchronize()

    quad_ms, step_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        run_step(p, w, args.precision)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        tm = p.timing()
        quad_ms.append(tm["quad_ms"])
        last_timing = tm
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress(f"{args.steps} timed steps, {elapsed * 1e3 / args.steps:.2f} ms per step")
    layout = p.layout_for(args.precision)
    factored = layout != "general"
    launch = p.launch(args.precision)
    # the same step with its results handed back in host memory: spectral E, B and the time
    # samples copied to (pageable) numpy arrays through the C ABI's host-output path
    host_ms = []
    for _ in range(5):
        ts = time.perf_counter()
        p.set_mirror(w.f, w.a, w.n_r, w.n_phi)
        p.set_frequencies(w.k)
        p.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
        p.set_observation(w.obs)
        p.evaluate(args.precision)
        p.to_time_at(w.dk, w.t)
        host_ms.append((time.perf_counter() - ts) * 1e3)
    p.close()

    evals = w.evals
    ms_per_step = elapsed * 1e3 / args.steps
    value = evals * args.steps / elapsed
    quad_avg = float(np.mean(quad_ms))
    fpe = flops_per_eval(layout, launch["freq_per_lane"], args.precision == "fp64")
    achieved = fpe * evals / (quad_avg * 1e-3) / 1e12
    peak = PEAK_FP64 if args.precision == "fp64" else PEAK_FP32
    # the counters were taken on the full FP32-split workload with the default launch
    traffic = measured_traffic() if (args.precision == "fp32_split" and args.shard == 1) else None
    out = {
        "metric": "integrand evals/s (obs x freq x node), whole step, one GPU",
        "value": value,
        "unit": "integrand evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (seeded parameters; Gaussian beam generated on the device)",
        "config": {
            "workload": f"broadband pulse, 800 nm carrier, 10 fs FWHM, f=0.1 m, aperture radius 0.075 m, "
                        f"w0=0.05 m, 400x400 GL x trapezoid nodes, 64x64 focal plane +-4 lambda0 + 64 axial, "
                        f"256 time samples; {shard_desc}",
            "precision": args.precision, "launch": (f"obs_per_lane={launch['obs_per_lane']}, freq_per_lane={launch['freq_per_lane']}, "
                                                 f"{launch['waves_per_block']} waves/block, chunk {launch['chunk']}"),
            "current": {"tied": "factored with the tied charge (Jt = u s, rho_t = -i beta s / k: n x B keeps "
                                 "one real direction per node and n.E carries its amplitude)",
                        "factored": "factored (Jt = u s: the current n x B keeps one real direction per node)",
                        "general": "general tables"}[layout],
            "n_obs": w.n_obs, "n_freq": w.n_k, "n_nodes": w.n_nodes, "n_time": len(w.t),
            "evals_per_step": evals,
        },
        "roofline": {
            "bound": "alu",
            "kernel": ("k_quad (split-form surface quadrature" + (" in FP64" if args.precision == "fp64" else "")
                       + {"tied": ", factored current, tied charge)", "factored": ", factored current)",
                          "general": ")"}[layout]),
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "flops_per_eval": fpe,
            "quad_ms_avg": quad_avg,
            "quad_launches": len(quad_ms),
        },
        "phases_ms": {k: last_timing[k] for k in ("prep_ms", "quad_ms", "reduce_ms", "time_ms")},
        # one step is one complete solve of the workload (set-up to time samples on the device);
        # the latency of requests of mixed sizes under load is `python bench.py --mode serve`
        "solve_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                             "max": float(np.max(step_ms))},
        # not `value`: the step above keeps its results in HBM
        "pcie_inclusive": {"value": w.evals / (float(np.median(host_ms)) * 1e-3), "unit": "integrand evals/s",
                           "ms_per_step": float(np.median(host_ms)), "steps": len(host_ms),
                           "note": "the same step with E, B and the time samples returned in host memory"},
    }

    if not args.no_fp64_form and args.precision != "fp64":
        # the plain FP64 form on the same workload, for the speed ratio
        w64 = w
        p = Problem(ctx)
        p.set_mirror(w64.f, w64.a, w64.n_r, w64.n_phi)
        p.set_frequencies(w64.k)
        p.set_incident_gaussian(w64.w0, 0.0, w64.spectrum, False)
        p.set_observation(w64.obs)
        p.evaluate("fp64", keep_on_device=True)
        torch.cuda.synchronize()
        q64 = p.timing()["quad_ms"]
        layout64 = p.layout_for("fp64")
        fact64 = layout64 != "general"
        fpl64 = p.launch("fp64")["freq_per_lane"]
        # error of every output component of the chosen form against the FP64 form (itself held to the
        # oracle at 1e-12 by the tests) over the whole grid: max |F_c - F_c,64| / max |F_c,64| (the
        # paper's e_rel, Sec. IV-A) and the same maximum over the peak |F| of the field
        E64, B64 = p.result()
        E32, B32 = p.evaluate(args.precision)
        p.close()
        per_comp = {}
        for lab, F, F64 in (("E", E32, E64), ("B", B32, B64)):
            peak = float(np.max(np.linalg.norm(F64, axis=-1)))
            for c, ax in enumerate("xyz"):
                err = float(np.max(np.abs(F[..., c] - F64[..., c])))
                per_comp[f"{lab}_{ax}"] = {"e_rel": err / float(np.max(np.abs(F64[..., c]))),
                                           "max_err_over_field_peak": err / peak}
        progress(f"FP64 form {q64:.1f} ms")
        r64 = w64.evals / (q64 * 1e-3)
        rq = evals / (quad_avg * 1e-3)
        fpg64 = flops_per_eval("general", fpl64, True)
        f64 = flops_per_eval(layout64, fpl64, True)
        out["forms"] = {
            "fp64": {"quad_evals_per_s": r64, "quad_ms": q64, "n_freq": w64.n_k,
                     "current": layout64, "flops_per_eval": f64,
                     "tflops": f64 * r64 / 1e12, "frac_fp64_peak": f64 * r64 / 1e12 / PEAK_FP64},
            args.precision: {"quad_evals_per_s": rq, "per_component_vs_fp64": per_comp},
            "speedup_vs_fp64": rq / r64,
        }
        if layout == "tied":
            # the factored current without the tied charge (a beam with a longitudinal E, such as the
            # curl-consistent radial one, takes this layout): its quadrature on the same workload
            qu = []
            p = Problem(ctx)
            p.set_factoring(True, tie_charge=False)
            for _ in range(4):
                run_step(p, w, args.precision)
                torch.cuda.synchronize()
                qu.append(p.timing()["quad_ms"])
            fpu = flops_per_eval("factored", p.launch(args.precision)["freq_per_lane"])
            p.close()
            ru = evals / (min(qu[1:]) * 1e-3)
            out["forms"]["fp32_split_factored_untied"] = {
                "quad_evals_per_s": ru, "quad_ms": min(qu[1:]), "flops_per_eval": fpu, "tflops": fpu * ru / 1e12,
                "frac_fp32_peak": fpu * ru / 1e12 / PEAK_FP32}
        if layout64 == "tied":
            # the FP64 form on the factored current without the tied charge
            p = Problem(ctx)
            p.set_factoring(True, tie_charge=False)
            p.set_mirror(w64.f, w64.a, w64.n_r, w64.n_phi)
            p.set_frequencies(w64.k)
            p.set_incident_gaussian(w64.w0, 0.0, w64.spectrum, False)
            p.set_observation(w64.obs)
            p.evaluate("fp64", keep_on_device=True)
            torch.cuda.synchronize()
            qu64 = p.timing()["quad_ms"]
            fpu64 = flops_per_eval("factored", p.launch("fp64")["freq_per_lane"], True)
            p.close()
            ru64 = w64.evals / (qu64 * 1e-3)
            out["forms"]["fp64_factored_untied"] = {
                "quad_evals_per_s": ru64, "quad_ms": qu64, "flops_per_eval": fpu64, "tflops": fpu64 * ru64 / 1e12,
                "frac_fp64_peak": fpu64 * ru64 / 1e12 / PEAK_FP64}
        if factored:
            # the same split form on the general tables (what an arbitrary incident field costs): the
            # whole step, timed like the headline over a few steps, and its quadrature
            qg, sg = [], []
            p = Problem(ctx)
            p.set_factoring(False)
            run_step(p, w, args.precision)
            torch.cuda.synchronize()
            for _ in range(4):
                ts = time.perf_counter()
                run_step(p, w, args.precision)
                torch.cuda.synchronize()
                sg.append(time.perf_counter() - ts)
                qg.append(p.timing()["quad_ms"])
            fpg = flops_per_eval("general", p.launch(args.precision)["freq_per_lane"])
            p.close()
            rg = evals / (min(qg) * 1e-3)
            out["value_general_tables"] = evals / float(np.mean(sg))
            out["forms"]["fp32_split_general_tables"] = {
                "step_evals_per_s": evals / float(np.mean(sg)), "ms_per_step": 1e3 * float(np.mean(sg)),
                "quad_evals_per_s": rg, "quad_ms": min(qg), "flops_per_eval": fpg, "tflops": fpg * rg / 1e12,
                "frac_fp32_peak": fpg * rg / 1e12 / PEAK_FP32}
        if fact64:
            # the FP64 form on the general tables
            p = Problem(ctx)
            p.set_factoring(False)
            p.set_mirror(w64.f, w64.a, w64.n_r, w64.n_phi)
            p.set_frequencies(w64.k)
            p.set_incident_gaussian(w64.w0, 0.0, w64.spectrum, False)
            p.set_observation(w64.obs)
            p.evaluate("fp64", keep_on_device=True)
            torch.cuda.synchronize()
            qg64 = p.timing()["quad_ms"]
            p.close()
            rg64 = w64.evals / (qg64 * 1e-3)
            out["forms"]["fp64_general_tables"] = {
                "quad_evals_per_s": rg64, "quad_ms": qg64, "tflops": fpg64 * rg64 / 1e12,
                "frac_fp64_peak": fpg64 * rg64 / 1e12 / PEAK_FP64}

    ctx.close()
    if args.serve_seconds > 0 and args.shard == 1:
        # the request stream as specified (200 per second for 60 s: an overload) and one sustainable rate
        out["serving"] = []
        # the sustainable rate first, and both before the batch: for about half a minute after a run
        # that freed a large part of the device memory (the overload stream's 200 GB, the batch's
        # 80 GB), a new server's request preparation runs slower
        for rate, secs in ((args.serve_rate_low, args.serve_seconds_low), (args.serve_rate, args.serve_seconds)):
            if secs <= 0:
                continue
            sv = serve_run(rate, secs)
            progress(f"serving at {rate:g}/s: p50 {sv['p50_ms']:.0f} ms, p99 {sv['p99_ms']:.0f} ms")
            row = {k: sv[k] for k in ("rate_hz", "duration_s", "arrivals", "completed", "cancelled", "rejected",
                                      "p50_ms", "p99_ms", "evals_per_s", "device_busy_frac",
                                      "quanta_evals_per_device_s", "prep_ms_per_request")}
            row["workload"] = ("seeded Poisson stream of sweep-like requests (mean 3.6e10 evaluations), FP32-split "
                               "with time transform, 200 GB admission budget")
            out["serving"].append(row)

    if not args.no_batch and args.shard == 1:
        # the 256-instance sweep in one persistent launch, library and tuned batch launch
        b = batch_run(256, tune=True, tune_budget_ms=20000.0)
        progress(f"batch of {b['instances']} instances done")
        out["batch"] = {"workload": "seeded sweep of 256 uneven instances (f 2-20 cm, 1-256 frequencies, "
                                    "100^2-600^2 nodes, 16^2-128^2 + 16-128 axial points) in one persistent launch, "
                                    "FP32-split, FP32-only tables",
                        "instances": b["instances"], "evals": b["evals"], "setup_s": b["setup_s"],
                        "runs": [{k: r[k] for k in ("label", "quad_evals_per_s", "quad_ms", "seconds", "launch",
                                                      "frac_fp32_peak", "partial_bytes", "tune_seconds", "tuned_on")
                                  if k in r} for r in b["runs"]]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
