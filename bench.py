"""Benchmark of the Stratton-Chu mirror-focusing hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--shard S] [--precision fp32_split]

One step is one pass of the whole path over the broadband workload (800 nm,
10 fs Gaussian spectrum, f = 0.1 m, aperture radius 0.075 m, w0 = 0.05 m,
400 x 400 mirror nodes, 64 x 64 focal-plane points over +-4 lambda0 plus 64
axial points): mirror node tables, incident / current tables for every
frequency, the surface quadrature for every (point, frequency), the split-K
reduction, and the transform to 256 time samples.  By default the step covers
one GPU's share of the 128-frequency spectrum under frequency sharding over
8 GPUs (16 frequencies, every 8th sample); ``--shard 1`` runs all 128.

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

# Algorithmic FP32 work per evaluation of the split form (FMA = 2 flops; the
# four transcendental instructions rsq, rcp, sin, cos are not counted):
#   geometry R, |R|^2, 1/R, R, r_s.r', delta, phase      22
#   g = e^{ik delta}/R, h = (ik - 1/R) g / R              10
#   E += Jt g                                             24
#   E += rho_t h R                                        18
#   B += (Jt h) x R                                       42
FLOPS_PER_EVAL = 114
PEAK_FP32_NONPACKED = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6 TFLOP/s: 256 CU x 4 SIMD16 x FMA x 2.4 GHz
PEAK_FP32_PACKED = 157.3                                 # published, needs packed FP32 (not used here)
PEAK_FP64 = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shard", type=int, default=8, help="frequency shards (1 = the full 128-frequency spectrum)")
    ap.add_argument("--precision", default="fp32_split", choices=["fp32_split", "fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    return ap.parse_args()


def shard_workload(shard: int):
    full = workloads.broadband()
    if shard <= 1:
        return full, "all 128 frequencies"
    kidx = np.arange(0, full.n_k, shard)
    return full.subset(k_idx=kidx, name="broadband-shard"), f"frequency shard 1/{shard} ({len(kidx)} of 128, every {shard}th)"


def run_step(ctx, w, precision):
    """One pass of the whole path; returns the problem (kept alive for timing)."""
    from paper_1609_08146_amd import Problem
    p = Problem(ctx)
    p.set_mirror(w.f, w.a, w.n_r, w.n_phi)
    p.set_frequencies(w.k)
    p.set_incident_gaussian(w.w0, w.pol, w.spectrum, False)
    p.set_observation(w.obs)
    p.evaluate(precision, keep_on_device=True)
    p.to_time(w.dk, w.t, out=_time_out(w, precision))
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


def cpu_baseline(w, target_s):
    import oracle
    oracle.build()
    threads = oracle.max_threads()
    # calibrate on a tiny sample, then size the sample to ~target_s of work
    probe = w.subset(obs_idx=np.arange(0, w.n_obs, w.n_obs // 8)[:8], k_idx=[0])
    t0 = time.perf_counter()
    oracle.solve(probe)
    rate = probe.evals / (time.perf_counter() - t0)
    n_obs = int(max(8, min(w.n_obs, target_s * rate / (w.n_k * w.n_nodes))))
    idx = np.linspace(0, w.n_obs - 1, n_obs).astype(int)
    sample = w.subset(obs_idx=idx)
    t0 = time.perf_counter()
    oracle.solve(sample)
    dt = time.perf_counter() - t0
    return {"value": sample.evals / dt, "unit": "integrand evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_obs} evenly spaced observation points x all {w.n_k} shard frequencies x "
                      f"{w.n_nodes} surface nodes (+ rim), FP64 with long-double phase, {dt:.1f} s"}


def main():
    args = parse()
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

    for _ in range(args.warmup):
        run_step(ctx, w, args.precision).close()
    torch.cuda.synchronize()

    quad_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        p = run_step(ctx, w, args.precision)
        torch.cuda.synchronize()
        tm = p.timing()
        quad_ms.append(tm["quad_ms"])
        last_timing = tm
        p.close()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    evals = w.evals
    ms_per_step = elapsed * 1e3 / args.steps
    value = evals * args.steps / elapsed
    quad_avg = float(np.mean(quad_ms))
    achieved = FLOPS_PER_EVAL * evals / (quad_avg * 1e-3) / 1e12
    peak = PEAK_FP64 if args.precision == "fp64" else PEAK_FP32_NONPACKED
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
            "precision": args.precision,
            "n_obs": w.n_obs, "n_freq": w.n_k, "n_nodes": w.n_nodes, "n_time": len(w.t),
            "evals_per_step": evals,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_quad (split-form surface quadrature)",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "flops_per_eval": FLOPS_PER_EVAL,
            "quad_ms_avg": quad_avg,
            "peak_note": "FP32 vector peak without packed FP32 (the build disables packed-FP32 instruction "
                         "selection); the published 157.3 TFLOP/s needs packed FP32",
            "frac_of_packed_peak": achieved / PEAK_FP32_PACKED if args.precision != "fp64" else None,
        },
        "phases_ms": {k: last_timing[k] for k in ("prep_ms", "quad_ms", "reduce_ms", "time_ms")},
    }

    if not args.no_fp64_form and args.precision != "fp64":
        # the plain FP64 form on two frequencies of the same shard, for the speed ratio
        w64 = w.subset(k_idx=[0, w.n_k // 2])
        p = Problem(ctx)
        p.set_mirror(w64.f, w64.a, w64.n_r, w64.n_phi)
        p.set_frequencies(w64.k)
        p.set_incident_gaussian(w64.w0, 0.0, w64.spectrum, False)
        p.set_observation(w64.obs)
        p.evaluate("fp64", keep_on_device=True)
        torch.cuda.synchronize()
        q64 = p.timing()["quad_ms"]
        p.close()
        r64 = w64.evals / (q64 * 1e-3)
        rq = evals / (quad_avg * 1e-3)
        out["forms"] = {
            "fp64": {"quad_evals_per_s": r64, "quad_ms": q64, "n_freq": w64.n_k,
                     "tflops": FLOPS_PER_EVAL * r64 / 1e12, "frac_fp64_peak": FLOPS_PER_EVAL * r64 / 1e12 / PEAK_FP64},
            args.precision: {"quad_evals_per_s": rq},
            "speedup_vs_fp64": rq / r64,
        }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)

    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
