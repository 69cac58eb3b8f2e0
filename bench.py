"""Benchmark of the multi-channel VEGAS sample pass on one MI355X.

Workload: d = 10, K = 32 channels, 100 bins per axis, 1e8 calls per iteration
(24 isotropic Gaussian peaks with sigma log-uniform in [0.01, 0.1] and 8
Breit-Wigner ridges of width 1e-3 on a random pair of axes; one channel per
peak; problem seed 3).  A step is one adaptation iteration: allocation, the
sample pass, its reduction, grid rebinning and the channel-weight update.
Both precision modes run with the same seed and number of calls, so their
statistical errors are equal; the headline value is the FP32-mixed mode.

Prints one JSON line (see the design notes for every field).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "samples/s at d=10, 32 channels (FP32 vs FP64 mode, equal rel. error); p99 job latency"
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def flops_per_call(p) -> float:
    """Algorithmic floating-point operations of one call of the method, with
    every channel term of the multi-channel density evaluated (eq. g(p)).
    Cost model: add, sub, mul, div, compare = 1; fused multiply-add = 2;
    exp, tan, erfcinv = 1.
      - each 1-d density factor (Gauss or BW) of a channel or a peak: 4;
        per channel / peak: exp argument, exp, normalisation, division = 4;
        each peak adds 1 for the mixture sum;
      - each other channel: per axis a binary search of ceil(log2 n)
        compares plus 1 density product, then 3 for g += alpha G q;
      - the call's own forward map per axis: 6 for x and 1 - x, 7 for a
        Gauss or BW map, 1 for the grid density; averaged over channels;
      - the weight f/g and its accumulation: 1 + 10 + d.
    """
    import numpy as np
    d, K, P, n = p.dim, p.n_channels, p.n_peaks, p.n_bins
    steps = max(1, math.ceil(math.log2(n)))
    q = sum(4 * int(np.count_nonzero(p.chan_kind[c])) + 4 for c in range(K))
    f = sum(4 * int(np.count_nonzero(p.peak_kind[i])) + 5 for i in range(P))
    lookups = (K - 1) * (d * (steps + 1) + 3)
    own = sum(6 * d + 7 * int(np.count_nonzero(p.chan_kind[c])) + d for c in range(K)) / K
    return float(q + f + lookups + own + 11 + d)


def run_mode(precision: int, n_points: int, steps: int, warmup: int):
    import numpy as np
    import torch

    import workloads
    from paper_1811_09711_amd import mcv

    p = workloads.config3(precision=precision)
    integ = mcv.Integrator(p, max_iterations=steps + warmup + 4)
    what = mcv.MCV_REFINE_GRID | mcv.MCV_REFINE_ALPHA
    for _ in range(warmup):
        integ.sample_iteration(n_points)
        integ.refine(what)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        integ.sample_iteration(n_points)
        integ.refine(what)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = integ.history
    timed = hist[warmup:]
    calls = float(timed[:, 2].sum())
    kernel_ms = [integ.pass_timing(warmup + s)[0] for s in range(steps)]
    groups = integ.pass_timing(warmup)[1]
    res = integ.result(warmup)
    out = {
        "precision": "fp32-mixed" if precision else "fp64",
        "samples_per_s": calls / (t1 - t0),
        "ms_per_step": 1e3 * (t1 - t0) / steps,
        "calls_per_step": calls / steps,
        "sample_kernel_ms": float(np.mean(kernel_ms)),
        "sample_kernel_ms_min": float(np.min(kernel_ms)),
        "workgroups": groups,
        "integral": res["integral"],
        "error": res["error"],
        "rel_error": res["error"] / abs(res["integral"]),
        "chi2_ndf": res["chi2_ndf"],
        "n_bad": res["n_bad"],
        "per_step_E": [float(x) for x in timed[:, 0]],
        "per_step_sigma": [float(x) for x in timed[:, 1]],
    }
    integ.close()
    return p, out


def cpu_baseline(precision: int, seconds: float = 10.0):
    """The FP64 CPU oracle on a bounded sample of the same workload, in its
    threaded timing mode on the host's cores."""
    import oracle
    import workloads
    p = workloads.config3(precision=precision)
    threads = min(16, os.cpu_count() or 1)
    o = oracle.Oracle(p)
    probe = 2000 * threads
    t0 = time.perf_counter()
    o.sample_iteration(probe, threads)
    rate = probe / (time.perf_counter() - t0)
    n = max(probe, int(rate * seconds))
    o2 = oracle.Oracle(p)
    t0 = time.perf_counter()
    o2.sample_iteration(n, threads)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"one pass of {n} calls of the same workload (fresh grids, alpha = 1/K), "
                      f"{'FP32' if precision else 'FP64'} rules, {dt:.1f} s wall on "
                      f"{threads} threads of {platform.processor() or platform.machine()}"}


def copy_calibration(nbytes: int):
    """A plain device copy of known size (for HBM counter scaling)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--points", type=float, default=1e8)
    ap.add_argument("--mode", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a plain device copy of this many bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "see the design notes for how the pass would shard.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    n_points = int(args.points)
    modes = {"both": [1, 0], "fp32": [1], "fp64": [0]}[args.mode]
    results = {}
    problem = None
    for prec in modes:
        problem, results[prec] = run_mode(prec, n_points, args.steps, args.warmup)
        print(json.dumps({"mode": results[prec]["precision"],
                          "samples_per_s": results[prec]["samples_per_s"],
                          "sample_kernel_ms": results[prec]["sample_kernel_ms"]}),
              file=sys.stderr, flush=True)
    head = results.get(1) or results.get(0)
    head_prec = 1 if 1 in results else 0
    fpc = flops_per_call(problem)
    achieved = fpc * head["calls_per_step"] / (head["sample_kernel_ms"] * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if head_prec else PEAK_FP64_TFLOPS
    line = {
        "metric": METRIC,
        "value": head["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head_prec else "f64",
        "data": "synthetic",
        "config": {
            "workload": "d=10, K=32 channels (24 Gaussian + 8 Breit-Wigner peaks, channel per "
                        "peak), 100 bins/axis, 1e8 calls/iteration, seed 3",
            "precision": head["precision"],
            "accumulate": "f64 compensated",
            "calls_per_step": head["calls_per_step"],
            "step": "allocate + sample pass + reduce + rebin grids + update alpha",
        },
        "modes": {results[k]["precision"]: {kk: v for kk, v in results[k].items()
                                            if kk not in ("per_step_E", "per_step_sigma")}
                  for k in results},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "kernel": "k_sample",
            "flops_per_call": fpc,
        },
    }
    if 0 in results and 1 in results:
        i32, i64 = results[1]["integral"], results[0]["integral"]
        line["fp32_vs_fp64"] = {
            "rel_diff": abs(i32 - i64) / abs(i64),
            "rel_error_fp32": results[1]["rel_error"],
            "rel_error_fp64": results[0]["rel_error"],
            "speedup": results[1]["samples_per_s"] / results[0]["samples_per_s"],
        }
    line["p99_job_latency_ms"] = None
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(head_prec, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
