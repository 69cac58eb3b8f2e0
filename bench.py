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
import re
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "samples/s at d=10, 32 channels (FP32 vs FP64 mode, equal rel. error); p99 job latency"
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6

# Hardware counters of one k_sample launch (FP32-mixed, d=10 / K=32 / n=100,
# 1e8 calls) from rocprofv3 --pmc runs of this script
# (profiles/k_sample_fp32_d10_K32_n100_counters.md): FETCH_SIZE and WRITE_SIZE
# (KiB per dispatch), each scaled by what the same counter reads for a plain
# device copy of known size; SQ_INSTS_VALU_FLOPS_FP32 (FP32 operations per
# wavefront instruction, FMA = 2, summed over the launch's wavefront
# instructions: x64 lanes gives the operations executed); SQ_ACTIVE_INST_VALU
# and SQ_INSTS_VALU per CU-cycle (CUs x GPU-active cycles per XCD).  Valid only for
# the kernel sources the counters were taken on (SHA-256 of their code
# without comments and whitespace: the kernel template and launch shape, its
# FP32 instantiation and the device headers it includes); otherwise null.
KERNEL_SOURCES = ["sample_kernel.h", "single_f32.hip", "mcv_point.h", "mcv_device.h"]
# Taken on d=10 / 32 channels / 100 bins, FP32 mode, 1e8 calls per launch
# (profiles/k_sample_fp32_d10_K32_n100_counters.md).
COUNTERS = {"sha256": "37043441b91977b1a4c0a79955d01bd417ffe0ddaa39c2d8095b69af0af32e25",
            "fetch_kib": 136896.0, "write_kib": 882510.0,
            "fetch_factor": 524307.9375 / 1048576.0, "write_factor": 1048576.0 / 1048576.0,
            "valu_flops_fp32_waves": 2.36732e9, "valu_active": 1.105,
            "valu_insts_per_cu_cycle": 1.080, "kernel_ms": 4.996}


def kernel_sources_digest() -> str:
    """SHA-256 of the kernel sources with comments and whitespace removed."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1811_09711_amd", "csrc", f)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update("".join(text.split()).encode())
    return h.hexdigest()


def counters_valid() -> bool:
    return COUNTERS["sha256"] is not None and kernel_sources_digest() == COUNTERS["sha256"]


def kernel_traffic_bytes():
    if not counters_valid():
        return None
    kib = COUNTERS["fetch_kib"] / COUNTERS["fetch_factor"] + \
        COUNTERS["write_kib"] / COUNTERS["write_factor"]
    return kib * 1024.0


def _same_shape(p, c, i) -> bool:
    """Channel c maps with exactly the shape of peak i (their density kernels
    are one and the same function of p)."""
    import numpy as np
    if not np.array_equal(p.chan_kind[c], p.peak_kind[i]):
        return False
    m = p.chan_kind[c] != 0
    return bool(np.array_equal(p.chan_loc[c][m], p.peak_loc[i][m]) and
                np.array_equal(p.chan_width[c][m], p.peak_width[i][m]))


def flops_per_call(p) -> dict:
    """Algorithmic arithmetic of one call of the method (Sec. 3.5: the VEGAS
    step map of the call's channel, every channel's density and grid density
    in eq. g(p), the integrand, w = f/g), with a fused multiply-add counted
    as 2, every other add, subtract, multiply or divide as 1, and no
    comparisons (bin searches and skip tests are not arithmetic of the
    method).  Transcendental calls (erfcinv, tan, exp, reciprocal) are
    counted apart.  A channel and a peak with the same shape share one
    density kernel (the same function of p), which is counted once.
      - the call's own map, per axis: bin width and x (3), the own grid
        density product (1), then 6 (Gaussian: t, 2t, sqrt(2) z, mu + sigma
        z) or 4 (Breit-Wigner: theta, m + h tan) plus one erfcinv / tan;
        averaged over the channels in proportion to their weights alpha =
        1/K;
      - every channel's density kernel: 4 per Gaussian axis (z' = ga p + gb,
        accumulate z'^2), 4 per Breit-Wigner axis ((p - m)^2 + h^2 and the
        product), 1 normalisation, plus one exp2 (any Gaussian axis) and one
        reciprocal (any Breit-Wigner axis);
      - every other channel's grid density: 1 product per axis;
      - every term alpha_c G_c q_c of g: 3 products and 1 add;
      - every peak of f: 2 (weight times kernel, add) when it shares a
        channel's kernel, else its own kernel as above plus 2;
      - w = f/g: 1.
    The accumulation (w^2, the sums of w and w^2, one per-bin sum per axis)
    is FP64: 3 + d operations, reported apart."""
    import numpy as np
    d, K, P = p.dim, p.n_channels, p.n_peaks
    GAUSS, BW = 1, 2

    def kernel(kinds):
        ng, nb = int(np.count_nonzero(kinds == GAUSS)), int(np.count_nonzero(kinds == BW))
        return 4 * ng + 4 * nb + 1, (1 if ng else 0) + (1 if nb else 0)

    own = trans_own = 0.0
    for c in range(K):
        kinds = p.chan_kind[c]
        ng, nb = int(np.count_nonzero(kinds == GAUSS)), int(np.count_nonzero(kinds == BW))
        own += 4 * d + 6 * ng + 4 * nb
        trans_own += ng + nb
    own /= K
    trans_own /= K
    dens = trans = 0
    for c in range(K):
        f_, t_ = kernel(p.chan_kind[c])
        dens += f_
        trans += t_
    peaks = 0
    for i in range(P):
        if any(_same_shape(p, c, i) for c in range(K)):
            peaks += 2
        else:
            f_, t_ = kernel(p.peak_kind[i])
            peaks += f_ + 2
            trans += t_
    grid = (K - 1) * d
    gsum = 4 * K
    fp32 = own + dens + grid + gsum + peaks + 1
    return {"fp32": float(fp32), "transcendental": float(trans + trans_own),
            "fp64": float(3 + d)}


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
    edges, alpha, _ = integ.get_state()
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
    return p, out, (edges, alpha)


def run_options(n_points: int, steps: int, warmup: int, n_events: int):
    """The optional parts of the method on the d=10, 32-channel workload in
    FP32 mode (the headline pass's precision): MRG32k3a streams in place of
    Philox words, pseudo-stratified passes (2 or more calls per box), a
    channel-equivalence list in the grid adaptation (every channel pooled
    with itself: the cost of the pooling, not a physics symmetry), and
    unweighting after adaptation (plain and with signs).  Passes: samples/s
    of whole iterations and the sample kernel's time; unweighting: events/s
    and trials/s."""
    import numpy as np
    import torch

    import workloads
    from paper_1811_09711_amd import mcv
    base = workloads.config3(precision=1)
    what = mcv.MCV_REFINE_GRID | mcv.MCV_REFINE_ALPHA
    out = {}

    def timed_run(name, p, setup=None):
        integ = mcv.Integrator(p, max_iterations=steps + warmup + 4)
        if setup:
            setup(integ)
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
        hist = integ.history[warmup:]
        res = integ.result(warmup)
        out[name] = {
            "samples_per_s": float(hist[:, 2].sum()) / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / steps,
            "sample_kernel_ms": float(np.mean([integ.pass_timing(warmup + s)[0]
                                               for s in range(steps)])),
            "integral": res["integral"], "rel_error": res["error"] / abs(res["integral"]),
            "chi2_ndf": res["chi2_ndf"]}
        print(json.dumps({"option": name, "samples_per_s": out[name]["samples_per_s"]}),
              file=sys.stderr, flush=True)
        return integ

    integ = timed_run("philox", base)
    integ.unweight(1000, batch=262_144)  # first calls set up their buffers
    integ.unweight_signed(1000, batch=262_144)
    for signed in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = integ.unweight_signed(n_events, batch=262_144)[2] if signed else \
            integ.unweight(n_events, batch=262_144)[1]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["unweighting_signed" if signed else "unweighting"] = {
            "events": n_events, "events_per_s": n_events / dt, "trials_per_s": st["trials"] / dt,
            "efficiency": st["efficiency"], "batch": 262_144}
    integ.close()
    timed_run("mrg32k3a", base.with_(rng=mcv.MCV_RNG_MRG32K3A)).close()
    timed_run("stratified_s2", base.with_(strat=2)).close()
    d = base.dim
    eq = [[c, c] + list(range(d)) + [mcv.MCV_EQ_IDENTITY] * d for c in range(base.n_channels)]
    timed_run("equivalences", base, lambda i: i.set_equivalences(eq)).close()
    return out


def run_config(problem, n_points: int, iterations: int):
    """A whole adaptation run of a smaller configuration (C1: d=2, K=2, 5 x
    1e4; C2: d=6, K=8, 10 x 1e6), FP64: samples per second of wall time over
    all iterations (pass, reduction, rebinning, channel weights), and of the
    sample kernel alone."""
    import numpy as np
    import torch

    from paper_1811_09711_amd import mcv
    integ = mcv.Integrator(problem, max_iterations=iterations + 2)
    what = mcv.MCV_REFINE_GRID | mcv.MCV_REFINE_ALPHA
    integ.sample_iteration(n_points)  # warm-up (first launches)
    integ.refine(what)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iterations):
        integ.sample_iteration(n_points)
        integ.refine(what)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hist = integ.history[1:]
    calls = float(hist[:, 2].sum())
    kms = [integ.pass_timing(1 + s)[0] for s in range(iterations)]
    res = integ.result(1)
    integ.close()
    return {"workload": problem.name, "precision": "fp64", "iterations": iterations,
            "calls_per_iteration": n_points, "samples_per_s": calls / wall,
            "ms_per_iteration": 1e3 * wall / iterations,
            "sample_kernel_samples_per_s": calls / (sum(kms) * 1e-3),
            "integral": res["integral"], "error": res["error"]}


def run_batch(precision: int, n_jobs: int, iterations: int, tune_cache: str,
              unbatched: bool = True):
    """The batched workload: n_jobs independent jobs (d ~ U{2..12}, K ~ U{1..64},
    N log-uniform in [1e4, 1e7], n = 50, job j seeded 4,000,000 + j), each
    `iterations` adaptation iterations, all advancing together: one graph
    replay per iteration.  Also the same jobs one at a time through the
    single-job integrator, for comparison."""
    import numpy as np
    import torch

    import workloads
    from paper_1811_09711_amd import mcv

    ps = [p.with_(precision=precision) for p in workloads.config4(n_jobs)]
    npts = [p.n_points for p in ps]
    t0 = time.perf_counter()
    tuning, tune_ms = mcv.autotune(ps, npts, cache_path=tune_cache)
    tune_s = time.perf_counter() - t0
    what = mcv.MCV_REFINE_GRID | mcv.MCV_REFINE_ALPHA
    b = mcv.Batch(ps, npts, tuning=tuning, max_iterations=iterations + 2)
    info = b.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iterations):
        b.iterate(what, graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iter_ms = [b.timing(i)[0] for i in range(iterations)]
    calls = 0.0
    for j in range(n_jobs):
        calls += float(b.history(j)[:, 2].sum())
    flops = sum(flops_per_call(p)["fp32"] * n for p, n in zip(ps, npts))
    b.close()
    # sample-kernel time from direct launches of a fresh batch (same first pass)
    e = mcv.Batch(ps, npts, tuning=tuning, max_iterations=4)
    e.iterate(what, graph=False)
    e.iterate(what, graph=False)
    sample_ms = [e.timing(i)[1] for i in range(2)]
    e.close()
    out = {
        "jobs": n_jobs,
        "iterations": iterations,
        "precision": "fp32-mixed" if precision else "fp64",
        "calls_per_iteration": float(sum(npts)),
        "samples_per_s": calls / (sum(iter_ms) * 1e-3),
        "samples_per_s_wall": calls / wall,
        "ms_per_iteration": float(np.mean(iter_ms)),
        "first_iteration_ms": iter_ms[0],
        "sample_kernel_ms": float(np.mean(sample_ms)),
        "tflops_sample_kernel": flops / (np.mean(sample_ms) * 1e-3) / 1e12,
        "tuning": tuning,
        "tuning_ms": tune_ms,
        "tuning_wall_s": tune_s,
        "units": info["units"],
        "workgroups": info["workgroups"],
        "lds_bytes": info["lds_bytes"],
    }
    if unbatched:
        # the same jobs one after another, each on its own single-job launches
        integs = [mcv.Integrator(p, max_iterations=iterations + 2) for p in ps]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(iterations):
            for g, n in zip(integs, npts):
                g.sample_iteration(n)
                g.refine(what)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        for g in integs:
            g.close()
        out["unbatched_samples_per_s"] = calls / dt
        out["batching_speedup"] = out["samples_per_s_wall"] / out["unbatched_samples_per_s"]
    return out


def run_serving(precision: int, rate: float, warm_s: float, measure_s: float, n_events: int,
                batch: int, tuning, budget: int, drain_s: float, max_active: int,
                tune_cache: str, unit_calls: int = 0):
    """Open-loop serving: Poisson arrivals at `rate` per second for warm_s +
    measure_s seconds, request q = job 5,000,000 + q of the batched workload
    with 8 iterations and n_events unweighted events; latency = completion
    minus scheduled arrival, over the requests that arrive in the measured
    window."""
    import numpy as np

    import workloads
    from paper_1811_09711_amd import mcv

    arrivals = workloads.config5_arrivals(duration_s=warm_s + measure_s, rate=rate)
    if tuning is None:  # the batched workload's tuning (a cache hit when tuned before)
        ps = [p.with_(precision=precision) for p in workloads.config4(256)]
        tuning, _ = mcv.autotune(ps, [p.n_points for p in ps], cache_path=tune_cache)
    if unit_calls > 0:  # shorter steps: latency, not pass time, is what serving minimises
        tuning = dict(tuning, unit_calls=max(unit_calls, int(tuning["block"])))
    srv = mcv.Server(precision=precision, unweight_batch=batch, tuning=tuning,
                     hbm_budget=budget, max_active=max_active)
    t0 = srv.clock()
    q = 0
    tick2q, lat, work, trials = {}, {}, {}, {}
    steps, max_active_seen, max_queued, peak_bytes = 0, 0, 0, 0
    active = queued = 0
    deadline = warm_s + measure_s + drain_s
    last_progress = time.perf_counter()
    while True:
        now = srv.clock() - t0
        while q < len(arrivals) and arrivals[q] <= now:
            p = workloads.config5_job(q).with_(precision=precision)
            tick2q[srv.submit(p, p.n_points, 8, n_events)] = q
            q += 1
            queued += 1
        if active == 0 and queued == 0:
            if q >= len(arrivals):
                break
            time.sleep(max(0.0, min(arrivals[q] - now, 0.002)))
            continue
        info = srv.step()
        steps += 1
        active, queued = info["n_active"], info["n_queued"]
        max_active_seen = max(max_active_seen, active)
        max_queued = max(max_queued, queued)
        peak_bytes = max(peak_bytes, info["bytes_in_use"])
        for t in srv.finished():
            r = srv.report(t)
            k = tick2q[t]
            lat[k] = r["finish_time"] - t0 - arrivals[k]
            work[k] = r["result"]["n_points"] + r["trials"]
            trials[k] = r["trials"]
        if time.perf_counter() - last_progress > 10.0:
            print(json.dumps({"serving_progress_s": round(now, 1), "submitted": q,
                              "finished": len(lat), "active": active, "queued": queued}),
                  file=sys.stderr, flush=True)
            last_progress = time.perf_counter()
        if now > deadline:
            break
    wall = srv.clock() - t0
    srv.close()
    measured = [k for k in range(len(arrivals)) if warm_s <= arrivals[k] < warm_s + measure_s]
    done = [k for k in measured if k in lat]
    L = np.array([lat[k] for k in done]) * 1e3
    total_work = float(sum(work.values()))
    return {
        "precision": "fp32-mixed" if precision else "fp64",
        "rate_per_s": rate,
        "window_s": [warm_s, warm_s + measure_s],
        "requests_measured": len(measured),
        "completed": len(done),
        "incomplete": len(measured) - len(done),
        "p50_ms": float(np.percentile(L, 50)) if len(L) else None,
        "p99_ms": float(np.percentile(L, 99)) if len(L) else None,
        "mean_ms": float(L.mean()) if len(L) else None,
        "samples_per_s": total_work / wall,
        "integration_calls": float(sum(work.values()) - sum(trials.values())),
        "unweight_trials": float(sum(trials.values())),
        "wall_s": wall,
        "samples_note": "integration calls + unweighting trials of every finished request",
        "steps": steps,
        "max_active_seen": max_active_seen,
        "max_queued": max_queued,
        "peak_device_bytes": peak_bytes,
        "unweight_batch": batch,
        "events_per_request": n_events,
        "max_active": max_active,
        "tuning": tuning,
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(precision: int, seconds: float = 10.0, state=None):
    """The FP64 CPU oracle (never tuned for this) on a bounded sample of the
    same workload, in its threaded timing mode on every core of the host, and
    on one core.  state: the grids and channel weights the GPU's last timed
    pass used, so that both time the same per-call work; else fresh grids."""
    import oracle
    import workloads
    p = workloads.config3(precision=precision)
    threads = os.cpu_count() or 1

    def timed(n, th):
        o = oracle.Oracle(p)
        if state is not None:
            o.edges, o.alpha = state
        t0 = time.perf_counter()
        o.sample_iteration(n, th)
        return time.perf_counter() - t0

    probe = 2000 * threads
    rate = probe / timed(probe, threads)
    n = max(probe, int(rate * seconds))
    dt = timed(n, threads)
    n1 = max(2000, int(2000 / timed(2000, 1) * min(seconds, 5.0)))
    dt1 = timed(n1, 1)
    return {"value": n / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "one_core_value": n1 / dt1, "cpu_model": _cpu_model(), "nproc": threads,
            "sample": f"one pass of {n} calls of the same workload "
                      f"({'the GPU run adapted grids and weights' if state is not None else 'fresh grids, alpha = 1/K'}), "
                      f"{'FP32' if precision else 'FP64'} rules, {dt:.1f} s wall on {threads} threads; "
                      f"{n1} calls on 1 thread in {dt1:.1f} s"}


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
    ap.add_argument("--batch-jobs", type=int, default=256)
    ap.add_argument("--batch-iterations", type=int, default=10)
    ap.add_argument("--batch-precision", choices=["both", "fp64", "fp32"], default="both")
    ap.add_argument("--no-small", action="store_true", help="skip the C1 / C2 FP64 legs")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-unbatched", action="store_true",
                    help="skip the one-job-at-a-time comparison of the batched workload")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-options", action="store_true",
                    help="skip the MRG32k3a, stratified, equivalence and unweighting legs")
    ap.add_argument("--option-events", type=int, default=2_000_000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-drain", type=float, default=60.0)
    ap.add_argument("--serve-events", type=int, default=100_000)
    ap.add_argument("--serve-batch", type=int, default=262_144)
    ap.add_argument("--serve-precision", choices=["fp64", "fp32"], default="fp32")
    ap.add_argument("--serve-max-active", type=int, default=512,
                    help="requests admitted at once (the rest wait in arrival order)")
    ap.add_argument("--serve-budget", type=int, default=0,
                    help="device bytes for admitted requests (0: 90%% of free memory)")
    ap.add_argument("--serve-unit-calls", type=int, default=1024,
                    help="calls per work unit of the serving steps (0: the batch tuning's; "
                         "1024 gave p50 11.7 / p99 79 ms against 15.2 / 85 at the tuned 2048)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1811_09711_amd",
                                                         "tuning_cache.json"))
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
    states = {}
    for prec in modes:
        problem, results[prec], states[prec] = run_mode(prec, n_points, args.steps, args.warmup)
        print(json.dumps({"mode": results[prec]["precision"],
                          "samples_per_s": results[prec]["samples_per_s"],
                          "sample_kernel_ms": results[prec]["sample_kernel_ms"]}),
              file=sys.stderr, flush=True)
    head = results.get(1) or results.get(0)
    head_prec = 1 if 1 in results else 0
    fpc = flops_per_call(problem)
    kernel_s = head["sample_kernel_ms"] * 1e-3
    achieved = fpc["fp32"] * head["calls_per_step"] / kernel_s / 1e12
    peak = PEAK_FP32_TFLOPS if head_prec else PEAK_FP64_TFLOPS
    counted = None
    if head_prec and counters_valid():
        executed = 64.0 * COUNTERS["valu_flops_fp32_waves"]  # FP32 operations per launch
        counted = {"fp32_flops_per_call_executed": executed / head["calls_per_step"],
                   "achieved_executed": executed / kernel_s / 1e12,
                   "frac_executed": executed / kernel_s / 1e12 / peak,
                   "valu_active_per_cu_cycle": COUNTERS["valu_active"],
                   "valu_insts_per_cu_cycle": COUNTERS["valu_insts_per_cu_cycle"],
                   "profiled_kernel_ms": COUNTERS["kernel_ms"]}
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
            "traffic": kernel_traffic_bytes() if head_prec else None,
            "traffic_unit": "bytes per launch (HBM, counter-scaled)",
            "kernel": "k_sample",
            "flops_per_call": fpc["fp32"],
            "transcendentals_per_call": fpc["transcendental"],
            "fp64_ops_per_call": fpc["fp64"],
            "counters": counted,
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
    if not args.no_batch:
        precs = {"both": [0, 1], "fp64": [0], "fp32": [1]}[args.batch_precision]
        line["batch"] = {}
        for bp in precs:
            r = run_batch(bp, args.batch_jobs, args.batch_iterations, args.tune_cache,
                          unbatched=(bp == precs[0] and not args.no_unbatched))
            line["batch"][r["precision"]] = r
            print(json.dumps({"batch": {k: r[k] for k in
                                        ("precision", "samples_per_s", "ms_per_iteration",
                                         "tuning")}}), file=sys.stderr, flush=True)
    line["p99_job_latency_ms"] = None
    if not args.no_serve:
        sp = 1 if args.serve_precision == "fp32" else 0
        tuning = line.get("batch", {}).get("fp32-mixed" if sp else "fp64", {}).get("tuning")
        line["serving"] = run_serving(sp, args.serve_rate, args.serve_warmup, args.serve_seconds,
                                      args.serve_events, args.serve_batch, tuning,
                                      args.serve_budget, args.serve_drain,
                                      args.serve_max_active, args.tune_cache,
                                      args.serve_unit_calls)
        line["p99_job_latency_ms"] = line["serving"]["p99_ms"]
        print(json.dumps({"serving": {k: line["serving"][k] for k in
                                      ("p50_ms", "p99_ms", "completed", "incomplete",
                                       "samples_per_s")}}), file=sys.stderr, flush=True)
    if not args.no_small:
        import workloads
        line["other_configs"] = {}
        for pr, n, it in ((workloads.config1(), 10_000, 5), (workloads.config2(), 1_000_000, 10)):
            r = run_config(pr, n, it)
            line["other_configs"][pr.name] = r
            print(json.dumps({"config": pr.name, "samples_per_s": r["samples_per_s"]}),
                  file=sys.stderr, flush=True)
    if not args.no_options:
        line["options"] = run_options(n_points, 5, 2, args.option_events)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(head_prec, args.cpu_seconds, states.get(head_prec))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
