"""Benchmark of the fused adaptive-relaxation LBM step on one MI355X.

Default run (one JSON line on stdout, progress on stderr):

* main line: 2D Euler, 2048 x 2048 four-quadrant Riemann data (seed 0),
  transmissive, CFL 0.5, FP32 storage and arithmetic: W warm-up steps, then
  K timed steps (default K = 1000, the configuration's run length);
  ``value`` = lattice updates per second (GLUPS) with the state resident in
  HBM; ``roofline`` = algorithmic bytes of the fused step / average kernel
  time from HIP events on the launch stream, against 8 TB/s;
* beside it: the FP64 plain path on the same inputs (and its FP32-vs-FP64
  error), 2D shallow water 4096 x 4096 with the bed source (FP32), 1D Euler
  N=4096 solve latency, the serving mix (continuous batching, p50/p99
  latency), the same arrivals solved one at a time on the plain path (FP64
  and FP32), and the FP64 CPU oracle timed on a bounded sample.

``--only NAME`` runs one workload (for profilers); ``--copy-calibration``
times a plain device copy of known size (HBM counter calibration).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2609_18177_amd import arlbm as A  # noqa: E402
from paper_2609_18177_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "GLUPS + HBM GB/s, FP32 batched vs FP64 plain; p50/p99 solve latency"
# algorithmic bytes per lattice update: one read + one write of Q*m values
# (+ the bed plane read for shallow water with a bed)
ALG_BYTES = {("euler2d", 4): 160, ("euler2d", 8): 320, ("swe2d", 4): 124, ("swe2d", 8): 248,
             ("euler1d", 4): 72, ("euler1d", 8): 144, ("adv1d", 4): 24, ("adv1d", 8): 48,
             ("euler3d", 4): 280, ("euler3d", 8): 560}
KERNEL_SOURCES = ["paper_2609_18177_amd/csrc/step.hpp", "paper_2609_18177_amd/csrc/physics.hpp",
                  "paper_2609_18177_amd/csrc/step3d.hpp",
                  "paper_2609_18177_amd/csrc/kernels.hip", "paper_2609_18177_amd/build.py"]


def alg_bytes_per_lup(p, size):
    """One read and one write of the Q*m populations (Q = 2d+1; m = 1 for
    advection, d+2 for Euler, d+1 for shallow water, d+3 for reactive Euler),
    plus the bed plane's read when the problem has a bed."""
    q = 2 * p.dim + 1
    m = {W.ADVECTION: 1, W.EULER: p.dim + 2, W.SWE: p.dim + 1, W.REACTIVE: p.dim + 3}[p.system]
    return 2 * q * m * size + (size if p.bed is not None else 0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(workload):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), or
    None when the summary is missing or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


class Timer:
    """HIP events recorded on the stream the library launches on (torch's
    current stream, handed to the library at creation)."""

    def __init__(self, torch):
        self.torch = torch
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.e0.record(self.torch.cuda.current_stream())
        return self

    def __exit__(self, *exc):
        self.e1.record(self.torch.cuda.current_stream())
        self.e1.synchronize()
        self.torch.cuda.synchronize()
        self.ms = self.e0.elapsed_time(self.e1)


def time_steps(torch, problem, precision, steps, warmup):
    cfg = A.config_from(problem, precision=precision)
    L = A.Lattice(cfg, owner="torch")
    L.set_state(problem.U0, problem.bed)
    L.step(warmup)
    L.sync(check=False)
    with Timer(torch) as tm:
        L.step(steps)
    st = L.sync(check=False)
    return L, tm.ms, st


def run_main(torch, args):
    p = W.euler_seeded_2d(0, n=2048, steps=1000)
    log(f"[main] 2D Euler 2048^2 FP32: warmup {args.warmup}, timed {args.steps}")
    L32, ms32, st32 = time_steps(torch, p, A.F32, args.steps, args.warmup)
    U32 = L32.moments()
    L32.close()
    res = {"ms": ms32, "steps": args.steps, "cells": p.cells, "flags": st32["flags"], "t": st32["t"]}
    if args.only:
        return res, p
    log(f"[main] FP64 plain path, same inputs and step count")
    L64, ms64, st64 = time_steps(torch, p, A.F64, args.steps, args.warmup)
    U64 = L64.moments()
    L64.close()
    res["fp64"] = {"ms": ms64, "flags": st64["flags"], "t": st64["t"]}
    res["fp32_vs_fp64_rel_l1"] = float(np.sum(np.abs(U32 - U64)) / np.sum(np.abs(U64)))
    res["fp32_vs_fp64_rel_l1_per_field"] = [float(np.sum(np.abs(U32[c] - U64[c])) / np.sum(np.abs(U64[c])))
                                            for c in range(U64.shape[0])]
    return res, p


def run_swe(torch, args, steps=None):
    p = W.swe_bed_2d(0, n=4096, steps=2000)
    steps = steps or args.swe_steps
    log(f"[swe] 2D shallow water 4096^2 with bed, FP32: warmup {args.warmup}, timed {steps}")
    L, ms, st = time_steps(torch, p, A.F32, steps, args.warmup)
    sums = L.conservation()
    L.close()
    m0 = math.fsum(p.U0[0].ravel().tolist())
    return {"ms": ms, "steps": steps, "cells": p.cells, "flags": st["flags"],
            "mass_drift_rel": float(sums[0] / m0 - 1.0)}


def run_euler3d(torch, args, steps=None):
    """3D Euler (D3Q7), seeded octant data on 256^3 cells, FP32: the
    three-pass step (indicator, relaxation, collide-and-pull with the moments
    of the new state)."""
    p = W.euler_octants_3d(seed=0, n=256, steps=100)
    steps = steps or args.steps3d
    log(f"[euler3d] 256^3 FP32: warmup {args.warmup}, timed {steps}")
    L, ms, st = time_steps(torch, p, A.F32, steps, args.warmup)
    L.close()
    ms_step = ms / steps
    return {"glups": p.cells / (ms_step * 1e-3) / 1e9, "ms_per_step": ms_step, "cells": p.cells,
            "alg_gbs": ALG_BYTES[("euler3d", 4)] * p.cells / (ms_step * 1e-3) / 1e9,
            "alg_frac": ALG_BYTES[("euler3d", 4)] * p.cells / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "flags": st["flags"]}


def run_latency_1d(torch, args):
    """Solve latency of the 1D Euler configuration: set_state (H2D) ->
    2000 steps -> read_moments (D2H), FP32 and FP64."""
    p = W.euler_seeded_1d(0, n=4096, steps=2000)
    out = {}
    for prec, name in ((A.F32, "fp32"), (A.F64, "fp64")):
        cfg = A.config_from(p, precision=prec)
        L = A.Lattice(cfg, owner="torch")
        lat = []
        for i in range(args.latency_solves + 2):
            t0 = time.perf_counter()
            L.set_state(p.U0)
            L.step(p.steps)
            U = L.moments()
            dt = time.perf_counter() - t0
            if i >= 2:
                lat.append(dt)
        L.close()
        lat = np.array(lat) * 1e3
        out[name] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                     "glups": p.cells * p.steps / (np.median(lat) * 1e-3) / 1e9}
    log(f"[latency] 1D Euler N=4096, 2000 steps: {out}")
    return out


def run_latency_advection(torch, args):
    """Solve latency of the advection configuration (N=256, sin 2 pi x,
    periodic, CFL 0.5, 512 steps to t=1), FP64 as configured: set_state ->
    steps -> read_moments; with the relative L2 error against the exact
    solution (the initial profile after one period)."""
    p = W.advection_sine(n=256, steps=512)
    L = A.Lattice(A.config_from(p, precision=A.F64), owner="torch")
    lat = []
    U = None
    for i in range(args.latency_solves + 2):
        t0 = time.perf_counter()
        L.set_state(p.U0)
        L.step(p.steps)
        U = L.moments()
        dt = time.perf_counter() - t0
        if i >= 2:
            lat.append(dt)
    st = L.sync(check=False)
    L.close()
    lat = np.array(lat) * 1e3
    err = float(np.linalg.norm(U.ravel() - p.U0.ravel()) / np.linalg.norm(p.U0.ravel()))
    out = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)), "t": st["t"],
           "rel_l2_vs_exact": err}
    log(f"[latency] advection N=256, 512 steps, FP64: {out}")
    return out


def run_serving(torch, args, n_requests, rate_hz, fp64_check, tag="serving", budget_gib=None):
    """Continuous batching: Poisson arrivals admitted by HBM budget into the
    batched FP32 kernel; latency = result read back - arrival."""
    budget_gib = args.budget_gib if budget_gib is None else budget_gib
    reqs = W.serving_requests(n_requests, rate_hz=rate_hz, seed=0)
    log(f"[{tag}] generating {len(reqs)} requests")
    t0 = time.perf_counter()
    probs = [r.problem() for r in reqs]
    log(f"[{tag}] generated in {time.perf_counter() - t0:.1f}s; budget {budget_gib} GiB")
    srv = A.Server(int(budget_gib * 2 ** 30), A.F32)
    cfgs = [A.config_from(p, precision=A.F32) for p in probs]
    results = {}
    nxt = 0
    peak_mem = 0
    iters = 0
    busy = 0.0
    start = time.perf_counter()
    while len(results) < len(reqs):
        now = time.perf_counter() - start
        while nxt < len(reqs) and reqs[nxt].arrival_s <= now:
            p = probs[nxt]
            reqs[nxt].server_id = srv.submit(cfgs[nxt], p.U0, p.bed, reqs[nxt].steps)
            nxt += 1
        ti = time.perf_counter()
        resident, queued = srv.iterate(args.launches_per_iterate)
        if resident:
            busy += time.perf_counter() - ti
        iters += 1
        peak_mem = max(peak_mem, srv.memory())
        for c in srv.poll(256):
            results[c["id"]] = c
        if resident == 0 and queued == 0 and nxt < len(reqs):
            time.sleep(max(0.0, min(0.001, reqs[nxt].arrival_s - (time.perf_counter() - start))))
    wall = time.perf_counter() - start
    torch.cuda.synchronize()
    lat = []
    lups = 0
    by_id = {r.server_id: r for r in reqs}
    bad = 0
    nbytes = 0
    for rid, c in results.items():
        r = by_id[rid]
        if c["status"] != 0:
            bad += 1
            continue
        # latency from the request's Poisson arrival time: perf_counter and the
        # library's steady clock both read CLOCK_MONOTONIC
        lat.append(c["done_s"] - (start + r.arrival_s))
        lups += probs[r.rid].cells * r.steps
        nbytes += probs[r.rid].cells * r.steps * alg_bytes_per_lup(probs[r.rid], 4)
    lat = np.array(lat) * 1e3
    span = max(reqs[-1].arrival_s, 1e-9)
    out = {"requests": len(reqs), "failed": bad, "wall_s": wall, "glups": lups / wall / 1e9,
           "alg_gbs_whole_job": nbytes / wall / 1e9,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "iterations": iters, "peak_resident_bytes": int(peak_mem), "offered_lups": int(lups),
           "offered_glups_over_arrivals": lups / span / 1e9, "arrival_span_s": span,
           "iterate_time_fraction_with_work": busy / wall, "rate_hz": rate_hz, "budget_gib": budget_gib,
           "launches_per_iterate": args.launches_per_iterate}
    # FP32 (batched) against the FP64 plain path on a subsample of requests
    errs = []
    for r in reqs[:fp64_check]:
        p = probs[r.rid]
        L = A.Lattice(A.config_from(p, precision=A.F64), owner="torch")
        L.set_state(p.U0, p.bed)
        L.step(r.steps)
        U64 = L.moments()
        L.close()
        U32 = results[r.server_id]["U"].reshape(U64.shape)
        errs.append(float(np.sum(np.abs(U32 - U64)) / np.sum(np.abs(U64))))
    out["fp32_batched_vs_fp64_plain_rel_l1"] = {"n": len(errs), "max": max(errs) if errs else None,
                                                "median": float(np.median(errs)) if errs else None}
    srv.close()
    log(f"[{tag}] {out}")
    return out


def run_plain(torch, args, n_requests, rate_hz, precision, tag):
    """The same arrival stream as run_serving, solved one request at a time
    in arrival order on the plain single-lattice path (no batching, no
    admission: a request waits until the one before it has been read back).
    Latency = moments read back - arrival, as for the server."""
    reqs = W.serving_requests(n_requests, rate_hz=rate_hz, seed=0)
    probs = [r.problem() for r in reqs]
    cfgs = [A.config_from(p, precision=precision) for p in probs]
    log(f"[{tag}] {len(reqs)} requests, one at a time")
    lat, lups, nbytes, bad = [], 0, 0, 0
    start = time.perf_counter()
    for r, p, cfg in zip(reqs, probs, cfgs):
        wait = r.arrival_s - (time.perf_counter() - start)
        if wait > 0:
            time.sleep(wait)
        L = A.Lattice(cfg, owner="torch")
        L.set_state(p.U0, p.bed)
        L.step(r.steps)
        st = L.sync(check=False)
        L.moments()
        L.close()
        if st["rc"] not in (0, A.EPOSITIVITY):
            bad += 1
            continue
        lat.append(time.perf_counter() - (start + r.arrival_s))
        lups += p.cells * r.steps
        nbytes += p.cells * r.steps * alg_bytes_per_lup(p, 8 if precision == A.F64 else 4)
    wall = time.perf_counter() - start
    lat = np.array(lat) * 1e3
    out = {"requests": len(reqs), "failed": bad, "wall_s": wall, "glups": lups / wall / 1e9,
           "alg_gbs_whole_job": nbytes / wall / 1e9,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "precision": "f64" if precision == A.F64 else "f32", "rate_hz": rate_hz}
    log(f"[{tag}] {out}")
    return out


def run_cpu_baseline(args):
    """The FP64 oracle (single-threaded C) on a bounded sample of the main
    workload: a few steps of the same 2048^2 lattice."""
    import oracle as O

    p = W.euler_seeded_2d(0, n=2048, steps=args.cpu_steps)
    c = O.make_cfg(p.system, p.dim, p.nx, p.ny, p.x0, p.x1, p.y0, p.y1, p.bc, p.cfl, p.eps, p.gamma)
    L = O.Lattice(c).init(p.U0)
    t0 = time.perf_counter()
    L.run(args.cpu_steps)
    dt = time.perf_counter() - t0
    glups = p.cells * args.cpu_steps / dt / 1e9
    log(f"[cpu] oracle {args.cpu_steps} steps of 2048^2 in {dt:.1f}s: {glups * 1e3:.2f} MLUPS")
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": glups, "unit": "GLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{args.cpu_steps} steps of the 2048x2048 2D Euler lattice (seed 0), FP64, "
                      f"single-threaded C oracle, {dt:.1f} s",
            "host_cpu": model, "host_logical_cpus": os.cpu_count()}


def copy_calibration(torch, args):
    """Plain device copy of known size for HBM counter calibration."""
    n = 1 << 28  # 1 GiB of float32 read + 1 GiB written per copy
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    with Timer(torch) as tm:
        for _ in range(10):
            b.copy_(a)
    gbs = 10 * 2 * n * 4 / (tm.ms * 1e-3) / 1e9
    log(f"[copy] {gbs:.0f} GB/s for a 1 GiB -> 1 GiB device copy")
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 10, "gbs": gbs}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--only", choices=["euler2d_f32", "euler2d_f64", "swe2d_f32", "euler3d_f32", "serving"],
                    default=None)
    ap.add_argument("--steps3d", type=int, default=100)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--swe-steps", type=int, default=2000)
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    # a budget above the whole mix's footprint (about 30 GB at its peak), so
    # that admission never waits for memory
    ap.add_argument("--unlimited-gib", type=float, default=192.0)
    ap.add_argument("--fp64-check", type=int, default=12)
    # batched launches per server iteration at most (capped by the resident
    # lattices' remaining steps): the host loop keeps that much work queued
    ap.add_argument("--launches-per-iterate", type=int, default=32)
    ap.add_argument("--low-requests", type=int, default=64)
    ap.add_argument("--low-rate", type=float, default=8.0)
    ap.add_argument("--latency-solves", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the method is built for a single MI355X here "
              f"(--gpus {args.gpus} requested). Multi-GPU sharding is described, not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch, args)
        return
    if args.only == "swe2d_f32":
        r = run_swe(torch, args, steps=args.steps)
        log(f"[only] swe2d_f32 {r}")
        return
    if args.only == "euler3d_f32":
        r = run_euler3d(torch, args, steps=args.steps)
        log(f"[only] euler3d_f32 {r}")
        return
    if args.only == "serving":
        r = run_serving(torch, args, args.requests, args.rate, 0)
        log(f"[only] serving {r}")
        return
    if args.only == "euler2d_f64":
        p = W.euler_seeded_2d(0, n=2048, steps=1000)
        L, ms, st = time_steps(torch, p, A.F64, args.steps, args.warmup)
        log(f"[only] euler2d_f64 ms/step {ms / args.steps:.4f}")
        return
    main_res, p = run_main(torch, args)
    if args.only:
        log(f"[only] euler2d_f32 ms/step {main_res['ms'] / args.steps:.4f}")
        return
    ms_step = main_res["ms"] / args.steps
    glups = p.cells / (ms_step * 1e-3) / 1e9
    alg = ALG_BYTES[("euler2d", 4)] * p.cells
    achieved = alg / (ms_step * 1e-3) / 1e9
    traffic = read_traffic("euler2d_2048_f32")
    extra = {}
    extra["fp64_plain"] = {
        "glups": p.cells / (main_res["fp64"]["ms"] / args.steps * 1e-3) / 1e9,
        "ms_per_step": main_res["fp64"]["ms"] / args.steps,
        "alg_gbs": ALG_BYTES[("euler2d", 8)] * p.cells / (main_res["fp64"]["ms"] / args.steps * 1e-3) / 1e9,
        "fp32_vs_fp64_rel_l1": main_res["fp32_vs_fp64_rel_l1"],
        "fp32_vs_fp64_rel_l1_per_field": main_res["fp32_vs_fp64_rel_l1_per_field"]}
    sw = run_swe(torch, args)
    ms_sw = sw["ms"] / sw["steps"]
    extra["swe2d_4096_f32"] = {"glups": sw["cells"] / (ms_sw * 1e-3) / 1e9, "ms_per_step": ms_sw,
                               "alg_gbs": ALG_BYTES[("swe2d", 4)] * sw["cells"] / (ms_sw * 1e-3) / 1e9,
                               "mass_drift_rel": sw["mass_drift_rel"], "flags": sw["flags"]}
    extra["euler3d_256_f32"] = run_euler3d(torch, args)
    extra["euler1d_4096_latency"] = run_latency_1d(torch, args)
    extra["advection_256_latency_f64"] = run_latency_advection(torch, args)
    if not args.no_serving:
        extra["serving"] = run_serving(torch, args, args.requests, args.rate, args.fp64_check)
        # the default mix offers several times the capacity, so its latency is
        # queueing; a run at a fraction of the capacity shows service latency
        extra["serving_low_rate"] = run_serving(torch, args, args.low_requests, args.low_rate, 4,
                                                tag="serving-low")
        # the default mix with a budget that never binds: every request is
        # admitted on arrival
        extra["serving_unlimited_budget"] = run_serving(torch, args, args.requests, args.rate, 4,
                                                        tag="serving-unlimited", budget_gib=args.unlimited_gib)
        if not args.no_plain:
            # the metric's comparison: the same arrivals on the plain path,
            # FP64 and FP32, one solve at a time (the FP32 run isolates what
            # the batched server gains from batching alone)
            extra["plain_fp64_sequential"] = run_plain(torch, args, args.requests, args.rate, A.F64,
                                                       "plain-f64")
            extra["plain_fp32_sequential"] = run_plain(torch, args, args.requests, args.rate, A.F32,
                                                       "plain-f32")
            extra["plain_fp64_sequential_low_rate"] = run_plain(torch, args, args.low_requests, args.low_rate,
                                                                A.F64, "plain-f64-low")
    cpu = None if args.no_cpu else run_cpu_baseline(args)
    line = {
        "metric": METRIC, "value": glups, "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded four-quadrant Riemann data)",
        "config": {"workload": "euler2d_2048x2048_quadrants_seed0_fp32", "system": "euler", "dim": 2,
                   "nx": 2048, "ny": 2048, "cfl": 0.5, "bc": "transmissive", "gamma": 1.4,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_step_single<EULER,2D,float>", "alg_bytes_per_lup": ALG_BYTES[("euler2d", 4)],
                     "lups_per_launch": p.cells, "avg_kernel_ms": ms_step},
        "cpu_baseline": cpu,
        "flags": main_res["flags"],
        "kernel_source_sha256_16": kernel_source_hash(),
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
