"""Benchmark of the adaptive-relaxation LBM step on one MI355X.

Default run (one JSON line on stdout, progress on stderr):

* main line: configuration 3, 2D Euler on 2048 x 2048 cells, four-quadrant
  Riemann data (seed 0), transmissive, CFL 0.5, stepped by the FP32 batched
  path: the lattice is a request of the serving runtime and every step is one
  launch of the batched kernel.  W warm-up steps, then K timed steps
  (default K = 1000, the configuration's run length); ``value`` = lattice
  updates per second (GLUPS) with the state resident in HBM; ``roofline`` =
  algorithmic bytes of the step / average launch time from HIP events on the
  launch stream, against 8 TB/s;
* beside it: the same lattice on the single-lattice FP32 kernel and on the
  FP64 plain path (the metric's comparison); configuration 4 (4096^2 shallow
  water with the bed source) the same way; FP32-vs-FP64 error per field at
  each configuration's own step count, with the problem's own conditioning
  (how far FP64 moves when the initial data is rounded to FP32); solve
  latency p50/p99 for configurations 1-4; the serving mix (continuous
  batching, p50/p99 latency) and the same arrivals solved one at a time on
  the plain path, with the FP32-vs-FP64 error of every served request; a
  fixed serving mix for per-launch HBM counters; 3D Euler; the FP64 CPU
  oracle on a bounded sample, single-threaded and on all host cores.

``--only NAME`` runs one workload (for profilers); ``--copy-calibration``
times a plain device copy of known size (HBM counter calibration).
"""
import argparse
import dataclasses
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
# the kernels, their build, and the runtime that deals the batched kernel's
# work (its schedule decides the batched launch's traffic)
KERNEL_SOURCES = ["paper_2609_18177_amd/csrc/step.hpp", "paper_2609_18177_amd/csrc/physics.hpp",
                  "paper_2609_18177_amd/csrc/step3d.hpp", "paper_2609_18177_amd/csrc/kernels.hip",
                  "paper_2609_18177_amd/csrc/runtime.cpp", "paper_2609_18177_amd/build.py"]
ONLY = ["euler2d_batched_f32", "euler2d_f32", "euler2d_f64", "swe2d_batched_f32", "swe2d_f32", "euler3d_f32",
        "serving", "serving_fixed_f32"]
# FP32-vs-FP64 bounds per served system (relative L1 over all fields of a
# request's result), set above the largest error measured over the served
# requests; shallow water's is loose because a wet/dry front moves with a
# single cell's rounding, so the FP64 result itself changes by about as much
# when its initial data are rounded to FP32
SERVED_FP32_TOL = {"euler1d": 5e-3, "euler2d": 2e-3, "swe2d": 1.5e-1}


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


def read_profile(workload):
    """rocprofv3 summary of a workload (profiles/), or None when it is
    missing or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d


def per_field(a, b):
    """Relative L1 and largest pointwise difference (over the field's largest
    magnitude) of each field of a against b."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    l1 = [float(np.sum(np.abs(a[c] - b[c])) / max(np.sum(np.abs(b[c])), 1e-300)) for c in range(b.shape[0])]
    mx = [float(np.max(np.abs(a[c] - b[c])) / max(np.max(np.abs(b[c])), 1e-300)) for c in range(b.shape[0])]
    return l1, mx


def rounded_to_fp32(p):
    """The problem with its initial data (and bed) rounded to FP32."""
    r = lambda a: None if a is None else a.astype(np.float32).astype(np.float64)  # noqa: E731
    return dataclasses.replace(p, U0=r(p.U0), bed=r(p.bed))


class Timer:
    """HIP events recorded on the stream the library launches on (torch's
    current stream, handed to the library and the server at creation)."""

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


# ---------------------------------------------------------------- timing --

def time_plain(torch, problem, precision, steps, warmup):
    """Steps of the single-lattice kernel: K launches timed with events."""
    cfg = A.config_from(problem, precision=precision)
    L = A.Lattice(cfg, owner="torch")
    L.set_state(problem.U0, problem.bed)
    L.step(warmup)
    L.sync(check=False)
    with Timer(torch) as tm:
        L.step(steps)
    st = L.sync(check=False)
    L.close()
    return tm.ms, st


def _drain(srv, want):
    """Iterate the server until the requests in `want` completed."""
    res = {}
    while len(res) < len(want):
        srv.iterate(32)
        for c in srv.poll(64):
            res[c["id"]] = c
    return res


def time_batched(torch, problems, precision, steps, warmup, repeats=None):
    """Steps of the batched kernel over the given lattices, all resident:
    the server admits them and runs the warm-up launches in one call, then
    one call makes the K timed launches (each a batched step of every
    lattice), timed with events on the server's stream.  repeats=(r, k):
    afterwards r more timed calls of k launches each, whose times per launch
    are appended to the list `repeats_ms` returned as a third value."""
    need = sum(A.query_sizes(A.config_from(p, precision=precision)).total_bytes for p in problems)
    srv = A.Server(int(need * 1.3) + (64 << 20), precision)
    warmup = max(warmup, 1)
    extra = repeats[0] * repeats[1] if repeats else 0
    ids = [srv.submit(A.config_from(p, precision=precision), p.U0, p.bed, warmup + steps + extra + 1)
           for p in problems]
    srv.iterate(warmup)
    with Timer(torch) as tm:
        srv.iterate(steps)
    reps = []
    for _ in range(repeats[0] if repeats else 0):
        with Timer(torch) as tr:
            srv.iterate(repeats[1])
        reps.append(tr.ms / repeats[1])
    res = _drain(srv, ids)
    srv.close()
    bad = [res[i]["status"] for i in ids if res[i]["status"] != 0]
    if repeats:
        return tm.ms, bad, reps
    return tm.ms, bad


def run_throughput(torch, args, p, tag):
    """FP32 batched (the metric's path), FP32 single-lattice and FP64 plain
    on the same lattice, K timed steps each."""
    log(f"[{tag}] {p.name}: FP32 batched, warmup {args.warmup}, timed {args.steps}")
    if args.only:
        ms_b, bad = time_batched(torch, [p], A.F32, args.steps, args.warmup)
        return {"fp32_batched": {"ms_per_step": ms_b / args.steps, "failed": bad}}
    # then 5 repeats of 200 launches each: their median and spread beside
    # the K-launch figure
    ms_b, bad, reps = time_batched(torch, [p], A.F32, args.steps, args.warmup, repeats=(5, 200))
    out = {"fp32_batched": {"ms_per_step": ms_b / args.steps, "failed": bad,
                            "repeats_ms_per_step": {"n": len(reps), "launches_each": 200,
                                                    "median": float(np.median(reps)), "min": float(min(reps)),
                                                    "max": float(max(reps))}}}
    log(f"[{tag}] FP32 single-lattice kernel")
    ms_s, st = time_plain(torch, p, A.F32, args.steps, args.warmup)
    out["fp32_single"] = {"ms_per_step": ms_s / args.steps, "flags": st["flags"]}
    log(f"[{tag}] FP64 plain path")
    ms_p, st = time_plain(torch, p, A.F64, args.steps, args.warmup)
    out["fp64_plain"] = {"ms_per_step": ms_p / args.steps, "flags": st["flags"]}
    for k, v in out.items():
        size = 8 if k == "fp64_plain" else 4
        v["glups"] = p.cells / (v["ms_per_step"] * 1e-3) / 1e9
        v["alg_gbs"] = alg_bytes_per_lup(p, size) * p.cells / (v["ms_per_step"] * 1e-3) / 1e9
        v["alg_frac_of_peak"] = v["alg_gbs"] / HBM_PEAK_GBS
    return out


# --------------------------------------------------------------- latency --

def solve_plain(p, precision, steps):
    """One solve on the plain path: set_state (H2D) -> steps -> moments (D2H)."""
    L = A.Lattice(A.config_from(p, precision=precision), owner="torch")
    t0 = time.perf_counter()
    L.set_state(p.U0, p.bed)
    L.step(steps)
    U = L.moments()
    dt = time.perf_counter() - t0
    st = L.sync(check=False)
    L.close()
    return dt, U, st


def solve_batched(srv, p, precision, steps):
    """One solve through a server: submit (the initial state is copied) ->
    admission, batched steps, retirement -> result polled."""
    t0 = time.perf_counter()
    rid = srv.submit(A.config_from(p, precision=precision), p.U0, p.bed, steps)
    r = _drain(srv, [rid])[rid]
    dt = time.perf_counter() - t0
    return dt, r["U"].reshape(p.U0.shape) if r["U"] is not None else None, r


def latency(ts):
    ts = np.array(ts) * 1e3
    return {"solves": len(ts), "p50_ms": float(np.percentile(ts, 50)), "p99_ms": float(np.percentile(ts, 99))}


def run_config_solves(torch, args, p, steps, n32, n64, tag):
    """Solve latency of a configuration at its own step count, FP32 batched
    and FP64 plain, and the FP32-vs-FP64 error of the results per field,
    with the FP64 result's own movement when the initial data is rounded to
    FP32 (the problem's conditioning at that precision)."""
    log(f"[{tag}] solve latency, {steps} steps: FP32 batched x{n32}, FP64 plain x{n64}")
    t32, t64 = [], []
    # one server for the solves, as a serving process keeps it: the first
    # solve warms its pool of device blocks and is not counted
    srv = A.Server(int(A.query_sizes(A.config_from(p, precision=A.F32)).total_bytes * 1.3) + (64 << 20), A.F32)
    for i in range(n32 + 1):
        dt, U32, r = solve_batched(srv, p, A.F32, steps)
        if i:
            t32.append(dt)
    srv.close()
    for i in range(n64 + 1):
        dt, U64, st = solve_plain(p, A.F64, steps)
        if i:
            t64.append(dt)
    _, U64r, _ = solve_plain(rounded_to_fp32(p), A.F64, steps)
    e_l1, e_max = per_field(U32, U64)
    c_l1, c_max = per_field(U64r, U64)
    out = {"steps": steps, "fp32_batched": latency(t32), "fp64_plain": latency(t64),
           "fp32_batched_vs_fp64_plain": {"rel_l1_per_field": e_l1, "rel_max_per_field": e_max},
           "fp64_conditioning": {"rel_l1_per_field": c_l1, "rel_max_per_field": c_max},
           "fp32_flags": r["flags"]}
    if p.system == W.SWE:
        wet = U64[0] > 1e-3
        out["fp32_wet_rel_l1_per_field"] = [float(np.sum(np.abs(U32[c][wet] - U64[c][wet])) /
                                                  np.sum(np.abs(U64[c][wet]))) for c in range(U64.shape[0])]
        out["fp32_volume_drift"] = float((math.fsum(U32[0].ravel().tolist()) -
                                          math.fsum(p.U0[0].ravel().tolist())) / math.fsum(p.U0[0].ravel().tolist()))
    log(f"[{tag}] {out}")
    return out


def run_latency_small(args):
    """Configurations 1 and 2 (lattices of a few kilobytes, launch-bound):
    solve latency on the plain path, with their errors (configuration 1
    against the exact solution, configuration 2 FP32 against FP64)."""
    out = {}
    p = W.advection_sine(n=256, steps=512)
    ts = []
    for i in range(args.latency_solves + 2):
        dt, U, st = solve_plain(p, A.F64, p.steps)
        if i >= 2:
            ts.append(dt)
    err = float(np.linalg.norm(U.ravel() - p.U0.ravel()) / np.linalg.norm(p.U0.ravel()))
    out["advection_256_fp64"] = {**latency(ts), "t": st["t"], "rel_l2_vs_exact": err}
    p = W.euler_seeded_1d(0, n=4096, steps=2000)
    res = {}
    for prec, name in ((A.F32, "fp32"), (A.F64, "fp64")):
        ts = []
        for i in range(args.latency_solves + 2):
            dt, U, st = solve_plain(p, prec, p.steps)
            if i >= 2:
                ts.append(dt)
        res[name] = U
        out[f"euler1d_4096_{name}"] = latency(ts)
    out["euler1d_4096_fp32_vs_fp64_rel_l1_per_field"] = per_field(res["fp32"], res["fp64"])[0]
    log(f"[latency] configurations 1, 2: {out}")
    return out


# ------------------------------------------------------------------- 3D ---

def run_euler3d(torch, args, steps=None):
    """3D Euler (D3Q7), seeded octant data on 256^3 cells, FP32: the
    fused one-pass step; FP32 against FP64 after the timed steps."""
    p = W.euler_octants_3d(seed=0, n=256, steps=100)
    steps = steps or args.steps3d
    log(f"[euler3d] 256^3 FP32: warmup {args.warmup}, timed {steps}")
    cfg = A.config_from(p, precision=A.F32)
    L = A.Lattice(cfg, owner="torch")
    L.set_state(p.U0)
    L.step(args.warmup)
    L.sync(check=False)
    with Timer(torch) as tm:
        L.step(steps)
    st = L.sync(check=False)
    out = {}
    if not args.only:
        U32 = L.moments()
        L.close()
        L = A.Lattice(A.config_from(p, precision=A.F64), owner="torch")
        L.set_state(p.U0)
        L.step(args.warmup + steps)
        U64 = L.moments()
        out["fp32_vs_fp64_rel_l1_per_field"], out["fp32_vs_fp64_rel_max_per_field"] = per_field(U32, U64)
        out["error_after_steps"] = args.warmup + steps
    L.close()
    ms_step = tm.ms / steps
    b = alg_bytes_per_lup(p, 4)
    out.update({"glups": p.cells / (ms_step * 1e-3) / 1e9, "ms_per_step": ms_step, "cells": p.cells,
                "alg_bytes_per_lup": b,
                "alg_gbs": b * p.cells / (ms_step * 1e-3) / 1e9,
                "alg_frac": b * p.cells / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, "flags": st["flags"]})
    return out


# --------------------------------------------------------------- serving --

def system_of(p):
    return {(W.EULER, 1): "euler1d", (W.EULER, 2): "euler2d", (W.SWE, 2): "swe2d"}.get((p.system, p.dim), "other")


def run_serving(torch, args, n_requests, rate_hz, tag="serving", budget_gib=None, keep=False):
    """Continuous batching: Poisson arrivals admitted by HBM budget into the
    batched FP32 kernel; latency = result read back - arrival.  keep: return
    the results for the FP32-vs-FP64 comparison."""
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
    peak_mem = peak_pool = 0
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
        peak_pool = max(peak_pool, srv.pool_bytes())
        for c in srv.poll(256):
            results[c["id"]] = c
        if resident == 0 and queued == 0 and nxt < len(reqs):
            time.sleep(max(0.0, min(0.001, reqs[nxt].arrival_s - (time.perf_counter() - start))))
    wall = time.perf_counter() - start
    torch.cuda.synchronize()
    srv.close()
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
           "iterations": iters, "peak_charged_bytes": int(peak_mem), "peak_pool_bytes": int(peak_pool),
           "offered_lups": int(lups), "offered_glups_over_arrivals": lups / span / 1e9, "arrival_span_s": span,
           "iterate_time_fraction_with_work": busy / wall, "rate_hz": rate_hz, "budget_gib": budget_gib,
           "launches_per_iterate": args.launches_per_iterate}
    log(f"[{tag}] {out}")
    kept = None
    if keep:
        kept = {r.rid: results[r.server_id] for r in reqs}
    return out, kept


def run_plain(torch, args, n_requests, rate_hz, precision, tag, served=None, cond_sample=0):
    """The same arrival stream as run_serving, solved one request at a time
    in arrival order on the plain single-lattice path (no batching, no
    admission: a request waits until the one before it has been read back).
    Latency = moments read back - arrival, as for the server.  With the
    served FP32 results, every request's FP32-vs-FP64 error (relative L1 of
    each field, its largest) is compared with the bound of its system; for
    the first cond_sample requests of each system the FP64 result's own
    movement under FP32 rounding of the initial data is measured too."""
    reqs = W.serving_requests(n_requests, rate_hz=rate_hz, seed=0)
    probs = [r.problem() for r in reqs]
    cfgs = [A.config_from(p, precision=precision) for p in probs]
    log(f"[{tag}] {len(reqs)} requests, one at a time")
    lat, lups, nbytes, bad = [], 0, 0, 0
    errs = {}
    start = time.perf_counter()
    for r, p, cfg in zip(reqs, probs, cfgs):
        wait = r.arrival_s - (time.perf_counter() - start)
        if wait > 0:
            time.sleep(wait)
        L = A.Lattice(cfg, owner="torch")
        L.set_state(p.U0, p.bed)
        L.step(r.steps)
        st = L.sync(check=False)
        U = L.moments()
        L.close()
        if st["rc"] not in (0, A.EPOSITIVITY):
            bad += 1
            continue
        lat.append(time.perf_counter() - (start + r.arrival_s))
        lups += p.cells * r.steps
        nbytes += p.cells * r.steps * alg_bytes_per_lup(p, 8 if precision == A.F64 else 4)
        if served is not None and served[r.rid]["status"] == 0:
            U32 = served[r.rid]["U"].reshape(U.shape)
            e = float(np.sum(np.abs(U32 - U)) / np.sum(np.abs(U)))
            ef = max(per_field(U32, U)[0])
            errs.setdefault(system_of(p), []).append((r.rid, e, ef))
    wall = time.perf_counter() - start
    lat = np.array(lat) * 1e3
    out = {"requests": len(reqs), "failed": bad, "wall_s": wall, "glups": lups / wall / 1e9,
           "alg_gbs_whole_job": nbytes / wall / 1e9,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "precision": "f64" if precision == A.F64 else "f32", "rate_hz": rate_hz}
    if served is not None:
        summary = {}
        for sysname, lst in sorted(errs.items()):
            v = np.array([e for _, e, _ in lst])
            vf = np.array([ef for _, _, ef in lst])
            tol = SERVED_FP32_TOL.get(sysname)
            summary[sysname] = {"requests": len(v), "max": float(v.max()), "median": float(np.median(v)),
                                "p99": float(np.percentile(v, 99)), "bound": tol,
                                "within_bound": int(np.sum(v <= tol)) if tol else None,
                                "largest_field_rel_l1": {"max": float(vf.max()), "median": float(np.median(vf))}}
            if cond_sample:
                ratios = []
                for rid, e, _ in lst[:cond_sample]:
                    p, rq = probs[rid], reqs[rid]
                    _, U64, _ = solve_plain(p, A.F64, rq.steps)
                    _, U64r, _ = solve_plain(rounded_to_fp32(p), A.F64, rq.steps)
                    c = float(np.sum(np.abs(U64r - U64)) / np.sum(np.abs(U64)))
                    ratios.append(e / max(c, 1e-300))
                summary[sysname]["error_over_conditioning_sample"] = {
                    "requests": len(ratios), "median": float(np.median(ratios)), "max": float(np.max(ratios))}
        out["fp32_batched_vs_fp64_plain_rel_l1"] = summary
    log(f"[{tag}] {out}")
    return out


def run_serving_fixed(torch, args, steps=None):
    """A fixed mix for per-launch figures: the default mix's requests in
    arrival order, as many as the 4 GiB budget admits at once, all resident
    for the timed launches, so that every launch does the same work."""
    reqs = W.serving_requests(args.requests, rate_hz=args.rate, seed=0)
    budget = int(args.budget_gib * 2 ** 30)
    probs, used = [], 0
    for r in reqs:
        p = r.problem()
        b = A.query_sizes(A.config_from(p, precision=A.F32)).total_bytes * 1.25
        if used + b > budget:
            break
        probs.append(p)
        used += b
    steps = steps or args.steps
    log(f"[serving-fixed] {len(probs)} lattices resident, warmup {args.warmup}, timed {steps}")
    ms, bad = time_batched(torch, probs, A.F32, steps, args.warmup)
    cells = sum(p.cells for p in probs)
    alg = sum(p.cells * alg_bytes_per_lup(p, 4) for p in probs)
    ms_step = ms / steps
    waves = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    _, groups = A.plan_groups([A.config_from(p, precision=A.F32) for p in probs], waves)
    return {"lattices": len(probs), "cells_per_step": cells, "alg_bytes_per_step": alg,
            "launches_per_step": groups, "ms_per_step": ms_step, "glups": cells / (ms_step * 1e-3) / 1e9,
            "alg_gbs": alg / (ms_step * 1e-3) / 1e9, "alg_frac": alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "failed": bad,
            "systems": {s: sum(1 for p in probs if system_of(p) == s) for s in ("euler1d", "euler2d", "swe2d")}}


# ------------------------------------------------------------------- CPU ---

def run_cpu_baseline(args):
    """The FP64 oracle on a bounded sample of the main workload (a few steps
    of the same 2048^2 lattice): the single-threaded build and the OpenMP
    build on every host core (the same source and the same bits)."""
    import oracle as O

    p = W.euler_seeded_2d(0, n=2048, steps=args.cpu_steps)
    c = O.make_cfg(p.system, p.dim, p.nx, p.ny, p.x0, p.x1, p.y0, p.y1, p.bc, p.cfl, p.eps, p.gamma)
    rates = {}
    for parallel, steps in ((False, args.cpu_steps), (True, args.cpu_steps_omp)):
        L = O.Lattice(c, parallel=parallel).init(p.U0)
        t0 = time.perf_counter()
        L.run(steps)
        dt = time.perf_counter() - t0
        rates[parallel] = (p.cells * steps / dt / 1e9, steps, dt, O.threads(parallel))
        log(f"[cpu] oracle ({O.threads(parallel)} threads) {steps} steps of 2048^2 in {dt:.1f}s: "
            f"{rates[parallel][0] * 1e3:.2f} MLUPS")
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    g, steps, dt, threads = rates[True]
    g1, steps1, dt1, _ = rates[False]
    return {"value": g, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} steps of the 2048x2048 2D Euler lattice (seed 0), FP64, C oracle built with OpenMP "
                      f"over rows on {threads} threads, {dt:.1f} s; single-threaded build: {steps1} steps in "
                      f"{dt1:.1f} s",
            "single_thread_value": g1, "host_cpu": model, "host_logical_cpus": os.cpu_count()}


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


def roofline(kernel, workload, alg_bytes, lups, ms):
    prof = read_profile(workload)
    achieved = alg_bytes * lups / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": prof["hbm_bytes_per_launch"] if prof else None,
            "kernel": kernel, "alg_bytes_per_lup": alg_bytes, "lups_per_launch": lups,
            "alg_bytes_per_launch": alg_bytes * lups, "avg_kernel_ms": ms,
            "avg_kernel_ms_rocprof": prof["avg_kernel_ns"] / 1e6 if prof else None,
            # counter traffic over the profiled kernel time: the DRAM rate
            "traffic_gbs": prof["hbm_bytes_per_launch"] / prof["avg_kernel_ns"] if prof else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--only", choices=ONLY, default=None)
    ap.add_argument("--steps3d", type=int, default=100)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    # a budget above the whole mix's footprint (about 30 GB at its peak), so
    # that admission never waits for memory
    ap.add_argument("--unlimited-gib", type=float, default=192.0)
    # batched launches per server iteration at most (capped by the resident
    # lattices' remaining steps): the host loop keeps that much work queued
    ap.add_argument("--launches-per-iterate", type=int, default=32)
    ap.add_argument("--low-requests", type=int, default=64)
    ap.add_argument("--low-rate", type=float, default=8.0)
    ap.add_argument("--latency-solves", type=int, default=20)
    ap.add_argument("--c4-solves", type=int, default=10)
    ap.add_argument("--cond-sample", type=int, default=8)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu-steps-omp", type=int, default=40)
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
    c3 = W.euler_seeded_2d(0, n=2048, steps=1000)
    c4 = W.swe_bed_2d(0, n=4096, steps=2000)
    if args.only:
        if args.only == "euler2d_batched_f32":
            ms, _ = time_batched(torch, [c3], A.F32, args.steps, args.warmup)
        elif args.only == "swe2d_batched_f32":
            ms, _ = time_batched(torch, [c4], A.F32, args.steps, args.warmup)
        elif args.only in ("euler2d_f32", "euler2d_f64", "swe2d_f32"):
            p = c4 if args.only.startswith("swe") else c3
            ms, _ = time_plain(torch, p, A.F64 if args.only.endswith("f64") else A.F32, args.steps, args.warmup)
        elif args.only == "euler3d_f32":
            r = run_euler3d(torch, args, steps=args.steps)
            ms = r["ms_per_step"] * args.steps
        elif args.only == "serving_fixed_f32":
            r = run_serving_fixed(torch, args)
            log(f"[only] serving_fixed_f32 {r}")
            ms = r["ms_per_step"] * args.steps
        else:
            r, _ = run_serving(torch, args, args.requests, args.rate)
            log(f"[only] serving {r}")
            return
        log(f"[only] {args.only} ms/step {ms / args.steps:.4f}")
        return

    extra = {}
    main_res = run_throughput(torch, args, c3, "c3")
    ms_step = main_res["fp32_batched"]["ms_per_step"]
    extra["c3_euler2d_2048"] = main_res
    extra["c4_swe2d_4096"] = run_throughput(torch, args, c4, "c4")
    extra["c3_solves"] = run_config_solves(torch, args, c3, 1000, args.latency_solves, args.latency_solves, "c3")
    extra["c4_solves"] = run_config_solves(torch, args, c4, 2000, args.c4_solves, max(3, args.c4_solves // 2), "c4")
    extra["c1_c2_solves"] = run_latency_small(args)
    extra["euler3d_256_f32"] = run_euler3d(torch, args)
    extra["serving_fixed_mix"] = run_serving_fixed(torch, args, steps=max(args.steps, 50))
    if not args.no_serving:
        extra["serving"], served = run_serving(torch, args, args.requests, args.rate, keep=not args.no_plain)
        # the default mix offers several times the capacity, so its latency is
        # queueing; a run at a fraction of the capacity shows service latency
        extra["serving_low_rate"], _ = run_serving(torch, args, args.low_requests, args.low_rate, tag="serving-low")
        # the default mix with a budget that never binds: every request is
        # admitted on arrival
        extra["serving_unlimited_budget"], _ = run_serving(torch, args, args.requests, args.rate,
                                                           tag="serving-unlimited", budget_gib=args.unlimited_gib)
        if not args.no_plain:
            # the metric's comparison: the same arrivals on the plain path,
            # FP64 (with the FP32 error of every served request) and FP32,
            # one solve at a time (the FP32 run isolates what the batched
            # server gains from batching alone)
            extra["plain_fp64_sequential"] = run_plain(torch, args, args.requests, args.rate, A.F64, "plain-f64",
                                                       served=served, cond_sample=args.cond_sample)
            served = None
            extra["plain_fp32_sequential"] = run_plain(torch, args, args.requests, args.rate, A.F32, "plain-f32")
            extra["plain_fp64_sequential_low_rate"] = run_plain(torch, args, args.low_requests, args.low_rate,
                                                                A.F64, "plain-f64-low")
    cpu = None if args.no_cpu else run_cpu_baseline(args)
    glups = c3.cells / (ms_step * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": glups, "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded four-quadrant Riemann data)",
        "config": {"workload": "euler2d_2048x2048_quadrants_seed0_fp32_batched", "system": "euler", "dim": 2,
                   "nx": 2048, "ny": 2048, "cfl": 0.5, "bc": "transmissive", "gamma": 1.4,
                   "path": "FP32 batched (serving runtime, one batched launch per step)",
                   "parallelism": "single GPU"},
        "roofline": roofline("k_step_batched<float>", "euler2d_2048_batched_f32", alg_bytes_per_lup(c3, 4),
                             c3.cells, ms_step),
        "cpu_baseline": cpu,
        "kernel_source_sha256_16": kernel_source_hash(),
        "extra": extra,
    }
    extra["roofline_single_kernel_c3"] = roofline("k_step_single<EULER,2D,float>", "euler2d_2048_f32",
                                                  alg_bytes_per_lup(c3, 4), c3.cells,
                                                  main_res["fp32_single"]["ms_per_step"])
    extra["roofline_fp64_plain_c3"] = roofline("k_step_single<EULER,2D,double>", "euler2d_2048_f64",
                                               alg_bytes_per_lup(c3, 8), c3.cells,
                                               main_res["fp64_plain"]["ms_per_step"])
    extra["roofline_batched_c4"] = roofline("k_step_batched<float>", "swe2d_4096_batched_f32",
                                            alg_bytes_per_lup(c4, 4), c4.cells,
                                            extra["c4_swe2d_4096"]["fp32_batched"]["ms_per_step"])
    e3 = extra["euler3d_256_f32"]
    extra["roofline_euler3d_256"] = roofline("k3_step<EULER,float>", "euler3d_256_f32", e3["alg_bytes_per_lup"],
                                             e3["cells"], e3["ms_per_step"])
    fx = extra["serving_fixed_mix"]
    prof = read_profile("serving_fixed_f32")
    # the mix is stepped in one batched launch per group of lattices: its
    # figures are per step (all the step's launches)
    extra["roofline_batched_serving_fixed_mix"] = {
        "bound": "hbm", "achieved": fx["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fx["alg_frac"],
        "traffic": prof["hbm_bytes_per_step"] if prof else None, "alg_bytes_per_step": fx["alg_bytes_per_step"],
        "launches_per_step": fx["launches_per_step"], "ms_per_step": fx["ms_per_step"],
        "kernel_ms_per_step_rocprof": prof["kernel_ns_per_step"] / 1e6 if prof else None,
        "traffic_gbs": prof["hbm_bytes_per_step"] / prof["kernel_ns_per_step"] if prof else None}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
