"""Profile the fused step kernel with rocprofv3 and summarise into profiles/.

Runs, each as its own rocprofv3 process on the benchmark's single-workload
mode (the launch configuration bench.py times):

1. ``--kernel-trace --stats``: average kernel duration;
2. ``--pmc FETCH_SIZE`` and 3. ``--pmc WRITE_SIZE``: HBM kilobytes per
   dispatch of the step kernel;
4./5. the same two counters for a plain 1 GiB device copy, which calibrate
   the counters (bytes the copy must move / what the counter reports).

Writes ``profiles/<workload>_pmc.json`` (HBM bytes per launch, keyed to a
hash of the kernel sources) and ``profiles/<workload>_rocprof.md`` (the
figures and the commands).  ``--workload serving`` runs only a kernel trace
of the serving mix and writes ``profiles/serving_mix_f32_rocprof.md``.  Usage, on a GPU machine, from the repository
root::

    python -m paper_2609_18177_amd.profile_step --workload euler2d_f32 --raw gpurun_out/prof
"""
import argparse
import ast
import csv
import collections
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (kernel source hash; bench imports no GPU module at import time)

# 2D kernels end in the columns per lane (2 for advection and shallow water
# on lattices of even nx) and the buffer-resource addressing flag (populations
# below 4 GiB)
KERNELS = {"euler2d_batched_f32": "k_step_batched<float>",
           "euler2d_f32": "k_step_single<1, 2, false, float, 1, true>",
           "euler2d_f64": "k_step_single<1, 2, false, double, 1, true>",
           "swe2d_batched_f32": "k_step_batched<float>",
           "swe2d_f32": "k_step_single<2, 2, true, float, 2, true>",
           "euler3d_f32": "k3_step<1, float>",
           "serving_fixed_f32": "k_step_batched<float>"}
# further kernels of a step (3D: the indicator and relaxation passes)
EXTRA_KERNELS = {}
WORKLOAD_NAMES = {"euler2d_batched_f32": "euler2d_2048_batched_f32", "euler2d_f32": "euler2d_2048_f32",
                  "euler2d_f64": "euler2d_2048_f64", "swe2d_batched_f32": "swe2d_4096_batched_f32",
                  "swe2d_f32": "swe2d_4096_f32", "euler3d_f32": "euler3d_256_f32",
                  "serving_fixed_f32": "serving_fixed_f32"}


FROM_RAW = False  # --from-raw: summarise the CSVs an earlier run left in --raw


def rocprof(args, raw, tag, prog, timeout):
    out = os.path.join(raw, tag)
    cmd = ["rocprofv3", *args, "--output-format", "csv", "-d", out, "-o", "run", "--", sys.executable, "-u", *prog]
    if not FROM_RAW:
        print("+", " ".join(cmd), flush=True)
        with open(os.path.join(raw, tag + ".log"), "w") as log:
            subprocess.run(cmd, cwd=ROOT, stdout=log, stderr=subprocess.STDOUT, timeout=timeout, check=True)
    rel = os.path.relpath(out, ROOT)
    return out, " ".join(["rocprofv3", *args, "--output-format csv -d", rel, "-o run --", "python3 -u", *prog])


def per_dispatch(csv_path, counter, name_part):
    vals = collections.defaultdict(float)
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]:
                vals[int(r["Dispatch_Id"])] += float(r["Counter_Value"])
    v = sorted(vals.values())
    return (sum(v) / len(v), len(v)) if v else (None, 0)


def timed_launch_ns(trace_csv, name_part, warmup, steps, per_step):
    """Average duration of the launches in the benchmark's timed region:
    dispatches warmup*per_step .. (warmup+steps)*per_step-1 of the kernel, in
    start order (the warm-up launches, the first of a process among them, are
    left out)."""
    spans = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            if name_part in r["Kernel_Name"]:
                spans.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    spans.sort()
    timed = spans[warmup * per_step:(warmup + steps) * per_step]
    return sum(e - b for b, e in timed) / len(timed) if timed else None


def kernel_stats(csv_path, name_part):
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if name_part in r["Name"]:
                return {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]), "min_ns": float(r["MinNs"]),
                        "max_ns": float(r["MaxNs"])}
    return None


def serving_profile(args, raw):
    """Kernel trace of the default serving mix (bench.py --only serving):
    time per kernel, and how much of the run the GPU spent in kernels.  The
    batched kernel's work differs from launch to launch (the resident mix
    changes), so no per-launch counters are taken."""
    prog = ["bench.py", "--only", "serving"]
    d, cmd = rocprof(["--kernel-trace", "--stats"], raw, "serving_trace", prog, 300)
    with open(os.path.join(raw, "serving_trace.log")) as f:
        line = [ln for ln in f if "[only] serving " in ln][-1]
    res = ast.literal_eval(line.split("[only] serving ", 1)[1].strip())
    starts, ends = [], []
    with open(os.path.join(d, "run_kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            starts.append(int(r["Start_Timestamp"]))
            ends.append(int(r["End_Timestamp"]))
    span_s = (max(ends) - min(starts)) / 1e9
    busy_s = sum(e - b for b, e in zip(starts, ends)) / 1e9
    rows = []
    with open(os.path.join(d, "run_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"].split("(")[0].replace("void ", ""), int(r["Calls"]), float(r["TotalDurationNs"]),
                         float(r["AverageNs"])))
    rows.sort(key=lambda x: -x[2])
    pdir = os.path.abspath(args.profiles_dir)
    os.makedirs(pdir, exist_ok=True)
    with open(os.path.join(pdir, "serving_mix_f32_rocprof.md"), "w") as f:
        f.write("# rocprofv3 summary: k_step_batched<float>, workload serving_mix_f32\n\n")
        f.write("Made by `python -m paper_2609_18177_amd.profile_step --workload serving` (kernel source hash "
                f"{bench.kernel_source_hash()}); the pass it ran:\n\n    {cmd}\n\n")
        f.write("512 requests (Poisson arrivals at 200/s; 1D Euler, 2D Euler and shallow water) admitted by a 4 GiB "
                "budget, served by the batched FP32 kernel.\n\n")
        f.write("| quantity | value |\n|---|---|\n")
        f.write(f"| requests served / failed | {res['requests']} / {res['failed']} |\n")
        f.write(f"| serving wall time (bench) | {res['wall_s']:.2f} s |\n")
        f.write(f"| throughput (bench) | {res['glups']:.2f} GLUPS |\n")
        f.write(f"| latency p50 / p99 (bench) | {res['p50_ms'] / 1e3:.2f} / {res['p99_ms'] / 1e3:.2f} s |\n")
        f.write(f"| batched launches per server call at most | {res.get('launches_per_iterate', 1)} |\n")
        f.write(f"| first kernel start to last kernel end | {span_s:.2f} s |\n")
        f.write(f"| time in kernels (all kinds) | {busy_s:.2f} s ({100 * busy_s / span_s:.1f}% of the span) |\n")
        f.write("\n| kernel | calls | total (s) | average (us) |\n|---|---|---|---|\n")
        for name, calls, tot, avg in rows[:8]:
            f.write(f"| {name} | {calls} | {tot / 1e9:.3f} | {avg / 1e3:.1f} |\n")
    print(json.dumps({"span_s": span_s, "busy_s": busy_s, "bench": res}, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=sorted(KERNELS) + ["serving"], default="euler2d_batched_f32")
    ap.add_argument("--no-calibration", action="store_true",
                    help="reuse the copy calibration of profiles/euler2d_2048_batched_f32_pmc.json")
    ap.add_argument("--raw", default="gpurun_out/prof")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--profiles-dir", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--from-raw", action="store_true",
                    help="write the summaries from the CSVs of an earlier run in --raw (no profiling)")
    args = ap.parse_args()
    global FROM_RAW
    FROM_RAW = args.from_raw
    raw = os.path.abspath(args.raw)
    os.makedirs(raw, exist_ok=True)
    if args.workload == "serving":
        serving_profile(args, raw)
        return
    prog = ["bench.py", "--only", args.workload, "--steps", str(args.steps), "--warmup", "10"]
    kname = KERNELS[args.workload]
    d, cmd_trace = rocprof(["--kernel-trace", "--stats"], raw, "trace", prog, 300)
    stats = kernel_stats(os.path.join(d, "run_kernel_stats.csv"), kname)
    if stats is None:
        raise SystemExit(f"kernel {kname} not found in the trace")
    # the benchmark's own event-timed figure of the traced run
    event_ms = None
    with open(os.path.join(raw, "trace.log")) as f:
        for ln in f:
            if ln.startswith(f"[only] {args.workload} ms/step "):
                event_ms = float(ln.split()[-1])
    extra_names = EXTRA_KERNELS.get(args.workload, [])
    extra_stats = {k: kernel_stats(os.path.join(d, "run_kernel_stats.csv"), k) for k in extra_names}
    pmc_prog = ["bench.py", "--only", args.workload, "--steps", "10", "--warmup", "2"]
    d, cmd_fetch = rocprof(["--pmc", "FETCH_SIZE"], raw, "fetch", pmc_prog, 120)
    fetch_kib, nf = per_dispatch(os.path.join(d, "run_counter_collection.csv"), "FETCH_SIZE", kname)
    extra_fetch = {k: per_dispatch(os.path.join(d, "run_counter_collection.csv"), "FETCH_SIZE", k)[0]
                   for k in extra_names}
    d, cmd_write = rocprof(["--pmc", "WRITE_SIZE"], raw, "write", pmc_prog, 120)
    write_kib, nw = per_dispatch(os.path.join(d, "run_counter_collection.csv"), "WRITE_SIZE", kname)
    extra_write = {k: per_dispatch(os.path.join(d, "run_counter_collection.csv"), "WRITE_SIZE", k)[0]
                   for k in extra_names}
    if args.no_calibration:
        with open(os.path.join(os.path.abspath(args.profiles_dir), "euler2d_2048_batched_f32_pmc.json")) as f:  # noqa: E501
            cal = json.load(f)
        copy_fetch_kib, copy_write_kib = cal["copy_fetch_kib_for_1GiB"], cal["copy_write_kib_for_1GiB"]
        cmd_cf, cmd_cw = cal["commands"][3], cal["commands"][4]
    else:
        cal_prog = ["bench.py", "--copy-calibration"]
        d, cmd_cf = rocprof(["--pmc", "FETCH_SIZE"], raw, "copy_fetch", cal_prog, 120)
        copy_fetch_kib, _ = per_dispatch(os.path.join(d, "run_counter_collection.csv"), "FETCH_SIZE", "copyBuffer")
        d, cmd_cw = rocprof(["--pmc", "WRITE_SIZE"], raw, "copy_write", cal_prog, 120)
        copy_write_kib, _ = per_dispatch(os.path.join(d, "run_counter_collection.csv"), "WRITE_SIZE", "copyBuffer")
    gib = float(1 << 30)
    read_scale = gib / (copy_fetch_kib * 1024.0)
    write_scale = gib / (copy_write_kib * 1024.0)
    read_b = fetch_kib * 1024.0 * read_scale
    write_b = write_kib * 1024.0 * write_scale
    wl = WORKLOAD_NAMES[args.workload]
    # launches of the kernel per step: the trace run's calls over its steps
    # (the served mix is stepped in one launch per group of lattices)
    dps = max(1, round(stats["calls"] / (args.steps + 10)))
    timed_ns = timed_launch_ns(os.path.join(raw, "trace", "run_kernel_trace.csv"), kname, 10, args.steps, dps)
    rec = {"workload": wl, "kernel": kname, "kernel_source_sha256_16": bench.kernel_source_hash(),
           "avg_kernel_ns": timed_ns, "avg_kernel_ns_all_calls": stats["avg_ns"],
           "kernel_calls": stats["calls"] if stats else None,
           "launches_per_step": dps, "kernel_ns_per_step": timed_ns * dps,
           "hbm_bytes_per_step": (read_b + write_b) * dps,
           "event_ms_per_step_same_run": event_ms,
           "fetch_kib_per_dispatch": fetch_kib, "write_kib_per_dispatch": write_kib,
           "copy_fetch_kib_for_1GiB": copy_fetch_kib, "copy_write_kib_for_1GiB": copy_write_kib,
           "read_scale": read_scale, "write_scale": write_scale,
           "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
           "hbm_bytes_per_launch": read_b + write_b,
           "commands": [cmd_trace, cmd_fetch, cmd_write, cmd_cf, cmd_cw]}
    if extra_names:
        rec["other_kernels_of_the_step"] = {
            k: {"avg_kernel_ns": extra_stats[k]["avg_ns"] if extra_stats[k] else None,
                "hbm_read_bytes": extra_fetch[k] * 1024.0 * read_scale if extra_fetch[k] else None,
                "hbm_write_bytes": extra_write[k] * 1024.0 * write_scale if extra_write[k] else None}
            for k in extra_names}
    pdir = os.path.abspath(args.profiles_dir)
    os.makedirs(pdir, exist_ok=True)
    with open(os.path.join(pdir, f"{wl}_pmc.json"), "w") as f:
        json.dump(rec, f, indent=1)
    with open(os.path.join(pdir, f"{wl}_rocprof.md"), "w") as f:
        f.write(f"# rocprofv3 summary: {kname}, workload {wl}\n\n")
        f.write(f"Made by `python -m paper_2609_18177_amd.profile_step --workload {args.workload}` "
                f"(kernel source hash {rec['kernel_source_sha256_16']}); the passes it ran:\n\n")
        for c in rec["commands"]:
            f.write(f"    {c}\n")
        f.write("\n| quantity | value |\n|---|---|\n")
        if stats:
            f.write(f"| kernel calls (trace run) | {stats['calls']} |\n")
            f.write(f"| average kernel duration, timed launches (the warm-up left out) | {timed_ns / 1e3:.2f} us |\n")
            f.write(f"| average kernel duration, all calls | {stats['avg_ns'] / 1e3:.2f} us |\n")
            f.write(f"| min / max duration | {stats['min_ns'] / 1e3:.2f} / {stats['max_ns'] / 1e3:.2f} us |\n")
        if event_ms is not None:
            f.write(f"| bench.py's event-timed time per step, same traced run | {event_ms * 1e3:.2f} us |\n")
        f.write(f"| FETCH_SIZE per dispatch | {fetch_kib:.4g} KiB ({nf} dispatches) |\n")
        f.write(f"| WRITE_SIZE per dispatch | {write_kib:.4g} KiB ({nw} dispatches) |\n")
        f.write(f"| 1 GiB copy: FETCH_SIZE / WRITE_SIZE | {copy_fetch_kib:.4g} / {copy_write_kib:.4g} KiB |\n")
        f.write(f"| calibration (bytes moved / counter bytes) read, write | {read_scale:.3f}, {write_scale:.3f} |\n")
        f.write(f"| HBM read / write per launch (calibrated) | {read_b / 1e6:.1f} / {write_b / 1e6:.1f} MB |\n")
        f.write(f"| HBM bytes per launch | {(read_b + write_b) / 1e6:.1f} MB |\n")
        if dps > 1:
            f.write(f"| launches per step (trace calls / steps) | {dps} |\n")
            f.write(f"| kernel time per step (launches x timed average) | {timed_ns * dps / 1e3:.2f} us |\n")
            f.write(f"| HBM bytes per step | {(read_b + write_b) * dps / 1e6:.1f} MB |\n")
        for k, v in rec.get("other_kernels_of_the_step", {}).items():
            ns = v["avg_kernel_ns"]
            rb, wb = v["hbm_read_bytes"], v["hbm_write_bytes"]
            f.write(f"| other kernel of the step: {k} | {ns / 1e3 if ns else float('nan'):.2f} us, "
                    f"HBM read/write {rb / 1e6 if rb else float('nan'):.1f} / {wb / 1e6 if wb else float('nan'):.1f} MB |\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
