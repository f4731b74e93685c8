#!/usr/bin/env python3
"""DBSCAN throughput on one MI355X: Mpoints/s of the full FDBSCAN path.

Workload (default): the 2^24-point halo field -- half the points in
Plummer-profile halos with a power-law mass function, half uniform, in the
box [0,256)^3 (mean spacing 1), eps = 0.2, minPts = 2 (friends-of-friends).
It stands in for the paper's HACC snapshot benchmark, which is not
available.  One step is one complete ``dbscan_cluster`` call (bounds,
Morton codes, radix sort, BVH build, pair traversal with union-find,
labels) on points already resident in device memory.

Prints one JSON line.  ``roofline`` is for the kernel that takes the most
time per step: algorithmic bytes per launch (points x bytes per point, see
BYTES_PER_POINT) over its average launch time, from HIP events recorded on
the library's stream inside the timed region.  ``cpu_baseline`` times the
CPU oracle (single-threaded C) on the same field and checks the GPU labels
against it bit for bit.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3]

Besides the headline line (plain FDBSCAN on the 2^24-point field) the same
JSON line carries, unless switched off:
  "densebox": the DenseBox variant on the same field;
  "batched":  4,096 independent single-halo sets (~133M points, eps 0.05,
              minPts 5) in one batched call (FDBSCAN, DenseBox, and the
              autotuner's pick, which "batched_ms" times) vs one plain call
              per set;
  "halo134M": the 2^27-point field at minPts 2 and 10 (--no-large skips it);
  "serving":  an open-loop replay of Poisson arrivals (200 jobs/s, sizes
              log-uniform in [1e3, 2^24], minPts in {2,5,10}) through the
              continuous-batching server: p50/p99 latency and Mpoints/s,
              beside a FIFO single-slot replay without batching.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E

# Algorithmic (compulsory) bytes each kernel moves per point, minPts <= 2.
# Reads and writes of whole arrays only; tree nodes count once per point
# (n-1 nodes of 32 bytes); caches, re-reads and atomics are not counted.
BYTES_PER_POINT = {
    "prep": 0.0,
    "bounds": 12.0,                 # read xyz
    "morton": 12.0 + 4.0,           # read xyz, write the code's high half (the halves
                                    # when more than 32 code bits are kept: sort_bytes)
    "sort": 16.0,                   # per pass over the code's high half: read and
                                    # write a 32-bit code word and the index
    "gather": 4 + 12 + 16 + 4 + 4 + 1,  # DenseBox: read index, xyz; write point,
                                        # parent, minlab, flag
    "build_frame": 4 + 12 + 8 + 16 + 32 + 4 + 4 + 1 + 4,  # index, xyz (gathered), codes;
                                  # leaves and nodes out (with ropes), exchange slots of
                                  # pending splits, parent, flag, label -1
    "build_levels": 0.0,            # a few nodes per 256-leaf frame
    "cells": 0.0,                   # DenseBox only
    "count": 16 + 32 + 1,           # leaves, nodes, core flag
    "pairs": 16 + 32 + 4 + 4 + 1,   # leaves, nodes, parent read/write, member flag
    "final_roots": 0.0,             # (the label pass is one kernel with minPts <= 2)
    "final_labels": 1.0,            # member flag; + parent, perm, label for clustered
                                    # points only (labels start at -1 from the build)
}


def sort_bytes(passes: int) -> float:
    """Algorithmic bytes per point of the clustering call's sort with
    `passes` working 8-bit passes (the last ones of 8): a pass over the low
    half of the codes moves a 32-bit code word, the high half and the index
    (24 bytes read and written), the last of them drops the low word (20),
    a pass over the high half moves the high word and the index (16); the
    first pass that runs reads no index (they are the identity)."""
    total = 0.0
    for p in range(8 - passes, 8):
        b = 24.0 if p < 3 else 20.0 if p == 3 else 16.0
        total += b - (4.0 if p == 8 - passes else 0.0)
    return total


def morton_bytes(passes: int) -> float:
    """Read xyz, write the code: both 32-bit halves when the sort runs
    passes over the low half, else the high half alone."""
    return 12.0 + (8.0 if passes > 4 else 4.0)

KERNEL_OF_PHASE = {f"sort{p}": "sort" for p in range(8)}
KERNEL_NAME = {  # device function names, as rocprofv3 reports them
    "sort": "k_onesweep", "pairs": "k_pairs", "build_frame": "k_build_frame",
    "build_levels": "k_build_level", "gather": "k_gather", "cells": "k_cell_stats",
    "morton": "k_morton", "bounds": "k_bounds", "count": "k_count",
    "final_roots": "k_final_roots", "final_labels": "k_final_labels", "prep": "k_prep",
}
KERNEL_SOURCE = {  # files whose text decides the kernel's code (plus common.hpp)
    "sort": "radix_sort.hip", "pairs": ("traverse.hip", "walk.hpp"),
    "count": ("traverse.hip", "walk.hpp"),
    "build_frame": "lbvh.hip", "build_levels": "lbvh.hip",
    "cells": "densebox.hip",
    "gather": "morton.hip", "morton": "morton.hip",
    "bounds": "morton.hip", "prep": "morton.hip", "final_roots": "finalize.hip",
    "final_labels": "finalize.hip",
}
METRIC = "Mpoints/s DBSCAN (16.8M pts, minPts=2) plain vs batched; p50/p99 job latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(kernel: str) -> str:
    srcs = KERNEL_SOURCE[kernel]
    srcs = (srcs,) if isinstance(srcs, str) else srcs
    h = hashlib.sha256()
    for f in (*srcs, "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2409_10743_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, if it was taken on the current source."""
    path = os.path.join(ROOT, "profiles", f"pmc_{KERNEL_NAME[kernel]}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_sha(kernel):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---- rocprofv3 summaries (what profiles/ holds) ------------------------------
# The profiles are taken on the GPU with these commands (from the repository
# root, TMPDIR=/tmp; <OUT> is any scratch folder, each summary names the one
# its command used):
#   rocprofv3 --kernel-trace --stats --output-format csv -d <OUT>/trace_<W> -o run \
#       -- python3 -u bench.py --workload <W> [--algorithm A] --steps 5 --warmup 1 \
#       --no-cpu-baseline --no-extras
#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <OUT>/pmc_FETCH_SIZE_<W> -o run \
#       -- python3 -u bench.py --workload <W> --steps 2 --warmup 1 --no-cpu-baseline --no-extras
#   (the same with WRITE_SIZE), and for the calibration
#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <OUT>/copy_FETCH_SIZE -o run \
#       -- python3 -u bench.py --copy-calibration        (and WRITE_SIZE)
# and summarised with --summarize-trace / --summarize-pmc below.

def _csv_rows(d: str, suffix: str):
    """Rows of every rocprofv3 CSV file under `d` whose name ends in `suffix`."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _col(row: dict, *names):
    for nm in names:
        if nm in row:
            return row[nm]
    raise KeyError(f"none of {names} in {sorted(row)}")


def _short(name: str) -> str:
    """A kernel's name as rocprofv3 prints it, without the return type, the
    namespaces and the parameter list: "k_onesweep<false, 16>"."""
    if name.startswith("void "):
        name = name[5:]
    for ns in ("dbx::(anonymous namespace)::", "dbx::"):
        name = name.replace(ns, "")
    name = name.replace("unsigned long", "u64").replace("unsigned int", "u32")
    depth, cut = 0, len(name)
    for k, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = k
            break
    return name[:cut]


def _kernel_durations(d: str):
    """kernel name -> list of launch durations (us) from a kernel trace."""
    out = {}
    for r in _csv_rows(d, "kernel_trace.csv"):
        name = _short(_col(r, "Kernel_Name", "Name"))
        t = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        out.setdefault(name, []).append(t)
    return out


def _did_work(values, frac=0.25):
    """The launches whose figure is at least `frac` of the largest: a sort
    pass below the code bits eps needs returns at once and is left out."""
    top = max(values) if values else 0.0
    return [v for v in values if v >= frac * top]


def summarize_trace(d: str, workload: str, cmd: str, bench_line: str, out_path: str):
    """Kernel statistics of a rocprofv3 --kernel-trace --stats run."""
    stats = _csv_rows(d, "kernel_stats.csv")
    rows = []
    for r in stats:
        rows.append((_short(_col(r, "Name", "Kernel_Name")), int(_col(r, "Calls")),
                     float(_col(r, "AverageNs")) / 1e3, float(_col(r, "TotalDurationNs")) / 1e6,
                     float(_col(r, "Percentage"))))
    rows.sort(key=lambda x: -x[3])
    lines = [f"# rocprofv3 kernel statistics, {workload}, one MI355X",
             f"# command: {cmd}",
             f"# bench line of the same build: {bench_line}",
             f"{'kernel':<44}{'calls':>7}{'avg_us':>11}{'total_ms':>11}{'pct':>8}"]
    for name, calls, avg, tot, pct in rows[:16]:
        lines.append(f"{name[:43]:<44}{calls:>7}{avg:>11.2f}{tot:>11.3f}{pct:>8.2f}")
    dur = _kernel_durations(d)
    for name in sorted(dur, key=lambda k: -sum(dur[k]))[:6]:
        w = _did_work(dur[name])
        lines.append(f"# {name}: {len(w)} of {len(dur[name])} launches did work, "
                     f"avg {sum(w) / len(w):.2f} us over those")
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _pmc_per_kernel(d: str, counter: str):
    """kernel name -> list of per-dispatch counter values (KiB)."""
    out = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        if _col(r, "Counter_Name") != counter:
            continue
        out.setdefault(_short(_col(r, "Kernel_Name")), []).append(
            float(_col(r, "Counter_Value")))
    return out


def summarize_pmc(fetch_dir: str, write_dir: str, copy_fetch: str, copy_write: str,
                  workload: str, n: int, cmds, kernels, out_dir: str):
    """HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by what the counter reads for a plain 1 GiB
    device copy (1 GiB read, 1 GiB written: --copy-calibration)."""
    copy_bytes = float(1 << 30)
    cf = max(max(v) for v in _pmc_per_kernel(copy_fetch, "FETCH_SIZE").values())
    cw = max(max(v) for v in _pmc_per_kernel(copy_write, "WRITE_SIZE").values())
    f_scale = copy_bytes / (cf * 1024.0)  # bytes per KiB read by the counter
    w_scale = copy_bytes / (cw * 1024.0)
    fetch = _pmc_per_kernel(fetch_dir, "FETCH_SIZE")
    write = _pmc_per_kernel(write_dir, "WRITE_SIZE")
    head = [f"# HBM traffic per kernel launch from rocprofv3 counters, {workload} (n={n}), "
            "one MI355X",
            f"# commands: {cmds[0]}", f"#           {cmds[1]}",
            "# calibration: a plain 1 GiB device copy (bench.py --copy-calibration under "
            "rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)",
            f"#   reads FETCH_SIZE = {1 / f_scale:.4f} x its bytes and WRITE_SIZE = "
            f"{1 / w_scale:.4f} x, so fetched bytes = FETCH_SIZE KiB * 1024 * {f_scale:.4f}, "
            f"written = WRITE_SIZE KiB * 1024 * {w_scale:.4f}",
            "# per launch: averaged over the launches that did work (a skipped sort pass "
            "returns at once)"]
    table = [f"{'kernel':<44}{'launches':>9}{'fetch_KiB':>13}{'write_KiB':>13}{'hbm_MB':>10}"
             f"{'B/point':>9}"]
    per = {}
    for name in sorted(fetch, key=lambda k: -sum(fetch[k])):
        fw = _did_work(fetch[name])
        ww = _did_work(write.get(name, [0.0]))
        fk, wk = sum(fw) / len(fw), sum(ww) / len(ww)
        b = fk * 1024 * f_scale + wk * 1024 * w_scale
        per[name] = (len(fw), fk, wk, b)
        table.append(f"{name[:43]:<44}{len(fw):>9}{fk:>13.1f}{wk:>13.1f}{b / 1e6:>10.1f}"
                     f"{b / n:>9.1f}")
    open(os.path.join(out_dir, f"hbm_traffic_{workload}.txt"), "w").write(
        "\n".join(head + table) + "\n")
    print("\n".join(head + table))
    for k in kernels:  # per-kernel files that bench.py reads for roofline.traffic
        base = KERNEL_NAME[k]
        names = [nm for nm in per if nm.split("<")[0] == base]
        if not names:
            continue
        nm = max(names, key=lambda x: per[x][0] * per[x][3])
        cnt, fk, wk, b = per[nm]
        txt = [f"# HBM bytes per launch of {nm} (averaged over the launches that did work), "
               f"{workload} (n={n})",
               f"# commands: {cmds[0]}", f"#           {cmds[1]}",
               f"# scaled by the 1 GiB copy calibration: FETCH_SIZE x {f_scale:.4f}, "
               f"WRITE_SIZE x {w_scale:.4f}",
               f"# source_sha256 is bench.source_sha('{k}'): the figure is used only while "
               "it matches",
               f"kernel: {base}", f"launches: {cnt}", f"fetch_kib_per_launch: {fk:.1f}",
               f"write_kib_per_launch: {wk:.1f}", f"hbm_bytes_per_launch: {b:.0f}",
               f"hbm_bytes_per_point: {b / n:.2f}", f"source_sha256: {source_sha(k)}"]
        open(os.path.join(out_dir, f"pmc_{base}_{workload}.txt"), "w").write(
            "\n".join(txt) + "\n")


def summarize_counters(d: str, workload: str, cmd: str, out_path: str, kernels=8):
    """Every counter of a rocprofv3 --pmc run, per kernel (sum over the
    launches that did work, divided by their number)."""
    import collections
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in _csv_rows(d, "counter_collection.csv"):
        per[_short(_col(r, "Kernel_Name"))][_col(r, "Counter_Name")].append(
            float(_col(r, "Counter_Value")))
    names = sorted({c for k in per for c in per[k]})
    order = sorted(per, key=lambda k: -max(max(v) for v in per[k].values()))[:kernels]
    lines = [f"# rocprofv3 counters per launch, {workload}, one MI355X", f"# command: {cmd}",
             "kernel" + "".join(f"  {c}" for c in names)]
    for k in order:
        vals = []
        for c in names:
            v = _did_work(per[k].get(c, [0.0]))
            vals.append(sum(v) / len(v))
        lines.append(k + "".join(f"  {x:.4g}" for x in vals))
    if "TCC_HIT_sum" in names and "TCC_MISS_sum" in names:
        for k in order:
            h = sum(per[k]["TCC_HIT_sum"]) or 0.0
            m = sum(per[k]["TCC_MISS_sum"]) or 0.0
            if h + m:
                lines.append(f"# {k}: L2 hit rate {h / (h + m):.3f}")
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def copy_calibration():
    """A plain device copy of known size, for scaling the FETCH_SIZE /
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    n = 1 << 28  # 256 Mi floats = 1 GiB each way
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 3}))


def host_threads() -> int:
    """Host threads for the oracle legs: the CPUs this process may use, at
    most 16 (the host share of one GPU on a shared machine)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="halo16M",
                    choices=["halo16M", "clumps32k", "halo134M", "subhalo4096"])
    ap.add_argument("--min-pts", type=int, default=0, help="0: the workload's own")
    ap.add_argument("--algorithm", default="fdbscan", choices=["fdbscan", "densebox"])
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--pair-count", action="store_true",
                    help="core points by pair traversal (DBSCAN_FLAG_PAIR_COUNT; minPts > 2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline measurement of --workload")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2^27-point field (about a minute of host-side generation)")
    ap.add_argument("--serving-seconds", type=float, default=60.0)
    ap.add_argument("--knn-only", action="store_true",
                    help="only the k-nearest-neighbour leg on --workload (for profiling)")
    ap.add_argument("--mst-only", action="store_true",
                    help="only the minimum-spanning-tree leg on --workload (for profiling)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write profiles/trace_<workload>.txt from a rocprofv3 kernel trace")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH",
                                                         "COPY_WRITE"),
                    help="write profiles/hbm_traffic_<workload>.txt and pmc_*.txt from "
                         "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs and the copy runs")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("DIR", "NAME"),
                    help="write profiles/counters_<NAME>_<workload>.txt from any --pmc run")
    ap.add_argument("--profile-cmd", nargs="*", default=[],
                    help="the command(s) the profile came from, for the summary header")
    ap.add_argument("--bench-line", default="", help="figures of the profiled run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path "
              "is single-GPU by design: run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    tag = args.workload + ("" if args.algorithm == "fdbscan" else "_" + args.algorithm)
    tag += "_knn" if args.knn_only else ""
    tag += "_mst" if args.mst_only else ""
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, tag, " ".join(args.profile_cmd) or "?",
                        args.bench_line, os.path.join(ROOT, "profiles", f"trace_{tag}.txt"))
        return
    if args.summarize_counters:
        d, name = args.summarize_counters
        summarize_counters(d, tag, " ".join(args.profile_cmd) or "?",
                           os.path.join(ROOT, "profiles", f"counters_{name}_{tag}.txt"))
        return
    if args.summarize_pmc:
        import datagen
        n = (int(datagen.subhalo_sets(4096, 4)[1][-1]) if args.workload == "subhalo4096"
             else datagen.CONFIGS[args.workload]["n"])
        cmds = (args.profile_cmd + ["?", "?"])[:2]
        summarize_pmc(*args.summarize_pmc, tag, n, cmds,
                      ("pairs", "sort", "build_frame") if args.algorithm == "fdbscan" else (),
                      os.path.join(ROOT, "profiles"))
        return
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    import datagen
    import paper_2409_10743_amd as dbx

    cfg = datagen.CONFIGS[args.workload]
    eps = np.float32(cfg["eps"])
    mp = args.min_pts or cfg["min_pts"]
    log(f"[bench] generating {args.workload} ...")
    off = None
    if args.workload == "subhalo4096":
        pts, off = datagen.subhalo_sets(cfg["num_sets"], cfg["seed"])
    else:
        pts = datagen.config_points(args.workload)
    n = pts.shape[0]
    d = torch.from_numpy(pts).cuda()
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx = dbx.Context(0)

    def step(**kw):
        if off is None:
            ctx.cluster(d, float(eps), mp, algorithm=args.algorithm, block_size=args.block_size,
                        out=labels, pair_count=args.pair_count, **kw)
        else:
            ctx.cluster_batched(d, off, float(eps), mp, algorithm=args.algorithm,
                                block_size=args.block_size, out=labels,
                                pair_count=args.pair_count, **kw)

    if args.knn_only:
        log("[bench] k nearest neighbours only ...")
        print(json.dumps({"workload": args.workload, "n": n, "knn": bench_knn(ctx, d, pts)}),
              flush=True)
        return
    if args.mst_only:
        log("[bench] minimum spanning trees only ...")
        print(json.dumps({"workload": args.workload, "n": n, "mst": bench_mst(ctx, d, pts)}),
              flush=True)
        return
    log(f"[bench] n={n} eps={float(eps)} minPts={mp} {args.algorithm}: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the timed calls run as a user would call them, without per-kernel
    # events; the per-phase times come from the same number of calls with
    # events (DBSCAN_FLAG_TIMING) right after
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    value = n / (ms / 1000.0) / 1e6
    phase_sum = {k: 0.0 for k in dbx.PHASES}
    for _ in range(args.steps):
        step(timing=True)
        for k, v in ctx.phase_times().items():
            phase_sum[k] += v
    torch.cuda.synchronize()
    phases = {k: v / args.steps for k, v in phase_sum.items()}
    sort_ms = sum(phases[f"sort{p}"] for p in range(8))  # skipped passes included
    passes = ctx.sort_passes() if off is None else 8

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "eps": float(eps), "min_pts": mp,
                   "algorithm": args.algorithm, "pair_count": args.pair_count,
                   "parallelism": "single GPU"},
        "roofline": None,
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "sort_passes": passes,
        "sort_bits": 8 * passes,
        # keys sorted per second over the passes that ran: 8 bits of the key
        # each (the low code bits eps does not need are cleared, not sorted)
        "sort_keys_per_s": round(n / (sort_ms / 1000.0), 1) if sort_ms > 0 else None,
    }
    if off is None and args.algorithm == "fdbscan" and mp <= 2:
        out["roofline"] = roofline(phases, passes, n, args.workload)

    if off is None:
        # the same call replayed as a captured HIP graph (DBSCAN_FLAG_GRAPH) on
        # a side stream: what repeated calls of one shape cost without launch
        # gaps (no per-kernel events in this mode, so the headline stays the
        # eager run)
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            for _ in range(2):
                step(graph=True)
            gs.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step(graph=True)
            gs.synchronize()
            gms = (time.perf_counter() - t0) * 1000.0 / args.steps
        out["graph_replay"] = {"ms_per_step": round(gms, 4),
                               "mpoints_per_s": round(n / gms / 1e3, 2)}
        # node visits of one pair traversal (outside the timed region): what
        # the pairs kernel's time is spent on
        ts = ctx.traversal_stats(d, float(eps))
        out["traversal"] = {k: v for k, v in ts.items()}
        out["traversal"].update({"internal_visits_per_point": round(ts["internal_visits"] / n, 2),
                                 "descents_per_point": round(ts["descents"] / n, 2),
                                 "leaf_tests_per_point": round(ts["leaf_tests"] / n, 2)})
        # logical bytes of the pair walk: every record it reads (32-byte
        # nodes, 16-byte leaves, the query's own leaf) and two union-find
        # words per pair, against the compulsory bytes of the roofline
        logical = (ts["internal_visits"] * 32 + ts["leaf_tests"] * 16 + n * 16 +
                   ts["pairs"] * 8)
        out["traversal"]["logical_bytes"] = int(logical)
        out["traversal"]["compulsory_bytes"] = int(n * BYTES_PER_POINT["pairs"])
        out["tree"] = tree_diagnostics(ctx, d, pts, passes)

    if not args.no_cpu_baseline and off is None:
        out["cpu_baseline"], same = cpu_baseline(pts, eps, mp, labels.cpu().numpy())
        out["parity"] = "bit-exact" if same else "MISMATCH"

    if not args.no_extras and args.workload == "halo16M":
        out["densebox"] = bench_densebox(ctx, d, eps, mp, args.steps, labels)
        # the same figures for the strongly clustered 32,768-point field
        c32 = datagen.config_points("clumps32k")
        dc = torch.from_numpy(c32).cuda()
        ctx.cluster(dc, float(datagen.CONFIGS["clumps32k"]["eps"]), 2, algorithm="fdbscan")
        out["tree_clumps32k"] = tree_diagnostics(ctx, dc, c32, ctx.sort_passes())
        del dc
        log("[bench] k nearest neighbours ...")
        out["knn"] = bench_knn(ctx, d, pts)
        log("[bench] minimum spanning trees ...")
        out["mst"] = bench_mst(ctx, d, pts)
        del d, labels
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(ctx)
        torch.cuda.empty_cache()
        if not args.no_large:
            out["halo134M"] = bench_large(ctx)
            torch.cuda.empty_cache()
        out["serving"] = bench_serving(args.serving_seconds, threads=host_threads())
    print(json.dumps(out), flush=True)


def roofline(phases, passes, n, workload):
    """The roofline object for the kernel with the largest time per step."""
    per_kernel, launches = {}, {}
    for ph, t in phases.items():
        k = KERNEL_OF_PHASE.get(ph, ph)
        per_kernel[k] = per_kernel.get(k, 0.0) + t
        if t > 0:
            launches[k] = launches.get(k, 0) + 1
    # sort passes below the code bits eps needs return at once: the sort's
    # launches are the passes that ran (the last ones)
    ran = [f"sort{p}" for p in range(8 - passes, 8)]
    per_kernel["sort"] = sum(phases[p] for p in ran)
    launches["sort"] = passes
    dom = max(per_kernel, key=per_kernel.get)
    launch_ms = per_kernel[dom] / max(1, launches.get(dom, 1))
    if dom == "sort":
        bytes_launch = n * sort_bytes(passes) / passes
    elif dom == "morton":
        bytes_launch = n * morton_bytes(passes)
    else:
        bytes_launch = n * BYTES_PER_POINT[dom]
    achieved = bytes_launch / (launch_ms / 1000.0) / 1e9
    traffic = measured_traffic(dom, workload)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic, "kernel": KERNEL_NAME[dom],
            "launch_ms": round(launch_ms, 4),
            "algorithmic_bytes_per_launch": int(bytes_launch),
            "traffic_over_algorithmic": (round(traffic / bytes_launch, 2) if traffic else None)}


def cpu_baseline(pts, eps, mp, gpu_labels):
    """The C oracle on the same field on the host: once on one thread, once
    on host_threads() threads (its counting and border steps; the union-find
    merge stays sequential).  Returns (the object, labels identical)."""
    import oracle
    n = pts.shape[0]
    t = host_threads()
    log("[bench] CPU oracle on the same field, 1 thread ...")
    t0 = time.perf_counter()
    ref = oracle.dbscan(pts, eps, mp)
    t_one = time.perf_counter() - t0
    log(f"[bench] CPU oracle on the same field, {t} threads ...")
    oracle.set_threads(t)
    try:
        t0 = time.perf_counter()
        ref_t = oracle.dbscan(pts, eps, mp)
        t_many = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    same = bool(np.array_equal(gpu_labels, ref) and np.array_equal(ref_t, ref))
    return {"value": round(n / t_many / 1e6, 3), "unit": "Mpoints/s", "cores": t,
            "kind": "oracle",
            "sample": f"the whole {n}-point field, one run of the C oracle on {t} host threads "
                      f"({t_many:.1f} s); on one thread {t_one:.1f} s",
            "single_thread_mpoints_per_s": round(n / t_one / 1e6, 3),
            "cpu_model": cpu_model()}, same


def tree_diagnostics(ctx, d, pts, passes):
    """The figures of the paper's table on Morton code width (section
    4.2.2): codes that occur at least twice and more than three times,
    points that share their code with another, the largest multiplicity;
    for the full 63-bit codes and for the codes as the clustering call sorts
    them (the low bits eps does not need cleared: `passes` 8-bit digits
    kept), and the depth of the deepest leaf (edges from the root, plus one)
    of the tree over the full codes."""
    codes = ctx.morton_codes(d).cpu().numpy().view(np.uint64)

    def table(c):
        _, counts = np.unique(c, return_counts=True)
        return {"codes_at_least_twice": int((counts >= 2).sum()),
                "codes_more_than_3_times": int((counts > 3).sum()),
                "points_sharing_a_code": int(counts[counts >= 2].sum()),
                "max_multiplicity": int(counts.max())}

    kept = 8 * passes
    mask = np.uint64(((1 << 64) - 1) ^ ((1 << (64 - kept)) - 1)) if kept < 64 else \
        np.uint64((1 << 64) - 1)
    perm, leaf, nodes, root = ctx.build_tree(d)
    depth = leaf_depth(nodes.cpu().numpy(), int(root.cpu().numpy()[0]), pts.shape[0])
    return {"full_63_bit": table(codes),
            "as_sorted": dict(table(codes & mask), code_bits=max(0, kept - 1)),
            "max_leaf_depth_63_bit": depth}


def leaf_depth(nodes, root, n):
    """Levels (edges + 1) from the root to the deepest leaf of the tree, as
    the library lays it out: internal node k split at g has its left child
    in `left` (leaf g or node g) and its right child g + 1, a leaf exactly
    when g + 1 is the node's last leaf r, which its rope gives (r + 1, or
    the sentinel for the last leaf of the field).  Walked level by level on
    the host."""
    if n <= 1 or root < -1:
        return 1
    rec = nodes.view(np.int32)
    left, rope = rec[:, 3], rec[:, 7]
    frontier = np.array([root], dtype=np.int64)
    levels = 0
    while frontier.size:
        levels += 1
        lref, rp = left[frontier], rope[frontier]
        g = (lref & 0x7fffffff).astype(np.int64)
        last = np.where(rp == -1, n - 1, (rp & 0x7fffffff).astype(np.int64) - 1)
        left_internal = lref >= 0
        right_internal = g + 1 < last
        frontier = np.concatenate([g[left_internal], (g + 1)[right_internal]])
    return levels + 1


def bench_large(ctx, steps=3):
    """The 2^27-point halo field (one GPU's share at production shape) at
    minPts 2 and 10 (the latter also with core points found by pair
    traversal), plain FDBSCAN, points resident in device memory."""
    import torch

    import datagen
    import oracle
    log("[bench] generating halo134M ...")
    cfg = datagen.CONFIGS["halo134M"]
    pts = datagen.config_points("halo134M")
    d = torch.from_numpy(pts).cuda()
    n = d.shape[0]
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    res = {"workload": "halo134M", "n": n, "eps": float(cfg["eps"])}
    for mp, pc in ((2, False), (10, False), (10, True)):
        ctx.cluster(d, float(cfg["eps"]), mp, out=lab, pair_count=pc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.cluster(d, float(cfg["eps"]), mp, out=lab, pair_count=pc)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        res[f"min_pts_{mp}" + ("_pair_count" if pc else "")] = {
            "ms_per_step": round(ms, 3), "mpoints_per_s": round(n / ms / 1e3, 2),
            "clustered_fraction": round(float((lab >= 0).float().mean()), 4)}
        if mp == 2:
            got = lab.cpu().numpy()
    # the oracle on the whole field at minPts 2, on the host's threads: its
    # time, and the GPU labels against it
    threads = host_threads()
    log(f"[bench] oracle on the 2^27-point field, {threads} threads ...")
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        ref = oracle.dbscan(pts, cfg["eps"], 2)
        t_o = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    bad = int((got != ref).sum())
    res["min_pts_2"]["oracle_differing_labels"] = bad
    res["min_pts_2"]["parity"] = "bit-exact" if bad == 0 else "MISMATCH"
    res["cpu_oracle"] = {"min_pts": 2, "mpoints_per_s": round(n / t_o / 1e6, 3),
                         "cores": threads, "seconds": round(t_o, 2)}
    return res


def bench_knn(ctx, d, pts, k=8, min_pts=5, steps=3, rows=300):
    """k nearest neighbours of every point of the field and HDBSCAN*'s core
    distances (section 3.2 nearest search; section 5), timed, with sampled
    rows checked against the brute-force oracle."""
    import torch

    import oracle
    n = d.shape[0]
    res = {"k": k}
    for name, call in (("knn", lambda: ctx.knn(d, k)),
                       ("core_distances", lambda: ctx.core_distances(d, min_pts))):
        out = call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = {"ms_per_call": round(ms, 3), "mpoints_per_s": round(n / ms / 1e3, 2)}
    idx, d2 = ctx.knn(d, k)
    rng = np.random.default_rng(9)
    q = rng.choice(n, rows, replace=False)
    oracle.set_threads(host_threads())
    try:
        ri, rd = oracle.knn(pts, k, q)
    finally:
        oracle.set_threads(1)
    same = bool(np.array_equal(idx.cpu().numpy()[q], ri) and
                np.array_equal(d2.cpu().numpy()[q].view(np.uint32), rd.view(np.uint32)))
    res["sampled_rows_bit_exact"] = same
    res["rows_checked"] = rows
    res["core_distances"]["min_pts"] = min_pts
    return res


def bench_mst(ctx, d, pts, steps=3, min_pts=5, samples=100, subset=20000):
    """Minimum spanning trees of the field (the Euclidean tree of section
    3.2's algorithm list; HDBSCAN*'s mutual reachability tree, section 5),
    timed.  Checked: the Euclidean tree's weights are the binary32 D of its
    ends, it spans the field, and the least edge at each of `samples`
    sampled points (brute force over the whole field) is a tree edge; both
    trees of the first `subset` points equal the oracle's (Prim) bit for bit."""
    import torch
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    import oracle
    n = d.shape[0]
    res = {}
    for name, mp in (("euclidean", 1), ("mutual_reachability", min_pts)):
        e, w = ctx.mst(d, mp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            e, w = ctx.mst(d, mp)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = {"min_pts": mp, "ms_per_call": round(ms, 2),
                     "mpoints_per_s": round(n / ms / 1e3, 2)}
    e, w = ctx.mst(d, 1)
    e, w = e.cpu().numpy().astype(np.int64), w.cpu().numpy()
    lo, hi = e[:, 0], e[:, 1]

    def d2(a, b):
        x = a - b
        x = x * x
        return (x[..., 0] + x[..., 1]) + x[..., 2]
    ok = bool(np.array_equal(w.view(np.uint32), d2(pts[lo], pts[hi]).view(np.uint32)))
    g = coo_matrix((np.ones(n - 1, np.int8), (lo, hi)), shape=(n, n))
    ok = ok and connected_components(g, directed=False)[0] == 1
    tree = set(zip(lo.tolist(), hi.tolist()))
    rng = np.random.default_rng(12)
    for u in rng.choice(n, samples, replace=False).tolist():
        dd = d2(pts, pts[u])
        dd[u] = np.inf
        v = int(np.flatnonzero(dd == dd.min())[0])
        ok = ok and (min(u, v), max(u, v)) in tree
    res["euclidean"]["properties_hold"] = ok
    res["euclidean"]["sampled_points"] = samples
    sub = np.ascontiguousarray(pts[:subset])
    ds = torch.from_numpy(sub).cuda()
    same = True
    t0 = time.perf_counter()
    for mp in (1, min_pts):
        ge, gw = ctx.mst(ds, mp)
        re, rw = oracle.mst(sub, mp)
        same = same and np.array_equal(ge.cpu().numpy(), re) and np.array_equal(
            gw.cpu().numpy().view(np.uint32), rw.view(np.uint32))
    res["oracle_subset"] = {"points": subset, "bit_exact": same,
                            "oracle_seconds_both_trees": round(time.perf_counter() - t0, 2)}
    return res


def bench_densebox(ctx, d, eps, mp, steps, ref_labels):
    import torch
    lab = torch.empty_like(ref_labels)
    for _ in range(2):
        ctx.cluster(d, float(eps), mp, algorithm="densebox", out=lab)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.cluster(d, float(eps), mp, algorithm="densebox", out=lab)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    n = d.shape[0]
    return {"ms_per_step": round(ms, 4), "mpoints_per_s": round(n / ms / 1e3, 2),
            "labels_equal_fdbscan": bool(torch.equal(lab, ref_labels))}


def bench_batched(ctx, steps=3):
    """4,096 sets in one batched call (FDBSCAN, DenseBox, and the option set
    the batched autotuner picks) vs one plain call per set."""
    import torch

    import datagen
    log("[bench] generating subhalo4096 ...")
    cfg = datagen.CONFIGS["subhalo4096"]
    pts, off = datagen.subhalo_sets(cfg["num_sets"], cfg["seed"])
    n = int(off[-1])
    eps, mp = cfg["eps"], cfg["min_pts"]
    d = torch.from_numpy(pts).cuda()
    lab = torch.empty(n, dtype=torch.int32, device="cuda")

    def timed(**kw):
        ctx.cluster_batched(d, off, eps, mp, out=lab, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.cluster_batched(d, off, eps, mp, out=lab, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_f = timed(algorithm="fdbscan")
    lab_f = lab.clone()
    t_d = timed(algorithm="densebox")
    same_d = bool(torch.equal(lab, lab_f))
    t_auto = timed(algorithm="auto")  # the density probe's pick
    ctx.cluster_batched(d, off, eps, mp, out=lab, algorithm="auto", timing=True)
    auto_pick = "densebox" if ctx.phase_times()["cells"] > 0 else "fdbscan"
    log("[bench] batched autotuner ...")
    tuned = ctx.autotune_batched(d, off, eps, mp)
    t_b = timed(algorithm=tuned["algorithm"], block_size=tuned["block_size"],
                dense_threshold=tuned["dense_threshold"], sort_tile=tuned["sort_tile"],
                pair_count=tuned["pair_count"])
    # one call per set, in sequence on one stream (launch overheads included)
    log("[bench] one plain call per set ...")
    eps = float(eps)
    lab2 = torch.empty_like(lab)
    for s in range(8):
        ctx.cluster(d[off[s]:off[s + 1]], eps, mp, out=lab2[off[s]:off[s + 1]])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(len(off) - 1):
        ctx.cluster(d[off[s]:off[s + 1]], eps, mp, out=lab2[off[s]:off[s + 1]])
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    # every set against the oracle, sets spread over the host's threads
    import oracle
    threads = host_threads()
    log(f"[bench] oracle on all {len(off) - 1} sets, {threads} threads ...")
    t0 = time.perf_counter()
    ref = oracle.dbscan_sets(pts, off, cfg["eps"], mp, workers=threads)
    t_o = time.perf_counter() - t0
    bad = {"fdbscan": int((lab_f.cpu().numpy() != ref).sum()),
           "autotuned": int((lab.cpu().numpy() != ref).sum()),
           "per_set_calls": int((lab2.cpu().numpy() != ref).sum())}
    return {"workload": "subhalo4096", "sets": len(off) - 1, "points": n, "eps": float(eps),
            "min_pts": mp, "autotuned": {k: tuned[k] for k in
                                         ("algorithm", "block_size", "dense_threshold",
                                          "sort_tile", "pair_count")},
            "batched_ms": round(t_b * 1e3, 3),
            "batched_mpoints_per_s": round(n / t_b / 1e6, 2),
            "fdbscan_batched_ms": round(t_f * 1e3, 3),
            "densebox_batched_ms": round(t_d * 1e3, 3),
            "auto_batched_ms": round(t_auto * 1e3, 3), "auto_pick": auto_pick,
            "per_set_calls_ms": round(t_p * 1e3, 3),
            "per_set_calls_mpoints_per_s": round(n / t_p / 1e6, 2),
            "speedup": round(t_p / t_b, 2),
            "densebox_equals_fdbscan": same_d,
            "oracle_differing_labels": bad,
            "parity": "bit-exact" if not any(bad.values()) else "MISMATCH",
            "cpu_oracle": {"mpoints_per_s": round(n / t_o / 1e6, 3), "cores": threads,
                           "seconds": round(t_o, 2),
                           "sample": "all sets, one oracle call each, sets spread over "
                                     "host threads"}}


def _replay(server, jobs, pools, ring, keep, saturate=False):
    """Submit `jobs` at their arrival times (open loop; with `saturate`, as
    fast as the label ring allows, all due at once) and wait for them.
    Label buffers come from a ring of pinned host buffers, recycled once a
    job is done; a job in `keep` (job index -> array) writes into its own
    array instead.  Returns (t0, tickets): t0 on the monotonic clock the
    server's job times use, tickets in job order."""
    import collections
    free = collections.deque(range(len(ring)))
    pending = collections.deque()  # (ticket, ring buffer or -1)
    tickets = []
    t0 = time.monotonic()
    for k, j in enumerate(jobs):
        while True:  # recycle finished buffers
            while pending and server.poll(pending[0][0]) is not None:
                b = pending.popleft()[1]
                if b >= 0:
                    free.append(b)
            if free or k in keep:
                break
            server.wait(pending[0][0], 1.0)
        if not saturate:
            delay = t0 + j.t_arrival - time.monotonic()
            if delay > 0:
                time.sleep(delay)
        p = pools[j.pool][j.start:j.start + j.n]
        if k in keep:
            b, out = -1, keep[k]
        else:
            b = free.popleft()
            out = ring[b][:j.n]
        t = server.submit(p, float(j.eps), j.min_pts, out=out)
        pending.append((t, b))
        tickets.append(t)
    for t, _ in pending:
        server.wait(t, -1.0)
    return t0, tickets


def bench_serving(seconds, sat_jobs=1500, small_check=100_000, large_check=30, alone=200,
                  threads=16):
    """Open-loop replay of the serving trace through the continuous-batching
    server and, on the same trace, through one slot without batching (one
    job at a time, FIFO).  Latency runs from each job's scheduled arrival to
    its labels landing in host memory.  A saturating leg submits the first
    `sat_jobs` jobs at once (as fast as 32 label buffers allow) for each
    mode's capacity.  Gates: every job of at most `small_check` points and
    `large_check` random larger ones against the oracle; `alone` random jobs
    identical in the mix and alone (the FIFO replay runs every job alone)."""
    import torch

    import datagen
    import oracle
    import paper_2409_10743_amd as dbx
    log("[bench] generating serving pools ...")
    pools = []
    for k in range(8):
        a = torch.empty((1 << 24, 3), dtype=torch.float32, pin_memory=True)
        a.numpy()[:] = datagen.serving_pool(k)
        pools.append(a.numpy())
    ring = [torch.empty(1 << 24, dtype=torch.int32, pin_memory=True).numpy() for _ in range(32)]
    trace = datagen.serving_trace()
    jobs = [j for j in trace if j.t_arrival < seconds]
    rng = np.random.default_rng(60)
    ids = np.arange(len(jobs))
    sizes = np.array([j.n for j in jobs])
    checked = set(ids[sizes <= small_check].tolist())
    big = ids[sizes > small_check]
    checked |= set(rng.choice(big, min(large_check, big.size), replace=False).tolist())
    alone_ids = set(rng.choice(ids, min(alone, ids.size), replace=False).tolist())
    res = {"trace": "Poisson 200 jobs/s, sizes log-uniform [1e3, 2^24], minPts {2,5,10}, "
                    "eps 0.2 x mean spacing", "seconds": seconds,
           "latency": "labels in host memory minus the job's scheduled arrival"}
    kept = {}
    for slots, cut, key in ((4, 1 << 18, "continuous_batching"), (1, 1, "fifo_one_at_a_time")):
        srv = dbx.Server(0, slots=slots, batch_cut=cut, budget_bytes=200 * 10 ** 9)
        top = max(jobs, key=lambda j: j.n)
        warm = [srv.submit(pools[k][:top.n], float(top.eps), 10, out=ring[k][:top.n])
                for k in range(slots)]  # one per slot: every arena sized for the largest job
        for t in warm:
            srv.wait(t, -1)
        want = alone_ids | (checked if key == "continuous_batching" else set())
        keep = {k: np.empty(jobs[k].n, dtype=np.int32) for k in sorted(want)}
        kept[key] = keep
        log(f"[bench] serving replay {key}: {seconds:.0f} s")
        st0 = srv.stats()
        t0, tickets = _replay(srv, jobs, pools, ring, keep)
        times = [srv.job_times(t) for t in tickets]
        st = srv.stats()
        sub = np.array([a for a, _ in times])
        done = np.array([b for _, b in times])
        due = t0 + np.array([j.t_arrival for j in jobs])
        assert (sub >= t0 - 1e-3).all(), "server clock differs from time.monotonic"
        lat = done - due
        failed = int(st["failed"] - st0["failed"])
        res[key] = {"jobs": len(tickets), "points": int(sizes.sum()),
                    "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                    "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                    "mean_ms": round(float(lat.mean()) * 1e3, 3),
                    "mpoints_per_s": round(float(sizes.sum()) / (done.max() - due[0]) / 1e6, 2),
                    "batched_calls": int(st["batches"] - st0["batches"]),
                    "jobs_in_batches": int(st["batched_jobs"] - st0["batched_jobs"]),
                    "failed": failed}
        # capacity: the first sat_jobs jobs all due at once
        sj = jobs[:sat_jobs]
        st0 = srv.stats()
        log(f"[bench] serving saturation {key}: {len(sj)} jobs at once")
        t0, tickets = _replay(srv, sj, pools, ring, {}, saturate=True)
        done = max(srv.job_times(t)[1] for t in tickets)
        st = srv.stats()
        npts = sum(j.n for j in sj)
        res[key]["saturated"] = {
            "jobs": len(sj), "points": npts, "seconds": round(done - t0, 3),
            "mpoints_per_s": round(npts / (done - t0) / 1e6, 2),
            "jobs_per_s": round(len(sj) / (done - t0), 1),
            "jobs_in_batches": int(st["batched_jobs"] - st0["batched_jobs"])}
        srv.close()
    mix, solo = kept["continuous_batching"], kept["fifo_one_at_a_time"]
    diff = sum(int((mix[k] != solo[k]).sum()) for k in alone_ids)
    res["alone_vs_mix"] = {"jobs": len(alone_ids), "differing_labels": diff}
    log(f"[bench] serving: {len(checked)} jobs against the oracle on {threads} threads ...")
    order = sorted(checked, key=lambda k: -jobs[k].n)
    bad = 0

    def check(k):
        j = jobs[k]
        ref = oracle.dbscan(pools[j.pool][j.start:j.start + j.n], j.eps, j.min_pts)
        return int((ref != mix[k]).sum())

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        bad = sum(ex.map(check, order))
    res["oracle_check"] = {"jobs": len(checked),
                           "rule": f"every job of at most {small_check} points and "
                                   f"{large_check} random larger ones",
                           "points": int(sum(jobs[k].n for k in checked)),
                           "differing_labels": bad}
    return res


if __name__ == "__main__":
    main()
