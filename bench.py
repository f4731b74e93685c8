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
    "morton": 12.0 + 8.0,           # read xyz, write code
    "sort": 24.0,                   # per pass: read code+index, write code+index
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
# the first sort pass reads no values (they are the identity)
FIRST_SORT_PASS_BYTES = 20.0

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="halo16M", choices=["halo16M", "clumps32k"])
    ap.add_argument("--min-pts", type=int, default=2)
    ap.add_argument("--algorithm", default="fdbscan", choices=["fdbscan"])
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline plain FDBSCAN measurement")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2^27-point field (about a minute of host-side generation)")
    ap.add_argument("--serving-seconds", type=float, default=60.0)
    ap.add_argument("--baseline-seconds", type=float, default=20.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path "
              "is single-GPU by design: run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    import datagen
    import paper_2409_10743_amd as dbx

    cfg = datagen.CONFIGS[args.workload]
    eps = np.float32(cfg["eps"])
    mp = args.min_pts
    log(f"[bench] generating {args.workload} ...")
    pts = datagen.config_points(args.workload)
    n = pts.shape[0]
    d = torch.from_numpy(pts).cuda()
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx = dbx.Context(0)
    log(f"[bench] n={n} eps={float(eps)} minPts={mp}: warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.cluster(d, float(eps), mp, algorithm=args.algorithm, block_size=args.block_size,
                    timing=True, out=labels)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    phase_sum = {k: 0.0 for k in dbx.PHASES}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.cluster(d, float(eps), mp, algorithm=args.algorithm, block_size=args.block_size,
                    timing=True, out=labels)
        for k, v in ctx.phase_times().items():
            phase_sum[k] += v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    value = n / (ms / 1000.0) / 1e6
    phases = {k: v / args.steps for k, v in phase_sum.items()}

    # group launches by kernel, pick the one with the largest time per step
    per_kernel, launches = {}, {}
    for ph, t in phases.items():
        k = KERNEL_OF_PHASE.get(ph, ph)
        per_kernel[k] = per_kernel.get(k, 0.0) + t
        if t > 0:
            launches[k] = launches.get(k, 0) + 1
    # sort passes below the code bits eps needs return at once: the sort's
    # launches are the passes that ran (the last ones)
    passes = ctx.sort_passes()
    ran = [f"sort{p}" for p in range(8 - passes, 8)]
    per_kernel["sort"] = sum(phases[p] for p in ran)
    launches["sort"] = passes
    dom = max(per_kernel, key=per_kernel.get)
    launch_ms = per_kernel[dom] / max(1, launches.get(dom, 1))
    if dom == "sort":
        bytes_launch = n * (FIRST_SORT_PASS_BYTES + (passes - 1) * BYTES_PER_POINT["sort"]) / passes
    else:
        bytes_launch = n * BYTES_PER_POINT[dom]
    achieved = bytes_launch / (launch_ms / 1000.0) / 1e9
    traffic = measured_traffic(dom, args.workload)
    sort_ms = sum(phases[f"sort{p}"] for p in range(8))  # skipped passes included

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "eps": float(eps), "min_pts": mp,
                   "algorithm": args.algorithm, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "kernel": KERNEL_NAME[dom],
                     "launch_ms": round(launch_ms, 4),
                     "algorithmic_bytes_per_launch": int(bytes_launch)},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "sort_keys_per_s": round(n / (sort_ms / 1000.0), 1) if sort_ms > 0 else None,
        "sort_passes": passes,
    }

    # the same call replayed as a captured HIP graph (DBSCAN_FLAG_GRAPH) on a
    # side stream: what repeated calls of one shape cost without launch gaps
    # (no per-kernel events in this mode, so the headline stays the eager run)
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        for _ in range(2):
            ctx.cluster(d, float(eps), mp, algorithm=args.algorithm, block_size=args.block_size,
                        out=labels, graph=True)
        gs.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.cluster(d, float(eps), mp, algorithm=args.algorithm, block_size=args.block_size,
                        out=labels, graph=True)
        gs.synchronize()
        gms = (time.perf_counter() - t0) * 1000.0 / args.steps
    out["graph_replay"] = {"ms_per_step": round(gms, 4), "mpoints_per_s": round(n / gms / 1e3, 2)}

    # node visits of one pair traversal (outside the timed region): what the
    # pairs kernel's time is spent on
    ts = ctx.traversal_stats(d, float(eps))
    out["traversal"] = {k: v for k, v in ts.items()}
    out["traversal"].update({"internal_visits_per_point": round(ts["internal_visits"] / n, 2),
                             "descents_per_point": round(ts["descents"] / n, 2),
                             "leaf_tests_per_point": round(ts["leaf_tests"] / n, 2)})

    if not args.no_cpu_baseline:
        import oracle
        log("[bench] CPU oracle on the same field ...")
        t0 = time.perf_counter()
        ref = oracle.dbscan(pts, eps, mp)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(n / t_cpu / 1e6, 3), "unit": "Mpoints/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the whole {n}-point field, one run of the single-threaded C oracle "
                      f"({t_cpu:.1f} s)"}
        same = bool(np.array_equal(labels.cpu().numpy(), ref))
        out["parity"] = "bit-exact" if same else "MISMATCH"

    if not args.no_extras and args.workload == "halo16M":
        out["densebox"] = bench_densebox(ctx, d, eps, mp, args.steps, labels)
        del d, labels
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(ctx)
        torch.cuda.empty_cache()
        if not args.no_large:
            out["halo134M"] = bench_large(ctx)
            torch.cuda.empty_cache()
        out["serving"] = bench_serving(args.serving_seconds, args.baseline_seconds)
    print(json.dumps(out), flush=True)


def bench_large(ctx, steps=3):
    """The 2^27-point halo field (one GPU's share at production shape) at
    minPts 2 and 10 (the latter also with core points found by pair
    traversal), plain FDBSCAN, points resident in device memory."""
    import torch

    import datagen
    log("[bench] generating halo134M ...")
    cfg = datagen.CONFIGS["halo134M"]
    d = torch.from_numpy(datagen.config_points("halo134M")).cuda()
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
    eps, mp = float(cfg["eps"]), cfg["min_pts"]
    d = torch.from_numpy(pts).cuda()
    del pts
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
    log("[bench] batched autotuner ...")
    tuned = ctx.autotune_batched(d, off, eps, mp)
    t_b = timed(algorithm=tuned["algorithm"], block_size=tuned["block_size"],
                dense_threshold=tuned["dense_threshold"], sort_tile=tuned["sort_tile"])
    same_t = bool(torch.equal(lab, lab_f))
    # one call per set, in sequence on one stream (launch overheads included)
    log("[bench] one plain call per set ...")
    lab2 = torch.empty_like(lab)
    for s in range(8):
        ctx.cluster(d[off[s]:off[s + 1]], eps, mp, out=lab2[off[s]:off[s + 1]])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(len(off) - 1):
        ctx.cluster(d[off[s]:off[s + 1]], eps, mp, out=lab2[off[s]:off[s + 1]])
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    # per-set labels are set-local in both
    same = bool(torch.equal(lab_f, lab2))
    return {"workload": "subhalo4096", "sets": len(off) - 1, "points": n, "eps": eps,
            "min_pts": mp, "autotuned": {k: tuned[k] for k in
                                         ("algorithm", "block_size", "dense_threshold",
                                                  "sort_tile")},
            "batched_ms": round(t_b * 1e3, 3),
            "batched_mpoints_per_s": round(n / t_b / 1e6, 2),
            "fdbscan_batched_ms": round(t_f * 1e3, 3),
            "densebox_batched_ms": round(t_d * 1e3, 3),
            "per_set_calls_ms": round(t_p * 1e3, 3),
            "per_set_calls_mpoints_per_s": round(n / t_p / 1e6, 2),
            "speedup": round(t_p / t_b, 2), "labels_equal": same and same_d and same_t}


def _replay(server, jobs, pools, seconds, pinned_labels):
    """Submit jobs at their arrival times (open loop) for `seconds`; returns
    the tickets.  Label buffers come from a ring of pinned host buffers and
    are recycled once a job is done."""
    import collections
    free = collections.deque(range(len(pinned_labels)))
    pending = collections.deque()
    tickets = []
    t0 = time.perf_counter()
    for j in jobs:
        if j.t_arrival > seconds:
            break
        while True:  # recycle finished buffers
            while pending and server.poll(pending[0][0]) is not None:
                free.append(pending.popleft()[1])
            if free:
                break
            server.wait(pending[0][0], 1.0)
        delay = t0 + j.t_arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        b = free.popleft()
        p = pools[j.pool][j.start:j.start + j.n]
        t = server.submit(p, float(j.eps), j.min_pts, out=pinned_labels[b][:j.n])
        pending.append((t, b))
        tickets.append(t)
    for t, _ in pending:
        server.wait(t, -1.0)
    return tickets


def bench_serving(seconds, baseline_seconds):
    import torch

    import datagen
    import paper_2409_10743_amd as dbx
    log("[bench] generating serving pools ...")
    pools = []
    for k in range(8):
        a = torch.empty((1 << 24, 3), dtype=torch.float32, pin_memory=True)
        a.numpy()[:] = datagen.serving_pool(k)
        pools.append(a.numpy())
    ring = [torch.empty(1 << 24, dtype=torch.int32, pin_memory=True).numpy() for _ in range(24)]
    jobs = datagen.serving_trace()
    res = {"trace": "Poisson 200 jobs/s, sizes log-uniform [1e3, 2^24], minPts {2,5,10}, "
                    "eps 0.2 x mean spacing", "seconds": seconds}
    # warm the device arenas with the largest job size
    big = max(jobs, key=lambda j: j.n)
    for slots, cut, key, secs in ((4, 1 << 18, "continuous_batching", seconds),
                                  (1, 1, "fifo_one_at_a_time", baseline_seconds)):
        srv = dbx.Server(0, slots=slots, batch_cut=cut, budget_bytes=200 * 10 ** 9)
        warm = [srv.submit(pools[k][:big.n], float(big.eps), 10, out=ring[k][:big.n])
                for k in range(slots)]  # one per slot: every arena sized for the largest job
        for t in warm:
            srv.wait(t, -1)
        log(f"[bench] serving replay {key}: {secs:.0f} s")
        tickets = _replay(srv, jobs, pools, secs, ring)
        lat = np.array([np.subtract(*srv.job_times(t)[::-1]) for t in tickets])
        npts = sum(j.n for j in jobs[:len(tickets)])
        t_first = srv.job_times(tickets[0])[0]
        t_last = max(srv.job_times(t)[1] for t in tickets)
        st = srv.stats()
        res[key] = {"jobs": len(tickets), "seconds_of_trace": secs,
                    "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                    "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                    "mpoints_per_s": round(npts / (t_last - t_first) / 1e6, 2),
                    "batched_calls": st["batches"], "jobs_in_batches": st["batched_jobs"],
                    "failed": st["failed"]}
        srv.close()
    return res


if __name__ == "__main__":
    main()
