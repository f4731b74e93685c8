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
    "gather": 4 + 12 + 16 + 4 + 4 + 1 + 4,  # read perm, xyz; write leaf, parent,
                                            # minlab, flag, build slot
    "build": 8 + 16 + 32 + 4 + 4,   # codes, leaves, node, right child, slot
    "ropes": 4 + 4 + 4 + 4,         # range end, right child, rope (nodes + leaves)
    "count": 16 + 32 + 1,           # leaves, nodes, core flag
    "pairs": 16 + 32 + 4 + 4 + 1,   # leaves, nodes, parent read/write, member flag
    "final_roots": 1 + 4 + 4 + 4 + 4,
    "final_labels": 4 + 4 + 4 + 4,
}
# the first sort pass reads no values (they are the identity)
FIRST_SORT_PASS_BYTES = 20.0

KERNEL_OF_PHASE = {f"sort{p}": "sort" for p in range(8)}
KERNEL_NAME = {  # device function names, as rocprofv3 reports them
    "sort": "k_onesweep", "pairs": "k_pairs", "build": "k_build", "gather": "k_gather",
    "morton": "k_morton", "bounds": "k_bounds", "ropes": "k_ropes", "count": "k_count",
    "final_roots": "k_final_roots", "final_labels": "k_final_labels", "prep": "k_prep",
}
KERNEL_SOURCE = {
    "sort": "radix_sort.hip", "pairs": "traverse.hip", "count": "traverse.hip",
    "build": "lbvh.hip", "ropes": "lbvh.hip", "gather": "morton.hip", "morton": "morton.hip",
    "bounds": "morton.hip", "prep": "morton.hip", "final_roots": "finalize.hip",
    "final_labels": "finalize.hip",
}
METRIC = "Mpoints/s DBSCAN (16.8M pts, minPts=2) plain vs batched; p50/p99 job latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(kernel: str) -> str:
    src = os.path.join(ROOT, "paper_2409_10743_amd", "csrc", KERNEL_SOURCE[kernel])
    h = hashlib.sha256()
    for f in (src, os.path.join(ROOT, "paper_2409_10743_amd", "csrc", "common.hpp")):
        h.update(open(f, "rb").read())
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
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path "
              "is single-GPU by design and multi-GPU runs are not part of this build",
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
    dom = max(per_kernel, key=per_kernel.get)
    launch_ms = per_kernel[dom] / max(1, launches.get(dom, 1))
    if dom == "sort":
        bytes_launch = n * (FIRST_SORT_PASS_BYTES + 7 * BYTES_PER_POINT["sort"]) / 8.0
    else:
        bytes_launch = n * BYTES_PER_POINT[dom]
    achieved = bytes_launch / (launch_ms / 1000.0) / 1e9
    traffic = measured_traffic(dom, args.workload)
    sort_ms = sum(phases[f"sort{p}"] for p in range(8))

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
    }

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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
