"""CPU oracle for the DBSCAN hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it; it shares no code
with the GPU path (its C source is compiled by gcc on its own).

Functions
---------
dbscan(points, eps, min_pts)      labels, section 3.1 definition (C, grid +
                                  sequential union-find, see dbscan_oracle.c)
core_flags(points, eps, min_pts)  |N_eps(x)| >= minPts per point (C)
neighbour_counts(points, eps)     |N_eps(x)| per point, self included (C)
pair_count(points, eps)           number of unordered eps-pairs (C)
set_threads(t)                    host threads of the counting and border
                                  steps (default 1)
dbscan_sets(points, offsets, ...) independent sets, each clustered alone,
                                  sets spread over host threads
knn(points, k, queries)           k nearest neighbours, self included, ties
                                  to the smaller index (C, brute force)
core_distances(points, min_pts)   squared distance to the min_pts-th nearest
mst(points, min_pts)              minimum spanning tree: Euclidean for
                                  min_pts <= 1, else of HDBSCAN*'s mutual
                                  reachability graph (C, Prim, O(n^2))
morton63(points)                  the 63-bit Morton code of every point,
                                  section 4.2.2 (numpy, plain definition)
morton_order(codes)               stable sort permutation of the codes
                                  (numpy's stable argsort)

Status codes mirror the library's: 0 ok, -1 invalid argument, -2 non-finite
coordinate, -3 out of memory.

Pins: the C functions by tests/test_oracle_pins.py (brute force, hand cases,
binary32 boundary cases, metamorphic relations, planted mistakes); the
Morton functions by tests/test_oracle_morton_pins.py (codes worked out by
hand, binary32 grid coordinates decided with exact rationals, a de-interleave
round trip, planted mistakes); the spanning trees by
tests/test_oracle_mst_pins.py (every spanning tree of tiny inputs, scipy's
minimum spanning tree, the cycle property, closed forms, planted mistakes).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dbscan_oracle.c")
_KNN_SRC = os.path.join(_HERE, "knn_oracle.c")
_MST_SRC = os.path.join(_HERE, "mst_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

# The predicate must be evaluated exactly as written: no contraction into
# fused multiply-adds, no fast-math, subnormals kept (x86-64 SSE, no -m flags).
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(extra_flags=(), out=None) -> str:
    """Compile the oracle with gcc; returns the path of the shared object."""
    out = out or _LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, *extra_flags, _SRC, _KNN_SRC, _MST_SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__({-1: "invalid argument", -2: "non-finite coordinate",
                          -3: "out of memory"}.get(code, f"status {code}"))
        self.code = code


def load(path: str | None = None) -> ctypes.CDLL:
    path = path or _LIB
    if not os.path.exists(path):
        build(out=path)
    lib = ctypes.CDLL(path)
    f32p = ctypes.POINTER(ctypes.c_float)
    lib.oracle_dbscan.argtypes = [f32p, ctypes.c_int64, ctypes.c_float,
                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_uint8)]
    lib.oracle_dbscan.restype = ctypes.c_int
    lib.oracle_neighbour_counts.argtypes = [f32p, ctypes.c_int64, ctypes.c_float,
                                            ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_neighbour_counts.restype = ctypes.c_int
    lib.oracle_pair_count.argtypes = [f32p, ctypes.c_int64, ctypes.c_float,
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_pair_count.restype = ctypes.c_int
    lib.oracle_version.restype = ctypes.c_char_p
    lib.oracle_knn.argtypes = [f32p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                               ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                               f32p]
    lib.oracle_knn.restype = ctypes.c_int
    lib.oracle_mst.argtypes = [f32p, ctypes.c_int64, f32p, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), f32p]
    lib.oracle_mst.restype = ctypes.c_int
    lib.knn_set_threads.argtypes = [ctypes.c_int]
    lib.knn_set_threads.restype = ctypes.c_int
    lib.knn_set_threads(1)
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    lib.oracle_set_threads(1)  # sequential unless asked otherwise
    return lib


_lib = None


def _get():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _as_points(points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.float32)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("points must be float32[N,3]")
    return p


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def dbscan(points, eps, min_pts, lib=None, return_core=False):
    """Labels (int32[N], -1 for noise, else the smallest member index)."""
    lib = lib or _get()
    p = _as_points(points)
    n = p.shape[0]
    lab = np.empty(n, dtype=np.int32)
    core = np.empty(n, dtype=np.uint8)
    st = lib.oracle_dbscan(_ptr(p, ctypes.c_float), n, ctypes.c_float(eps),
                           int(min_pts), _ptr(lab, ctypes.c_int32),
                           _ptr(core, ctypes.c_uint8))
    if st != 0:
        raise OracleError(st)
    return (lab, core.astype(bool)) if return_core else lab


def dbscan_sets(points, offsets, eps, min_pts, workers: int = 1, lib=None) -> np.ndarray:
    """Labels of independent sets points[offsets[k]:offsets[k+1]], each
    clustered alone (set-local indices), with eps and min_pts scalars or one
    value per set.  `workers` host threads take sets in turn (each call
    sequential inside); the result does not depend on it."""
    from concurrent.futures import ThreadPoolExecutor
    p = _as_points(points)
    off = np.asarray(offsets, dtype=np.int64)
    k = off.size - 1
    e = np.broadcast_to(np.asarray(eps, dtype=np.float32), (k,))
    m = np.broadcast_to(np.asarray(min_pts, dtype=np.int64), (k,))
    out = np.empty(int(off[-1]), dtype=np.int32)

    def one(s):
        a, b = int(off[s]), int(off[s + 1])
        out[a:b] = dbscan(p[a:b], e[s], int(m[s]), lib=lib)

    if workers <= 1:
        for s in range(k):
            one(s)
    else:  # largest sets first, so the last ones to finish are small
        order = np.argsort(-np.diff(off), kind="stable")
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, order.tolist()))
    return out


def set_threads(t: int, lib=None) -> int:
    """Host threads of the counting and border steps (the union-find merge is
    always sequential) and of the kNN queries; 1 by default.  Results do not
    depend on it."""
    lib = lib or _get()
    lib.knn_set_threads(int(t))
    return int(lib.oracle_set_threads(int(t)))


def knn(points, k: int, queries=None, lib=None):
    """k nearest neighbours of each query (all points, or the given point
    indices), the query itself included: (indices int32[nq, k], squared
    distances float32[nq, k]) in increasing (D, index) order; -1 / inf past
    the number of points.  See knn_oracle.c."""
    lib = lib or _get()
    p = _as_points(points)
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = p.shape[0] if q is None else q.size
    idx = np.empty((nq, int(k)), dtype=np.int32)
    d2 = np.empty((nq, int(k)), dtype=np.float32)
    st = lib.oracle_knn(_ptr(p, ctypes.c_float), p.shape[0],
                        None if q is None else _ptr(q, ctypes.c_int64), nq, int(k),
                        _ptr(idx, ctypes.c_int32), _ptr(d2, ctypes.c_float))
    if st != 0:
        raise OracleError(st)
    return idx, d2


def core_distances(points, min_pts: int, queries=None, lib=None) -> np.ndarray:
    """HDBSCAN*'s core distance, squared: D to the min_pts-th nearest
    neighbour, the point itself counted (inf if there are fewer points)."""
    return knn(points, min_pts, queries, lib)[1][:, int(min_pts) - 1].copy()


def mst(points, min_pts: int = 1, core=None, lib=None):
    """Minimum spanning tree of the complete graph with weights
    max(c_i, c_j, D(i, j)), c the squared core distances at min_pts (none
    for min_pts <= 1: the Euclidean tree) or the given `core`.  Returns
    (edges int32[n-1, 2] as (lo, hi) input indices, squared weights
    float32[n-1]) in increasing (w, lo, hi) order.  See mst_oracle.c."""
    lib = lib or _get()
    p = _as_points(points)
    n = p.shape[0]
    if core is None and int(min_pts) > 1 and n > 0:
        core = core_distances(p, int(min_pts), lib=lib)
    c = None if core is None else np.ascontiguousarray(core, dtype=np.float32)
    m = max(n - 1, 0)
    lo = np.empty(m, dtype=np.int32)
    hi = np.empty(m, dtype=np.int32)
    w = np.empty(m, dtype=np.float32)
    st = lib.oracle_mst(_ptr(p, ctypes.c_float), n, None if c is None else _ptr(c, ctypes.c_float),
                        _ptr(lo, ctypes.c_int32), _ptr(hi, ctypes.c_int32),
                        _ptr(w, ctypes.c_float))
    if st != 0:
        raise OracleError(st)
    return np.stack([lo, hi], axis=1), w


def core_flags(points, eps, min_pts, lib=None) -> np.ndarray:
    return neighbour_counts(points, eps, lib) >= int(min_pts)


def neighbour_counts(points, eps, lib=None) -> np.ndarray:
    lib = lib or _get()
    p = _as_points(points)
    cnt = np.empty(p.shape[0], dtype=np.int64)
    st = lib.oracle_neighbour_counts(_ptr(p, ctypes.c_float), p.shape[0],
                                     ctypes.c_float(eps), _ptr(cnt, ctypes.c_int64))
    if st != 0:
        raise OracleError(st)
    return cnt


def pair_count(points, eps, lib=None) -> int:
    lib = lib or _get()
    p = _as_points(points)
    out = ctypes.c_int64(0)
    st = lib.oracle_pair_count(_ptr(p, ctypes.c_float), p.shape[0],
                               ctypes.c_float(eps), ctypes.byref(out))
    if st != 0:
        raise OracleError(st)
    return int(out.value)


# ---- Morton codes (section 4.2.2), plain definition in numpy -------------

MORTON_BITS = 21  # per axis: 3 x 21 = 63 bits of a 64-bit code


def morton_quantise(points) -> np.ndarray:
    """Per-axis grid coordinate q_a = min(floor((p_a - lo_a) * s_a), 2^21-1)
    with s_a = 2^21 / (hi_a - lo_a) (s_a = 0 for a zero extent), all in
    float32, where lo/hi are the per-axis min/max of the points (the scene
    bounding volume of section 3.2)."""
    p = _as_points(points)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    ext = (hi - lo).astype(np.float32)
    s = np.zeros(3, dtype=np.float32)
    nz = ext > 0
    s[nz] = np.float32(1 << MORTON_BITS) / ext[nz]
    t = (p - lo).astype(np.float32) * s
    q = np.floor(t).astype(np.int64)
    return np.minimum(q, (1 << MORTON_BITS) - 1).astype(np.uint64)


def morton63(points) -> np.ndarray:
    """63-bit Morton code: bit b of the x, y, z grid coordinates goes to bit
    3b+2, 3b+1, 3b of the code."""
    q = morton_quantise(points)
    code = np.zeros(q.shape[0], dtype=np.uint64)
    for b in range(MORTON_BITS):
        for a in range(3):
            bit = (q[:, a] >> np.uint64(b)) & np.uint64(1)
            code |= bit << np.uint64(3 * b + 2 - a)
    return code


def morton_order(codes) -> np.ndarray:
    """Permutation sorting the codes, ties kept in input order."""
    return np.argsort(np.asarray(codes), kind="stable")
