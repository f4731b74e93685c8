"""MI355X-native DBSCAN (FDBSCAN, section 4.3.3 of "Advances in ArborX to
support exascale applications"), Python binding of the C ABI declared in
``include/dbscan_mi355x.h``.

Argument marshalling only: every step of the clustering runs in the HIP
kernels of ``libdbscan_mi355x.so``.  PyTorch supplies device memory and the
current stream.  If the shared library is missing the import of any entry
point raises: there is no CPU fallback.

    import torch, paper_2409_10743_amd as dbx
    labels = dbx.cluster(points_cuda_f32_nx3, eps=0.2, min_pts=2)
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["cluster", "cluster_noalloc", "Context", "Server", "DbscanError", "library_path",
           "load_library", "PHASES", "ALGO", "NOALLOC_MAX_POINTS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libdbscan_mi355x.so"

ALGO = {"auto": 0, "fdbscan": 1, "densebox": 2}
ALGO_NAME = {v: k for k, v in ALGO.items()}
FLAG_TIMING = 1
FLAG_GRAPH = 2
FLAG_PAIR_COUNT = 4
STATUS = {0: "ok", -1: "invalid argument", -2: "non-finite coordinate",
          -3: "out of device memory", -4: "device error", -5: "job exceeds budget"}


def library_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


class DbscanError(RuntimeError):
    def __init__(self, code: int, detail: str = ""):
        super().__init__(f"{STATUS.get(code, code)} ({code}): {detail}")
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("algorithm", ctypes.c_int32), ("dense_threshold", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("sort_tile", ctypes.c_int32)]


class _ServerOptions(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("batch_cut", ctypes.c_int64),
                ("batch_max_points", ctypes.c_int64), ("batch_max_jobs", ctypes.c_int32),
                ("fake_executor", ctypes.c_int32), ("fake_us_per_mpoint", ctypes.c_double)]


class _ServingStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("points", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("batched_jobs", ctypes.c_uint64),
                ("peak_in_flight_bytes", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("mpoints_per_s", ctypes.c_double)]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2409_10743_amd.csrc.build`")
    L = ctypes.CDLL(path)
    vp, i64, i32, f32, u64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_float, ctypes.c_uint64)
    sig = {
        "dbscan_ctx_create": ([ctypes.c_int, u64, ctypes.POINTER(vp)], ctypes.c_int),
        "dbscan_ctx_destroy": ([vp], ctypes.c_int),
        "dbscan_scratch_bytes": ([i64, i32, i32], u64),
        "dbscan_cluster": ([vp, i64, f32, i32, vp, vp], ctypes.c_int),
        "dbscan_cluster_ex": ([vp, vp, i64, f32, i32, vp, vp, ctypes.POINTER(_Options)],
                              ctypes.c_int),
        "dbscan_cluster_host": ([vp, i64, f32, i32, vp], ctypes.c_int),
        "dbscan_cluster_noalloc": ([vp, i64, f32, i32, vp, vp], ctypes.c_int),
        "dbscan_cluster_batched": ([vp, vp, ctypes.POINTER(i64), i32, ctypes.POINTER(f32),
                                    ctypes.POINTER(i32), vp, vp, ctypes.POINTER(_Options)],
                                   ctypes.c_int),
        "dbscan_phase_times": ([vp, ctypes.POINTER(f32), i32], ctypes.c_int),
        "dbscan_phase_name": ([i32], ctypes.c_char_p),
        "dbscan_sort_passes": ([vp], ctypes.c_int),
        "dbscan_morton_codes": ([vp, vp, i64, vp, vp], ctypes.c_int),
        "dbscan_sort_pairs": ([vp, vp, vp, i64, vp], ctypes.c_int),
        "dbscan_build_tree": ([vp, vp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "dbscan_core_flags": ([vp, vp, i64, f32, i32, vp, vp], ctypes.c_int),
        "dbscan_pair_count": ([vp, vp, i64, f32, ctypes.POINTER(i64), vp], ctypes.c_int),
        "dbscan_traversal_stats": ([vp, vp, i64, f32, ctypes.POINTER(i64), vp], ctypes.c_int),
        "dbscan_server_create": ([ctypes.POINTER(_ServerOptions), ctypes.POINTER(vp)],
                                 ctypes.c_int),
        "dbscan_server_submit": ([vp, vp, i64, f32, i32, vp, ctypes.POINTER(u64)], ctypes.c_int),
        "dbscan_server_poll": ([vp, u64, ctypes.POINTER(i32)], ctypes.c_int),
        "dbscan_server_wait": ([vp, u64, ctypes.c_double, ctypes.POINTER(i32)], ctypes.c_int),
        "dbscan_server_job_times": ([vp, u64, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "dbscan_server_stats": ([vp, ctypes.POINTER(_ServingStats)], ctypes.c_int),
        "dbscan_server_destroy": ([vp], ctypes.c_int),
        "dbscan_autotune": ([vp, vp, i64, f32, i32, i32, vp, ctypes.POINTER(_Options),
                             ctypes.POINTER(f32), vp], ctypes.c_int),
        "dbscan_autotune_batched": ([vp, vp, ctypes.POINTER(i64), i32, ctypes.POINTER(f32),
                                     ctypes.POINTER(i32), vp, ctypes.POINTER(_Options),
                                     ctypes.POINTER(f32), vp], ctypes.c_int),
        "dbscan_knn": ([vp, vp, i64, i32, vp, vp, vp], ctypes.c_int),
        "dbscan_core_distances": ([vp, vp, i64, i32, vp, vp], ctypes.c_int),
        "dbscan_mst": ([vp, vp, i64, i32, vp, vp, vp], ctypes.c_int),
        "dbscan_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "dbscan_last_error": ([], ctypes.c_char_p),
        "dbscan_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(code: int):
    if code != 0:
        raise DbscanError(code, load_library().dbscan_last_error().decode())


def _torch():
    import torch
    return torch


def _points(points):
    torch = _torch()
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
        raise TypeError("points must be float32 [N, 3]")
    return points.contiguous()


def _labels_out(out, n: int, device):
    """The label buffer of a call: a new int32 tensor, or the caller's `out`,
    which must be an int32 tensor on the points' device, contiguous and
    holding at least n elements (the library writes n labels through the
    bare pointer and cannot check its size)."""
    torch = _torch()
    if out is None:
        return torch.empty(n, dtype=torch.int32, device=device)
    if not isinstance(out, torch.Tensor):
        raise TypeError("out must be a torch tensor")
    if out.dtype != torch.int32:
        raise TypeError(f"out must be int32, not {out.dtype}")
    if out.device != torch.device(device):
        raise ValueError(f"out is on {out.device}, the points on {device}")
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    if out.numel() < n:
        raise ValueError(f"out holds {out.numel()} labels, {n} are written")
    return out


def _offsets(offsets, npoints: int):
    """CSR set offsets as int64: offsets[0] = 0, non-decreasing, and the last
    equal to the number of points (the library reads points and writes
    labels up to offsets[-1])."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if off.ndim != 1 or off.size < 1:
        raise ValueError("offsets must be a 1-D array of num_sets + 1 values")
    if off[0] != 0:
        raise ValueError("offsets[0] must be 0")
    if off.size > 1 and bool((np.diff(off) < 0).any()):
        raise ValueError("offsets must not decrease")
    if int(off[-1]) != int(npoints):
        raise ValueError(f"offsets[-1] = {int(off[-1])} but there are {npoints} points")
    return off


def _host_labels_out(out, n: int):
    """A host label buffer for the server: numpy int32, C-contiguous,
    writable, at least n elements (results land there after submit
    returns, through its bare pointer)."""
    import numpy as np
    if out is None:
        return np.empty(n, dtype=np.int32)
    if not isinstance(out, np.ndarray):
        raise TypeError("out must be a numpy array")
    if out.dtype != np.int32:
        raise TypeError(f"out must be int32, not {out.dtype}")
    if not out.flags.c_contiguous or not out.flags.writeable:
        raise ValueError("out must be C-contiguous and writable")
    if out.size < n:
        raise ValueError(f"out holds {out.size} labels, {n} are written")
    return out


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(_torch().cuda.current_stream(device).cuda_stream)


# one timing slot per kernel launch, in launch order
PHASES = ("prep", "bounds", "morton", "sort0", "sort1", "sort2", "sort3", "sort4", "sort5",
          "sort6", "sort7", "gather", "cells", "build_frame", "build_levels", "count", "pairs",
          "final_roots", "final_labels")


class Context:
    """Device scratch (arena) + timing events, reused across calls."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        L = load_library()
        h = ctypes.c_void_p()
        _check(L.dbscan_ctx_create(int(device), int(budget_bytes), ctypes.byref(h)))
        self.handle = h
        self.device = int(device)

    def close(self):
        if getattr(self, "handle", None):
            load_library().dbscan_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cluster(self, points, eps: float, min_pts: int, algorithm: str = "auto",
                block_size: int = 0, dense_threshold: int = 0, timing: bool = False,
                out=None, graph: bool = False, pair_count: bool = False, sort_tile: int = 0):
        """``graph``: enqueue as a HIP graph replayed by later calls of the
        same shape (needs a non-default current stream; see
        DBSCAN_FLAG_GRAPH).  ``pair_count``: core points by pair traversal
        (DBSCAN_FLAG_PAIR_COUNT).  ``sort_tile``: keys per radix-sort
        workgroup (0 = 4096, 2048, 3072, 4096)."""
        p = _points(points)
        n = p.shape[0]
        labels = _labels_out(out, n, p.device)
        o = _Options(ALGO[algorithm], int(dense_threshold), int(block_size),
                     (FLAG_TIMING if timing else 0) | (FLAG_GRAPH if graph else 0) |
                     (FLAG_PAIR_COUNT if pair_count else 0), int(sort_tile))
        _check(load_library().dbscan_cluster_ex(
            self.handle, ctypes.c_void_p(p.data_ptr()), n, ctypes.c_float(eps), int(min_pts),
            ctypes.c_void_p(labels.data_ptr()), _stream(p.device), ctypes.byref(o)))
        return labels

    def cluster_batched(self, points, offsets, eps, min_pts, block_size: int = 0,
                        timing: bool = False, out=None, graph: bool = False,
                        algorithm: str = "auto", dense_threshold: int = 0, sort_tile: int = 0,
                        pair_count: bool = False):
        """Cluster the sets points[offsets[k]:offsets[k+1]] independently in
        one pass; ``eps`` and ``min_pts`` are scalars or one value per set.
        Labels are set-local (-1 noise, else the smallest index within the
        set of the point's cluster).  ``algorithm``: "auto"/"fdbscan" or
        "densebox" (``dense_threshold`` 0 = each set's min_pts).
        ``pair_count``: DenseBox core points by pair traversal
        (DBSCAN_FLAG_PAIR_COUNT)."""
        import numpy as np
        p = _points(points)
        off = _offsets(offsets, p.shape[0])
        k = off.size - 1
        e = np.ascontiguousarray(np.broadcast_to(np.float32(eps) if np.ndim(eps) == 0
                                                 else np.asarray(eps, np.float32), (k,)),
                                 dtype=np.float32)
        m = np.ascontiguousarray(np.broadcast_to(np.asarray(min_pts, np.int32), (k,)),
                                 dtype=np.int32)
        labels = _labels_out(out, p.shape[0], p.device)
        o = _Options(ALGO[algorithm], int(dense_threshold), int(block_size),
                     (FLAG_TIMING if timing else 0) | (FLAG_GRAPH if graph else 0) |
                     (FLAG_PAIR_COUNT if pair_count else 0), int(sort_tile))
        _check(load_library().dbscan_cluster_batched(
            self.handle, ctypes.c_void_p(p.data_ptr()),
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k,
            e.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            ctypes.c_void_p(labels.data_ptr()), _stream(p.device), ctypes.byref(o)))
        return labels

    def autotune(self, points, eps: float, min_pts: int, algorithm: str = "fdbscan",
                 cache=None):
        """Fastest options for this input (block_size, dense_threshold,
        pair_count, sort_tile), with its time in ms; see dbscan_autotune.
        ``cache``: a TuneCache or a JSON file path; a workload of the same
        device, size class, eps, minPts and algorithm found there is not
        tuned again (the result then has ``"cached": True``)."""
        torch = _torch()
        p = _points(points)
        key = None
        if cache is not None:
            from .tuning import TuneCache, plain_key
            cache = cache if isinstance(cache, TuneCache) else TuneCache(cache)
            key = plain_key(torch.cuda.get_device_name(p.device), p.shape[0], eps, min_pts,
                            algorithm)
            hit = cache.get(key)
            if hit is not None:
                return dict(hit, cached=True)
        lab = torch.empty(p.shape[0], dtype=torch.int32, device=p.device)
        o, ms = _Options(), ctypes.c_float(0)
        _check(load_library().dbscan_autotune(
            self.handle, ctypes.c_void_p(p.data_ptr()), p.shape[0], ctypes.c_float(eps),
            int(min_pts), ALGO[algorithm], ctypes.c_void_p(lab.data_ptr()), ctypes.byref(o),
            ctypes.byref(ms), _stream(p.device)))
        res = {"block_size": o.block_size, "dense_threshold": o.dense_threshold,
               "pair_count": bool(o.flags & FLAG_PAIR_COUNT), "sort_tile": o.sort_tile,
               "ms": ms.value}
        if key is not None:
            cache.put(key, res)
        return dict(res, cached=False) if key is not None else res

    def autotune_batched(self, points, offsets, eps, min_pts, cache=None):
        """Fastest options for this batch (algorithm, block_size,
        dense_threshold, sort_tile, pair_count), with its time in ms; see
        dbscan_autotune_batched.  ``cache`` as for autotune, keyed by the
        device, the set count, the size class of the total and the exact
        per-set eps and minPts."""
        import numpy as np
        torch = _torch()
        p = _points(points)
        off = _offsets(offsets, p.shape[0])
        k = off.size - 1
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float32), (k,)))
        m = np.ascontiguousarray(np.broadcast_to(np.asarray(min_pts, np.int32), (k,)))
        key = None
        if cache is not None:
            from .tuning import TuneCache, batched_key
            cache = cache if isinstance(cache, TuneCache) else TuneCache(cache)
            key = batched_key(torch.cuda.get_device_name(p.device), off, e, m)
            hit = cache.get(key)
            if hit is not None:
                return dict(hit, cached=True)
        lab = torch.empty(p.shape[0], dtype=torch.int32, device=p.device)
        o, ms = _Options(), ctypes.c_float(0)
        _check(load_library().dbscan_autotune_batched(
            self.handle, ctypes.c_void_p(p.data_ptr()),
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k,
            e.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.c_void_p(lab.data_ptr()),
            ctypes.byref(o), ctypes.byref(ms), _stream(p.device)))
        res = {"algorithm": ALGO_NAME[o.algorithm], "block_size": o.block_size,
               "dense_threshold": o.dense_threshold, "sort_tile": o.sort_tile,
               "pair_count": bool(o.flags & FLAG_PAIR_COUNT), "ms": ms.value}
        if key is not None:
            cache.put(key, res)
        return dict(res, cached=False) if key is not None else res

    def sort_passes(self) -> int:
        """Sort passes the last plain clustering call ran (the rest skipped)."""
        return int(load_library().dbscan_sort_passes(self.handle))

    def phase_times(self) -> dict:
        buf = (ctypes.c_float * len(PHASES))()
        k = load_library().dbscan_phase_times(self.handle, buf, len(PHASES))
        return {PHASES[i]: float(buf[i]) for i in range(k)}

    # ---- stages, for testing -------------------------------------------
    def morton_codes(self, points):
        torch = _torch()
        p = _points(points)
        codes = torch.empty(p.shape[0], dtype=torch.int64, device=p.device)
        _check(load_library().dbscan_morton_codes(
            self.handle, ctypes.c_void_p(p.data_ptr()), p.shape[0],
            ctypes.c_void_p(codes.data_ptr()), _stream(p.device)))
        return codes

    def sort_pairs(self, keys, vals):
        """Sort int64 keys (as unsigned) with int32 values, in place."""
        torch = _torch()
        if keys.dtype != torch.int64 or vals.dtype != torch.int32:
            raise TypeError("keys must be int64 and vals int32")
        if not (keys.is_cuda and vals.device == keys.device):
            raise TypeError("keys and vals must be on the same HIP device")
        if not (keys.is_contiguous() and vals.is_contiguous()) or keys.numel() != vals.numel():
            raise ValueError("keys and vals must be contiguous and of equal length")
        _check(load_library().dbscan_sort_pairs(
            self.handle, ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
            keys.numel(), _stream(keys.device)))
        return keys, vals

    def build_tree(self, points):
        torch = _torch()
        p = _points(points)
        n = p.shape[0]
        dev = p.device
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        leaf = torch.empty((n, 4), dtype=torch.float32, device=dev)
        nodes = torch.empty((max(n - 1, 1), 8), dtype=torch.float32, device=dev)
        root = torch.empty(1, dtype=torch.int32, device=dev)
        _check(load_library().dbscan_build_tree(
            self.handle, ctypes.c_void_p(p.data_ptr()), n, ctypes.c_void_p(perm.data_ptr()),
            ctypes.c_void_p(leaf.data_ptr()), ctypes.c_void_p(nodes.data_ptr()),
            ctypes.c_void_p(root.data_ptr()), _stream(dev)))
        return perm, leaf, nodes[: max(n - 1, 0)], root

    def core_flags(self, points, eps: float, min_pts: int):
        torch = _torch()
        p = _points(points)
        core = torch.empty(p.shape[0], dtype=torch.uint8, device=p.device)
        _check(load_library().dbscan_core_flags(
            self.handle, ctypes.c_void_p(p.data_ptr()), p.shape[0], ctypes.c_float(eps),
            int(min_pts), ctypes.c_void_p(core.data_ptr()), _stream(p.device)))
        return core

    def traversal_stats(self, points, eps: float) -> dict:
        p = _points(points)
        out = (ctypes.c_int64 * 4)()
        _check(load_library().dbscan_traversal_stats(
            self.handle, ctypes.c_void_p(p.data_ptr()), p.shape[0], ctypes.c_float(eps), out,
            _stream(p.device)))
        return {"pairs": out[0], "internal_visits": out[1], "descents": out[2],
                "leaf_tests": out[3]}

    def knn(self, points, k: int):
        """k nearest neighbours of every point, itself included: (indices
        int32 [n, k], squared distances float32 [n, k]) on the points'
        device, ranked by (squared distance, index); -1 / inf past n."""
        torch = _torch()
        p = _points(points)
        n = p.shape[0]
        idx = torch.empty((n, int(k)), dtype=torch.int32, device=p.device)
        d2 = torch.empty((n, int(k)), dtype=torch.float32, device=p.device)
        _check(load_library().dbscan_knn(
            self.handle, ctypes.c_void_p(p.data_ptr()), n, int(k),
            ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()), _stream(p.device)))
        return idx, d2

    def core_distances(self, points, min_pts: int):
        """HDBSCAN*'s squared core distance of every point: the squared
        distance to its min_pts-th nearest neighbour, itself counted."""
        torch = _torch()
        p = _points(points)
        d2 = torch.empty(p.shape[0], dtype=torch.float32, device=p.device)
        _check(load_library().dbscan_core_distances(
            self.handle, ctypes.c_void_p(p.data_ptr()), p.shape[0], int(min_pts),
            ctypes.c_void_p(d2.data_ptr()), _stream(p.device)))
        return d2

    def mst(self, points, min_pts: int = 1):
        """Minimum spanning tree: Euclidean for min_pts = 1, else of
        HDBSCAN*'s mutual reachability graph at min_pts.  Returns (edges
        int32 [n-1, 2] as (lo, hi) input indices, squared weights float32
        [n-1]) on the points' device, in increasing (w, lo, hi) order."""
        torch = _torch()
        p = _points(points)
        m = max(p.shape[0] - 1, 0)
        edges = torch.empty((m, 2), dtype=torch.int32, device=p.device)
        w = torch.empty(m, dtype=torch.float32, device=p.device)
        _check(load_library().dbscan_mst(
            self.handle, ctypes.c_void_p(p.data_ptr()), p.shape[0], int(min_pts),
            ctypes.c_void_p(edges.data_ptr()), ctypes.c_void_p(w.data_ptr()),
            _stream(p.device)))
        return edges, w

    def pair_count(self, points, eps: float) -> int:
        p = _points(points)
        out = ctypes.c_int64(0)
        _check(load_library().dbscan_pair_count(
            self.handle, ctypes.c_void_p(p.data_ptr()), p.shape[0], ctypes.c_float(eps),
            ctypes.byref(out), _stream(p.device)))
        return int(out.value)


class Server:
    """Continuous-batching job server (C++ scheduler in the library).  Jobs
    are host arrays (numpy float32 [n, 3]); results land in host int32
    arrays.  With ``fake_us_per_mpoint`` set, no GPU is used: jobs "run" for
    that many microseconds per million points and return all -1 labels."""

    def __init__(self, device: int = 0, slots: int = 4, budget_bytes: int = 0,
                 batch_cut: int = 0, batch_max_points: int = 0, batch_max_jobs: int = 0,
                 fake_us_per_mpoint=None):
        o = _ServerOptions(int(device), int(slots), int(budget_bytes), int(batch_cut),
                           int(batch_max_points), int(batch_max_jobs),
                           1 if fake_us_per_mpoint is not None else 0,
                           float(fake_us_per_mpoint or 0.0))
        h = ctypes.c_void_p()
        _check(load_library().dbscan_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, points, eps: float, min_pts: int, out=None) -> int:
        import numpy as np
        p = np.ascontiguousarray(points, dtype=np.float32)
        if p.ndim != 2 or p.shape[1] != 3:
            raise TypeError("points must be float32 [N, 3]")
        lab = _host_labels_out(out, p.shape[0])
        t = ctypes.c_uint64(0)
        _check(load_library().dbscan_server_submit(
            self.handle, ctypes.c_void_p(p.ctypes.data), p.shape[0], ctypes.c_float(eps),
            int(min_pts), ctypes.c_void_p(lab.ctypes.data), ctypes.byref(t)))
        self._keep[t.value] = (p, lab)
        return t.value

    def labels(self, ticket: int):
        return self._keep[ticket][1]

    def poll(self, ticket: int):
        """None while pending, else the job's status code."""
        st = ctypes.c_int32(0)
        r = load_library().dbscan_server_poll(self.handle, ticket, ctypes.byref(st))
        if r < 0:
            raise DbscanError(r, "unknown ticket")
        return None if r == 0 else st.value

    def wait(self, ticket: int, timeout: float = -1.0):
        st = ctypes.c_int32(0)
        r = load_library().dbscan_server_wait(self.handle, ticket, float(timeout),
                                              ctypes.byref(st))
        if r < 0:
            raise DbscanError(r, "unknown ticket")
        return None if r == 0 else st.value

    def job_times(self, ticket: int):
        a, b = ctypes.c_double(0), ctypes.c_double(0)
        _check(load_library().dbscan_server_job_times(self.handle, ticket, ctypes.byref(a),
                                                      ctypes.byref(b)))
        return a.value, b.value

    def stats(self) -> dict:
        st = _ServingStats()
        _check(load_library().dbscan_server_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServingStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            load_library().dbscan_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cluster(points, eps: float, min_pts: int, out=None):
    """Labels (int32 CUDA tensor, input order): -1 for noise, otherwise the
    smallest input index in the point's cluster.  Uses the device's default
    context."""
    p = _points(points)
    n = p.shape[0]
    labels = _labels_out(out, n, p.device)
    _check(load_library().dbscan_cluster(
        ctypes.c_void_p(p.data_ptr()), n, ctypes.c_float(eps), int(min_pts),
        ctypes.c_void_p(labels.data_ptr()), _stream(p.device)))
    return labels


NOALLOC_MAX_POINTS = 1048576  # DBSCAN_NOALLOC_MAX_POINTS


def cluster_noalloc(points, eps: float, min_pts: int, out=None):
    """As ``cluster``, through dbscan_cluster_noalloc: the library's fixed
    per-GPU scratch array instead of an allocated arena (at most
    NOALLOC_MAX_POINTS points).  Pass ``out`` to keep the call itself free
    of allocations on the Python side too."""
    p = _points(points)
    n = p.shape[0]
    labels = _labels_out(out, n, p.device)
    _check(load_library().dbscan_cluster_noalloc(
        ctypes.c_void_p(p.data_ptr()), n, ctypes.c_float(eps), int(min_pts),
        ctypes.c_void_p(labels.data_ptr()), _stream(p.device)))
    return labels
