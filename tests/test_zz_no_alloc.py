"""dbscan_cluster_noalloc (the entry point that allocates nothing) against
dbscan_cluster, both called through the C ABI with ctypes: bit-exact labels
on two calls in a row, the second on a smaller input (the fixed scratch
array keeps the first call's contents), at the maximum size, and after a
rejected oversized call."""
import ctypes

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(p, eps, mp):
    """Labels of the plain entry point and of the no-allocation one."""
    lib = dbx.load_library()
    d = torch.from_numpy(p).cuda()
    n = p.shape[0]
    ref = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    got = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    st = lib.dbscan_cluster(_vp(d), n, ctypes.c_float(eps), mp, _vp(ref), None)
    assert st == 0, lib.dbscan_last_error()
    st = lib.dbscan_cluster_noalloc(_vp(d), n, ctypes.c_float(eps), mp, _vp(got), None)
    assert st == 0, lib.dbscan_last_error()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_two_calls_second_smaller():
    big = datagen.clumps(300_007, seed=11)
    small = datagen.clumps(50_001, seed=12)
    print("[noalloc] 300,007 points, minPts 5", flush=True)
    ref, got = _both(big, F32(0.004), 5)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.dbscan(big, F32(0.004), 5))
    print("[noalloc] 50,001 points, minPts 2", flush=True)
    ref, got = _both(small, F32(0.006), 2)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.dbscan(small, F32(0.006), 2))


def test_maximum_size_then_rejection_then_smaller():
    n = dbx.NOALLOC_MAX_POINTS
    p = datagen.clumps(n, seed=13)
    print(f"[noalloc] {n} points (the maximum), minPts 10", flush=True)
    ref, got = _both(p, F32(0.003), 10)
    assert np.array_equal(got, ref)
    lib = dbx.load_library()
    d = torch.from_numpy(p).cuda()
    lab = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    st = lib.dbscan_cluster_noalloc(_vp(d), n + 1, ctypes.c_float(0.003), 10, _vp(lab), None)
    assert st == -5  # ETOOBIG, nothing launched
    assert int((lab != -7).sum()) == 0
    q = datagen.clumps(3_071, seed=14)
    print("[noalloc] 3,071 points, minPts 3", flush=True)
    ref, got = _both(q, F32(0.02), 3)
    assert np.array_equal(got, ref)


def test_on_a_torch_stream():
    p = datagen.clumps(70_000, seed=15)
    d = torch.from_numpy(p).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = dbx.cluster_noalloc(d, 0.006, 2)
    s.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.dbscan(p, F32(0.006), 2))
