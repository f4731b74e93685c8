"""GPU parity of the batched path: many independent sets in one pass, each
result bit-identical to the oracle's clustering of that set alone, with
FDBSCAN and with DenseBox (per-set cell grids and thresholds)."""
import os

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32
ALGOS = ["fdbscan", "densebox"]


@pytest.fixture(scope="module")
def ctx():
    c = dbx.Context(0)
    yield c
    c.close()


def dev(p):
    return torch.from_numpy(np.ascontiguousarray(p, dtype=F32)).cuda()


def check(ctx, pts, off, eps, mp, **kw):
    got = ctx.cluster_batched(dev(pts), off, eps, mp, **kw).cpu().numpy()
    k = len(off) - 1
    eps = np.broadcast_to(np.asarray(eps, F32), (k,))
    mp = np.broadcast_to(np.asarray(mp), (k,))
    for s in range(k):
        a, b = off[s], off[s + 1]
        ref = oracle.dbscan(pts[a:b], F32(eps[s]), int(mp[s])) if b > a else np.zeros(0)
        np.testing.assert_array_equal(got[a:b], ref, err_msg=f"set {s}")


@pytest.mark.parametrize("algo", ALGOS)
def test_subhalo_sets_small(ctx, algo):
    pts, off = datagen.subhalo_sets(64, 4, nmin=64, nmax=8192)
    check(ctx, pts, off, 0.05, 5, algorithm=algo)


def test_subhalo_sets_pair_count(ctx):
    """DenseBox core points by pair traversal over many sets (persistent
    walks, counts cut at set ends)."""
    pts, off = datagen.subhalo_sets(64, 4, nmin=64, nmax=65536)
    check(ctx, pts, off, 0.05, 5, algorithm="densebox", pair_count=True)


@pytest.mark.parametrize("algo,thresh,pc", [("fdbscan", 0, False), ("densebox", 0, False),
                                            ("densebox", 10, False), ("densebox", 40, False),
                                            ("densebox", 0, True), ("densebox", 10, True)])
def test_mixed_params_and_empty_sets(ctx, algo, thresh, pc):
    rng = np.random.Generator(np.random.PCG64(3))
    sizes = [0, 1, 2, 700, 0, 5000, 33, 4096, 4097, 1]
    parts = [datagen.clumps(max(s, 1), 10 + i)[:s] for i, s in enumerate(sizes)]
    pts = np.concatenate(parts).astype(F32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps = rng.uniform(0.005, 0.05, len(sizes)).astype(F32)
    mp = np.array([1, 2, 3, 5, 10, 2, 1, 4, 2, 7], np.int32)
    check(ctx, pts, off, eps, mp, algorithm=algo, dense_threshold=thresh, pair_count=pc)


@pytest.mark.parametrize("algo", ALGOS)
def test_overlapping_identical_sets(ctx, algo):
    """Sets occupying the same space (ropes must not leak across sets)."""
    p = datagen.clumps(3000, 9)
    pts = np.concatenate([p, p, p]).astype(F32)
    off = np.array([0, 3000, 6000, 9000], np.int64)
    check(ctx, pts, off, [0.01, 0.02, 0.01], [2, 5, 3], algorithm=algo)


def test_dense_sets_mixed_with_sparse(ctx):
    """DenseBox: sets of piled-up duplicates (one dense cell each), tight
    balls and sparse sets in one call, minPts on both sides of 2."""
    rng = np.random.Generator(np.random.PCG64(12))
    parts = [np.repeat(rng.uniform(0, 1, (1, 3)), 500, 0),
             rng.normal(0.5, 0.002, (3000, 3)),
             rng.uniform(0, 1, (2000, 3)),
             np.repeat(rng.uniform(0, 1, (1, 3)), 3, 0),
             rng.normal(0.2, 0.01, (4000, 3))]
    pts = np.concatenate(parts).astype(F32)
    off = np.concatenate([[0], np.cumsum([len(q) for q in parts])]).astype(np.int64)
    check(ctx, pts, off, [0.01, 0.003, 0.05, 0.0, 0.004], [5, 2, 3, 4, 1],
          algorithm="densebox")


@pytest.mark.parametrize("algo", ALGOS)
def test_single_set_equals_plain_call(ctx, algo):
    p = datagen.config_points("clumps32k")
    got = ctx.cluster_batched(dev(p), [0, p.shape[0]], 0.006, 2, algorithm=algo).cpu().numpy()
    np.testing.assert_array_equal(got, ctx.cluster(dev(p), 0.006, 2,
                                                   algorithm=algo).cpu().numpy())


@pytest.mark.parametrize("algo", ALGOS)
def test_many_sets_block_sizes(ctx, algo):
    pts, off = datagen.subhalo_sets(300, 8, nmin=64, nmax=20000)
    for bs in (64, 256, 1024):
        check(ctx, pts, off, 0.05, 5, block_size=bs, algorithm=algo)


def test_autotune_batched_keeps_labels(ctx):
    pts, off = datagen.subhalo_sets(40, 5, nmin=64, nmax=20000)
    best = ctx.autotune_batched(dev(pts), off, 0.05, 5)
    assert best["algorithm"] in ALGOS and best["block_size"] in (64, 128, 256, 512)
    assert best["dense_threshold"] in (0, 10, 20) and best["ms"] > 0
    if best["algorithm"] == "fdbscan":
        assert best["dense_threshold"] == 0
    assert best["sort_tile"] in (0, 2048, 3072)
    if best["algorithm"] == "fdbscan":
        assert not best["pair_count"]  # (batched FDBSCAN counts by walk)
    check(ctx, pts, off, 0.05, 5, algorithm=best["algorithm"], block_size=best["block_size"],
          dense_threshold=best["dense_threshold"], sort_tile=best["sort_tile"],
          pair_count=best["pair_count"])


@pytest.mark.parametrize("tile", [2048, 3072, 4096])
def test_sort_tiles_keep_labels(ctx, tile):
    """Every radix-sort tile size gives the same set-local labels (sets of
    ragged sizes, so the tiles end mid-set)."""
    pts, off = datagen.subhalo_sets(30, 13, nmin=1, nmax=9000)
    for algo in ALGOS:
        check(ctx, pts, off, 0.05, 3, algorithm=algo, sort_tile=tile)


def test_autotune_batched_cache(ctx, tmp_path):
    pts, off = datagen.subhalo_sets(16, 6, nmin=64, nmax=5000)
    path = tmp_path / "tune.json"
    a = ctx.autotune_batched(dev(pts), off, 0.05, 5, cache=path)
    b = ctx.autotune_batched(dev(pts), off, 0.05, 5, cache=path)
    assert a["cached"] is False and b["cached"] is True
    assert {k: a[k] for k in a if k != "cached"} == {k: b[k] for k in b if k != "cached"}
    # other per-set parameters: tuned again
    c = ctx.autotune_batched(dev(pts), off, 0.06, 5, cache=path)
    assert c["cached"] is False


def test_invalid_offsets(ctx):
    """The binding rejects bad offsets before the call (ValueError), and so
    does the C ABI itself (EINVAL) when called directly."""
    import ctypes
    p = dev(datagen.clumps(100, 1))
    for off in ([1, 100], [0, 60, 50, 100], [0, 50, 101], [0, 50, 99]):
        with pytest.raises(ValueError):
            ctx.cluster_batched(p, off, 0.01, 2)
    lab = torch.empty(100, dtype=torch.int32, device="cuda")
    lib = dbx.load_library()
    for off in ([1, 100], [0, 60, 50, 100]):
        o = np.array(off, dtype=np.int64)
        k = o.size - 1
        e = np.full(k, 0.01, np.float32)
        m = np.full(k, 2, np.int32)
        st = lib.dbscan_cluster_batched(
            ctx.handle, ctypes.c_void_p(p.data_ptr()),
            o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k,
            e.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            ctypes.c_void_p(lab.data_ptr()), None, None)
        assert st == -1


@pytest.fixture(scope="module")
def subhalo4096():
    print("[batched] generating the 4,096 sets", flush=True)
    pts, off = datagen.subhalo_sets(4096, 4)
    print("[batched] oracle on every set", flush=True)
    ref = oracle.dbscan_sets(pts, off, F32(0.05), 5, workers=min(16, os.cpu_count() or 1))
    return pts, off, ref


def _first_bad_sets(got, ref, off, limit=5):
    bad = np.flatnonzero(got != ref)
    return sorted(set(np.searchsorted(off, bad, side="right") - 1))[:limit]


@pytest.mark.parametrize("algo,pc", [("fdbscan", False), ("densebox", False),
                                     ("densebox", True)])
def test_subhalo4096_every_set_bit_exact(ctx, subhalo4096, algo, pc):
    """The full 4,096-set workload (~133M points): every set's labels
    against the oracle's clustering of that set alone."""
    pts, off, ref = subhalo4096
    d = dev(pts)
    got = ctx.cluster_batched(d, off, 0.05, 5, algorithm=algo, pair_count=pc).cpu().numpy()
    del d
    assert np.array_equal(got, ref), f"sets differ: {_first_bad_sets(got, ref, off)}"
