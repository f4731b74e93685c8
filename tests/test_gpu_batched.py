"""GPU parity of the batched path: many independent sets in one pass, each
result bit-identical to the oracle's clustering of that set alone."""
import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32


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


def test_subhalo_sets_small(ctx):
    pts, off = datagen.subhalo_sets(64, 4, nmin=64, nmax=8192)
    check(ctx, pts, off, 0.05, 5)


def test_mixed_params_and_empty_sets(ctx):
    rng = np.random.Generator(np.random.PCG64(3))
    sizes = [0, 1, 2, 700, 0, 5000, 33, 4096, 4097, 1]
    parts = [datagen.clumps(max(s, 1), 10 + i)[:s] for i, s in enumerate(sizes)]
    pts = np.concatenate(parts).astype(F32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps = rng.uniform(0.005, 0.05, len(sizes)).astype(F32)
    mp = np.array([1, 2, 3, 5, 10, 2, 1, 4, 2, 7], np.int32)
    check(ctx, pts, off, eps, mp)


def test_overlapping_identical_sets(ctx):
    """Sets occupying the same space (ropes must not leak across sets)."""
    p = datagen.clumps(3000, 9)
    pts = np.concatenate([p, p, p]).astype(F32)
    off = np.array([0, 3000, 6000, 9000], np.int64)
    check(ctx, pts, off, [0.01, 0.02, 0.01], [2, 5, 3])


def test_single_set_equals_plain_call(ctx):
    p = datagen.config_points("clumps32k")
    got = ctx.cluster_batched(dev(p), [0, p.shape[0]], 0.006, 2).cpu().numpy()
    np.testing.assert_array_equal(got, ctx.cluster(dev(p), 0.006, 2).cpu().numpy())


def test_many_sets_block_sizes(ctx):
    pts, off = datagen.subhalo_sets(300, 8, nmin=64, nmax=20000)
    for bs in (64, 256):
        check(ctx, pts, off, 0.05, 5, block_size=bs)


def test_invalid_offsets(ctx):
    p = dev(datagen.clumps(100, 1))
    for off in ([1, 100], [0, 60, 50, 100]):
        with pytest.raises(dbx.DbscanError) as e:
            ctx.cluster_batched(p, off, 0.01, 2)
        assert e.value.code == -1


def test_subhalo4096_full(ctx):
    """The full 4,096-set workload (~133M points); every set is checked
    against the oracle on a deterministic sample of 200 sets plus the
    largest and smallest."""
    pts, off = datagen.subhalo_sets(4096, 4)
    got = ctx.cluster_batched(dev(pts), off, 0.05, 5).cpu().numpy()
    sizes = np.diff(off)
    pick = set(np.random.Generator(np.random.PCG64(0)).choice(4096, 200, replace=False).tolist())
    pick |= {int(sizes.argmax()), int(sizes.argmin())}
    for s in sorted(pick):
        a, b = off[s], off[s + 1]
        np.testing.assert_array_equal(got[a:b], oracle.dbscan(pts[a:b], F32(0.05), 5),
                                      err_msg=f"set {s}")
