"""Minimum spanning trees on the GPU (the Euclidean tree of section 3.2's
algorithm list; the mutual reachability tree of HDBSCAN*, section 5)
against the oracle's Prim, bit for bit: the n-1 edges (lo, hi) in (w, lo,
hi) order and the bits of every weight.  At the 2^24-point field, where the
oracle's O(n^2) is out of reach: properties that hold at any size."""
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


def _check(ctx, p, min_pts):
    p = np.ascontiguousarray(p, dtype=F32)
    e, w = ctx.mst(torch.from_numpy(p).cuda(), min_pts)
    e, w = e.cpu().numpy(), w.cpu().numpy()
    re, rw = oracle.mst(p, min_pts)
    assert np.array_equal(e, re)
    assert np.array_equal(w.view(np.uint32), rw.view(np.uint32))


@pytest.mark.parametrize("min_pts", [1, 2, 5, 16])
def test_clumps(ctx, min_pts):
    print(f"[mst] clumps 20,000 minPts={min_pts}", flush=True)
    _check(ctx, datagen.clumps(20_000, seed=90 + min_pts), min_pts)


@pytest.mark.parametrize("n", [2, 3, 17, 64, 65, 1000, 4099])
def test_uniform_sizes(ctx, n):
    print(f"[mst] uniform n={n}", flush=True)
    p = np.random.default_rng(n).random((n, 3)).astype(F32)
    for mp in (1, 3):
        _check(ctx, p, mp)


def test_ties_on_a_lattice(ctx):
    g = np.arange(10, dtype=F32)
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p = p[np.random.default_rng(3).permutation(len(p))]
    for mp in (1, 2, 7, 27):
        print(f"[mst] lattice 1,000 minPts={mp}", flush=True)
        _check(ctx, p, mp)


def test_duplicates_flat_and_fewer_points_than_min_pts(ctx):
    rng = np.random.default_rng(4)
    base = rng.random((60, 3)).astype(F32)
    p = np.concatenate([base, base, base[:9]])[rng.permutation(129)]
    for mp in (1, 2, 4):
        _check(ctx, p, mp)
    flat = rng.random((700, 3)).astype(F32)
    flat[:, 1] = 0.25
    _check(ctx, flat, 1)
    _check(ctx, flat, 6)
    _check(ctx, base[:5], 8)                 # every core distance +inf
    _check(ctx, np.zeros((50, 3), F32), 3)   # all identical: every weight 0


def test_empty_and_one_point(ctx):
    for n in (0, 1):
        e, w = ctx.mst(torch.zeros((n, 3), dtype=torch.float32, device="cuda"), 1)
        assert e.shape == (0, 2) and w.shape == (0,)


def _d2(a, b):
    d = a - b
    sq = d * d
    return (sq[..., 0] + sq[..., 1]) + sq[..., 2]


def test_halo16m_properties(ctx):
    """The Euclidean tree of the 2^24-point field: n-1 edges in strictly
    increasing (w, lo, hi) order, each weight the binary32 D of its ends,
    one connected tree, and for 300 sampled points the least edge at the
    point (brute force over all n points) is a tree edge."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    p = datagen.config_points("halo16M")
    n = p.shape[0]
    print(f"[mst] halo16M n={n}", flush=True)
    e, w = ctx.mst(torch.from_numpy(p).cuda(), 1)
    e, w = e.cpu().numpy(), w.cpu().numpy()
    assert e.shape == (n - 1, 2)
    lo, hi = e[:, 0].astype(np.int64), e[:, 1].astype(np.int64)
    assert (lo < hi).all() and lo.min() >= 0 and hi.max() < n
    assert np.array_equal(w.view(np.uint32), _d2(p[lo], p[hi]).view(np.uint32))
    key = np.lexsort((hi, lo, w))
    assert np.array_equal(key, np.arange(n - 1))
    same = (w[1:] == w[:-1]) & (lo[1:] == lo[:-1]) & (hi[1:] == hi[:-1])
    assert not same.any()
    g = coo_matrix((np.ones(n - 1, np.int8), (lo, hi)), shape=(n, n))
    assert connected_components(g, directed=False)[0] == 1
    tree = set(zip(lo.tolist(), hi.tolist()))
    rng = np.random.default_rng(11)
    for u in rng.choice(n, 300, replace=False).tolist():
        d = _d2(p, p[u])
        d[u] = np.inf
        m = d.min()
        cand = np.flatnonzero(d == m)
        pairs = sorted((min(u, int(v)), max(u, int(v))) for v in cand)
        assert pairs[0] in tree
