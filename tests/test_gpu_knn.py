"""k nearest neighbours and HDBSCAN* core distances on the GPU (section 3.2
nearest search; section 5) against the oracle's brute force, bit for bit:
indices and squared distances, ties to the smaller index."""
import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = dbx.Context(0)
    yield c
    c.close()


def _check(ctx, p, k, sample=None):
    d = torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()
    idx, d2 = ctx.knn(d, k)
    idx, d2 = idx.cpu().numpy(), d2.cpu().numpy()
    q = None if sample is None else np.asarray(sample, dtype=np.int64)
    ri, rd = oracle.knn(p, k, q)
    if q is not None:
        idx, d2 = idx[q], d2[q]
    assert np.array_equal(d2.view(np.uint32), rd.view(np.uint32))
    assert np.array_equal(idx, ri)


@pytest.mark.parametrize("k", [1, 2, 4, 5, 8, 13, 16, 31, 32])
def test_clumps(ctx, k):
    print(f"[knn] clumps 20,000 k={k}", flush=True)
    _check(ctx, datagen.clumps(20_000, seed=70 + k), k)


def test_ties_on_a_lattice(ctx):
    g = np.arange(12, dtype=np.float32)
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p = p[np.random.default_rng(3).permutation(len(p))]
    for k in (1, 6, 7, 19, 27, 32):
        print(f"[knn] lattice 1,728 k={k}", flush=True)
        _check(ctx, p, k)


def test_duplicates_and_fewer_points_than_k(ctx):
    rng = np.random.default_rng(4)
    base = rng.random((40, 3)).astype(np.float32)
    p = np.concatenate([base, base, base[:7]])[rng.permutation(87)]
    _check(ctx, p, 32)
    _check(ctx, p[:5], 8)      # -1 / inf past n
    _check(ctx, p[:1], 3)
    _check(ctx, np.zeros((9, 3), np.float32), 4)  # all identical: ties by index


def test_flat_axis_and_far_points(ctx):
    rng = np.random.default_rng(6)
    p = rng.random((3000, 3)).astype(np.float32)
    p[:, 2] = 0.5
    _check(ctx, p, 10)
    q = rng.random((3000, 3)).astype(np.float32) * np.float32(1e4)
    _check(ctx, q, 10)


def test_halo_field_sampled(ctx):
    import os
    p = datagen.config_points("halo16M", n=1 << 21)
    rng = np.random.default_rng(8)
    print("[knn] halo field 2^21 points, k=8, 1,000 sampled rows", flush=True)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    try:
        _check(ctx, p, 8, sample=rng.choice(p.shape[0], 1000, replace=False))
    finally:
        oracle.set_threads(1)


@pytest.mark.parametrize("mp", [1, 2, 5, 10, 32])
def test_core_distances(ctx, mp):
    p = datagen.clumps(30_000, seed=90 + mp)
    d = torch.from_numpy(p).cuda()
    got = ctx.core_distances(d, mp).cpu().numpy()
    ref = oracle.core_distances(p, mp)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_invalid_k(ctx):
    d = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    for k in (0, 33):
        with pytest.raises(dbx.DbscanError):
            ctx.knn(d, k)
    d[3, 1] = float("nan")
    with pytest.raises(dbx.DbscanError):
        ctx.knn(d, 4)
