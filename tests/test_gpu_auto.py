"""DBSCAN_ALGO_AUTO: the density probe picks DenseBox where points have
many neighbours and FDBSCAN where they have few; the labels are the
oracle's either way.  Which algorithm ran is seen in the per-phase times:
only DenseBox has a "cells" phase."""
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


def ran_densebox(ctx):
    return ctx.phase_times()["cells"] > 0


def test_sparse_field_runs_fdbscan(ctx):
    """FDBSCAN; at minPts > 2 with core points by pair traversal (fewer
    neighbours than minPts on average): the labels do not change."""
    p = datagen.config_points("halo16M", n=1 << 20)
    d = torch.from_numpy(p).cuda()
    for mp in (2, 3, 5):
        got = ctx.cluster(d, 0.2, mp, algorithm="auto", timing=True).cpu().numpy()
        assert not ran_densebox(ctx)
        assert np.array_equal(got, oracle.dbscan(p, F32(0.2), mp)), mp


def test_dense_clumps_run_densebox(ctx):
    # 200,000 points in 20 tight clumps: hundreds of neighbours each at eps 0.01
    p = datagen.clumps(200_000, seed=21, n_clumps=20, clump_frac=0.95, sigma=(0.01, 0.02))
    d = torch.from_numpy(p).cuda()
    for mp in (2, 10):
        got = ctx.cluster(d, 0.01, mp, algorithm="auto", timing=True).cpu().numpy()
        assert ran_densebox(ctx), mp
        assert np.array_equal(got, oracle.dbscan(p, F32(0.01), mp))


def test_batched_subhalo_sets_run_densebox(ctx):
    pts, off = datagen.subhalo_sets(96, 4, nmin=20_000, nmax=200_000)
    d = torch.from_numpy(pts).cuda()
    got = ctx.cluster_batched(d, off, 0.05, 5, timing=True).cpu().numpy()  # default: auto
    assert ran_densebox(ctx)
    ref = oracle.dbscan_sets(pts, off, F32(0.05), 5, workers=8)
    assert np.array_equal(got, ref)


def test_batched_sparse_sets_run_fdbscan(ctx):
    rng = np.random.default_rng(5)
    sizes = rng.integers(500, 5000, 64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts = rng.random((int(off[-1]), 3)).astype(F32)
    d = torch.from_numpy(pts).cuda()
    got = ctx.cluster_batched(d, off, 0.01, 3, timing=True).cpu().numpy()
    assert not ran_densebox(ctx)
    assert np.array_equal(got, oracle.dbscan_sets(pts, off, F32(0.01), 3, workers=8))


def test_pick_is_kept_for_graph_replays(ctx):
    p = datagen.clumps(100_000, seed=22, n_clumps=10, clump_frac=0.95, sigma=(0.01, 0.02))
    d = torch.from_numpy(p).cuda()
    ref = oracle.dbscan(p, F32(0.01), 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(3):
            got = ctx.cluster(d, 0.01, 4, algorithm="auto", graph=True)
            s.synchronize()
            assert np.array_equal(got.cpu().numpy(), ref)
