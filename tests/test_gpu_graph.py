"""HIP-graph replays of the plain and batched calls (DBSCAN_FLAG_GRAPH), with
FDBSCAN and DenseBox: every replay, with eager work and synchronisations
between replays, must give the eager labels; a batched replay picks up new
per-set parameters (for DenseBox also new cell grids and primitive counts,
which stay on the device)."""
import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32


@pytest.mark.parametrize("algo", ["fdbscan", "densebox"])
def test_plain_graph_replays_match_eager(algo):
    p = datagen.clumps(200003, 41)
    ctx = dbx.Context(0)
    d = torch.from_numpy(p).cuda()
    eager = ctx.cluster(d, 0.01, 3, algorithm=algo).cpu().numpy()
    np.testing.assert_array_equal(eager, oracle.dbscan(p, F32(0.01), 3))
    stream = torch.cuda.Stream()
    out = torch.empty(p.shape[0], dtype=torch.int32, device="cuda")
    for k in range(4):
        with torch.cuda.stream(stream):
            out.fill_(-7)
            ctx.cluster(d, 0.01, 3, out=out, graph=True, algorithm=algo)
        stream.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), eager)
        # eager work of other shapes in between, on the default stream
        small = datagen.clumps(5000 + k, 60 + k)
        np.testing.assert_array_equal(ctx.cluster(torch.from_numpy(small).cuda(), 0.02, 2,
                                                  algorithm=algo).cpu().numpy(),
                                      oracle.dbscan(small, F32(0.02), 2))
    ctx.close()


@pytest.mark.parametrize("algo", ["fdbscan", "densebox"])
def test_batched_graph_replay_takes_new_parameters(algo):
    pts, off = datagen.subhalo_sets(64, 9, nmin=64, nmax=20000)
    ctx = dbx.Context(0)
    d = torch.from_numpy(pts).cuda()
    stream = torch.cuda.Stream()
    out = torch.empty(pts.shape[0], dtype=torch.int32, device="cuda")
    rng = np.random.Generator(np.random.PCG64(3))
    for k in range(4):
        eps = rng.uniform(0.03, 0.08, 64).astype(F32)
        mp = rng.choice([2, 5, 10], 64).astype(np.int32)
        eager = ctx.cluster_batched(d, off, eps, mp, algorithm=algo).cpu().numpy()
        with torch.cuda.stream(stream):
            out.fill_(-7)
            ctx.cluster_batched(d, off, eps, mp, out=out, graph=True, algorithm=algo)
        stream.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), eager)
        for s in (0, 17, 63):
            a, b = int(off[s]), int(off[s + 1])
            np.testing.assert_array_equal(eager[a:b], oracle.dbscan(pts[a:b], eps[s], int(mp[s])))
    ctx.close()
