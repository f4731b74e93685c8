"""GPU parity of the DenseBox path (dense grid cells taken whole) against the
CPU oracle, bit for bit, and against the FDBSCAN path on the same input."""
import os

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = dbx.Context(0)
    yield c
    c.close()


def dev(p):
    return torch.from_numpy(np.ascontiguousarray(p, dtype=F32)).cuda()


def db(ctx, p, eps, mp, **kw):
    return ctx.cluster(dev(p), float(eps), mp, algorithm="densebox", **kw).cpu().numpy()


def clumpy(n, seed, k=8, sigma=0.02):
    rng = np.random.Generator(np.random.PCG64(seed))
    cen = rng.random((k, 3))
    p = cen[rng.integers(0, k, n)] + rng.standard_normal((n, 3)) * sigma
    m = n // 5
    p[:m] = rng.random((m, 3))
    return p[rng.permutation(n)].astype(F32)


def _pts(*rows):
    return np.array(rows, dtype=F32).reshape(-1, 3)


def test_hand_cases(ctx):
    assert db(ctx, _pts((0, 0, 0), (0.5, 0, 0)), 0.5, 2).tolist() == [0, 0]
    x = np.nextafter(F32(0.5), F32(1))
    assert db(ctx, _pts((0, 0, 0), (x, 0, 0)), 0.5, 2).tolist() == [-1, -1]
    c = np.zeros((1000, 3), F32)
    c[:, 0] = np.arange(1000, dtype=F32) * F32(0.25)
    assert (db(ctx, c, 0.25, 2) == 0).all()
    assert (db(ctx, c, np.nextafter(F32(0.25), F32(0)), 2) == -1).all()
    assert db(ctx, _pts((0, 0, 0), (2e-20, 0, 0)), F32(1e-20), 2).tolist() == [-1, -1]
    assert db(ctx, _pts((1e-30, 0, 0), (2e-30, 0, 0), (5e-30, 0, 0)), 0.0, 2).tolist() == [0, 0, 0]
    assert db(ctx, _pts((-1e30, 0, 0), (1e30, 0, 0), (1e30, 0, 0)), 1e18, 2).tolist() == [-1, 1, 1]
    assert db(ctx, _pts((1, 2, 3)), 1.0, 1).tolist() == [0]
    assert db(ctx, _pts((1, 2, 3)), 1.0, 2).tolist() == [-1]


def test_border_rules(ctx):
    A = [(0.0, 0, 0), (-0.1, 0, 0), (-0.2, 0, 0), (-0.3, 0, 0)]
    B = [(2.0, 0, 0), (2.1, 0, 0), (2.2, 0, 0), (2.3, 0, 0)]
    b = [(1.0, 0, 0)]
    for pts in (B + A + b, A + B + b, b + B + A, b + A + B):
        p = _pts(*pts)
        np.testing.assert_array_equal(db(ctx, p, 1.0, 4), oracle.dbscan(p, F32(1.0), 4))


def test_fp_boundary_golden_cases(ctx):
    with open(os.path.join(GOLDEN, "fp_boundary_cases.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            v = [F32(float.fromhex(x)) for x in t[1:8]]
            p = np.array([v[0:3], v[3:6]], F32)
            exp = [0, 0] if int(t[8]) else [-1, -1]
            assert db(ctx, p, v[6], 2).tolist() == exp, line


@pytest.mark.parametrize("k", [1, 7, 3000])
def test_identical_points_one_dense_cell(ctx, k):
    p = np.tile(_pts((0.3, -1.25, 7.0)), (k, 1))
    assert (db(ctx, p, 0.0, min(k, 5)) == 0).all()
    assert (db(ctx, p, 0.0, k + 1) == -1).all()
    assert (db(ctx, p, 1.0, min(k, 5)) == 0).all()


def test_dense_ball(ctx):
    rng = np.random.Generator(np.random.PCG64(14))
    d = rng.standard_normal((100000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p = (d * rng.random((100000, 1)) * 0.1).astype(F32)
    for mp in (2, 10):
        assert (db(ctx, p, 1.0, mp) == 0).all()


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mp", [1, 2, 3, 5, 10])
def test_random_clumpy(ctx, seed, mp):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    n = int(rng.integers(10, 30000))
    p = clumpy(n, seed, sigma=float(rng.uniform(0.005, 0.03)))
    eps = F32(rng.uniform(0.005, 0.05))
    np.testing.assert_array_equal(db(ctx, p, eps, mp), oracle.dbscan(p, eps, mp))


@pytest.mark.parametrize("thresh", [0, 6, 40, 1 << 20])
def test_dense_threshold_does_not_change_labels(ctx, thresh):
    p = clumpy(60000, 11, sigma=0.01)
    ref = oracle.dbscan(p, F32(0.02), 5)
    np.testing.assert_array_equal(db(ctx, p, 0.02, 5, dense_threshold=thresh), ref)


def test_dense_threshold_below_minpts_rejected(ctx):
    with pytest.raises(dbx.DbscanError) as e:
        db(ctx, clumpy(100, 1), 0.02, 5, dense_threshold=3)
    assert e.value.code == -1


@pytest.mark.parametrize("mp", [2, 5, 10])
def test_clumps32k(ctx, mp):
    p = datagen.config_points("clumps32k")
    np.testing.assert_array_equal(db(ctx, p, F32(0.006), mp), oracle.dbscan(p, F32(0.006), mp))


def test_subhalo_sets_dense_subclumps(ctx):
    """Single Plummer halos with dense sub-clumps (the batched workload's
    sets): many dense cells, cell-cell and point-cell pairs."""
    pts, off = datagen.subhalo_sets(6, 4, nmin=20000, nmax=200000)
    for s in range(6):
        p = pts[off[s]:off[s + 1]]
        np.testing.assert_array_equal(db(ctx, p, F32(0.05), 5), oracle.dbscan(p, F32(0.05), 5))


def test_densebox_equals_fdbscan_and_block_sizes(ctx):
    p = clumpy(80001, 5, sigma=0.01)
    ref = ctx.cluster(dev(p), 0.015, 4).cpu().numpy()
    for bs in (64, 256, 1024):
        np.testing.assert_array_equal(db(ctx, p, 0.015, 4, block_size=bs), ref)


def test_halo16m_densebox_bit_exact(ctx):
    p = datagen.config_points("halo16M")
    np.testing.assert_array_equal(db(ctx, p, F32(0.2), 2), oracle.dbscan(p, F32(0.2), 2))


# ---- core points by pair traversal (DBSCAN_FLAG_PAIR_COUNT) -----------------
# The counts come from every pair of primitives met once (point-point adds
# one to both, a point and a dense cell add the cell's points within eps to
# the point): the same labels as the counting walk, checked against the
# oracle where points, cells and mixed pairs all occur.

@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("mp", [3, 5, 10])
def test_pair_count_random_clumpy(ctx, seed, mp):
    rng = np.random.Generator(np.random.PCG64(200 + seed))
    n = int(rng.integers(10, 30000))
    p = clumpy(n, seed, sigma=float(rng.uniform(0.005, 0.03)))
    eps = F32(rng.uniform(0.005, 0.05))
    np.testing.assert_array_equal(db(ctx, p, eps, mp, pair_count=True),
                                  oracle.dbscan(p, eps, mp))


@pytest.mark.parametrize("thresh", [0, 6, 40])
def test_pair_count_dense_thresholds(ctx, thresh):
    p = clumpy(60000, 11, sigma=0.01)
    ref = oracle.dbscan(p, F32(0.02), 5)
    np.testing.assert_array_equal(
        db(ctx, p, 0.02, 5, dense_threshold=thresh, pair_count=True), ref)


def test_pair_count_hand_cases(ctx):
    # a border point between two dense cells, and one that only reaches
    # part of a cell (the queued count of the cell's points within eps)
    A = [(0.0, 0, 0), (-0.1, 0, 0), (-0.2, 0, 0), (-0.3, 0, 0)]
    B = [(2.0, 0, 0), (2.1, 0, 0), (2.2, 0, 0), (2.3, 0, 0)]
    b = [(1.0, 0, 0)]
    for pts in (B + A + b, A + B + b, b + B + A, b + A + B):
        p = _pts(*pts)
        for mp in (3, 4, 5):
            np.testing.assert_array_equal(db(ctx, p, 1.0, mp, pair_count=True),
                                          oracle.dbscan(p, F32(1.0), mp))
    c = np.tile(_pts((0.3, -1.25, 7.0)), (50, 1))
    assert (db(ctx, c, 0.0, 50, pair_count=True) == 0).all()
    assert (db(ctx, c, 0.0, 51, pair_count=True) == -1).all()


def test_pair_count_subhalo_sets(ctx):
    pts, off = datagen.subhalo_sets(6, 4, nmin=20000, nmax=200000)
    for s in range(6):
        p = pts[off[s]:off[s + 1]]
        np.testing.assert_array_equal(db(ctx, p, F32(0.05), 5, pair_count=True),
                                      oracle.dbscan(p, F32(0.05), 5))
