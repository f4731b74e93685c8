"""GPU parity: the HIP path against the CPU oracle, element by element.

Integer / index / label outputs must match bit for bit.  Stages are checked
first (Morton codes, sort, tree structure, pair count, core flags) so that a
failure names the stage, then full labels on hand-built, boundary, seeded
and full-size inputs.
"""
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


def run(ctx, p, eps, mp, **kw):
    return ctx.cluster(dev(p), float(eps), mp, **kw).cpu().numpy()


def clumpy(n, seed, k=8):
    rng = np.random.Generator(np.random.PCG64(seed))
    cen = rng.random((k, 3))
    p = cen[rng.integers(0, k, n)] + rng.standard_normal((n, 3)) * 0.02
    m = n // 5
    p[:m] = rng.random((m, 3))
    return p[rng.permutation(n)].astype(F32)


SIZES = [1, 2, 3, 64, 255, 4095, 4096, 4097, 50001]


# ---- stages ----------------------------------------------------------------

# 5000011: several grid-stride rounds of the bounds pass (axis phase
# carried across strides) and a scalar tail
@pytest.mark.parametrize("n", SIZES + [300007, 5000011])
def test_morton_codes_match_oracle(ctx, n):
    p = clumpy(n, n)
    got = ctx.morton_codes(dev(p)).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, oracle.morton63(p))


@pytest.mark.parametrize("n", [1, 6, 4097, 50001])
def test_unaligned_points(ctx, n):
    """A point array that is not 16-byte aligned takes the scalar load path
    of the bounds and Morton kernels: same codes, same labels."""
    p = clumpy(n, 77 + n)
    buf = torch.zeros((n + 1, 3), dtype=torch.float32, device="cuda")
    buf[1:] = dev(p)
    view = buf[1:]
    assert view.data_ptr() % 16 != 0
    got = ctx.morton_codes(view).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, oracle.morton63(p))
    lab = ctx.cluster(view, 0.02, 3).cpu().numpy()
    np.testing.assert_array_equal(lab, oracle.dbscan(p, F32(0.02), 3))
    buf[n, 2] = float("nan")  # last coordinate: the scalar tail
    with pytest.raises(dbx.DbscanError):
        ctx.cluster(view, 0.02, 3)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7])
def test_nonfinite_in_vector_tail(ctx, n):
    """Every coordinate position of small arrays, which lie in the float4
    part or the scalar tail of the bounds kernel, is checked."""
    p = clumpy(n, 5)
    for k in range(3 * n):
        q = p.copy()
        q.reshape(-1)[k] = np.inf
        with pytest.raises(dbx.DbscanError):
            ctx.cluster(dev(q), 0.02, 2)


def test_morton_zero_extent_axis(ctx):
    p = clumpy(5000, 9)
    p[:, 1] = F32(3.5)
    got = ctx.morton_codes(dev(p)).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, oracle.morton63(p))


@pytest.mark.parametrize("n", [1, 5, 4096, 4097, 12345, 1 << 20])
def test_sort_is_stable_and_complete(ctx, n):
    rng = np.random.Generator(np.random.PCG64(n))
    keys = rng.integers(0, 2 ** 63, n, dtype=np.uint64)
    keys[: n // 3] = keys[rng.integers(0, max(1, n // 50), n // 3)]   # many ties
    if n > 10:
        keys[5] = np.uint64(2 ** 64 - 1)                               # top bit set
    vals = np.arange(n, dtype=np.int32)[rng.permutation(n)]
    k = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    v = torch.from_numpy(vals.copy()).cuda()
    ctx.sort_pairs(k, v)
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(k.cpu().numpy().view(np.uint64), keys[order])
    np.testing.assert_array_equal(v.cpu().numpy(), vals[order])


@pytest.mark.parametrize("n", [3000, 4096 * 5 + 17])
@pytest.mark.parametrize("spread", ["low_bits", "middle_constant", "all_equal"])
def test_sort_with_constant_digits(ctx, n, spread):
    """Passes whose digit is the same for every key only copy their tile:
    keys confined to the low 20 bits, keys whose bits 24..47 are constant,
    and all keys equal (every pass a copy; values must keep their order)."""
    rng = np.random.Generator(np.random.PCG64(n + len(spread)))
    if spread == "low_bits":
        keys = rng.integers(0, 2 ** 20, n, dtype=np.uint64)
    elif spread == "middle_constant":
        lo = rng.integers(0, 2 ** 24, n, dtype=np.uint64)
        hi = rng.integers(0, 2 ** 16, n, dtype=np.uint64) << np.uint64(48)
        keys = lo | hi | (np.uint64(0xA5) << np.uint64(32))
    else:
        keys = np.full(n, np.uint64(0x0123456789ABCDEF))
    vals = np.arange(n, dtype=np.int32)[rng.permutation(n)]
    k = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    v = torch.from_numpy(vals.copy()).cuda()
    ctx.sort_pairs(k, v)
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(k.cpu().numpy().view(np.uint64), keys[order])
    np.testing.assert_array_equal(v.cpu().numpy(), vals[order])


def _walk(nodes, leaf, root, n):
    """Pre-order walk that always descends: internal -> left child, leaf ->
    its rope.  Returns the visit sequence (node refs)."""
    left = nodes[:, 3].view(np.int32) if n > 1 else None
    lrope = leaf[:, 3].view(np.int32)
    seq = []
    node = int(root)
    while node != -1:
        seq.append(node)
        if len(seq) > 2 * n + 5:
            raise AssertionError("walk does not terminate")
        node = int(lrope[node & 0x7FFFFFFF]) if node < -1 else int(left[node])
    return seq


@pytest.mark.parametrize("n", [1, 2, 3, 17, 4097, 50001])
def test_tree_structure(ctx, n):
    p = clumpy(n, 100 + n)
    perm, leaf, nodes, root = ctx.build_tree(dev(p))
    perm, leaf, nodes = perm.cpu().numpy(), leaf.cpu().numpy(), nodes.cpu().numpy()
    root = int(root.cpu().numpy()[0])
    # leaves are the points in stable Morton order
    np.testing.assert_array_equal(perm, oracle.morton_order(oracle.morton63(p)))
    np.testing.assert_array_equal(leaf[:, :3], p[perm])
    seq = _walk(nodes, leaf, root, n)
    assert len(seq) == 2 * n - 1
    lv = [s & 0x7FFFFFFF for s in seq if s < -1]
    assert lv == list(range(n))                        # leaves in order, once each
    iv = sorted(s for s in seq if s >= 0)
    assert iv == list(range(n - 1))                    # every internal node once
    if n > 1:
        rope = nodes[:, 7].view(np.int32)
        left = nodes[:, 3].view(np.int32)
        lrope = leaf[:, 3].view(np.int32)

        def box(ref):
            if ref < -1:
                q = leaf[ref & 0x7FFFFFFF, :3]
                return q, q
            return nodes[ref, 0:3], nodes[ref, 4:7]

        for k in range(n - 1):
            lc = int(left[k])
            rc = int(lrope[lc & 0x7FFFFFFF]) if lc < -1 else int(rope[lc])
            (a0, a1), (b0, b1) = box(lc), box(rc)
            np.testing.assert_array_equal(nodes[k, 0:3], np.minimum(a0, b0))
            np.testing.assert_array_equal(nodes[k, 4:7], np.maximum(a1, b1))
        np.testing.assert_array_equal(nodes[root, 0:3], p.min(0))
        np.testing.assert_array_equal(nodes[root, 4:7], p.max(0))
        # Karras order: the root is number 0, and every rope leads to the
        # subtree starting right after the last leaf of the one it leaves,
        # numbered (leaf or node) by that first leaf
        assert root == 0
        first = np.full(n - 1, -1, np.int64)
        last = np.full(n - 1, -1, np.int64)
        order = [s for s in seq if s >= 0]
        for k in reversed(order):  # children before parents
            lc = int(left[k])
            rc = int(lrope[lc & 0x7FFFFFFF]) if lc < -1 else int(rope[lc])
            first[k] = (lc & 0x7FFFFFFF) if lc < -1 else first[lc]
            last[k] = (rc & 0x7FFFFFFF) if rc < -1 else last[rc]
            assert k in (first[k], last[k]) or k == 0
        for k in range(n - 1):
            t = int(rope[k])
            if t != -1:
                assert (t & 0x7FFFFFFF if t < -1 else t) == last[k] + 1
                assert t < -1 or first[t] == last[k] + 1
        for j in range(n):
            t = int(lrope[j])
            if t != -1:
                assert (t & 0x7FFFFFFF if t < -1 else t) == j + 1


@pytest.mark.parametrize("n,eps", [(2, 0.5), (4097, 0.03), (50001, 0.02), (300007, 0.01)])
def test_pair_traversal_finds_each_pair_once(ctx, n, eps):
    p = clumpy(n, 7 + n)
    assert ctx.pair_count(dev(p), eps) == oracle.pair_count(p, F32(eps))


@pytest.mark.parametrize("eps,passes", [(1e-6, 8), (5e-6, 7), (2e-5, 6), (1e-4, 5), (4e-4, 4),
                                         (0.02, 3)])
def test_code_bits_dropped_by_eps(ctx, eps, passes):
    """In a unit cube these radii let the clustering call clear 0 to 40 low
    code bits (0 to 5 skipped sort passes, odd and even; the last two only
    by the sparse-cell rule): pairs and labels must not change.  Near-copies
    of some points at several small offsets give every radius some pairs."""
    base = clumpy(40000, 123)
    rng = np.random.Generator(np.random.PCG64(5))
    # 49,003 points: an odd count, so the sort's second 32-bit words (at n + i)
    # are not 16-byte aligned
    extra = [base[rng.integers(0, 40000, m)] + rng.normal(0, d, (m, 3)).astype(F32)
             for d, m in ((2e-6, 3000), (1e-5, 3001), (5e-5, 3002))]
    p = np.clip(np.concatenate([base] + extra), 0, 1).astype(F32)
    p = p[rng.permutation(p.shape[0])]
    assert ctx.pair_count(dev(p), eps) == oracle.pair_count(p, F32(eps))
    np.testing.assert_array_equal(run(ctx, p, eps, 2, algorithm="fdbscan"),
                                  oracle.dbscan(p, F32(eps), 2))
    assert ctx.sort_passes() == passes
    np.testing.assert_array_equal(run(ctx, p, eps, 4, algorithm="fdbscan"),
                                  oracle.dbscan(p, F32(eps), 4))


def test_traversal_stats_counts(ctx):
    """The instrumented traversal finds the same pairs; every pair is one
    leaf test that passed, and each query but the last visits at least one
    node (its leaf's rope)."""
    n, eps = 50001, 0.02
    p = clumpy(n, 31)
    st = ctx.traversal_stats(dev(p), eps)
    assert st["pairs"] == oracle.pair_count(p, F32(eps))
    assert st["leaf_tests"] >= st["pairs"]
    assert st["internal_visits"] >= st["descents"]
    assert st["internal_visits"] + st["leaf_tests"] >= n - 1
    assert st["descents"] > 0  # pairs exist, so some walks entered subtrees


@pytest.mark.parametrize("mp", [1, 2, 3, 5, 10, 50])
def test_core_flags(ctx, mp):
    p = clumpy(40000, 5)
    got = ctx.core_flags(dev(p), 0.02, mp).cpu().numpy().astype(bool)
    np.testing.assert_array_equal(got, oracle.core_flags(p, F32(0.02), mp))


# ---- labels ----------------------------------------------------------------

def _pts(*rows):
    return np.array(rows, dtype=F32).reshape(-1, 3)


def test_hand_cases(ctx):
    # exact boundary, one ulp beyond
    assert run(ctx, _pts((0, 0, 0), (0.5, 0, 0)), 0.5, 2).tolist() == [0, 0]
    x = np.nextafter(F32(0.5), F32(1))
    assert run(ctx, _pts((0, 0, 0), (x, 0, 0)), 0.5, 2).tolist() == [-1, -1]
    # chain at exact spacing, and just below it
    c = np.zeros((1000, 3), F32)
    c[:, 0] = np.arange(1000, dtype=F32) * F32(0.25)
    assert (run(ctx, c, 0.25, 2) == 0).all()
    assert (run(ctx, c, np.nextafter(F32(0.25), F32(0)), 2) == -1).all()
    # subnormal threshold, underflow at eps = 0, overflow
    assert run(ctx, _pts((0, 0, 0), (2e-20, 0, 0)), F32(1e-20), 2).tolist() == [-1, -1]
    assert run(ctx, _pts((0, 0, 0), (1e-20, 0, 0)), F32(1e-20), 2).tolist() == [0, 0]
    assert run(ctx, _pts((1e-30, 0, 0), (2e-30, 0, 0), (5e-30, 0, 0)), 0.0, 2).tolist() == [0, 0, 0]
    assert run(ctx, _pts((0, 0, 0), (1e-22, 0, 0)), 0.0, 2).tolist() == [-1, -1]
    assert run(ctx, _pts((-1e30, 0, 0), (1e30, 0, 0), (1e30, 0, 0)), 1e18, 2).tolist() == [-1, 1, 1]
    # tiny inputs
    assert run(ctx, _pts((1, 2, 3)), 1.0, 1).tolist() == [0]
    assert run(ctx, _pts((1, 2, 3)), 1.0, 2).tolist() == [-1]


def test_border_rules(ctx):
    A = [(0.0, 0, 0), (-0.1, 0, 0), (-0.2, 0, 0), (-0.3, 0, 0)]
    B = [(2.0, 0, 0), (2.1, 0, 0), (2.2, 0, 0), (2.3, 0, 0)]
    b = [(1.0, 0, 0)]
    for pts in (B + A + b, A + B + b, b + B + A, b + A + B):
        p = _pts(*pts)
        np.testing.assert_array_equal(run(ctx, p, 1.0, 4), oracle.dbscan(p, F32(1.0), 4))


def test_fp_boundary_golden_cases(ctx):
    with open(os.path.join(GOLDEN, "fp_boundary_cases.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            v = [F32(float.fromhex(x)) for x in t[1:8]]
            p = np.array([v[0:3], v[3:6]], F32)
            exp = [0, 0] if int(t[8]) else [-1, -1]
            assert run(ctx, p, v[6], 2).tolist() == exp, line


@pytest.mark.parametrize("k", [1, 7, 3000])
def test_identical_points(ctx, k):
    """All points equal: one cluster (minPts <= k); union-find contention on
    k(k-1)/2 pairs."""
    p = np.tile(_pts((0.3, -1.25, 7.0)), (k, 1))
    assert (run(ctx, p, 0.0, min(k, 5)) == 0).all()
    assert (run(ctx, p, 0.0, k + 1) == -1).all()


def test_dense_ball_one_cluster(ctx):
    rng = np.random.Generator(np.random.PCG64(14))
    d = rng.standard_normal((5000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p = (d * rng.random((5000, 1)) * 0.1).astype(F32)
    for mp in (2, 10):
        assert (run(ctx, p, 1.0, mp) == 0).all()


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("mp", [1, 2, 3, 5, 10])
def test_random_clumpy_labels(ctx, seed, mp):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(10, 20000))
    p = clumpy(n, seed)
    eps = F32(rng.uniform(0.005, 0.05))
    np.testing.assert_array_equal(run(ctx, p, eps, mp), oracle.dbscan(p, eps, mp))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mp", [3, 5, 10, 40])
def test_pair_count_core_flags(ctx, seed, mp):
    """Core points found by pair traversal (DBSCAN_FLAG_PAIR_COUNT): the same
    labels as the oracle, across sizes that span tiles and a ragged tail."""
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    n = int(rng.integers(10, 70000))
    p = clumpy(n, 100 + seed)
    eps = F32(rng.uniform(0.004, 0.04))
    np.testing.assert_array_equal(run(ctx, p, eps, mp, pair_count=True),
                                  oracle.dbscan(p, eps, mp))


@pytest.mark.parametrize("mp", [3, 6])
def test_pair_count_sparse_dense_and_mixed(ctx, mp):
    """With counting by pair traversal the main phase starts no walk at a
    point with no neighbour: a sparse field (most points have none), a tight
    clump (thousands of neighbours a point) and both together."""
    rng = np.random.Generator(np.random.PCG64(77 + mp))
    sparse = rng.random((60000, 3)).astype(F32)
    clump = (0.5 + rng.standard_normal((8000, 3)) * 0.004).astype(F32)
    both = np.concatenate([sparse, clump])[rng.permutation(68000)]
    for p, eps in ((sparse, 0.012), (clump, 0.01), (both, 0.012)):
        np.testing.assert_array_equal(run(ctx, p, eps, mp, pair_count=True),
                                      oracle.dbscan(p, F32(eps), mp))


def test_pair_count_no_core_point(ctx):
    """Counting by pair traversal on a field with no core point (the main
    phase starts no walk: every label is noise), between calls that have
    core points (the core-point count starts from zero on every call)."""
    rng = np.random.Generator(np.random.PCG64(79))
    sparse = rng.random((60000, 3)).astype(F32)
    ref = oracle.dbscan(sparse, F32(0.012), 12)
    assert (ref == -1).all()
    for eps, mp in ((0.012, 12), (0.012, 3), (0.012, 12), (0.05, 12)):
        np.testing.assert_array_equal(run(ctx, sparse, eps, mp, pair_count=True),
                                      ref if mp == 12 and eps == 0.012
                                      else oracle.dbscan(sparse, F32(eps), mp))


@pytest.mark.parametrize("mp", [2, 5, 10])
def test_clumps32k(ctx, mp):
    p = datagen.config_points("clumps32k")
    np.testing.assert_array_equal(run(ctx, p, F32(0.006), mp), oracle.dbscan(p, F32(0.006), mp))


def test_ragged_and_block_sizes_deterministic(ctx):
    p = clumpy(70001, 3)
    ref = oracle.dbscan(p, F32(0.01), 4)
    for bs in (64, 128, 256, 512, 1024):
        np.testing.assert_array_equal(run(ctx, p, 0.01, 4, block_size=bs), ref)


def test_default_context_and_host_entry(ctx):
    p = clumpy(9000, 4)
    ref = oracle.dbscan(p, F32(0.02), 3)
    np.testing.assert_array_equal(dbx.cluster(dev(p), 0.02, 3).cpu().numpy(), ref)
    lib = dbx.load_library()
    lab = np.empty(p.shape[0], np.int32)
    import ctypes
    st = lib.dbscan_cluster_host(p.ctypes.data_as(ctypes.c_void_p), p.shape[0],
                                 ctypes.c_float(0.02), 3, lab.ctypes.data_as(ctypes.c_void_p))
    assert st == 0
    np.testing.assert_array_equal(lab, ref)


def test_nonfinite_rejected(ctx):
    p = clumpy(1000, 1)
    p[500, 1] = np.nan
    with pytest.raises(dbx.DbscanError) as e:
        run(ctx, p, 0.01, 2)
    assert e.value.code == -2
    p[500, 1] = np.inf
    with pytest.raises(dbx.DbscanError) as e:
        run(ctx, p, 0.01, 2)
    assert e.value.code == -2
    # the context still works afterwards
    q = clumpy(1000, 2)
    np.testing.assert_array_equal(run(ctx, q, 0.02, 2), oracle.dbscan(q, F32(0.02), 2))


def test_budget_too_small():
    c = dbx.Context(0, budget_bytes=1 << 20)
    with pytest.raises(dbx.DbscanError) as e:
        c.cluster(dev(clumpy(100000, 1)), 0.01, 2)
    assert e.value.code == -5
    c.close()


# ---- full size -----------------------------------------------------------------

def oracle_threads(fn):
    """Run an oracle call with its counting and border steps on the host's
    cores (at most 16, the box's share); labels do not depend on it."""
    oracle.set_threads(min(16, os.cpu_count() or 1))
    try:
        return fn()
    finally:
        oracle.set_threads(1)


@pytest.fixture(scope="module")
def halo16m():
    p = datagen.config_points("halo16M")
    return p, oracle_threads(lambda: oracle.dbscan(p, F32(0.2), 2))


def test_halo16m_minpts2_bit_exact(ctx, halo16m):
    p, ref = halo16m
    np.testing.assert_array_equal(run(ctx, p, F32(0.2), 2), ref)


def test_halo16m_minpts3_both_core_modes_bit_exact(ctx, halo16m):
    """minPts 3 on the 2^24-point field: core points from the counting walk
    and from the pair traversal, each against the oracle."""
    p, _ = halo16m
    ref = oracle_threads(lambda: oracle.dbscan(p, F32(0.2), 3))
    assert (ref >= 0).any() and (ref < 0).any()
    d = dev(p)
    np.testing.assert_array_equal(ctx.cluster(d, 0.2, 3).cpu().numpy(), ref)
    np.testing.assert_array_equal(ctx.cluster(d, 0.2, 3, pair_count=True).cpu().numpy(), ref)


def test_autotune_returns_options_that_keep_labels(ctx):
    p = clumpy(60000, 21)
    ref = oracle.dbscan(p, F32(0.01), 4)
    for algo in ("fdbscan", "densebox"):
        best = ctx.autotune(dev(p), 0.01, 4, algorithm=algo)
        assert best["block_size"] in (64, 128, 256, 512) and best["ms"] > 0
        assert best["sort_tile"] in (0, 2048, 3072)
        got = run(ctx, p, 0.01, 4, algorithm=algo, block_size=best["block_size"],
                  dense_threshold=best["dense_threshold"], pair_count=best["pair_count"],
                  sort_tile=best["sort_tile"])
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("tile", [2048, 3072, 4096])
@pytest.mark.parametrize("n", [1, 3071, 3073, 50001])
def test_sort_tiles_keep_labels(ctx, tile, n):
    """Each radix-sort tile size (one tile, a ragged last tile, many tiles)
    gives the oracle's labels with both algorithms."""
    p = clumpy(n, 300 + n)
    ref = oracle.dbscan(p, F32(0.02), 3)
    for algo in ("fdbscan", "densebox"):
        np.testing.assert_array_equal(run(ctx, p, 0.02, 3, algorithm=algo, sort_tile=tile), ref)


def test_sort_tile_rejected(ctx):
    p = dev(clumpy(100, 1))
    for t in (-1, 1024, 4097, 8192):
        with pytest.raises(dbx.DbscanError) as e:
            ctx.cluster(p, 0.02, 2, sort_tile=t)
        assert e.value.code == -1


def test_autotune_cache(ctx, tmp_path):
    p = clumpy(40000, 23)
    path = tmp_path / "tune.json"
    a = ctx.autotune(dev(p), 0.01, 4, cache=path)
    b = ctx.autotune(dev(p), 0.01, 4, cache=path)
    assert a["cached"] is False and b["cached"] is True
    assert {k: a[k] for k in a if k != "cached"} == {k: b[k] for k in b if k != "cached"}
    # same size class, same parameters: the cached pick; another minPts: tuned
    assert ctx.autotune(dev(clumpy(41000, 24)), 0.01, 4, cache=path)["cached"] is True
    assert ctx.autotune(dev(p), 0.01, 5, cache=path)["cached"] is False
