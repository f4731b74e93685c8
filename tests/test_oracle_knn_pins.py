"""Pins for the oracle's k-nearest-neighbour search (section 3.2, nearest
search) and the core distances built on it (HDBSCAN*, section 5), against
values that do not come from the oracle itself:

* hand cases worked out from the definition: points on a line, ties in D
  going to the smaller index, exact duplicates, k larger than the set;
* a numpy brute force (float32 arithmetic rounds every operation, and a
  stable lexicographic sort orders (D, index));
* scipy's k-d tree (float64) on inputs whose neighbour distances are far
  apart, where the float32 order cannot differ;
* exact metamorphic relations: scaling by 2^k, reflection, swapping x and y,
  input permutation;
* the DBSCAN oracle: a point has at least minPts neighbours within eps (self
  included) exactly when its minPts-th nearest neighbour has D <= fl(eps^2);
* planted mistakes: each mutant build of the kNN oracle fails a pin.
"""
import os
import tempfile

import numpy as np
import pytest
from scipy.spatial import cKDTree

import datagen
import oracle

F32 = np.float32


def _pts(*rows):
    return np.array(rows, dtype=F32).reshape(-1, 3)


def brute_knn(p, k):
    """The definition in numpy: D in binary32 per operation, then the k
    smallest (D, j) per row by a stable lexicographic sort."""
    p = np.asarray(p, dtype=F32)
    n = p.shape[0]
    d = [(p[:, None, a] - p[None, :, a]).astype(F32) for a in range(3)]
    sq = [(x * x).astype(F32) for x in d]
    D = ((sq[0] + sq[1]).astype(F32) + sq[2]).astype(F32)
    idx = np.full((n, k), -1, np.int32)
    dd = np.full((n, k), np.inf, F32)
    for i in range(n):
        order = np.lexsort((np.arange(n), D[i]))[:k]
        idx[i, :order.size] = order
        dd[i, :order.size] = D[i, order]
    return idx, dd


def test_line_by_hand():
    p = _pts((0, 0, 0), (1, 0, 0), (3, 0, 0), (6, 0, 0), (10, 0, 0))
    idx, d2 = oracle.knn(p, 3)
    np.testing.assert_array_equal(idx, [[0, 1, 2], [1, 0, 2], [2, 1, 0], [3, 2, 4], [4, 3, 2]])
    np.testing.assert_array_equal(d2, [[0, 1, 9], [0, 1, 4], [0, 4, 9], [0, 9, 16],
                                       [0, 16, 49]])


def test_ties_go_to_the_smaller_index():
    # the query (index 2) has neighbours at distance 1 on both sides
    p = _pts((1, 0, 0), (-1, 0, 0), (0, 0, 0), (0, 1, 0), (0, 0, -1))
    idx, d2 = oracle.knn(p, 4, queries=[2])
    np.testing.assert_array_equal(idx, [[2, 0, 1, 3]])
    np.testing.assert_array_equal(d2, [[0, 1, 1, 1]])


def test_duplicates_and_k_beyond_n():
    p = _pts((5, 5, 5), (5, 5, 5), (5, 5, 6), (5, 5, 5))
    idx, d2 = oracle.knn(p, 6)
    np.testing.assert_array_equal(idx[0], [0, 1, 3, 2, -1, -1])
    np.testing.assert_array_equal(idx[3], [0, 1, 3, 2, -1, -1])
    np.testing.assert_array_equal(idx[2], [2, 0, 1, 3, -1, -1])
    np.testing.assert_array_equal(d2[2], [0, 1, 1, 1, np.inf, np.inf])
    assert oracle.core_distances(p, 3).tolist() == [0, 0, 1, 0]
    assert np.isinf(oracle.core_distances(p, 5)).all()


def test_invalid_arguments():
    with pytest.raises(oracle.OracleError) as e:
        oracle.knn(_pts((0, 0, 0)), 0)
    assert e.value.code == -1
    with pytest.raises(oracle.OracleError) as e:
        oracle.knn(_pts((0, 0, np.nan)), 2)
    assert e.value.code == -2
    with pytest.raises(oracle.OracleError) as e:
        oracle.knn(_pts((0, 0, 0)), 1, queries=[1])
    assert e.value.code == -1


@pytest.mark.parametrize("seed,k", [(s, k) for s in range(6) for k in (1, 4, 16)])
def test_matches_numpy_brute_force(seed, k):
    rng = np.random.Generator(np.random.PCG64(400 + seed))
    n = int(rng.integers(20, 600))
    if seed % 3 == 0:  # a lattice: many exact ties
        p = (rng.integers(0, 6, (n, 3)) * 0.5).astype(F32)
    elif seed % 3 == 1:  # duplicates
        base = rng.random((max(1, n // 4), 3)).astype(F32)
        p = base[rng.integers(0, base.shape[0], n)]
    else:
        p = datagen.clumps(n, seed)
    idx, d2 = oracle.knn(p, k)
    bi, bd = brute_knn(p, k)
    np.testing.assert_array_equal(idx, bi)
    np.testing.assert_array_equal(d2, bd)


def test_matches_kdtree_without_near_ties():
    """On well-separated neighbour distances the float32 order is the real
    one: the index lists equal scipy's (float64) k-d tree answer."""
    rng = np.random.Generator(np.random.PCG64(11))
    p = (rng.random((3000, 3)) * 100).astype(F32)
    k = 8
    dist, nb = cKDTree(p.astype(np.float64)).query(p.astype(np.float64), k=k + 1)
    gaps = np.diff(dist, axis=1).min(axis=1)
    ok = gaps > 1e-3  # no two of the k + 1 nearest are within 1e-3
    assert ok.sum() > 2000
    idx, _ = oracle.knn(p, k)
    np.testing.assert_array_equal(idx[ok], nb[ok, :k])


def test_metamorphic_exact():
    p = datagen.clumps(4000, 5)
    k = 7
    idx, d2 = oracle.knn(p, k)
    for s in (F32(2.0 ** -4), F32(2.0 ** 6)):  # D scales by 4^k exactly
        i2, d = oracle.knn(p * s, k)
        np.testing.assert_array_equal(i2, idx)
        np.testing.assert_array_equal(d, d2 * s * s)
    q = p.copy()
    q[:, 2] = -q[:, 2]  # reflection: fl(-a - -b) = -fl(a - b)
    np.testing.assert_array_equal(oracle.knn(q, k)[0], idx)
    np.testing.assert_array_equal(oracle.knn(p[:, [1, 0, 2]], k)[1], d2)  # x <-> y
    # permutation: the same neighbour sets, up to the order of equal D
    pi = np.random.Generator(np.random.PCG64(3)).permutation(p.shape[0])
    ip, dp = oracle.knn(p[pi], k)
    np.testing.assert_array_equal(dp, d2[pi])
    strict = d2[pi][:, :-1] < d2[pi][:, 1:]
    ok = strict.all(axis=1)  # rows without ties: the same neighbours in the same order
    np.testing.assert_array_equal(pi[ip[ok]], idx[pi][ok])


@pytest.mark.parametrize("min_pts", [2, 3, 5, 10])
def test_core_distance_agrees_with_dbscan_counts(min_pts):
    """|N_eps(x)| >= minPts (self included) iff the minPts-th nearest
    neighbour of x has D <= fl(eps*eps)."""
    p = datagen.clumps(20000, 8)
    eps = F32(0.01)
    core = oracle.neighbour_counts(p, eps) >= min_pts
    cd = oracle.core_distances(p, min_pts)
    np.testing.assert_array_equal(cd <= F32(eps * eps), core)


def test_threads_do_not_change_the_result():
    p = datagen.clumps(5000, 9)
    a = oracle.knn(p, 9)
    try:
        oracle.set_threads(4)
        b = oracle.knn(p, 9)
    finally:
        oracle.set_threads(1)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def _knn_pin_failures(lib):
    fails = []
    p = _pts((0, 0, 0), (1, 0, 0), (3, 0, 0), (6, 0, 0), (10, 0, 0))
    i, d = oracle.knn(p, 3, lib=lib)
    if i.tolist() != [[0, 1, 2], [1, 0, 2], [2, 1, 0], [3, 2, 4], [4, 3, 2]]:
        fails.append("line")
    i, _ = oracle.knn(_pts((1, 0, 0), (-1, 0, 0), (0, 0, 0), (0, 1, 0), (0, 0, -1)), 4,
                     queries=[2], lib=lib)
    if i.tolist() != [[2, 0, 1, 3]]:
        fails.append("ties")
    rng = np.random.Generator(np.random.PCG64(77))
    for t in range(3):
        q = (rng.random((300, 3)) * [1, 1, 3] + rng.random(3)).astype(F32)
        a, b = oracle.knn(q, 5, lib=lib)
        bi, bd = brute_knn(q, 5)
        if not (np.array_equal(a, bi) and np.array_equal(b, bd)):
            fails.append(f"brute-{t}")
    return fails


def test_knn_pins_pass_on_the_real_oracle(oracle_lib):
    assert _knn_pin_failures(oracle_lib) == []


@pytest.mark.parametrize("mutant", ["TIE_LARGER", "NO_SELF", "FMA", "NO_DZ"])
def test_knn_pins_catch_planted_mistake(mutant):
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build(extra_flags=[f"-DKNN_MUTANT_{mutant}"],
                            out=os.path.join(d, "liboracle_knn_mutant.so"))
        lib = oracle.load(path)
        assert _knn_pin_failures(lib), f"mutant {mutant} passed every pin"
