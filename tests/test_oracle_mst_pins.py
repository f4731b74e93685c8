"""Pins for the oracle's minimum spanning trees (the Euclidean tree of
section 3.2's algorithm list, and the mutual reachability tree HDBSCAN*
clusters from, section 5), against values that do not come from the oracle:

* every spanning tree of tiny inputs enumerated by brute force: the tree
  under the strict order (w, lo, hi) is the one whose sorted edge list is
  lexicographically smallest (the greedy basis of a matroid), with core
  distances taken from a numpy sort of each point's distance row;
* scipy's minimum spanning tree on inputs without equal weights;
* the cycle property on every edge outside the tree: each edge on the tree
  path between its ends comes before it;
* closed forms: equally spaced points on a line, with and without core
  distances (ties at the line's ends);
* planted mistakes: each mutant build of the MST oracle fails a pin.
"""
import itertools
import os
import tempfile

import numpy as np
import pytest
from scipy.sparse.csgraph import minimum_spanning_tree

import oracle

F32 = np.float32


def _d2(p):
    """binary32 squared distances, every operation rounded (numpy does not
    contract float32 expressions)."""
    d = p[:, None, :] - p[None, :, :]
    sq = d * d
    return (sq[..., 0] + sq[..., 1]) + sq[..., 2]


def _core(p, min_pts):
    d = _d2(p)
    if min_pts <= 1:
        return np.zeros(p.shape[0], F32)
    s = np.sort(d, axis=1)
    return np.where(min_pts <= p.shape[0], s[:, min(min_pts, p.shape[0]) - 1], np.inf).astype(F32)


def _weights(p, core):
    d = _d2(p)
    return np.maximum(np.maximum(d, core[:, None]), core[None, :]).astype(F32)


def _brute_tree(p, min_pts):
    n = p.shape[0]
    w = _weights(p, _core(p, min_pts))
    edges = [(float(w[i, j]), i, j) for i in range(n) for j in range(i + 1, n)]
    best = None
    for sub in itertools.combinations(range(len(edges)), n - 1):
        parent = list(range(n))

        def find(x):
            while parent[x] != x:
                x = parent[x]
            return x
        ok = True
        for k in sub:
            _, a, b = edges[k]
            ra, rb = find(a), find(b)
            if ra == rb:
                ok = False
                break
            parent[ra] = rb
        if not ok:
            continue
        seq = sorted(edges[k] for k in sub)
        if best is None or seq < best:
            best = seq
    return best


def _as_list(edges, w):
    return [(float(x), int(a), int(b)) for (a, b), x in zip(edges, w)]


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("min_pts", [1, 2, 3])
def test_every_spanning_tree_of_tiny_inputs(n, min_pts):
    rng = np.random.Generator(np.random.PCG64(100 * n + min_pts))
    cases = [rng.random((n, 3)).astype(F32),
             rng.integers(0, 2, (n, 3)).astype(F32),            # lattice: many ties
             np.repeat(rng.random((1, 3)).astype(F32), n, 0)]   # all duplicates
    for p in cases:
        e, w = oracle.mst(p, min_pts)
        assert _as_list(e, w) == _brute_tree(p, min_pts)


def test_scipy_without_ties():
    iu = np.triu_indices(70, 1)
    done = 0
    for seed in range(40):  # inputs without equal weights (most of them at 70 points)
        p = np.random.Generator(np.random.PCG64(seed)).random((70, 3)).astype(F32)
        w = _d2(p)
        if np.unique(w[iu]).size != iu[0].size:
            continue
        t = minimum_spanning_tree(np.triu(w.astype(np.float64), 1)).tocoo()
        ref = sorted((float(x), int(min(a, b)), int(max(a, b))) for a, b, x in
                     zip(t.row, t.col, t.data))
        e, ww = oracle.mst(p)
        assert _as_list(e, ww) == ref
        done += 1
    assert done >= 20


def _cycle_property_failures(p, min_pts, lib=None):
    n = p.shape[0]
    e, w = oracle.mst(p, min_pts, lib=lib)
    if e.shape != (n - 1, 2):
        return ["size"]
    W = _weights(p, _core(p, min_pts))
    adj = [[] for _ in range(n)]
    for (a, b), x in zip(e, w):
        if x != W[a, b] or a >= b:
            return ["weight"]
        adj[a].append(b)
        adj[b].append(a)
    fails = []
    for s in range(n):
        # parent pointers of the tree rooted at s
        par = [-1] * n
        par[s] = s
        stack = [s]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if par[y] < 0:
                    par[y] = x
                    stack.append(y)
        if min(par) < 0:
            return ["not spanning"]
        for t in range(s + 1, n):
            key = (float(W[s, t]), s, t)
            x = t
            while x != s:
                y = par[x]
                k = (float(W[x, y]), min(x, y), max(x, y))
                if k > key:
                    fails.append((s, t))
                    break
                x = y
    return fails


@pytest.mark.parametrize("min_pts", [1, 2, 4])
def test_cycle_property(min_pts):
    rng = np.random.Generator(np.random.PCG64(9 + min_pts))
    for p in (rng.random((80, 3)).astype(F32),
              rng.integers(0, 3, (60, 3)).astype(F32),
              np.concatenate([rng.random((30, 3)), rng.random((30, 3))]).astype(F32)):
        assert _cycle_property_failures(p, min_pts) == []


def test_line_closed_form():
    perm = np.random.Generator(np.random.PCG64(3)).permutation(12)
    x = perm.astype(F32)
    p = np.stack([x, np.zeros(12, F32), np.zeros(12, F32)], 1)
    inv = np.argsort(perm)  # inv[k]: the input index of the point at x = k
    pairs = sorted((min(inv[k], inv[k + 1]), max(inv[k], inv[k + 1])) for k in range(11))
    e, w = oracle.mst(p)
    assert [tuple(r) for r in e.tolist()] == pairs and (w == 1).all()
    # minPts 3: interior core 1 (self, two neighbours at 1), the ends 4.
    # The nine inner edges weigh 1; an end point joins at weight 4 through
    # its neighbour or the one after (D = 4, both weigh max(4, 1, D) = 4),
    # whichever pair (lo, hi) is smaller
    e, w = oracle.mst(p, 3)

    def pr(a, b):
        return (min(inv[a], inv[b]), max(inv[a], inv[b]))
    inner = sorted(pr(k, k + 1) for k in range(1, 10))
    ends = sorted([min(pr(0, 1), pr(0, 2)), min(pr(11, 10), pr(11, 9))])
    assert [tuple(r) for r in e.tolist()] == inner + ends
    assert w.tolist() == [1.0] * 9 + [4.0, 4.0]


def test_small_and_invalid():
    assert oracle.mst(np.zeros((0, 3), F32))[0].shape == (0, 2)
    assert oracle.mst(np.zeros((1, 3), F32))[0].shape == (0, 2)
    p = np.zeros((3, 3), F32)
    p[1, 0] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.mst(p)


def _mst_pin_failures(lib):
    fails = []
    rng = np.random.Generator(np.random.PCG64(41))
    for n, mp in ((5, 1), (5, 3), (6, 2)):
        for p in (rng.integers(0, 2, (n, 3)).astype(F32), rng.random((n, 3)).astype(F32)):
            e, w = oracle.mst(p, mp, lib=lib)
            if _as_list(e, w) != _brute_tree(p, mp):
                fails.append(f"brute-{n}-{mp}")
    if _cycle_property_failures(rng.random((40, 3)).astype(F32), 4, lib=lib):
        fails.append("cycle")
    return fails


def test_mst_pins_pass_on_the_real_oracle(oracle_lib):
    assert _mst_pin_failures(oracle_lib) == []


@pytest.mark.parametrize("mutant", ["TIE_HI_FIRST", "NO_CORE", "ONE_CORE"])
def test_mst_pins_catch_planted_mistake(mutant):
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build(extra_flags=[f"-DMST_MUTANT_{mutant}"],
                            out=os.path.join(d, "liboracle_mst_mutant.so"))
        lib = oracle.load(path)
        assert _mst_pin_failures(lib), f"mutant {mutant} passed every pin"
