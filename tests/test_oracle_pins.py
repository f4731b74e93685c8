"""Pins for the CPU oracle: checks it against things other than itself.

* the definition evaluated by brute force (O(N^2) adjacency + scipy
  connected components) on small seeded inputs, with eps placed exactly on
  pair distances so the "<=" boundary is exercised;
* hand-built cases whose answer follows from the definition by hand
  (boundary equality, subnormals, underflow, overflow, the border and label
  rules);
* binary32 boundary cases found and decided with exact rational arithmetic
  (tests/golden/fp_boundary_cases.txt);
* special cases: minPts = 2 is connected components of the eps-graph minus
  singletons (section 4.3.1), minPts = 1 has no noise, eps = 0 groups exact
  duplicates;
* exact metamorphic relations (reflection, axis swap x<->y, scaling by 2^k,
  input permutation);
* planted mistakes: each mutant build of the oracle fails at least one pin.
"""
import os
import tempfile

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

import bruteforce
import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32


def _canon(groups):
    return bruteforce.canonical(np.asarray(groups))


# ---- random inputs against the brute-force definition ---------------------

def _family(kind, n, rng):
    if kind == "clumpy":
        k = rng.integers(1, 6)
        cen = rng.random((k, 3))
        idx = rng.integers(0, k, n)
        p = cen[idx] + rng.standard_normal((n, 3)) * rng.uniform(0.01, 0.05)
        bg = rng.random((n // 4, 3))
        return np.concatenate([p, bg]).astype(F32)
    if kind == "lattice":
        g = rng.integers(0, 8, (n, 3)).astype(F32) * F32(0.25)
        return g
    if kind == "dups":
        base = rng.random((max(1, n // 5), 3)).astype(F32)
        return base[rng.integers(0, base.shape[0], n)]
    if kind == "flat":  # zero extent in one axis
        p = rng.random((n, 3)).astype(F32)
        p[:, 2] = F32(5.0)
        return p
    raise KeyError(kind)


def _boundary_eps(p, rng):
    """eps such that fl(eps*eps) sits on (or next to) an actual pair's D."""
    i, j = rng.integers(0, p.shape[0], 2)
    d = p[i] - p[j]
    D = F32(F32(d[0] * d[0]) + F32(d[1] * d[1])) + F32(d[2] * d[2])
    e = F32(np.sqrt(np.float64(D)))
    if e == 0:
        e = F32(0.02)
    return F32(np.nextafter(e, F32(np.inf)) if rng.random() < 0.3 else e)


CASES = [(kind, seed, mp) for kind in ("clumpy", "lattice", "dups", "flat")
         for seed in range(6) for mp in (1, 2, 3, 5, 10)]


@pytest.mark.parametrize("kind,seed,min_pts", CASES)
def test_oracle_matches_bruteforce(kind, seed, min_pts):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    p = _family(kind, int(rng.integers(50, 700)), rng)
    eps = _boundary_eps(p, rng) if seed % 2 == 0 else F32(rng.uniform(0.01, 0.3))
    exp, exp_core = bruteforce.dbscan(p, eps, min_pts, return_core=True)
    got, got_core = oracle.dbscan(p, eps, min_pts, return_core=True)
    np.testing.assert_array_equal(got_core, exp_core)
    np.testing.assert_array_equal(got, exp)


def test_oracle_matches_bruteforce_3000():
    p = datagen.clumps(3000, 77)
    for mp in (2, 4):
        eps = F32(0.03)
        np.testing.assert_array_equal(oracle.dbscan(p, eps, mp),
                                      bruteforce.dbscan(p, eps, mp))


def test_counts_and_pairs_match_bruteforce():
    rng = np.random.Generator(np.random.PCG64(5))
    p = _family("clumpy", 800, rng)
    eps = F32(0.04)
    A = bruteforce.adjacency(p, eps)
    np.testing.assert_array_equal(oracle.neighbour_counts(p, eps), A.sum(1))
    assert oracle.pair_count(p, eps) == (int(A.sum()) - p.shape[0]) // 2


# ---- hand-built cases -------------------------------------------------------

def _pts(*rows):
    return np.array(rows, dtype=F32).reshape(-1, 3)


def test_h1_exact_boundary_is_inclusive():
    # D = 0.25 = fl(0.5*0.5) exactly: "<=" links them
    np.testing.assert_array_equal(
        oracle.dbscan(_pts((0, 0, 0), (0.5, 0, 0)), F32(0.5), 2), [0, 0])


def test_h2_one_ulp_beyond_is_noise():
    x = np.nextafter(F32(0.5), F32(1))
    np.testing.assert_array_equal(
        oracle.dbscan(_pts((0, 0, 0), (x, 0, 0)), F32(0.5), 2), [-1, -1])


def _fp_cases():
    rows = []
    with open(os.path.join(GOLDEN, "fp_boundary_cases.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            v = [F32(float.fromhex(x)) for x in t[1:8]]
            rows.append((t[0], np.array(v[0:3], F32), np.array(v[3:6], F32),
                         v[6], int(t[8]), int(t[9])))
    return rows


@pytest.mark.parametrize("case", range(16))
def test_h3_binary32_predicate_decides(case):
    kind, p, q, eps, plain, other = _fp_cases()[case]
    assert plain != other
    lab = oracle.dbscan(np.stack([p, q]), eps, 2)
    np.testing.assert_array_equal(lab, [0, 0] if plain else [-1, -1])


def test_h4_chain():
    p = np.zeros((1000, 3), F32)
    p[:, 0] = np.arange(1000, dtype=F32) * F32(0.25)
    np.testing.assert_array_equal(oracle.dbscan(p, F32(0.25), 2), np.zeros(1000))
    below = np.nextafter(F32(0.25), F32(0))
    np.testing.assert_array_equal(oracle.dbscan(p, below, 2), -np.ones(1000))


def test_h5_lattice_all_noise():
    g = np.stack(np.meshgrid(*[np.arange(6, dtype=F32)] * 3), -1).reshape(-1, 3)
    np.testing.assert_array_equal(oracle.dbscan(g, F32(0.5), 2), -np.ones(216))


@pytest.mark.parametrize("k", [1, 2, 7])
def test_h6_copies(k):
    p = np.tile(_pts((0.3, -1.25, 7.0)), (k, 1))
    for mp in range(1, k + 3):
        exp = np.zeros(k) if mp <= k else -np.ones(k)
        np.testing.assert_array_equal(oracle.dbscan(p, F32(0.0), mp), exp)


def _two_clusters_and_border(border_first=False, b_cluster_first=True):
    A = [(0.0, 0, 0), (-0.1, 0, 0), (-0.2, 0, 0), (-0.3, 0, 0)]
    B = [(2.0, 0, 0), (2.1, 0, 0), (2.2, 0, 0), (2.3, 0, 0)]
    b = [(1.0, 0, 0)]
    groups = (B + A) if b_cluster_first else (A + B)
    return _pts(*((b + groups) if border_first else (groups + b)))


def test_h7_border_goes_to_smallest_index_core():
    # the border point at x=1 is exactly eps from the cores at x=0 and x=2
    lab = oracle.dbscan(_two_clusters_and_border(), F32(1.0), 4)
    np.testing.assert_array_equal(lab, [0, 0, 0, 0, 4, 4, 4, 4, 0])
    lab = oracle.dbscan(_two_clusters_and_border(b_cluster_first=False), F32(1.0), 4)
    np.testing.assert_array_equal(lab, [0, 0, 0, 0, 4, 4, 4, 4, 0])
    lab, core = oracle.dbscan(_two_clusters_and_border(), F32(1.0), 4, return_core=True)
    assert not core[8] and core[:8].all()


def test_h8_label_is_min_over_borders_too():
    lab = oracle.dbscan(_two_clusters_and_border(border_first=True), F32(1.0), 4)
    np.testing.assert_array_equal(lab, [0, 0, 0, 0, 0, 5, 5, 5, 5])


def test_h9_tiny():
    assert oracle.dbscan(np.zeros((0, 3), F32), F32(1), 2).shape == (0,)
    np.testing.assert_array_equal(oracle.dbscan(_pts((1, 2, 3)), F32(1), 1), [0])
    np.testing.assert_array_equal(oracle.dbscan(_pts((1, 2, 3)), F32(1), 2), [-1])


def test_h10_subnormal_threshold_not_flushed():
    # e2 = fl(1e-20^2) and D = fl((2e-20)^2) are subnormal, D > e2; flushing
    # both to zero would link the points
    p = _pts((0, 0, 0), (F32(2e-20), 0, 0))
    np.testing.assert_array_equal(oracle.dbscan(p, F32(1e-20), 2), [-1, -1])
    p = _pts((0, 0, 0), (F32(1e-20), 0, 0))
    np.testing.assert_array_equal(oracle.dbscan(p, F32(1e-20), 2), [0, 0])


def test_h11_underflow_links_at_eps_zero():
    p = _pts((1e-30, 0, 0), (2e-30, 0, 0), (5e-30, 0, 0))
    np.testing.assert_array_equal(oracle.dbscan(p, F32(0), 2), [0, 0, 0])
    assert oracle.dbscan(_pts((0, 0, 0), (1e-22, 0, 0)), F32(0), 2).tolist() == [-1, -1]


def test_h12_overflow_is_not_a_neighbour():
    p = _pts((-1e30, 0, 0), (1e30, 0, 0), (1e30, 0, 0))
    np.testing.assert_array_equal(oracle.dbscan(p, F32(1e18), 2), [-1, 1, 1])


def test_h13_zero_extent_axis():
    rng = np.random.Generator(np.random.PCG64(13))
    p = _family("flat", 400, rng)
    np.testing.assert_array_equal(oracle.dbscan(p, F32(0.05), 3),
                                  bruteforce.dbscan(p, F32(0.05), 3))


def test_h14_dense_ball_one_cluster():
    rng = np.random.Generator(np.random.PCG64(14))
    d = rng.standard_normal((20000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    p = (d * rng.random((20000, 1)) * 0.1).astype(F32)
    np.testing.assert_array_equal(oracle.dbscan(p, F32(1.0), 10), np.zeros(20000))


def test_h15_invalid_arguments():
    p = _pts((0, 0, 0), (1, 1, 1))
    for eps, mp in [(F32(np.nan), 2), (F32(np.inf), 2), (F32(-1), 2),
                    (F32(1e20), 2), (F32(1), 0), (F32(1), -3)]:
        with pytest.raises(oracle.OracleError) as e:
            oracle.dbscan(p, eps, mp)
        assert e.value.code == -1
    for bad in (np.nan, np.inf, -np.inf):
        q = p.copy()
        q[1, 2] = bad
        with pytest.raises(oracle.OracleError) as e:
            oracle.dbscan(q, F32(1), 2)
        assert e.value.code == -2


# ---- special cases that reduce to library routines --------------------------

def test_minpts2_is_connected_components():
    """minPts = 2 (friends-of-friends, section 4.3.1): clusters are the
    connected components of the eps-graph, singletons are noise.  Candidate
    pairs from scipy's k-d tree, kept if the binary32 predicate holds."""
    p = datagen.config_points("clumps32k")
    eps = F32(0.006)
    pairs = cKDTree(p.astype(np.float64)).query_pairs(float(eps) * (1 + 1e-5) + 1e-20,
                                                      output_type="ndarray")
    d = p[pairs[:, 0]] - p[pairs[:, 1]]          # float32 throughout
    D = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    assert D.dtype == F32
    keep = D <= F32(eps * eps)
    e = pairs[keep]
    n = p.shape[0]
    g = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    deg = np.bincount(e.ravel(), minlength=n)
    comp[deg == 0] = -1
    np.testing.assert_array_equal(oracle.dbscan(p, eps, 2), _canon(comp))


def test_minpts1_has_no_noise_and_eps0_groups_duplicates():
    rng = np.random.Generator(np.random.PCG64(3))
    base = rng.random((50, 3)).astype(F32)
    idx = rng.integers(0, 50, 400)
    p = base[idx]
    lab = oracle.dbscan(p, F32(0), 1)
    assert (lab >= 0).all()
    np.testing.assert_array_equal(lab, _canon(np.unique(idx, return_inverse=True)[1]))
    p2 = oracle.dbscan(p, F32(0.2), 1)
    assert (p2 >= 0).all()


# ---- exact metamorphic relations -------------------------------------------

@pytest.mark.parametrize("min_pts", [2, 5])
def test_metamorphic_exact(min_pts):
    p = datagen.clumps(20000, 21)
    eps = F32(0.008)
    ref = oracle.dbscan(p, eps, min_pts)
    # reflection: fl(-a - -b) = -fl(a - b)
    q = p.copy()
    q[:, 0] = -q[:, 0]
    np.testing.assert_array_equal(oracle.dbscan(q, eps, min_pts), ref)
    # swapping x and y: fl(a + b) = fl(b + a)
    np.testing.assert_array_equal(oracle.dbscan(p[:, [1, 0, 2]], eps, min_pts), ref)
    # scaling by 2^k scales D and e2 by 4^k exactly (no over/underflow here)
    for k in (-3, 5):
        s = F32(2.0 ** k)
        np.testing.assert_array_equal(oracle.dbscan(p * s, eps * s, min_pts), ref)
    # permutation: cluster membership follows the points; with borders the
    # smallest-index rule depends on indices, so compare core/noise there
    pi = np.random.Generator(np.random.PCG64(9)).permutation(p.shape[0])
    got, core = oracle.dbscan(p[pi], eps, min_pts, return_core=True)
    _, core_ref = oracle.dbscan(p, eps, min_pts, return_core=True)
    np.testing.assert_array_equal(core, core_ref[pi])
    if min_pts <= 2:
        np.testing.assert_array_equal(got, _canon(ref[pi]))
    else:
        np.testing.assert_array_equal(got < 0, ref[pi] < 0)
        c = core
        np.testing.assert_array_equal(_canon(np.where(c, got, -1)),
                                      _canon(np.where(c, ref[pi], -1)))


# ---- the pins catch planted mistakes ---------------------------------------

def _pin_failures(lib):
    """A compact run of the pins above against one build of the oracle."""
    fails = []

    def check(name, got, exp):
        if not np.array_equal(np.asarray(got), np.asarray(exp)):
            fails.append(name)

    check("h1", oracle.dbscan(_pts((0, 0, 0), (0.5, 0, 0)), F32(0.5), 2, lib=lib), [0, 0])
    check("h7", oracle.dbscan(_two_clusters_and_border(), F32(1.0), 4, lib=lib),
          [0, 0, 0, 0, 4, 4, 4, 4, 0])
    check("h8", oracle.dbscan(_two_clusters_and_border(border_first=True), F32(1.0), 4,
                              lib=lib), [0, 0, 0, 0, 0, 5, 5, 5, 5])
    for kind, p, q, eps, plain, other in _fp_cases():
        check("h3" + kind, oracle.dbscan(np.stack([p, q]), eps, 2, lib=lib),
              [0, 0] if plain else [-1, -1])
    for kind, seed, mp in CASES[::7]:
        rng = np.random.Generator(np.random.PCG64(1000 + seed))
        p = _family(kind, int(rng.integers(50, 700)), rng)
        eps = _boundary_eps(p, rng) if seed % 2 == 0 else F32(rng.uniform(0.01, 0.3))
        check(f"bf-{kind}-{seed}-{mp}", oracle.dbscan(p, eps, mp, lib=lib),
              bruteforce.dbscan(p, eps, mp))
    return fails


def test_pins_pass_on_the_real_oracle(oracle_lib):
    assert _pin_failures(oracle_lib) == []


@pytest.mark.parametrize("mutant", ["STRICT", "FMA", "NOSELF", "BORDER_MAX",
                                    "LABEL_CORE", "NO_DZ", "INDEX"])
def test_pins_catch_planted_mistake(mutant):
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build(extra_flags=[f"-DORACLE_MUTANT_{mutant}"],
                            out=os.path.join(d, "liboracle_mutant.so"))
        lib = oracle.load(path)
        assert _pin_failures(lib), f"mutant {mutant} passed every pin"


# ---- the local spot-check used at sizes too large for the whole-field oracle

def test_local_check_agrees_with_whole_field_oracle():
    import localcheck
    p = datagen.halo_field(1 << 18, 256.0 * (1 / 64) ** (1 / 3), 5)
    for mp in (2, 3):
        full = oracle.dbscan(p, F32(0.2), mp)
        checked = localcheck.check_cube(p, full, (10, 10, 10), (30, 30, 30), 0.2, mp, 4.0)
        assert checked > 1000
        bad = full.copy()
        inner = np.all((p > 12) & (p < 28), axis=1)
        lab_k = np.flatnonzero(inner & (full >= 0))
        k = lab_k[0] if lab_k.size else np.flatnonzero(inner)[0]
        bad[k] = -1 if full[k] >= 0 else int(k)  # a clustered point as noise, or vice versa
        with pytest.raises(AssertionError):
            localcheck.check_cube(p, bad, (10, 10, 10), (30, 30, 30), 0.2, mp, 4.0)


# ---- threads do not change the result ----------------------------------------

def test_thread_count_does_not_change_labels():
    """The counting and border steps may run on several host threads; the
    labels and core flags are the same as with one."""
    p = datagen.halo_field(1 << 18, 256.0 * (1 / 64) ** (1 / 3), 8)
    try:
        for mp in (2, 3, 5):
            oracle.set_threads(1)
            ref, ref_core = oracle.dbscan(p, F32(0.2), mp, return_core=True)
            oracle.set_threads(4)
            got, got_core = oracle.dbscan(p, F32(0.2), mp, return_core=True)
            np.testing.assert_array_equal(got, ref)
            np.testing.assert_array_equal(got_core, ref_core)
            np.testing.assert_array_equal(oracle.neighbour_counts(p, F32(0.2)) >= mp, ref_core)
    finally:
        oracle.set_threads(1)


def test_dbscan_sets_equals_one_call_per_set():
    pts, off = datagen.subhalo_sets(24, 6, nmax=4096)
    eps = np.full(24, 0.05, F32)
    eps[::3] = F32(0.02)
    mp = np.array([2, 5, 10] * 8)
    one = np.concatenate([oracle.dbscan(pts[off[s]:off[s + 1]], eps[s], mp[s])
                          for s in range(24)])
    for w in (1, 4):
        np.testing.assert_array_equal(oracle.dbscan_sets(pts, off, eps, mp, workers=w), one)
