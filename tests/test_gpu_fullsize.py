"""The 2^27-point halo field (box [0,512)^3, eps 0.2) at full size on the
GPU, at minPts 2 and 10: every label against the oracle's whole-field run,
bit for bit.  Before that, as a fast first check that names a region, the
canonical form of the labels and exact sub-cube checks (tests/localcheck.py).
"""
import os

import numpy as np
import pytest

import datagen
import localcheck
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32
CUBES = [((100, 100, 100), (124, 124, 124)), ((300, 40, 460), (324, 64, 484)),
         ((0, 0, 0), (20, 20, 20))]


@pytest.fixture(scope="module")
def field():
    print("[fullsize] generating the 2^27-point field", flush=True)
    p = datagen.config_points("halo134M")
    return p, torch.from_numpy(p).cuda(), {}


def oracle_labels(field, mp):
    """The oracle's whole-field labels at this minPts (once per module), its
    counting and border steps on the host's cores (at most 16)."""
    p, _, cache = field
    if mp not in cache:
        print(f"[fullsize] oracle, minPts {mp}", flush=True)
        oracle.set_threads(min(16, os.cpu_count() or 1))
        try:
            cache[mp] = oracle.dbscan(p, F32(0.2), mp)
        finally:
            oracle.set_threads(1)
    return cache[mp]


def canonical_form(lab):
    """-1 or a label c with lab[c] == c and every member index >= c."""
    n = lab.shape[0]
    v = np.flatnonzero(lab >= 0)
    assert lab.min() >= -1 and lab.max() < n
    assert (lab[lab[v]] == lab[v]).all()
    assert (v >= lab[v]).all()


@pytest.mark.parametrize("algo,mp,pc", [("fdbscan", 2, False), ("fdbscan", 10, False),
                                        ("fdbscan", 10, True), ("densebox", 2, False)])
def test_halo134m(field, algo, mp, pc):
    p, d, _ = field
    ctx = dbx.Context(0)
    lab = ctx.cluster(d, 0.2, mp, algorithm=algo, pair_count=pc).cpu().numpy()
    ctx.close()
    canonical_form(lab)
    checked = 0
    for lo, hi in CUBES:
        checked += localcheck.check_cube(p, lab, lo, hi, F32(0.2), mp, margin=1.0)
    assert checked > 20000  # about 35,000 points lie in the trusted inner regions
    ref = oracle_labels(field, mp)
    bad = np.flatnonzero(lab != ref)
    assert bad.size == 0, f"{bad.size} labels differ, first at {bad[:5].tolist()}"
