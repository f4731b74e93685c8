"""The 2^27-point halo field (box [0,512)^3, eps 0.2) at full size on the
GPU: every label satisfies the canonical-form properties, and labels in
sub-cubes are checked exactly against the oracle (tests/localcheck.py)."""
import numpy as np
import pytest

import datagen
import localcheck

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32
CUBES = [((100, 100, 100), (124, 124, 124)), ((300, 40, 460), (324, 64, 484)),
         ((0, 0, 0), (20, 20, 20))]


@pytest.fixture(scope="module")
def field():
    p = datagen.config_points("halo134M")
    return p, torch.from_numpy(p).cuda()


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
    p, d = field
    ctx = dbx.Context(0)
    lab = ctx.cluster(d, 0.2, mp, algorithm=algo, pair_count=pc).cpu().numpy()
    ctx.close()
    canonical_form(lab)
    checked = 0
    for lo, hi in CUBES:
        checked += localcheck.check_cube(p, lab, lo, hi, F32(0.2), mp, margin=1.0)
    assert checked > 20000  # about 35,000 points lie in the trusted inner regions
