"""Exact spot checks of labels on fields too large for a whole-field oracle
run: the oracle clusters the points inside a cube plus a margin, and a point
is checked only where that sub-run cannot differ from the whole field.

Why 3*eps.  A point at least eps inside the region has its whole
eps-neighbourhood in the sub-run, so its core flag there is exact.  For a
sub-run cluster whose members all lie 3*eps inside: any core point of the
whole field within eps of one of its cores lies 2*eps inside, is core in
the sub-run too and joins the same sub-run cluster; any border point
attached to it lies 2*eps inside, so its neighbours (eps inside) have exact
core flags and it picks the same smallest-index core neighbour.  So the
sub-run cluster is exactly the field's cluster.  A sub-run noise point 3*eps
inside has an exact neighbourhood and exact neighbour core flags, so it is
noise in the field too.
Labels are compared as partitions mapped to global indices: the smallest
global index of a cluster wholly inside the sub-run is the whole field's
label for it.
"""
from __future__ import annotations

import numpy as np

import oracle


def check_cube(points, labels, lo, hi, eps, min_pts, margin):
    """Compare `labels` (whole field, global indices) with the oracle inside
    [lo, hi] (+ margin).  Returns the number of points checked; raises on a
    mismatch."""
    eps = np.float32(eps)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    sel = np.all((points >= lo - margin) & (points <= hi + margin), axis=1)
    idx = np.flatnonzero(sel)
    sub = points[idx]
    lab = oracle.dbscan(sub, eps, min_pts)
    # the float predicate accepts separations a hair above eps: pad 3*eps
    pad = 3.0 * float(eps) * (1 + 1e-5) + 1e-6
    inner_lo, inner_hi = lo - margin + pad, hi + margin - pad
    inside = np.all((sub >= inner_lo) & (sub <= inner_hi), axis=1)
    # clusters with every member inside the trusted region
    ok_cluster = {}
    for c in np.unique(lab[lab >= 0]):
        members = lab == c
        ok_cluster[int(c)] = bool(inside[members].all())
    checked = 0
    for k in range(sub.shape[0]):
        if not inside[k]:
            continue
        c = int(lab[k])
        if c < 0:
            expect = -1
        elif ok_cluster[c]:
            expect = int(idx[lab == c].min())
        else:
            continue
        g = int(labels[idx[k]])
        if g != expect:
            raise AssertionError(f"point {idx[k]}: label {g}, expected {expect}")
        checked += 1
    return checked
