"""O(N^2) DBSCAN straight from the definition (paper, section 3.1).

Used only to pin the oracle on small inputs.  It shares nothing with the
oracle's algorithm: a dense N x N adjacency matrix instead of a grid, scipy's
connected components instead of a union-find, and argmin instead of a
running minimum.  numpy float32 arithmetic rounds every operation on its
own and never fuses a multiply with an add, so the distance below is the
binary32 evaluation of ((dx*dx + dy*dy) + dz*dz).
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components


def adjacency(points: np.ndarray, eps) -> np.ndarray:
    p = np.asarray(points, dtype=np.float32)
    e2 = np.float32(np.float32(eps) * np.float32(eps))
    d = [(p[:, None, a] - p[None, :, a]).astype(np.float32) for a in range(3)]
    sq = [(x * x).astype(np.float32) for x in d]
    D = ((sq[0] + sq[1]).astype(np.float32) + sq[2]).astype(np.float32)
    return D <= e2


def canonical(groups: np.ndarray) -> np.ndarray:
    """Relabel group ids (-1 = none) by the smallest member index."""
    out = np.full(groups.shape, -1, dtype=np.int32)
    for g in np.unique(groups[groups >= 0]):
        members = np.flatnonzero(groups == g)
        out[members] = members.min()
    return out


def dbscan(points: np.ndarray, eps, min_pts: int, return_core=False):
    A = adjacency(points, eps)
    n = A.shape[0]
    cnt = A.sum(axis=1)
    core = cnt >= min_pts
    comp = np.full(n, -1, dtype=np.int64)
    ci = np.flatnonzero(core)
    if ci.size:
        _, cc = connected_components(csr_matrix(A[np.ix_(ci, ci)]), directed=False)
        comp[ci] = cc
    for i in np.flatnonzero(~core):
        nb = np.flatnonzero(A[i] & core)
        if nb.size:
            comp[i] = comp[nb.min()]
    lab = canonical(comp)
    return (lab, core) if return_core else lab
