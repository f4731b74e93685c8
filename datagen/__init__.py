"""Seeded synthetic point fields for the DBSCAN workloads.

This module only draws coordinates.  It holds none of the clustering
arithmetic, so both the CPU oracle (under ``oracle/``) and the GPU library
can be fed from it without sharing any code of the method itself.

The HACC snapshot the paper benchmarks on (section 4, the ~37M dark-matter
particle rank of a 2x1024^3 run, eps = 0.042, minPts = 2) is not available;
the halo-like fields below stand in for it:

* ``clumps``      -- Gaussian clumps plus a uniform background in the unit
                     cube (the small 32,768-point case and the serving pools).
* ``halo_field``  -- Plummer-profile halos with a power-law mass function
                     plus a uniform background in a periodic box (the 2^24
                     and 2^27 point fields, mean inter-particle spacing 1).
* ``subhalo_sets``-- many independent single-halo sets with Gaussian
                     sub-clumps (the batched workload).
* ``serving_trace``-- Poisson arrivals with log-uniform job sizes.

All draws use numpy's PCG64 ``Generator`` in float64 and cast to float32
last; every field is shuffled by a seeded permutation so that input order
carries no spatial information.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "clumps", "halo_field", "plummer_radius", "subhalo_sets",
    "serving_trace", "CONFIGS", "config_points", "mean_spacing_eps",
]

# Plummer profile truncated at 10 scale radii: enclosed-mass fraction
# m(r) = r^3 / (r^2 + a^2)^{3/2}, so m(10a) = 1000 / 101^{3/2}.
_PLUMMER_MMAX = 1000.0 / 101.0 ** 1.5


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _iso_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    nrm = np.sqrt((v * v).sum(axis=1, keepdims=True))
    nrm[nrm == 0.0] = 1.0
    return v / nrm


def plummer_radius(u: np.ndarray, a) -> np.ndarray:
    """Radius of a Plummer sphere of scale radius ``a`` at enclosed-mass
    fraction ``u`` (inverse of m(r) = r^3/(r^2+a^2)^{3/2})."""
    u = np.clip(u, 1e-300, None)
    return a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)


def _to_f32_box(x: np.ndarray, box: float) -> np.ndarray:
    """Wrap into [0, box) and cast to float32, clamping values that round up
    to ``box`` onto the largest float32 below it."""
    x = np.mod(x, box)
    out = x.astype(np.float32)
    top = np.nextafter(np.float32(box), np.float32(0.0))
    out[out >= np.float32(box)] = top
    return out


def clumps(n: int, seed: int, n_clumps: int = 64, clump_frac: float = 0.75,
           sigma=(0.01, 0.03)) -> np.ndarray:
    """``n`` points in [0,1)^3: ``clump_frac`` of them in isotropic Gaussian
    clumps (centres uniform, sigma uniform in ``sigma``, clump weights
    Dirichlet(1)), the rest uniform.  Periodic wrap, float32, shuffled."""
    rng = _rng(seed)
    n_cl = int(round(n * clump_frac))
    n_bg = n - n_cl
    centres = rng.random((n_clumps, 3))
    sig = rng.uniform(sigma[0], sigma[1], n_clumps)
    w = rng.dirichlet(np.ones(n_clumps))
    counts = rng.multinomial(n_cl, w)
    cid = np.repeat(np.arange(n_clumps), counts)
    pts_cl = centres[cid] + rng.standard_normal((n_cl, 3)) * sig[cid, None]
    pts_bg = rng.random((n_bg, 3))
    pts = np.concatenate([pts_cl, pts_bg], axis=0)
    pts = pts[rng.permutation(n)]
    return _to_f32_box(pts, 1.0)


def _halo_masses(rng: np.random.Generator, budget: int, mmin=20.0,
                 mmax=200000.0, slope=1.9) -> np.ndarray:
    """Integer halo sizes from dN/dM ~ M^-slope on [mmin, mmax] (inverse
    CDF), drawn until they hold ``budget`` particles; the last is trimmed."""
    k = slope - 1.0
    lo, hi = mmin ** (-k), mmax ** (-k)
    out = []
    total = 0
    while total < budget:
        u = rng.random(65536)
        m = np.rint((lo - u * (lo - hi)) ** (-1.0 / k)).astype(np.int64)
        m = np.maximum(m, 1)
        c = np.cumsum(m)
        need = budget - total
        if c[-1] >= need:
            cut = int(np.searchsorted(c, need))
            m = m[: cut + 1].copy()
            m[-1] -= int(c[cut] - need)
            out.append(m)
            total = budget
        else:
            out.append(m)
            total += int(c[-1])
    m = np.concatenate(out)
    return m[m > 0]


def halo_field(n: int, box: float, seed: int, halo_frac: float = 0.5,
               chunk: int = 1 << 22) -> np.ndarray:
    """``n`` points in [0, box)^3: ``halo_frac`` of them in Plummer halos
    (sizes from a M^-1.9 power law on [20, 200000], scale radius
    0.3*M^(1/3), truncated at 10 scale radii, centres uniform), the rest
    uniform.  Periodic wrap, float32, shuffled."""
    rng = _rng(seed)
    n_h = int(round(n * halo_frac))
    masses = _halo_masses(rng, n_h)
    centres = rng.random((masses.size, 3)) * box
    scale = 0.3 * np.cbrt(masses.astype(np.float64))
    out = np.empty((n, 3), dtype=np.float32)
    # halo particles, generated in chunks of whole halos to bound memory
    hid_all = np.repeat(np.arange(masses.size, dtype=np.int64), masses)
    pos = 0
    while pos < n_h:
        end = min(n_h, pos + chunk)
        hid = hid_all[pos:end]
        m = end - pos
        u = rng.random(m) * _PLUMMER_MMAX
        r = plummer_radius(u, scale[hid])
        x = centres[hid] + _iso_dirs(rng, m) * r[:, None]
        out[pos:end] = _to_f32_box(x, box)
        pos = end
    del hid_all
    pos = n_h
    while pos < n:
        end = min(n, pos + chunk)
        out[pos:end] = _to_f32_box(rng.random((end - pos, 3)) * box, box)
        pos = end
    perm = rng.permutation(n)
    return out[perm]


def subhalo_sets(num_sets: int, seed: int, nmin: int = 64,
                 nmax: int = 262144, a: float = 1.0, sub_frac: float = 0.1,
                 sizes_only: bool = False):
    """Independent point sets, sizes log-uniform in [nmin, nmax].  Each set
    is one Plummer halo of scale radius ``a`` centred at the origin
    (truncated at 10a, no wrap) with ``sub_frac`` of its particles in 3..20
    Gaussian sub-clumps (sigma uniform in [0.02, 0.08], centres drawn from
    the same Plummer profile, weights Dirichlet(1)).  Returns
    ``(points float32[total,3], offsets int64[num_sets+1])``; each set is
    shuffled on its own."""
    rng = _rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax),
                                       num_sets))).astype(np.int64)
    offsets = np.zeros(num_sets + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    if sizes_only:
        return None, offsets
    pts = np.empty((int(offsets[-1]), 3), dtype=np.float32)
    for s in range(num_sets):
        n = int(sizes[s])
        n_sub = n // 10 if sub_frac == 0.1 else int(n * sub_frac)
        n_pl = n - n_sub
        u = rng.random(n_pl) * _PLUMMER_MMAX
        x_pl = _iso_dirs(rng, n_pl) * plummer_radius(u, a)[:, None]
        k = int(rng.integers(3, 21))
        uc = rng.random(k) * _PLUMMER_MMAX
        cen = _iso_dirs(rng, k) * plummer_radius(uc, a)[:, None]
        sig = rng.uniform(0.02, 0.08, k)
        cnt = rng.multinomial(n_sub, rng.dirichlet(np.ones(k)))
        cid = np.repeat(np.arange(k), cnt)
        x_sub = cen[cid] + rng.standard_normal((n_sub, 3)) * sig[cid, None]
        x = np.concatenate([x_pl, x_sub], axis=0)[rng.permutation(n)]
        pts[offsets[s]:offsets[s + 1]] = x.astype(np.float32)
    return pts, offsets


def mean_spacing_eps(n: int, b: float = 0.2, volume: float = 1.0) -> np.float32:
    """eps = b * (V / n)^(1/3): the linking-length convention of the paper's
    benchmark (b = 0.168 there), rounded to float32."""
    return np.float32(b * (volume / n) ** (1.0 / 3.0))


@dataclass
class Job:
    t_arrival: float
    n: int
    min_pts: int
    eps: np.float32
    pool: int
    start: int


def serving_trace(seed: int = 59, rate: float = 200.0, duration: float = 60.0,
                  nmin: int = 1000, nmax: int = 1 << 24, pools: int = 8,
                  pool_size: int = 1 << 24):
    """Open-loop Poisson arrivals: exponential gaps at ``rate`` jobs/s over
    ``duration`` seconds, sizes log-uniform in [nmin, nmax], minPts uniform
    over {2, 5, 10}, eps = 0.2 * n^(-1/3) (0.2 of the mean spacing in the
    unit cube), points a window of one of ``pools`` clump pools."""
    rng = _rng(seed)
    jobs = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        n = min(n, pool_size)
        mp = int(rng.choice([2, 5, 10]))
        pool = int(rng.integers(0, pools))
        start = int(rng.integers(0, pool_size - n + 1))
        jobs.append(Job(t, n, mp, mean_spacing_eps(n), pool, start))
    return jobs


def serving_pool(k: int, pool_size: int = 1 << 24) -> np.ndarray:
    """The ``k``-th clump pool of the serving workload (seed 50 + k)."""
    return clumps(pool_size, 50 + k)


# The five workloads: name -> (description, eps, min_pts)
CONFIGS = {
    "clumps32k": dict(n=32768, eps=np.float32(0.006), min_pts=2, seed=1),
    "halo16M": dict(n=1 << 24, box=256.0, eps=np.float32(0.2), min_pts=2, seed=2),
    "halo134M": dict(n=1 << 27, box=512.0, eps=np.float32(0.2), min_pts=2, seed=3),
    "subhalo4096": dict(num_sets=4096, eps=np.float32(0.05), min_pts=5, seed=4),
}


def config_points(name: str, n: int | None = None) -> np.ndarray:
    """Points of a single-field workload; ``n`` overrides the size (the
    generator is the same, so density changes with it for the clump case
    and stays fixed for the halo case only if the box is rescaled)."""
    c = CONFIGS[name]
    if name == "clumps32k":
        return clumps(n or c["n"], c["seed"])
    if name in ("halo16M", "halo134M"):
        nn = n or c["n"]
        box = c["box"] * (nn / c["n"]) ** (1.0 / 3.0)
        return halo_field(nn, box, c["seed"])
    raise KeyError(name)


# ---- input manifest -----------------------------------------------------------
MANIFEST = __import__("os").path.join(__import__("os").path.dirname(__file__), "manifest.json")


def digest(*arrays) -> str:
    """sha256 of the arrays' bytes, in order (C order, native little-endian)."""
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def input_digests(names=None) -> dict:
    """sha256 of each workload's generated input: the three fields, the
    4,096 sub-halo sets (points, offsets), the serving trace's job table
    and its eight point pools."""
    out = {}
    names = names or ["clumps32k", "halo16M", "halo134M", "subhalo4096", "serving_trace",
                      "serving_pools"]
    for nm in names:
        if nm in ("clumps32k", "halo16M", "halo134M"):
            out[nm] = digest(config_points(nm))
        elif nm == "subhalo4096":
            c = CONFIGS[nm]
            out[nm] = digest(*subhalo_sets(c["num_sets"], c["seed"]))
        elif nm == "serving_trace":
            jobs = serving_trace()
            tab = np.array([(j.t_arrival, j.n, j.min_pts, float(j.eps), j.pool, j.start)
                            for j in jobs], dtype=np.float64)
            out[nm] = digest(tab)
        elif nm == "serving_pools":
            out[nm] = digest(*[serving_pool(k) for k in range(8)])
    return out


def check_manifest(name: str, *arrays) -> bool | None:
    """True if the arrays hash to the manifest's digest for `name`, False if
    they differ, None if the manifest has no entry."""
    import json
    import os
    if not os.path.exists(MANIFEST):
        return None
    want = json.load(open(MANIFEST))["sha256"].get(name)
    return None if want is None else digest(*arrays) == want
