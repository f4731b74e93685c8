"""Synthetic workload generators: determinism, sizes, ranges, structure."""
import hashlib

import numpy as np
import pytest

import datagen


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_clumps_deterministic_and_in_unit_cube():
    a = datagen.clumps(32768, 1)
    b = datagen.clumps(32768, 1)
    assert a.dtype == np.float32 and a.shape == (32768, 3)
    assert _sha(a) == _sha(b)
    assert (a >= 0).all() and (a < 1).all()
    assert _sha(a) != _sha(datagen.clumps(32768, 2))


def test_halo_field_structure():
    n = 1 << 18
    box = 256.0 * (n / (1 << 24)) ** (1 / 3)
    p = datagen.halo_field(n, box, 2)
    assert p.shape == (n, 3) and p.dtype == np.float32
    assert (p >= 0).all() and (p < box).all()
    # half the points sit in halos: the share of points in unit cells holding
    # >= 6 points is far above a uniform field's (P(Poisson(1) >= 5) ~ 0.4%)
    c = np.floor(p).astype(np.int64)
    key = (c[:, 0] * 4096 + c[:, 1]) * 4096 + c[:, 2]
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    assert (cnt[inv] >= 6).mean() > 0.05


def test_halo_masses_power_law():
    rng = np.random.Generator(np.random.PCG64(0))
    m = datagen._halo_masses(rng, 5_000_000)
    assert m.sum() == 5_000_000
    assert m.min() >= 1 and m.max() <= 200000
    # mean of dN/dM ~ M^-1.9 on [20, 2e5] is about 272
    assert 200 < m.mean() < 350


def test_plummer_radius_inverts_enclosed_mass():
    a = 0.7
    r = np.array([0.1, 1.0, 3.0, 7.0])
    m = r ** 3 / (r ** 2 + a ** 2) ** 1.5
    np.testing.assert_allclose(datagen.plummer_radius(m, a), r, rtol=1e-12)


def test_subhalo_sets_sizes():
    _, off = datagen.subhalo_sets(4096, 4, sizes_only=True)
    sizes = np.diff(off)
    assert sizes.min() >= 64 and sizes.max() <= 262144
    assert 110e6 < off[-1] < 150e6
    pts, off2 = datagen.subhalo_sets(8, 4, nmax=4096)
    assert pts.shape[0] == off2[-1] and np.isfinite(pts).all()


def test_serving_trace_rate():
    jobs = datagen.serving_trace()
    assert 11000 < len(jobs) < 13000
    assert all(1000 <= j.n <= (1 << 24) for j in jobs)
    assert {j.min_pts for j in jobs} == {2, 5, 10}
    t = np.array([j.t_arrival for j in jobs])
    assert (np.diff(t) > 0).all() and t[-1] < 60.0


def test_eps_linking_length_closed_form():
    # the paper's benchmark: eps = 0.168 * (256^3 / 1024^3)^(1/3) = 0.042
    assert abs(float(datagen.mean_spacing_eps(1024 ** 3, 0.168, 256.0 ** 3)) - 0.042) < 1e-7


@pytest.mark.parametrize("name", ["clumps32k", "halo16M", "serving_trace"])
def test_inputs_match_the_manifest(name):
    """The generators give the bytes datagen/manifest.json records (the
    same bytes on every machine that reproduces them)."""
    import json
    want = json.load(open(datagen.MANIFEST))["sha256"][name]
    assert datagen.input_digests([name])[name] == want
