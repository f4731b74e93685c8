"""Pins for the oracle's 63-bit Morton codes (section 4.2.2, 64-bit codes;
section 3.2, the scene bounding volume) against values that do not come
from the oracle itself.

The definition being pinned: per axis a, lo_a and hi_a are the minimum and
maximum coordinate over the points, s_a = 2^21 / (hi_a - lo_a) (0 when the
extent is 0) and q_a = min(floor((p_a - lo_a) * s_a), 2^21 - 1), every
operation in binary32; bit b of q_x, q_y, q_z goes to bit 3b+2, 3b+1, 3b of
the code.

* codes worked out by hand on a grid whose extent is 2^21 (so s_a = 1 and
  q_a = p_a - lo_a exactly): the corners, one step along each axis, the top
  bit of each axis, the clamp at 2^21 - 1, a zero-extent axis;
* grid coordinates decided by exact rational arithmetic with binary32
  rounding (tests/fp32exact.py), on points where the binary32 result
  differs from the real-number one, so a float64 evaluation fails;
* a bit-by-bit de-interleave, written here independently of the oracle's
  interleave, gives back the grid coordinates;
* planted mistakes: each mutant (swapped axes, float64 arithmetic, no
  clamp, rounding instead of floor, 20 bits per axis, the other scale
  convention) is the oracle's own source with one change, and each fails
  at least one of the pins above.
"""
import math
import types
from fractions import Fraction

import numpy as np
import pytest

import fp32exact as fx
import oracle

F32 = np.float32
G = float(1 << 21)           # grid extent for which s_a = 1 exactly
ALL_X = 0x4924924924924924   # every x bit set: bits 2, 5, ..., 62
ALL_XY = 0x6DB6DB6DB6DB6DB6  # every x and y bit set


def _pts(*rows):
    return np.array(rows, dtype=F32).reshape(-1, 3)


# (point, code) on the grid [0, 2^21]^3, worked out by hand from the
# definition: q = p, so the code is the interleave of the point's integer
# coordinates.
HAND_GRID = [
    ((0, 0, 0), 0),                       # the lo corner
    ((G, G, G), (1 << 63) - 1),           # the hi corner: 2^21 clamps to 2^21 - 1
    ((1, 0, 0), 4),                       # x bit 0 -> code bit 2
    ((0, 1, 0), 2),                       # y bit 0 -> code bit 1
    ((0, 0, 1), 1),                       # z bit 0 -> code bit 0
    ((2, 0, 0), 32),                      # x bit 1 -> code bit 5
    ((0, 2, 0), 16),
    ((0, 0, 2), 8),
    ((1 << 20, 0, 0), 1 << 62),           # the top bit of each axis
    ((0, 1 << 20, 0), 1 << 61),
    ((0, 0, 1 << 20), 1 << 60),
    ((G - 1, 0, 0), ALL_X),               # the largest grid coordinate
    ((G, 0, 0), ALL_X),                   # clamped to the same
    ((5, 3, 6), 350),                     # 101, 011, 110 -> 110 011 101 (bits 8..0)
]


def _deinterleave(code: int):
    """Grid coordinates from a code, one bit at a time: code bit k belongs
    to axis x, y, z for k % 3 = 2, 1, 0, at bit k // 3."""
    q = [0, 0, 0]
    for k in range(63):
        if (code >> k) & 1:
            q[2 - k % 3] |= 1 << (k // 3)
    return q


def _q_exact(p, lo, hi):
    """One grid coordinate from the definition with exact rationals rounded
    to binary32 after every operation."""
    ext = fx.sub(hi, lo)
    if ext == 0:
        return 0
    s = fx.round32(Fraction(1 << 21) / fx.exact(ext))
    t = fx.mul(fx.sub(p, lo), s)
    return min(math.floor(fx.exact(t)), (1 << 21) - 1)


def _q_real(p, lo, hi):
    """The same coordinate in real arithmetic on the float32 inputs."""
    ext = fx.exact(hi) - fx.exact(lo)
    if ext == 0:
        return 0
    return min(math.floor((fx.exact(p) - fx.exact(lo)) * (1 << 21) / ext), (1 << 21) - 1)


def _binary32_cases(count=24, seed=42):
    """Point sets (lo corner, hi corner, then points inside) together with
    grid coordinates whose binary32 value differs from the real one on at
    least one axis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sets = []
    while len(sets) < count:
        lo = rng.uniform(-100, 100, 3).astype(F32)
        ext = (10.0 ** rng.uniform(-3, 3, 3)).astype(F32)
        hi = (lo + ext).astype(F32)
        inner = (lo + rng.random((64, 3)) * (hi - lo)).astype(F32)
        inner = np.minimum(np.maximum(inner, lo), hi)
        keep = []
        for p in inner:
            qe = [_q_exact(p[a], lo[a], hi[a]) for a in range(3)]
            qr = [_q_real(p[a], lo[a], hi[a]) for a in range(3)]
            if qe != qr:
                keep.append((p, qe))
        if keep:
            pts = np.stack([lo, hi] + [p for p, _ in keep]).astype(F32)
            q = np.array([[0, 0, 0], [(1 << 21) - 1] * 3] + [qe for _, qe in keep],
                         dtype=np.uint64)
            sets.append((pts, q))
    return sets


BINARY32 = _binary32_cases()


def _morton_pin_failures(mod):
    """The pins above, run against one version of the oracle module; returns
    the names of the pins it fails."""
    fails = []

    def check(name, got, exp):
        if not np.array_equal(np.asarray(got, dtype=np.uint64), np.asarray(exp, dtype=np.uint64)):
            fails.append(name)

    p = _pts(*[r for r, _ in HAND_GRID])
    check("hand-grid", mod.morton63(p), [c for _, c in HAND_GRID])
    # a zero-extent z axis: s_z = 0, every z bit clear
    flat = _pts((0, 0, 7), (G, G, 7), (1, 1, 7), (0, 0, 7))
    check("zero-extent", mod.morton63(flat), [0, ALL_XY, 6, 0])
    for k, (pts, q) in enumerate(BINARY32):
        check(f"binary32-{k}", mod.morton_quantise(pts), q)
    rng = np.random.Generator(np.random.PCG64(7))
    r = (rng.standard_normal((500, 3)) * [1.0, 30.0, 0.01]).astype(F32)
    codes = mod.morton63(r)
    check("round-trip", [_deinterleave(int(c)) for c in codes], mod.morton_quantise(r))
    if int(np.max(codes)) >= 1 << 63:
        fails.append("63-bit")
    return fails


def test_morton_codes_by_hand():
    p = _pts(*[r for r, _ in HAND_GRID])
    got = oracle.morton63(p)
    for (row, exp), g in zip(HAND_GRID, got):
        assert int(g) == exp, f"{row}: {int(g):#x} != {exp:#x}"


def test_morton_zero_extent_axis():
    flat = _pts((0, 0, 7), (G, G, 7), (1, 1, 7), (0, 0, 7))
    np.testing.assert_array_equal(oracle.morton_quantise(flat)[:, 2], 0)
    assert [int(c) for c in oracle.morton63(flat)] == [0, ALL_XY, 6, 0]


def test_binary32_cases_differ_from_real_arithmetic():
    # the cases are only a pin if a real-number (or float64) evaluation
    # would get them wrong
    assert sum(q.shape[0] - 2 for _, q in BINARY32) >= 24


@pytest.mark.parametrize("k", range(len(BINARY32)))
def test_morton_quantise_binary32_exact(k):
    pts, q = BINARY32[k]
    np.testing.assert_array_equal(oracle.morton_quantise(pts), q)


def test_morton_deinterleave_round_trip():
    rng = np.random.Generator(np.random.PCG64(8))
    p = datagen_like_points(rng)
    codes = oracle.morton63(p)
    q = oracle.morton_quantise(p)
    assert int(codes.max()) < 1 << 63
    for c, qq in zip(codes[:2000], q[:2000]):
        assert _deinterleave(int(c)) == [int(x) for x in qq]


def datagen_like_points(rng):
    """Clustered points with very different extents per axis."""
    c = rng.random((8, 3)) * [1.0, 1e3, 1e-3]
    return (c[rng.integers(0, 8, 3000)] + rng.standard_normal((3000, 3)) *
            [0.01, 5.0, 1e-5]).astype(F32)


def test_morton_pins_pass_on_the_real_oracle():
    assert _morton_pin_failures(oracle) == []


# (name, [(text in oracle/__init__.py, replacement), ...])
MUTANTS = [
    ("swap_xz", [("3 * b + 2 - a", "3 * b + a")]),
    ("swap_xy", [("bit = (q[:, a] >>", "bit = (q[:, (1, 0, 2)[a]] >>")]),
    ("float64_multiply", [("s = np.zeros(3, dtype=np.float32)",
                           "s = np.zeros(3, dtype=np.float64)")]),
    ("float64_everything", [("s = np.zeros(3, dtype=np.float32)",
                             "s = np.zeros(3, dtype=np.float64)"),
                            ("s[nz] = np.float32(1 << MORTON_BITS) / ext[nz]",
                             "s[nz] = float(1 << MORTON_BITS) / ext[nz].astype(np.float64)"),
                            ("t = (p - lo).astype(np.float32) * s",
                             "t = (p.astype(np.float64) - lo) * s")]),
    ("no_clamp", [("np.minimum(q, (1 << MORTON_BITS) - 1)", "q")]),
    ("round_not_floor", [("np.floor(t)", "np.round(t)")]),
    ("bits_20", [("MORTON_BITS = 21", "MORTON_BITS = 20")]),
    ("scale_2pow21_minus_1", [("np.float32(1 << MORTON_BITS) / ext",
                               "np.float32((1 << MORTON_BITS) - 1) / ext")]),
]


def _mutant_module(changes):
    src = open(oracle.__file__).read()
    for old, new in changes:
        assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
        src = src.replace(old, new)
    mod = types.ModuleType("oracle_morton_mutant")
    mod.__file__ = oracle.__file__
    exec(compile(src, "oracle_morton_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,changes", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_morton_pins_catch_planted_mistake(name, changes):
    assert _morton_pin_failures(_mutant_module(changes)), f"mutant {name} passed every pin"
