"""Correctly rounded IEEE binary32 arithmetic on exact rationals.

An implementation of round-to-nearest-even written from the IEEE 754
definition, independent of numpy and of any C compiler, used to decide
boundary cases of the distance predicate exactly (with and without a fused
multiply-add) when building and checking test fixtures.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

_EMIN = -126       # smallest normal exponent
_MANT = 23         # fraction bits
_MAXF = Fraction((2 ** 24 - 1) * 2 ** (127 - 23))


def exact(x) -> Fraction:
    """The exact rational value of a float32."""
    return Fraction(float(np.float32(x)))


def round32(x: Fraction) -> np.float32:
    """Round an exact rational to the nearest binary32, ties to even."""
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, _EMIN)                      # subnormals share the min exponent
    ulp = Fraction(2) ** (e - _MANT)
    q, r = divmod(a, ulp)                  # a = q*ulp + r, 0 <= r < ulp
    q = int(q)
    if r * 2 > ulp or (r * 2 == ulp and q % 2 == 1):
        q += 1
    v = q * ulp
    if v > _MAXF:
        return np.float32(sign * np.inf)
    return np.float32(sign * float(v))     # v is exactly representable


def add(a, b):
    return round32(exact(a) + exact(b))


def sub(a, b):
    return round32(exact(a) - exact(b))


def mul(a, b):
    return round32(exact(a) * exact(b))


def fma(a, b, c):
    return round32(exact(a) * exact(b) + exact(c))


def sqdist_plain(p, q):
    """((dx*dx + dy*dy) + dz*dz), every operation rounded."""
    dx, dy, dz = (sub(p[i], q[i]) for i in range(3))
    return add(add(mul(dx, dx), mul(dy, dy)), mul(dz, dz))


def sqdist_fused(p, q):
    """The same sum as a compiler contracting into fused multiply-adds would
    evaluate it: fma(dz, dz, fma(dy, dy, dx*dx))."""
    dx, dy, dz = (sub(p[i], q[i]) for i in range(3))
    return fma(dz, dz, fma(dy, dy, mul(dx, dx)))


def sqdist_real(p, q) -> Fraction:
    """The exact squared distance of the two float32 points."""
    return sum((exact(p[i]) - exact(q[i])) ** 2 for i in range(3))
