"""Writes fp_boundary_cases.txt: point pairs on which the binary32 predicate
dist^2 <= eps^2 (paper, section 3.1, with the squared distance evaluated as
((dx*dx + dy*dy) + dz*dz) in binary32 without fused multiply-add) gives a
different answer than

  kind "real"  : the exact real-number comparison of the same float inputs;
  kind "fused" : the same sum contracted into fused multiply-adds,
                 fma(dz, dz, fma(dy, dy, dx*dx)).

Expected answers come from exact rational arithmetic with correct rounding
(tests/fp32exact.py), never from any implementation under test.  Seeded, so
re-running reproduces the file.  Run from the repository root:

    python tests/golden/make_fp_cases.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import fp32exact as fx  # noqa: E402


def hexf(x) -> str:
    return float(np.float32(x)).hex()


def search(kind: str, want: int, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    found = []
    while len(found) < want:
        p = rng.uniform(-2, 2, 3).astype(np.float32)
        q = (p + rng.uniform(-0.7, 0.7, 3)).astype(np.float32)
        dp = fx.sqdist_plain(p, q)
        if not np.isfinite(dp) or dp == 0:
            continue
        e0 = np.float32(np.sqrt(np.float64(dp)))
        for k in range(-3, 4):
            eps = np.float32(e0)
            for _ in range(abs(k)):
                eps = np.nextafter(eps, np.float32(np.inf if k > 0 else 0))
            e2 = fx.mul(eps, eps)
            plain = bool(dp <= e2)
            if kind == "fused":
                other = bool(fx.sqdist_fused(p, q) <= e2)
            else:
                other = bool(fx.sqdist_real(p, q) <= fx.exact(eps) ** 2)
            if plain != other:
                found.append((p, q, eps, int(plain), int(other)))
                break
    return found


def main():
    out = os.path.join(HERE, "fp_boundary_cases.txt")
    rows = [("real", c) for c in search("real", 8, 11)] + \
           [("fused", c) for c in search("fused", 8, 12)]
    with open(out, "w") as f:
        f.write("# kind px py pz qx qy qz eps plain_neighbour other_neighbour\n")
        f.write("# written by tests/golden/make_fp_cases.py (exact arithmetic)\n")
        for kind, (p, q, eps, plain, other) in rows:
            f.write(" ".join([kind, *map(hexf, p), *map(hexf, q), hexf(eps),
                              str(plain), str(other)]) + "\n")
    print("wrote", out, len(rows), "cases")


if __name__ == "__main__":
    main()
