"""Writes predicate_order.txt: point pairs where the evaluation order matters.

The clustering's edge test (Eq. (1), strict) is evaluated in binary32 as
s = (dx*dx + dy*dy) + dz*dz and compared with fl(d*d).  This script searches
seeded random pairs very close to the threshold for ones where another
evaluation order -- dx*dx + (dy*dy + dz*dz), (dx*dx + dz*dz) + dy*dy, or a
fused multiply-add of the first product into the sum -- reaches the opposite
verdict, and stores each pair with the verdict of the fixed order.  The
verdict comes from oracle.bruteforce.adjacency (the brute-force definition);
the alternative orders are only used to select interesting pairs.

Run from the repository root:  python tests/golden/make_predicate_order.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.bruteforce import adjacency  # noqa: E402


def _alt_verdicts(a, b, d):
    f = np.float32
    dx, dy, dz = f(a[0] - b[0]), f(a[1] - b[1]), f(a[2] - b[2])
    sx, sy, sz = f(dx * dx), f(dy * dy), f(dz * dz)
    d2 = f(f(d) * f(d))
    right = f(sx + f(sy + sz))
    xz = f(f(sx + sz) + sy)
    # fused: dx*dx + sy rounded once (exact product in float64 then one rounding)
    fused = f(f(np.float64(dx) * np.float64(dx) + np.float64(sy)) + sz)
    return [right < d2, xz < d2, fused < d2]


def main():
    rng = np.random.default_rng(20220816)
    out = []
    kinds = {0: 0, 1: 0, 2: 0}
    tries = 0
    while min(kinds.values()) < 3 and tries < 2_000_000:
        tries += 1
        d = float(np.float32(rng.choice([0.2, 0.35, 0.5, 1.0])))
        a = (rng.uniform(-50, 50, 3)).astype(np.float32)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        b = (a.astype(np.float64) + d * (1 + rng.uniform(-3e-7, 3e-7)) * u).astype(np.float32)
        joined = bool(adjacency(np.stack([a, b]), d)[0, 1])
        alts = _alt_verdicts(a, b, d)
        for k, v in enumerate(alts):
            if v != joined and kinds[k] < 3:
                kinds[k] += 1
                out.append((a, b, d, joined, k))
    names = ["dx2+(dy2+dz2)", "(dx2+dz2)+dy2", "fma(dx,dx,dy2)+dz2"]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predicate_order.txt")
    with open(path, "w") as f:
        f.write("# Pairs near the threshold where the order of the binary32 evaluation\n")
        f.write("# decides Eq. (1)'s strict test.  Verdict (joined) of the fixed order\n")
        f.write("# s = (dx*dx + dy*dy) + dz*dz < fl(d*d), from oracle.bruteforce;\n")
        f.write("# the comment names the other order that disagrees.\n")
        f.write("# Written by tests/golden/make_predicate_order.py (seed 20220816).\n")
        for a, b, d, joined, k in out:
            f.write("# %s gives %d\n" % (names[k], 0 if joined else 1))
            f.write("pair %s %s %s  %s %s %s  d=%s joined=%d\n" % (
                *[repr(float(v)) for v in a], *[repr(float(v)) for v in b],
                repr(float(np.float32(d))), int(joined)))
    print("wrote %d pairs after %d tries" % (len(out), tries))


if __name__ == "__main__":
    main()
