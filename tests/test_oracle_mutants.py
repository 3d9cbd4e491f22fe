"""Planted mistakes in (a copy of) the oracle must fail at least one pin.

Each mutant is a plausible slip -- a dropped term, a wrong sign, a wrong index,
a non-strict comparison, another evaluation order, a missing relabel, the
printed "skip labelled points" test, the wrong canonical member, an
off-by-one size bound, an over-eager kd-tree prune.  The copy is compiled on
the CPU and run through the fixtures and a brute-force sample; the real
oracle is never modified.
"""

import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import goldens
import synth
from oracle import bruteforce

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "fec_oracle.cpp")

MUTANTS = [
    ("dropped dz term", "    s = s + sz;\n", "    s = s;\n"),
    ("wrong sign in dy", "float dy = a[1] - b[1];", "float dy = a[1] + b[1];"),
    ("wrong index in dz", "float dz = a[2] - b[2];", "float dz = a[2] - b[1];"),
    ("non-strict test", "return s < d2;", "return s <= d2;"),
    ("other sum order", "    float s = sx + sy;\n    s = s + sz;\n",
     "    float s = sy + sz;\n    s = s + sx;\n"),
    ("fused multiply-add", "    float s = sx + sy;\n", "    float s = std::fma(dx, dx, sy);\n"),
    ("max instead of min label", "if (l != 0 && l < m) m = l;", "if (l != 0 && l > m) m = l;"),
    ("no relabel", "else if (l > m) relabel(l, m);", "else if (l > m) {}"),
    ("skip labelled points", "if (skip && label(i) != 0) continue;",
     "if (label(i) != 0) continue;"),
    ("largest member as id", "if (first[l] < 0) first[l] = i;", "first[l] = i;"),
    ("exclusive max bound",
     "labels_out[i] = (size[l] >= lo && size[l] <= max_size)",
     "labels_out[i] = (size[l] >= lo && size[l] < max_size)"),
    ("tight kd prune", "double rc = (double)d * (1.0 + std::ldexp(1.0, -10));",
     "double rc = (double)d * 0.75;"),
]


def _build(src_text, tmp):
    cpp = os.path.join(tmp, "m.cpp")
    so = os.path.join(tmp, "m.so")
    with open(cpp, "w") as f:
        f.write(src_text)
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", so, cpp], check=True, capture_output=True)
    lib = ctypes.CDLL(so)
    lib.oracle_fec.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    lib.oracle_fec.restype = ctypes.c_int64
    return lib


def _run(lib, xyz, d, mn, mx):
    a = np.ascontiguousarray(xyz, dtype=np.float32)
    out = np.empty(a.shape[0], dtype=np.int32)
    k = lib.oracle_fec(a.ctypes.data, a.shape[0], ctypes.c_float(d), mn, mx, 0, out.ctypes.data)
    return out, int(k)


def _pins_fail(lib):
    for name, xyz, d, mn, mx, k, labels in goldens.all_cases():
        got, gk = _run(lib, xyz, d, mn, mx)
        if gk != k or not np.array_equal(got, labels):
            return "fixture " + name
    for seed in range(300):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(2, 120))
        x = synth.random_cloud(n, extent=(3, 3, 1.5), seed=seed)
        d = float(rng.uniform(0.3, 1.0))
        got, gk = _run(lib, x, d, 1, n)
        want, wk = bruteforce.cluster(x, d, 1, n)
        if gk != wk or not np.array_equal(got, want):
            return "brute force seed %d" % seed
    return None


def test_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build(open(SRC).read(), tmp)
        assert _pins_fail(lib) is None


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(mutant):
    name, old, new = mutant
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site for %r not found exactly once" % name
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build(src.replace(old, new), tmp)
        assert _pins_fail(lib) is not None, "mutant %r passed every pin" % name
