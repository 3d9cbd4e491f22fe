"""Pins of the oracle's property checkers (oracle/invariants.py and the
closure / component queries of oracle/fec_oracle.cpp).

The checkers carry the parity claims on clouds too large for a full oracle
run in a test, so each is shown to REPORT a planted violation, not only to
stay silent on correct labellings:

* a known-good labelling (the hand-worked 9-point fixture of
  tests/golden/filter9.txt, d = 1.5, clusters A = {0, 3, 5},
  B = {1, 2, 6, 8}, C = {4}, D = {7}) is broken in one way at a time --
  two clusters merged, one split, a non-minimal id, a label above its
  index, a label whose own point does not carry it, a mis-filtered size, a
  kept count off by one -- and the matching checker must report it;
* a 5-point chain (step 1, d = 1.5) with exactly one edge across two labels
  makes the closure count exactly 1 per sampled end point;
* mutant copies of the checkers (plausible slips: a dropped bound, a
  comparison of a value with itself, an off-by-one) must each fail one of
  these pins, as tests/test_oracle_mutants.py does for the clustering.
"""

import ctypes
import importlib.util
import os
import subprocess
import tempfile

import numpy as np
import pytest

import goldens
import oracle
from oracle import invariants

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INV_SRC = os.path.join(ROOT, "oracle", "invariants.py")
CPP_SRC = os.path.join(ROOT, "oracle", "fec_oracle.cpp")

G = goldens.load("filter9.txt")
XYZ, D = G["points"], G["d"]
GOOD = np.array([0, 1, 1, 0, 4, 0, 1, 7, 1], dtype=np.int32)  # unfiltered, min=1
CHAIN = np.array([[float(i), 0.0, 0.0] for i in range(5)], dtype=np.float32)


def _cases():
    """(name, check(inv, index, chain_index) -> True when the pin holds)."""
    merged = np.array([0, 0, 0, 0, 4, 0, 0, 7, 0], dtype=np.int32)   # A and B one label
    split = np.array([0, 1, 1, 0, 4, 0, 6, 7, 6], dtype=np.int32)    # B cut between 2 and 6
    nonmin = np.array([0, 2, 2, 0, 4, 0, 2, 7, 2], dtype=np.int32)   # B named by 2, not 1
    above = GOOD.copy()
    above[4] = 5                                                     # label 5 > index 4
    notself = GOOD.copy()
    notself[5] = 3                                                   # point 3 carries 0
    beyond = GOOD.copy()
    beyond[8] = 9                                                    # no point 9 (n = 9)
    below = GOOD.copy()
    below[7] = -2                                                    # only -1 marks filtered
    # filtered run with sizes 2..3: only A survives
    f23 = np.array([0, -1, -1, 0, -1, 0, -1, -1, -1], dtype=np.int32)
    kept_b = np.where(np.isin(GOOD, [0, 1]), GOOD, -1).astype(np.int32)  # B (size 4) kept
    dropped_a = np.full(9, -1, dtype=np.int32)                           # A (size 3) dropped
    f24 = np.array([0, 1, 1, 0, -1, 0, 1, -1, 1], dtype=np.int32)        # sizes 2..4: A, B
    cut = np.array([0, 0, 0, 3, 3], dtype=np.int32)                      # chain cut 2 | 3
    allp = np.arange(9)
    return [
        ("good labelling passes every checker",
         lambda inv, ix, cx: (inv.partition_problems(GOOD) == [] and
                              inv.size_problems(GOOD, 1, 100) == [] and
                              inv.filter_problems(f23, GOOD, 2, 3) == [] and
                              inv.closure_problems(ix, GOOD, allp) == [] and
                              inv.component_problems(ix, GOOD, allp, 100) == [] and
                              inv.count_kept(GOOD) == 4 and inv.count_kept(f24) == 2)),
        ("merged clusters: component checker",
         lambda inv, ix, cx: (inv.partition_problems(merged) == [] and
                              inv.closure_problems(ix, merged, allp) == [] and
                              inv.component_problems(ix, merged, [0], 100) != [] and
                              inv.component_problems(ix, merged, [1], 100) != [])),
        ("split cluster: closure and component checkers",
         lambda inv, ix, cx: (inv.partition_problems(split) == [] and
                              inv.closure_problems(ix, split, [2]) != [] and
                              inv.closure_problems(ix, split, [6]) != [] and
                              inv.closure_problems(ix, split, [0, 1, 3]) == [] and
                              inv.component_problems(ix, split, [8], 100) != [])),
        ("non-minimal id: partition and component checkers",
         lambda inv, ix, cx: (inv.partition_problems(nonmin) != [] and
                              inv.component_problems(ix, nonmin, [1], 100) != [])),
        ("label above its index: partition checker",
         lambda inv, ix, cx: inv.partition_problems(above) != []),
        ("label beyond the cloud or below -1: partition checker",
         lambda inv, ix, cx: (inv.partition_problems(beyond) != [] and
                              inv.partition_problems(below) != [])),
        ("label not carried by its own point: partition checker",
         lambda inv, ix, cx: inv.partition_problems(notself) != []),
        ("oversized cluster kept: size and filter checkers",
         lambda inv, ix, cx: (inv.size_problems(kept_b, 2, 3) != [] and
                              inv.filter_problems(kept_b, GOOD, 2, 3) != [])),
        ("in-range cluster dropped: filter checker",
         lambda inv, ix, cx: inv.filter_problems(dropped_a, GOOD, 2, 3) != []),
        ("undersized cluster kept: size checker",
         lambda inv, ix, cx: inv.size_problems(GOOD, 2, 100) != []),
        ("size bounds inclusive: size and filter checkers accept the bounds",
         lambda inv, ix, cx: (inv.size_problems(f24, 3, 4) == [] and
                              inv.filter_problems(f24, GOOD, 3, 4) == [])),
        ("unfiltered input with -1: filter checker",
         lambda inv, ix, cx: inv.filter_problems(f23, f23, 2, 3) != []),
        ("kept count off by one",
         lambda inv, ix, cx: (inv.count_kept(f24) == 2 and inv.count_kept(f23) == 1 and
                              inv.count_kept(dropped_a) == 0)),
        ("exactly one cross-label edge",
         lambda inv, ix, cx: (cx.closure_violations(cut, [2]) == 1 and
                              cx.closure_violations(cut, [3]) == 1 and
                              cx.closure_violations(cut, np.arange(5)) == 2 and
                              cx.closure_violations(cut, [0, 1, 4]) == 0 and
                              inv.closure_problems(cx, cut, [2]) != [])),
        ("component search stops after cap points",
         lambda inv, ix, cx: (cx.component(0, 4) == (5, 0) and cx.component(4, 5) == (5, 0) and
                              cx.component(2, 3) == (4, 0) and
                              inv.component_problems(cx, np.zeros(5, np.int32), [3], 4) == [] and
                              inv.component_problems(cx, cut, [3], 4) != [])),
    ]


CASES = _cases()


def _failing_pin(inv, ix, cx):
    for name, check in CASES:
        try:
            if not check(inv, ix, cx):
                return name
        except Exception as e:  # a crash is a failed pin too
            return "%s (%s)" % (name, type(e).__name__)
    return None


@pytest.fixture(scope="module")
def indexes():
    ix, cx = oracle.Index(XYZ, D), oracle.Index(CHAIN, 1.5)
    yield ix, cx
    ix.close()
    cx.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_checker_pin(case, indexes):
    ix, cx = indexes
    assert case[1](invariants, ix, cx), case[0]


def test_fixture_is_the_oracle_labelling():
    lab, k = oracle.fec(XYZ, D, 1, 100)
    assert np.array_equal(lab, GOOD) and k == 4


# ---------------------------------------------------------------- mutants

INV_MUTANTS = [
    ("lower bound off by one", "neg = lab < -1", "neg = lab < -2"),
    ("minimality compares names with themselves", "bad = kept[first] != uniq",
     "bad = uniq != uniq"),
    ("last carrier instead of first", "bad = kept[first] != uniq",
     "bad = kept[kept.size - 1 - np.unique(lab[kept][::-1], return_index=True)[1]] != uniq"),
    ("size max off by one", "bad = (cnt < lo) | (cnt > int(max_size))",
     "bad = (cnt < lo) | (cnt > int(max_size) + 1)"),
    ("size min bound dropped", "bad = (cnt < lo) | (cnt > int(max_size))",
     "bad = (cnt > int(max_size))"),
    ("filter min exclusive", "keep = (sizes[u] >= lo) & (sizes[u] <= int(max_size))",
     "keep = (sizes[u] > lo) & (sizes[u] <= int(max_size))"),
    ("filter compares expectation with itself", "if not np.array_equal(expect, f):",
     "if not np.array_equal(expect, expect):"),
    ("unfiltered -1 not refused", "    if (u < 0).any():\n        return",
     "    if (u < -1).any():\n        return"),
    ("closure tolerates one edge", "    if bad:\n", "    if bad > 1:\n"),
    ("component size not compared", "elif (c, m) != (have, lab):", "elif m != lab:"),
    ("component min not compared", "elif (c, m) != (have, lab):", "elif c != have:"),
    ("kept counts points", "return int(np.count_nonzero(lab == np.arange(lab.shape[0])))",
     "return int(np.count_nonzero(lab >= 0))"),
]


def _load_inv(text, tmp):
    path = os.path.join(tmp, "inv_mutant.py")
    with open(path, "w") as f:
        f.write(text)
    spec = importlib.util.spec_from_file_location("inv_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_unmutated_checker_copy_passes(indexes, tmp_path):
    mod = _load_inv(open(INV_SRC).read(), str(tmp_path))
    assert _failing_pin(mod, *indexes) is None


@pytest.mark.parametrize("mutant", INV_MUTANTS, ids=[m[0] for m in INV_MUTANTS])
def test_checker_mutant_is_caught(mutant, indexes, tmp_path):
    name, old, new = mutant
    src = open(INV_SRC).read()
    assert src.count(old) == 1, "mutation site for %r not found exactly once" % name
    mod = _load_inv(src.replace(old, new), str(tmp_path))
    assert _failing_pin(mod, *indexes) is not None, "mutant %r passed every pin" % name


CPP_MUTANTS = [
    ("closure compares a label with itself", "if (labels[j] != labels[i]) ++bad;",
     "if (labels[j] != labels[j]) ++bad;"),
    ("closure counts agreeing pairs", "if (labels[j] != labels[i]) ++bad;",
     "if (labels[j] == labels[i]) ++bad;"),
    ("component keeps the largest index", "if (j < mn) mn = j;", "if (j > mn) mn = j;"),
    ("component cap off by one", "while (head < q.size() && (int64_t)q.size() <= cap)",
     "while (head < q.size() && (int64_t)q.size() < cap)"),
    ("component never marks seen", "                seen[j] = 1;\n", "\n"),
]


class _MutIndex:
    """oracle.Index's closure and component queries over a mutant build."""

    def __init__(self, lib, xyz, d):
        self.lib, self.xyz = lib, np.ascontiguousarray(xyz, dtype=np.float32)
        self.h = lib.oracle_index_new(self.xyz.ctypes.data, self.xyz.shape[0], ctypes.c_float(d))

    def closure_violations(self, labels, sample):
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        s = np.ascontiguousarray(sample, dtype=np.int64)
        return int(self.lib.oracle_closure_violations(self.h, lab.ctypes.data, s.ctypes.data,
                                                      s.shape[0]))

    def component(self, seed, cap):
        mn = ctypes.c_int64(0)
        c = self.lib.oracle_component(self.h, int(seed), int(cap), ctypes.byref(mn), None)
        return int(c), int(mn.value)

    def close(self):
        self.lib.oracle_index_free(self.h)


def _build_cpp(text, tmp):
    cpp, so = os.path.join(tmp, "m.cpp"), os.path.join(tmp, "m.so")
    with open(cpp, "w") as f:
        f.write(text)
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    so, cpp], check=True, capture_output=True)
    lib = ctypes.CDLL(so)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_index_new.argtypes = [vp, i64, ctypes.c_float]
    lib.oracle_index_new.restype = vp
    lib.oracle_index_free.argtypes = [vp]
    lib.oracle_index_free.restype = None
    lib.oracle_closure_violations.argtypes = [vp, vp, vp, i64]
    lib.oracle_closure_violations.restype = i64
    lib.oracle_component.argtypes = [vp, i64, i64, vp, vp]
    lib.oracle_component.restype = i64
    return lib


def _cpp_failing_pin(text):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_cpp(text, tmp)
        ix, cx = _MutIndex(lib, XYZ, D), _MutIndex(lib, CHAIN, 1.5)
        try:
            return _failing_pin(invariants, ix, cx)
        finally:
            ix.close()
            cx.close()


def test_unmutated_oracle_queries_pass():
    assert _cpp_failing_pin(open(CPP_SRC).read()) is None


@pytest.mark.parametrize("mutant", CPP_MUTANTS, ids=[m[0] for m in CPP_MUTANTS])
def test_oracle_query_mutant_is_caught(mutant):
    name, old, new = mutant
    src = open(CPP_SRC).read()
    assert src.count(old) == 1, "mutation site for %r not found exactly once" % name
    assert _cpp_failing_pin(src.replace(old, new)) is not None, "mutant %r passed" % name
