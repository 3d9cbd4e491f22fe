"""CPU oracle for fixed-radius Euclidean clustering -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never links, loads or calls it,
and it shares no code with the GPU path.

Contents:

* ``fec``            -- the C++ oracle (``fec_oracle.cpp``): Alg. 1's
  point-wise loop over a kd-tree, then canonical labels and the size filter.
* ``fec_both``       -- one run, filtered and unfiltered labels together.
* ``fec_raw``        -- the raw Alg. 1 label values after any number of steps.
* ``Index``          -- the oracle's kd-tree kept alive for sampled checks on
  clouds too large to cluster in full (component of one point, neighbours
  of one point, closure on a sample).
* ``bruteforce``     -- an independent O(n^2) NumPy BFS (its own module).
* ``invariants``     -- property checks that hold at any size (own module).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fec_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

LITERAL_SCAN = 1
SKIP_LABELLED = 2

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction, no fast-math)."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    f32p = ctypes.c_void_p
    lib.oracle_fec_raw.argtypes = [f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_void_p]
    lib.oracle_fec_raw.restype = ctypes.c_int32
    lib.oracle_fec.argtypes = [f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    lib.oracle_fec.restype = ctypes.c_int64
    lib.oracle_fec_ex.argtypes = [f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_void_p]
    lib.oracle_fec_ex.restype = ctypes.c_int64
    lib.oracle_fec_full.argtypes = [f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_fec_full.restype = ctypes.c_int64
    lib.oracle_index_new.argtypes = [f32p, ctypes.c_int64, ctypes.c_float]
    lib.oracle_index_new.restype = ctypes.c_void_p
    lib.oracle_index_free.argtypes = [ctypes.c_void_p]
    lib.oracle_index_free.restype = None
    lib.oracle_index_neighbors.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_int64]
    lib.oracle_index_neighbors.restype = ctypes.c_int64
    lib.oracle_component.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_component.restype = ctypes.c_int64
    lib.oracle_closure_violations.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_int64]
    lib.oracle_closure_violations.restype = ctypes.c_int64
    lib.oracle_count_neighbors.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    lib.oracle_count_neighbors.restype = ctypes.c_int64
    _lib = lib
    return lib


def _as_xyz(xyz) -> np.ndarray:
    a = np.ascontiguousarray(xyz, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("xyz must be float32 [n, 3]")
    return a


def fec(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1, flags: int = 0,
        th_max: int = 0):
    """Canonical FEC labels (int32 [n]) and the number of kept clusters.

    ``flags`` and ``th_max`` (> 0: keep only the th_max nearest neighbours of
    each visited point, Alg. 1's cap) select fidelity variants of Alg. 1 for
    measuring their effect; the defaults are the exact clustering.
    """
    a = _as_xyz(xyz)
    n = a.shape[0]
    out = np.empty(n, dtype=np.int32)
    k = _load().oracle_fec_ex(a.ctypes.data, n, ctypes.c_float(d), int(min_size),
                              int(max_size), int(flags), int(th_max), out.ctypes.data)
    if k < 0:
        raise ValueError("oracle_fec rejected its arguments")
    return out, int(k)


def fec_both(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1):
    """One run of the exact clustering, two outputs: (filtered labels, kept
    clusters, unfiltered canonical labels, number of clusters)."""
    a = _as_xyz(xyz)
    n = a.shape[0]
    out = np.empty(n, dtype=np.int32)
    canon = np.empty(n, dtype=np.int32)
    nc = ctypes.c_int64(0)
    k = _load().oracle_fec_full(a.ctypes.data, n, ctypes.c_float(d), int(min_size),
                                int(max_size), 0, 0, out.ctypes.data, canon.ctypes.data,
                                ctypes.byref(nc))
    if k < 0:
        raise ValueError("oracle_fec rejected its arguments")
    return out, int(k), canon, int(nc.value)


def fec_raw(xyz, d: float, steps: int | None = None, flags: int = 0):
    """Raw Alg. 1 label values (int64 [n], 0 = unlabelled) after ``steps``."""
    a = _as_xyz(xyz)
    n = a.shape[0]
    steps = n if steps is None else int(steps)
    out = np.zeros(n, dtype=np.int64)
    rc = _load().oracle_fec_raw(a.ctypes.data, n, ctypes.c_float(d), steps, int(flags),
                                out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_fec_raw rejected its arguments")
    return out


class Index:
    """The oracle's kd-tree over one cloud, for sampled queries."""

    def __init__(self, xyz, d: float):
        self.xyz = _as_xyz(xyz)
        self.n = self.xyz.shape[0]
        self.d = float(d)
        self._h = _load().oracle_index_new(self.xyz.ctypes.data, self.n, ctypes.c_float(d))
        if not self._h:
            raise ValueError("oracle_index_new failed")

    def close(self):
        if self._h:
            _load().oracle_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def neighbors(self, i: int) -> np.ndarray:
        """Indices j != i with E(i, j), sorted."""
        lib = _load()
        cap = 256
        while True:
            buf = np.empty(cap, dtype=np.int64)
            c = lib.oracle_index_neighbors(self._h, int(i), buf.ctypes.data, cap)
            if c <= cap:
                return np.sort(buf[:c])
            cap = int(c)

    def component(self, seed: int, cap: int, members: bool = False):
        """(size, min index[, member indices]) of seed's component.

        Size is ``cap + 1`` when the search stopped after reaching more than
        ``cap`` points.
        """
        mn = ctypes.c_int64(0)
        buf = np.empty(cap if members else 0, dtype=np.int64)
        c = _load().oracle_component(self._h, int(seed), int(cap), ctypes.byref(mn),
                                     buf.ctypes.data if members else None)
        if members:
            return int(c), int(mn.value), buf[:min(c, cap)]
        return int(c), int(mn.value)

    def closure_violations(self, labels, sample) -> int:
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        s = np.ascontiguousarray(sample, dtype=np.int64)
        return int(_load().oracle_closure_violations(self._h, lab.ctypes.data, s.ctypes.data,
                                                     s.shape[0]))

    def count_neighbors(self, sample) -> int:
        s = np.ascontiguousarray(sample, dtype=np.int64)
        return int(_load().oracle_count_neighbors(self._h, s.ctypes.data, s.shape[0]))
