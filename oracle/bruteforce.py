"""Brute-force clustering in NumPy -- TEST INFRASTRUCTURE (pins the oracle).

An O(n^2) definition of the clustering, independent of the C++ oracle: every
pair is tested with the binary32 predicate of Eq. (1) written out in NumPy
float32 arithmetic in the fixed order ((dx*dx + dy*dy) + dz*dz), the
components of the resulting graph are found by breadth-first search, each
component is named by its smallest index, and clusters outside
[min_size, max_size] become -1.  Meant for clouds up to a few thousand points.
"""

from __future__ import annotations

import numpy as np


def adjacency(xyz, d: float) -> np.ndarray:
    """Boolean [n, n] matrix of E(i, j) (the diagonal is True for finite points)."""
    p = np.asarray(xyz, dtype=np.float32)
    d32 = np.float32(d)
    d2 = np.float32(d32 * d32)
    with np.errstate(invalid="ignore", over="ignore"):
        dx = p[:, None, 0] - p[None, :, 0]
        dy = p[:, None, 1] - p[None, :, 1]
        dz = p[:, None, 2] - p[None, :, 2]
        s = (dx * dx + dy * dy)
        s = s + dz * dz
        assert s.dtype == np.float32
        return s < d2


def components(adj: np.ndarray) -> np.ndarray:
    """Smallest member index of each vertex's component (BFS)."""
    n = adj.shape[0]
    comp = np.full(n, -1, dtype=np.int64)
    for s in range(n):
        if comp[s] >= 0:
            continue
        comp[s] = s
        frontier = np.array([s])
        while frontier.size:
            reach = adj[frontier].any(axis=0) & (comp < 0)
            frontier = np.nonzero(reach)[0]
            comp[frontier] = s
    return comp


def cluster(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1):
    """(labels int32 [n], kept cluster count) by brute force."""
    comp = components(adjacency(xyz, d))
    n = comp.shape[0]
    if n == 0:
        return np.zeros(0, dtype=np.int32), 0
    sizes = np.bincount(comp, minlength=n)
    lo = max(1, int(min_size))
    keep_root = (sizes >= lo) & (sizes <= int(max_size))
    labels = np.where(keep_root[comp], comp, -1).astype(np.int32)
    k = int(np.count_nonzero(keep_root & (sizes > 0)))
    return labels, k
