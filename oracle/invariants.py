"""Properties every correct labelling has, at any size -- TEST INFRASTRUCTURE.

For labels produced with the output convention of the clustering (each kept
cluster named by its smallest point index, -1 for points of clusters whose
size lies outside [min_size, max_size]):

* partition / minimality: no label is below -1, and the first point that
  carries a kept label L is point L (so 0 <= L <= i for every carrier i,
  and point L carries L itself);
* size filter: every kept label is carried by between min_size and max_size
  points;
* filter exactness: the filtered labelling equals the unfiltered one with
  clusters of out-of-range size masked to -1;
* closure (with an ``oracle.Index``): both ends of every edge of the graph
  carry the same label, checked on a sample of points (catches a split
  cluster, not a merge);
* components (with an ``oracle.Index``): for sampled seed points, the
  breadth-first component of the seed in the graph has as many points as
  the unfiltered labelling gives the seed's label, and its smallest index is
  that label (catches merges and splits alike).

Each check returns a list of human-readable problems (empty when it holds).
"""

from __future__ import annotations

import numpy as np


def partition_problems(labels: np.ndarray, max_report: int = 5) -> list[str]:
    """Labels that are not -1 or a valid cluster name: a value below -1, or a
    kept label L whose first carrier is not point L.  The second condition is
    the whole of partition and minimality: it means every point carrying L
    has index >= L (so L <= i, and L < n), and point L carries L itself."""
    lab = np.asarray(labels, dtype=np.int64)
    out = []
    neg = lab < -1
    if neg.any():
        out.append("labels below -1 at %s" % np.nonzero(neg)[0][:max_report].tolist())
    kept = np.nonzero(lab >= 0)[0]
    if kept.size:
        uniq, first = np.unique(lab[kept], return_index=True)
        bad = kept[first] != uniq
        if bad.any():
            out.append("kept labels whose first carrier is another point: %s"
                       % uniq[bad][:max_report].tolist())
    return out


def size_problems(labels: np.ndarray, min_size: int, max_size: int) -> list[str]:
    lab = np.asarray(labels, dtype=np.int64)
    kept = lab[lab >= 0]
    if kept.size == 0:
        return []
    uniq, cnt = np.unique(kept, return_counts=True)
    lo = max(1, int(min_size))
    bad = (cnt < lo) | (cnt > int(max_size))
    if bad.any():
        return ["%d kept clusters have sizes outside [%d, %d], e.g. label %d size %d"
                % (int(bad.sum()), lo, max_size, int(uniq[bad][0]), int(cnt[bad][0]))]
    return []


def filter_problems(filtered: np.ndarray, unfiltered: np.ndarray, min_size: int,
                    max_size: int) -> list[str]:
    f = np.asarray(filtered, dtype=np.int64)
    u = np.asarray(unfiltered, dtype=np.int64)
    if (u < 0).any():
        return ["unfiltered labelling contains -1"]
    sizes = np.bincount(u, minlength=u.shape[0])
    lo = max(1, int(min_size))
    keep = (sizes[u] >= lo) & (sizes[u] <= int(max_size))
    expect = np.where(keep, u, -1)
    if not np.array_equal(expect, f):
        w = np.nonzero(expect != f)[0][:5]
        return ["filtered labels differ from masked unfiltered labels at %s" % w.tolist()]
    return []


def closure_problems(index, labels: np.ndarray, sample: np.ndarray) -> list[str]:
    bad = index.closure_violations(labels, sample)
    if bad:
        return ["%d edges from sampled points join different labels" % bad]
    return []


def component_problems(index, unfiltered: np.ndarray, seeds, cap: int) -> list[str]:
    """Seeds whose true component (breadth-first search, stopped after
    ``cap`` points) does not match the unfiltered labelling: another size
    (clusters merged or split) or another smallest index.  Seeds whose
    component is larger than ``cap`` are compared only by being larger."""
    u = np.asarray(unfiltered, dtype=np.int64)
    sizes = np.bincount(u[u >= 0], minlength=u.shape[0])
    out = []
    for s in np.asarray(seeds, dtype=np.int64):
        c, m = index.component(int(s), int(cap))
        lab = int(u[s])
        have = int(sizes[lab]) if lab >= 0 else 0
        if c > cap:
            if have <= cap:
                out.append("seed %d: component larger than %d, label %d has %d points"
                           % (s, cap, lab, have))
        elif (c, m) != (have, lab):
            out.append("seed %d: component size %d min %d, labelling size %d label %d"
                       % (s, c, m, have, lab))
        if len(out) >= 5:
            break
    return out


def count_kept(labels: np.ndarray) -> int:
    lab = np.asarray(labels)
    return int(np.count_nonzero(lab == np.arange(lab.shape[0])))
