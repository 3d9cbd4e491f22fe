"""Properties every correct labelling has, at any size -- TEST INFRASTRUCTURE.

For labels produced with the output convention of the clustering (each kept
cluster named by its smallest point index, -1 for points of clusters whose
size lies outside [min_size, max_size]):

* partition / minimality: a kept label L satisfies 0 <= L <= i, point L
  carries L itself, and L is the smallest index carrying L;
* size filter: every kept label is carried by between min_size and max_size
  points;
* filter exactness: the filtered labelling equals the unfiltered one with
  clusters of out-of-range size masked to -1;
* closure (with an ``oracle.Index``): both ends of every edge of the graph
  carry the same label, checked on a sample of points.

Each check returns a list of human-readable problems (empty when it holds).
"""

from __future__ import annotations

import numpy as np


def partition_problems(labels: np.ndarray, max_report: int = 5) -> list[str]:
    lab = np.asarray(labels, dtype=np.int64)
    n = lab.shape[0]
    out = []
    idx = np.arange(n)
    bad_range = (lab < -1) | (lab > idx)
    if bad_range.any():
        w = np.nonzero(bad_range)[0][:max_report]
        out.append("labels outside {-1} U [0, i] at %s" % w.tolist())
        return out
    kept = lab >= 0
    roots = lab[kept]
    self_ok = lab[roots] == roots
    if not self_ok.all():
        w = np.nonzero(kept)[0][~self_ok][:max_report]
        out.append("label's own point does not carry it at %s" % w.tolist())
    # minimality: the first occurrence of each kept label is the label itself
    if kept.any():
        uniq, first = np.unique(lab[kept], return_index=True)
        first_idx = idx[kept][first]
        if not np.array_equal(uniq, first_idx):
            out.append("a kept label is not the smallest index carrying it")
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


def count_kept(labels: np.ndarray) -> int:
    lab = np.asarray(labels)
    return int(np.count_nonzero(lab == np.arange(lab.shape[0])))
