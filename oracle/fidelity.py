"""Fidelity variants of Alg. 1 against the exact clustering -- TEST INFRASTRUCTURE.

Measures how much the printed details of Alg. 1 that this project does not
follow (readings A1 and A2: skipping points that already carry a label, and
a neighbour cap Th_max) over-segment, compared with the exact connected
components, on the blob cloud and the LiDAR frame workloads.  Oracle only:

    python -m oracle.fidelity

For every variant: the number of clusters (no size filter), whether the
variant's partition refines the exact one (every variant cluster inside one
exact cluster), how many exact clusters it splits, and the share of points
outside the largest piece of their exact cluster.
"""

from __future__ import annotations

import json
import sys

import numpy as np

from . import SKIP_LABELLED, fec


def compare(exact: np.ndarray, variant: np.ndarray) -> dict:
    """Partition statistics of ``variant`` against ``exact`` (canonical labels, no filter)."""
    n = exact.shape[0]
    pairs = np.unique(np.stack([variant, exact], 1), axis=0)
    # refinement: each variant cluster maps to exactly one exact cluster
    refines = np.unique(pairs[:, 0]).shape[0] == pairs.shape[0]
    pieces = np.bincount(np.searchsorted(np.unique(exact), pairs[:, 1]))
    split = int((pieces > 1).sum())
    # points outside the largest piece of their exact cluster
    key = exact.astype(np.int64) * (n + 1) + variant.astype(np.int64)
    uk, cnt = np.unique(key, return_counts=True)
    ex = uk // (n + 1)
    order = np.lexsort((-cnt, ex))
    first = np.ones(order.shape[0], bool)
    first[1:] = ex[order][1:] != ex[order][:-1]
    moved = int(n - cnt[order][first].sum())
    return {"clusters": int(np.unique(variant).shape[0]), "refines_exact": bool(refines),
            "exact_clusters_split": split, "points_moved_share": moved / max(n, 1)}


def report(configs=("blobs20k", "lidar120k"), caps=(100, 50, 20, 10, 5)) -> list[dict]:
    import synth
    rows = []
    for name in configs:
        xyz, d, _, _ = synth.make_config(name)
        exact, _ = fec(xyz, d)
        base = {"workload": name, "n": int(xyz.shape[0]), "d": d,
                "exact_clusters": int(np.unique(exact).shape[0])}
        variants = [("skip labelled points (A1, as printed)", dict(flags=SKIP_LABELLED))]
        variants += [("Th_max = %d (A2)" % c, dict(th_max=c)) for c in caps]
        for label, kw in variants:
            lab, _ = fec(xyz, d, **kw)
            rows.append(dict(base, variant=label, **compare(exact, lab)))
    return rows


if __name__ == "__main__":
    for r in report():
        print(json.dumps(r))
        sys.stdout.flush()
