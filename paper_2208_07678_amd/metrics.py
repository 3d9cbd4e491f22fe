"""Segmentation quality: the average precision of Eq. (2) (host-side, NumPy).

AP = TP / (TP + FP) over the predicted clusters.  A predicted cluster is a
true positive when its point-wise intersection over union with the
ground-truth instance it overlaps most reaches the threshold (0.75 in the
paper's experiments); every other predicted cluster is a false positive.
Points labelled -1 (filtered out) belong to no predicted cluster.
"""

from __future__ import annotations

import numpy as np


def average_precision(labels, truth, iou: float = 0.75) -> float:
    """AP of predicted ``labels`` against ground-truth instance ids ``truth``.

    Both are integer arrays over the same points; ``labels`` may hold -1.
    Returns 1.0 when there is no predicted cluster.
    """
    lab = np.asarray(labels).astype(np.int64).ravel()
    gt = np.asarray(truth).astype(np.int64).ravel()
    if lab.shape != gt.shape:
        raise ValueError("labels and truth differ in length")
    _, gt_id = np.unique(gt, return_inverse=True)
    gt_size = np.bincount(gt_id)
    keep = lab >= 0
    if not keep.any():
        return 1.0
    _, pr_id = np.unique(lab[keep], return_inverse=True)
    pr_size = np.bincount(pr_id)
    g = gt_id[keep]
    # overlap of every (predicted, truth) pair that shares points
    pair = pr_id * (gt_size.shape[0] + 1) + g
    up, inter = np.unique(pair, return_counts=True)
    p = up // (gt_size.shape[0] + 1)
    t = up % (gt_size.shape[0] + 1)
    # the truth instance each predicted cluster overlaps most (ties: smaller id)
    order = np.lexsort((t, -inter, p))
    first = np.ones(order.shape[0], bool)
    first[1:] = p[order][1:] != p[order][:-1]
    best = order[first]
    i = inter[best]
    union = pr_size[p[best]] + gt_size[t[best]] - i
    tp = int((i >= iou * union).sum())
    return tp / pr_size.shape[0]
