"""The AP of Eq. (2) and the synthetic voxel clusters (host only)."""

import numpy as np
from scipy.spatial import cKDTree

import oracle
import synth
from paper_2208_07678_amd.metrics import average_precision


def test_ap_hand_cases():
    gt = np.array([0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2])
    assert average_precision(gt, gt) == 1.0
    assert average_precision(gt * 7 + 3, gt) == 1.0          # ids need not match
    # cluster 0 split 3 + 1: IoU 3/4 (exactly the threshold: TP) and 1/4 (FP)
    lab = np.array([0, 0, 0, 9, 1, 1, 1, 1, 2, 2, 2, 2])
    assert average_precision(lab, gt) == 3 / 4
    # split 2 + 2: two FPs
    lab = np.array([0, 0, 9, 9, 1, 1, 1, 1, 2, 2, 2, 2])
    assert average_precision(lab, gt) == 2 / 4
    # clusters 1 and 2 merged: IoU 4/8 with either, one FP among two predictions
    lab = np.array([0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1])
    assert average_precision(lab, gt) == 1 / 2
    # filtered points (-1) are in no predicted cluster
    lab = np.array([0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1])
    assert average_precision(lab, gt) == 1.0
    assert average_precision(np.full(12, -1), gt) == 1.0
    # a stricter threshold turns the 3/4 piece into a false positive
    lab = np.array([0, 0, 0, 9, 1, 1, 1, 1, 2, 2, 2, 2])
    assert average_precision(lab, gt, iou=0.8) == 2 / 4


def test_voxel_clusters_shape_and_separation():
    for sub in (0, 4):
        x, gt = synth.voxel_clusters(60, 50, subclusters=sub, seed=2)
        assert x.shape == (3000, 3) and x.dtype == np.float32
        assert np.array_equal(np.bincount(gt), np.full(60, 50))
        assert not np.all(np.diff(gt) >= 0)               # shuffled order
        # points of different clusters are at least one voxel apart
        pairs = cKDTree(x).query_pairs(0.999, output_type="ndarray")
        assert (gt[pairs[:, 0]] == gt[pairs[:, 1]]).all()
    assert np.array_equal(synth.voxel_clusters(10, 20, seed=1)[0],
                          synth.voxel_clusters(10, 20, seed=1)[0])


def test_exact_clustering_recovers_even_voxel_clusters():
    # d = 0.9 voxel joins the points of an evenly filled voxel and no two
    # voxels: the oracle's partition is the ground truth, AP 1
    for m in (10, 60):
        x, gt = synth.voxel_clusters(80, m, seed=m)
        lab, k = oracle.fec(x, synth.SWEEP_D)
        assert k == 80 and average_precision(lab, gt) == 1.0
