"""Fidelity variants of Alg. 1 in the oracle (measurement only): pins.

The exact clustering ignores two printed details of Alg. 1 (readings A1 and
A2).  The oracle keeps both as variants to measure their effect; these tests
pin the variants themselves.
"""

import numpy as np

import oracle
import synth
from oracle import bruteforce
from oracle.fidelity import compare


def test_cap_drops_an_edge_seen_from_both_sides():
    # A-B and C-D are 0.5 apart, B-C 0.9 (< d = 1): one exact cluster.  With
    # Th_max = 1, B keeps only A and C keeps only D, so the B-C edge is never
    # used and Alg. 1 returns two segments.
    x = np.array([[0, 0, 0], [0.5, 0, 0], [1.4, 0, 0], [1.9, 0, 0]], np.float32)
    exact, k = oracle.fec(x, 1.0)
    assert exact.tolist() == [0, 0, 0, 0] and k == 1
    capped, k1 = oracle.fec(x, 1.0, th_max=1)
    assert capped.tolist() == [0, 0, 2, 2] and k1 == 2
    assert oracle.fec(x, 1.0, th_max=2)[0].tolist() == [0, 0, 0, 0]


def test_cap_at_or_above_every_degree_is_exact():
    for seed in range(20):
        x = synth.random_cloud(300, extent=(3, 3, 3), seed=seed)
        want = bruteforce.cluster(x, 0.4)[0]
        got, _ = oracle.fec(x, 0.4, th_max=299)
        assert np.array_equal(got, want), seed


def test_variants_refine_the_exact_partition():
    for seed in range(30):
        rng = np.random.default_rng(seed)
        x = synth.random_cloud(int(rng.integers(50, 600)), extent=(4, 4, 2), seed=seed)
        x = x[rng.permutation(x.shape[0])]
        d = float(rng.uniform(0.2, 0.6))
        exact, _ = oracle.fec(x, d)
        for kw in (dict(flags=oracle.SKIP_LABELLED), dict(th_max=1), dict(th_max=3)):
            lab, _ = oracle.fec(x, d, **kw)
            st = compare(exact, lab)
            assert st["refines_exact"], (seed, kw)
            assert st["clusters"] >= np.unique(exact).shape[0]


def test_compare_statistics_on_a_hand_case():
    exact = np.array([0, 0, 0, 0, 4, 4], np.int32)
    variant = np.array([0, 0, 2, 2, 4, 4], np.int32)
    st = compare(exact, variant)
    assert st == {"clusters": 3, "refines_exact": True, "exact_clusters_split": 1,
                  "points_moved_share": 2 / 6}
    assert not compare(exact, np.array([0, 0, 0, 0, 0, 4], np.int32))["refines_exact"]
