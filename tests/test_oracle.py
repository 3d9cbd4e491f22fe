"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle (oracle/fec_oracle.cpp) is checked against
* hand-derived fixtures (tests/golden/*.txt, each with its derivation),
* an independent O(n^2) NumPy brute force on thousands of small clouds,
* scipy's kd-tree pair search + graph connected components,
* closed forms (Fig. 3's extreme cases, chains, separated blobs),
* invariants (partition, minimality, size filter, closure),
* the printed relabel-by-rescan loop of Alg. 1, step by step.
"""

import numpy as np
import pytest

import goldens
import oracle
import synth
from oracle import bruteforce, invariants


# ------------------------------------------------------------------ fixtures

@pytest.mark.parametrize("case", goldens.all_cases(), ids=lambda c: c[0] if isinstance(c, tuple) else None)
def test_golden_cases(case):
    name, xyz, d, mn, mx, k, labels = case
    got, gk = oracle.fec(xyz, d, mn, mx)
    assert np.array_equal(got, labels), (name, got, labels)
    assert gk == k
    bf, bk = bruteforce.cluster(xyz, d, mn, mx)
    assert np.array_equal(bf, labels) and bk == k


def test_chain4_raw_labels():
    g = goldens.load("chain4.txt")
    assert np.array_equal(oracle.fec_raw(g["points"], g["d"], flags=oracle.SKIP_LABELLED),
                          g["raw_skip"])
    assert np.array_equal(oracle.fec_raw(g["points"], g["d"]), g["raw_all"])
    assert np.array_equal(oracle.fec_raw(g["points"], g["d"], flags=oracle.LITERAL_SCAN),
                          g["raw_all"])


# ------------------------------------------------------------ brute force

def _small_cloud(seed):
    """A varied small cloud and threshold for brute-force comparison."""
    rng = np.random.default_rng(seed)
    kind = seed % 8
    n = int(rng.integers(1, 160))
    if kind == 0:      # uniform, sparse to dense
        ext = rng.uniform(0.5, 6.0)
        x = synth.random_cloud(n, extent=(ext, ext, ext * rng.uniform(0.1, 1)), seed=seed)
        d = float(rng.uniform(0.1, 1.5))
    elif kind == 1:    # a few Gaussian blobs
        c = rng.uniform(0, 10, size=(int(rng.integers(1, 6)), 3))
        x = (c[rng.integers(0, c.shape[0], n)] + rng.normal(0, 0.4, (n, 3))).astype(np.float32)
        d = float(rng.uniform(0.2, 1.0))
    elif kind == 2:    # chains with spacing around d
        d = float(rng.uniform(0.2, 1.0))
        x = synth.chain_cloud(n, d * float(rng.uniform(0.8, 1.2)), axis=int(rng.integers(0, 3)))
        x = x[rng.permutation(n)]
    elif kind == 3:    # near-threshold pairs
        d = float(rng.choice([0.5, 0.35, 0.2, 1.0, 0.1]))
        x = synth.near_threshold_cloud(max(1, n // 2), d, seed=seed, spread=3.0)
    elif kind == 4:    # duplicates and a grid at spacing exactly d
        d = 0.25
        g = np.stack(np.meshgrid(*[np.arange(4) * 0.25] * 3, indexing="ij"), -1).reshape(-1, 3)
        x = np.concatenate([g, g[rng.integers(0, g.shape[0], 8)]]).astype(np.float32)
        x = x[rng.permutation(x.shape[0])]
    elif kind == 5:    # far from the origin, negative coordinates
        x = synth.random_cloud(n, extent=(3, 3, 3), seed=seed, offset=(-2000.0, 1500.0, -40.0))
        d = float(rng.uniform(0.2, 1.0))
    elif kind == 6:    # with non-finite points mixed in
        x = synth.random_cloud(n, extent=(3, 3, 3), seed=seed)
        bad = rng.random(n) < 0.2
        vals = np.array([np.nan, np.inf, -np.inf], dtype=np.float32)
        x[bad, rng.integers(0, 3)] = vals[rng.integers(0, 3, int(bad.sum()))]
        d = float(rng.uniform(0.3, 1.2))
    else:              # flat plane (2-D) like the ground of a scan
        x = synth.random_cloud(n, extent=(4, 4, 0.0), seed=seed)
        d = float(rng.uniform(0.2, 0.8))
    mn = int(rng.integers(0, 4))
    lo = max(mn, 1)
    mx = int(rng.integers(lo, max(lo + 1, x.shape[0] + 2)))
    return x, d, mn, mx


def test_oracle_equals_bruteforce_small_clouds():
    bad = []
    for seed in range(2000):
        x, d, mn, mx = _small_cloud(seed)
        a, ka = oracle.fec(x, d, mn, mx)
        b, kb = bruteforce.cluster(x, d, mn, mx)
        if not (np.array_equal(a, b) and ka == kb):
            bad.append(seed)
    assert not bad, "oracle != brute force for seeds %s" % bad[:10]


@pytest.mark.parametrize("seed", range(6))
def test_oracle_equals_bruteforce_medium(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(800, 1600))
    x = synth.random_cloud(n, extent=(8, 8, 3), seed=100 + seed)
    d = float(rng.uniform(0.3, 0.7))
    a, ka = oracle.fec(x, d, 1, n)
    b, kb = bruteforce.cluster(x, d, 1, n)
    assert np.array_equal(a, b) and ka == kb


def test_literal_rescan_matches_member_lists_every_step():
    for seed in range(30):
        x, d, _, _ = _small_cloud(seed)
        n = x.shape[0]
        for flags in (0, oracle.SKIP_LABELLED):
            for steps in range(n + 1):
                fast = oracle.fec_raw(x, d, steps=steps, flags=flags)
                slow = oracle.fec_raw(x, d, steps=steps, flags=flags | oracle.LITERAL_SCAN)
                assert np.array_equal(fast, slow), (seed, flags, steps)


# ------------------------------------------------------------ library check

def _scipy_labels(xyz, d, mn, mx):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree

    p64 = xyz.astype(np.float64)
    n = xyz.shape[0]
    pairs = cKDTree(p64).query_pairs(float(d) * (1 + 1e-5), output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    a, b = xyz[i], xyz[j]
    dx, dy, dz = a[:, 0] - b[:, 0], a[:, 1] - b[:, 1], a[:, 2] - b[:, 2]
    s = (dx * dx + dy * dy) + dz * dz
    d32 = np.float32(d)
    keep = s < np.float32(d32 * d32)
    g = coo_matrix((np.ones(int(keep.sum())), (i[keep], j[keep])), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    first = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(first, comp, np.arange(n))
    size = np.bincount(comp)
    lo = max(1, mn)
    ok = (size >= lo) & (size <= mx)
    return np.where(ok[comp], first[comp], -1).astype(np.int32), int(ok.sum())


@pytest.mark.parametrize("name", ["blobs20k", "lidar120k"])
def test_oracle_equals_scipy_on_workloads(name):
    xyz, d, mn, mx = synth.make_config(name)
    a, ka = oracle.fec(xyz, d, mn, mx)
    b, kb = _scipy_labels(xyz, d, mn, mx)
    assert ka == kb and np.array_equal(a, b)


def test_oracle_equals_scipy_map_prefix():
    xyz = synth.lidar_map(frames=[0, 1])
    a, ka = oracle.fec(xyz, 0.2, 100, 5000000)
    b, kb = _scipy_labels(xyz, 0.2, 100, 5000000)
    assert ka == kb and np.array_equal(a, b)


def test_oracle_equals_scipy_random_200k():
    xyz = synth.random_cloud(200000, extent=(40, 40, 4), seed=7)
    a, ka = oracle.fec(xyz, 0.3, 1, 200000)
    b, kb = _scipy_labels(xyz, 0.3, 1, 200000)
    assert ka == kb and np.array_equal(a, b)


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("name", ["blobs20k", "lidar120k"])
def test_oracle_invariants(name):
    xyz, d, mn, mx = synth.make_config(name)
    lab, k = oracle.fec(xyz, d, mn, mx)
    unf, _ = oracle.fec(xyz, d, 1, xyz.shape[0])
    assert invariants.partition_problems(lab) == []
    assert invariants.partition_problems(unf) == []
    assert invariants.size_problems(lab, mn, mx) == []
    assert invariants.filter_problems(lab, unf, mn, mx) == []
    assert invariants.count_kept(lab) == k
    idx = oracle.Index(xyz, d)
    sample = np.random.default_rng(0).choice(xyz.shape[0], 3000, replace=False)
    assert invariants.closure_problems(idx, unf, sample) == []


def test_component_search_matches_full_run():
    xyz, d, mn, mx = synth.make_config("lidar120k")
    unf, _ = oracle.fec(xyz, d, 1, xyz.shape[0])
    idx = oracle.Index(xyz, d)
    for s in np.random.default_rng(1).choice(xyz.shape[0], 40, replace=False):
        size, mnidx = idx.component(int(s), cap=xyz.shape[0])
        assert mnidx == unf[s]
        assert size == int(np.count_nonzero(unf == unf[s]))
    big = int(np.bincount(unf).argmax())
    size, _ = idx.component(big, cap=1000)
    assert size == 1001


# ------------------------------------------------------------ closed forms

def test_fig3_case2_small_d_all_singletons():
    x = synth.random_cloud(500, extent=(10, 10, 10), seed=3)
    p = x.astype(np.float64)
    dmin = np.sqrt(((p[:, None] - p[None]) ** 2).sum(-1) + np.eye(500) * 1e9).min()
    lab, k = oracle.fec(x, float(dmin) * 0.99, 1, 500)
    assert k == 500 and np.array_equal(lab, np.arange(500))


def test_fig3_case1_large_d_one_cluster():
    x = synth.random_cloud(500, extent=(10, 10, 10), seed=4)
    lab, k = oracle.fec(x, 18.0, 1, 500)   # diagonal is 17.3
    assert k == 1 and (lab == 0).all()


def test_fig3_case3_collinear_chain():
    x = synth.chain_cloud(1000, 0.45, axis=1)
    x = x[np.random.default_rng(0).permutation(1000)]
    lab, k = oracle.fec(x, 0.5, 1, 1000)
    assert k == 1 and (lab == 0).all()
    # spacing exactly d (0.5 and multiples are exact): strict test splits all
    y = synth.chain_cloud(64, 0.5, axis=0)
    lab, k = oracle.fec(y, 0.5, 1, 64)
    assert k == 64 and np.array_equal(lab, np.arange(64))


def test_separated_blobs_count():
    rng = np.random.default_rng(5)
    centres = np.stack(np.meshgrid(np.arange(4) * 10.0, np.arange(5) * 10.0, [0.0],
                                   indexing="ij"), -1).reshape(-1, 3)
    x = np.concatenate([c + rng.uniform(-1, 1, (50, 3)) * 0.4 for c in centres])
    x = x.astype(np.float32)[rng.permutation(1000)]
    lab, k = oracle.fec(x, 3.0, 1, 1000)    # blobs span < 1.4 m, 10 m apart
    assert k == 20


def test_permutation_equivariance():
    xyz, d, mn, mx = synth.make_config("blobs20k")
    lab, k = oracle.fec(xyz, d, mn, mx)
    perm = np.random.default_rng(9).permutation(xyz.shape[0])
    lab2, k2 = oracle.fec(xyz[perm], d, mn, mx)
    assert k2 == k
    # same partition: relate clusters through the permutation
    a = lab[perm]
    assert np.array_equal(a < 0, lab2 < 0)
    m = a >= 0
    pairs = np.unique(np.stack([a[m], lab2[m]], 1), axis=0)
    assert pairs.shape[0] == len(np.unique(a[m])) == len(np.unique(lab2[m]))


def test_nonfinite_points_are_singletons():
    x = synth.random_cloud(300, extent=(2, 2, 2), seed=11)
    x[5] = [np.nan, 0, 0]
    x[17] = [np.inf, 1, 1]
    x[18] = [np.inf, 1, 1]
    x[40] = [0, -np.inf, 0]
    lab, k = oracle.fec(x, 0.8, 1, 300)
    for i in (5, 17, 18, 40):
        assert lab[i] == i and np.count_nonzero(lab == i) == 1
    lab, _ = oracle.fec(x, 0.8, 2, 300)
    for i in (5, 17, 18, 40):
        assert lab[i] == -1


def test_duplicates_are_joined():
    x = np.zeros((5, 3), dtype=np.float32) + np.float32(3.25)
    lab, k = oracle.fec(x, 1e-3, 1, 5)
    assert k == 1 and (lab == 0).all()


def test_empty_cloud():
    lab, k = oracle.fec(np.zeros((0, 3), np.float32), 0.5)
    assert lab.shape == (0,) and k == 0


def test_rejects_bad_arguments():
    x = synth.random_cloud(4, seed=0)
    for d in (0.0, -1.0, float("nan"), float("inf"), 1e-30):
        with pytest.raises(ValueError):
            oracle.fec(x, d)
    with pytest.raises(ValueError):
        oracle.fec(x, 0.5, 5, 2)


def test_fec_both_equals_two_single_runs():
    # one loop, two outputs: the filtered labels and count equal a filtered
    # run, the unfiltered labels and cluster count equal a run without bounds
    for seed, (mn, mx) in enumerate([(1, 10**9), (3, 40), (50, 60), (1, 1)]):
        xyz = synth.blobs_cloud(n=3000, n_blobs=6, seed=70 + seed)
        filt, k, unf, nc = oracle.fec_both(xyz, 0.4, mn, mx)
        f2, k2 = oracle.fec(xyz, 0.4, mn, mx)
        u2, n2 = oracle.fec(xyz, 0.4, 1, 2**31 - 1)
        assert np.array_equal(filt, f2) and k == k2
        assert np.array_equal(unf, u2) and nc == n2
