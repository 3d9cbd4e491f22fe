"""GPU parity: labels of the HIP path equal the CPU oracle's, bit for bit.

Every case runs through the C ABI (fec_cluster_async via the ctypes
binding) on cuda:0 and is compared element by element with oracle.fec on
the same seeded input.  Integer labels: the bar is exact equality.
"""

import numpy as np
import pytest

import goldens
import oracle
import synth
from gpu_helpers import describe_mismatch, gpu_cluster, say
from oracle import invariants

pytestmark = pytest.mark.gpu


def _check(xyz, d, mn, mx, tag):
    say("case", tag, "n=%d d=%g min=%d max=%d" % (xyz.shape[0], d, mn, mx))
    got, k = gpu_cluster(xyz, d, mn, mx)
    want, wk = oracle.fec(xyz, d, mn, mx)
    assert np.array_equal(got, want), "%s: %s" % (tag, describe_mismatch(got, want))
    assert k == wk, "%s: k gpu %d oracle %d" % (tag, k, wk)
    return got, k


def test_golden_fixtures():
    for name, xyz, d, mn, mx, k, labels in goldens.all_cases():
        say("fixture", name)
        got, gk = gpu_cluster(xyz, d, mn, mx)
        assert np.array_equal(got, labels), (name, got, labels)
        assert gk == k


def _small(seed):
    rng = np.random.default_rng(seed)
    kind = seed % 6
    n = int(rng.integers(1, 3000))
    if kind == 0:
        x = synth.random_cloud(n, extent=(6, 6, 2), seed=seed)
        d = float(rng.uniform(0.1, 0.8))
    elif kind == 1:
        c = rng.uniform(0, 20, size=(int(rng.integers(1, 12)), 3))
        x = (c[rng.integers(0, c.shape[0], n)] + rng.normal(0, 0.5, (n, 3))).astype(np.float32)
        d = float(rng.uniform(0.1, 0.6))
    elif kind == 2:
        d = float(rng.choice([0.5, 0.35, 0.2, 1.0]))
        x = synth.near_threshold_cloud(max(1, n // 2), d, seed=seed, spread=4.0)
    elif kind == 3:
        x = synth.random_cloud(n, extent=(30, 30, 0.0), seed=seed, offset=(-1800, 900, -3))
        d = float(rng.uniform(0.2, 1.5))
    elif kind == 4:
        x = synth.random_cloud(n, extent=(2, 2, 2), seed=seed)
        bad = rng.random(n) < 0.1
        vals = np.array([np.nan, np.inf, -np.inf], dtype=np.float32)
        x[bad, rng.integers(0, 3)] = vals[rng.integers(0, 3, int(bad.sum()))]
        d = float(rng.uniform(0.05, 0.4))
    else:
        d = float(rng.uniform(0.1, 0.5))
        x = synth.chain_cloud(n, d * float(rng.uniform(0.7, 1.3)), axis=int(rng.integers(0, 3)))
        x = x[rng.permutation(n)]
    mn = int(rng.integers(0, 5))
    mx = int(rng.integers(max(1, mn), n + 3))
    return x, d, mn, max(mn, mx)


def test_many_small_clouds():
    for seed in range(300):
        x, d, mn, mx = _small(seed)
        _check(x, d, mn, mx, "small seed %d" % seed)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 4095, 4096, 4097, 8191, 12289])
def test_ragged_sizes(n):
    x = synth.random_cloud(n, extent=(8, 8, 8), seed=n)
    _check(x, 0.45, 1, n, "ragged %d" % n)


def test_blobs20k():
    xyz, d, mn, mx = synth.make_config("blobs20k")
    _check(xyz, d, mn, mx, "blobs20k")
    _check(xyz, d, 1, xyz.shape[0], "blobs20k unfiltered")


def test_lidar120k_and_shuffled():
    xyz, d, mn, mx = synth.make_config("lidar120k")
    _check(xyz, d, mn, mx, "lidar120k")
    perm = np.random.default_rng(5).permutation(xyz.shape[0])
    _check(xyz[perm], d, mn, mx, "lidar120k shuffled")


def test_map_prefix_full_oracle():
    xyz = synth.lidar_map(frames=list(range(6)))
    _check(xyz, 0.2, 100, 5000000, "map 6 frames")


def test_degenerate_inputs():
    # all points identical: one cell, one cluster
    x = np.full((5000, 3), 7.25, dtype=np.float32)
    _check(x, 0.3, 1, 5000, "duplicates")
    _check(x, 0.3, 1, 4999, "duplicates filtered")
    # all non-finite
    y = np.full((100, 3), np.nan, dtype=np.float32)
    _check(y, 0.3, 1, 10, "all nan")
    _check(y, 0.3, 2, 10, "all nan filtered")
    # d below every distance / above the diagonal (Fig. 3 cases 2 and 1)
    z = synth.random_cloud(3000, extent=(10, 10, 10), seed=2)
    _check(z, 1e-4, 1, 3000, "tiny d")
    _check(z, 30.0, 1, 3000, "huge d")
    # points on a line (Fig. 3 case 3), both sides of the threshold
    c = synth.chain_cloud(10000, 0.25, axis=2)
    _check(c, 0.25, 1, 10000, "chain at d (strict)")
    _check(c, float(np.nextafter(np.float32(0.25), np.float32(1))), 1, 10000, "chain above d")


def test_wide_grid_pair_mode():
    # grid key + point index exceed 64 bits: keys and indices sorted as pairs
    rng = np.random.default_rng(8)
    centres = rng.uniform(0, 100, size=(500, 3))
    x = (np.repeat(centres, 10, axis=0) + rng.uniform(-3e-4, 3e-4, size=(5000, 3)))
    x = x.astype(np.float32)[rng.permutation(5000)]
    _check(x, 1e-3, 1, 5000, "wide grid, d=1e-3 over 100 m")
    _check(x, 1e-3, 10, 10, "wide grid, size filter")


def test_tall_sparse_columns_near_percolation():
    # a narrow box 20 m tall (32 x 32 columns of about 290 cells each) at
    # about 0.07 points per cell and 1.5 neighbours per point: columns
    # with long gaps, so both shells locate the cells in reach of a cell by
    # the tall-column seek rather than from the column's first cell
    x = synth.random_cloud(20000, extent=(2.2, 2.2, 20.0), seed=12)
    _check(x, 0.12, 1, 20000, "tall sparse columns")
    _check(x, 0.12, 3, 50, "tall sparse columns, filtered")


def test_dense_plane_one_cell_layer():
    # a plane of about one point per cell over 462 x 462 columns, about 9
    # neighbours per point (above the plane's percolation threshold): one
    # giant component spanning the plane with small pieces around it, which
    # exercises the giant-component bitmap and the far shell's backward
    # pairs towards it
    x = synth.random_cloud(200000, extent=(40.0, 40.0, 0.05), seed=13)
    _check(x, 0.15, 1, 200000, "dense plane")


def test_flat_plane_single_z_layer():
    # every point at z = 0 exactly: one cell layer (no z bits in the key)
    x = synth.random_cloud(30000, extent=(30.0, 30.0, 0.0), seed=14)
    assert (x[:, 2] == 0).all()
    _check(x, 0.2, 1, 30000, "flat plane z=0")
    y = synth.chain_cloud(500, 0.3, axis=1)  # a single line: one column per cell row
    _check(y, 0.35, 1, 500, "line along y")


def test_repeatable_bitwise():
    xyz, d, mn, mx = synth.make_config("lidar120k")
    first, k = gpu_cluster(xyz, d, mn, mx)
    for r in range(4):
        say("repeat", r)
        again, k2 = gpu_cluster(xyz, d, mn, mx)
        assert np.array_equal(first, again) and k == k2


def test_workspace_reuse_across_sizes():
    import torch

    import paper_2208_07678_amd as fec
    big = synth.random_cloud(50000, extent=(20, 20, 5), seed=3)
    ws = fec.new_workspace(50000, "cuda:0")
    for n in (50000, 1000, 37, 50000, 20000):
        x = big[:n]
        say("reuse n", n)
        got, k = gpu_cluster(x, 0.3, 1, n, workspace=ws)
        want, wk = oracle.fec(x, 0.3, 1, n)
        assert np.array_equal(got, want) and k == wk
    torch.cuda.synchronize()


def test_invariants_map_prefix():
    xyz = synth.lidar_map(frames=[10, 11, 12])
    got, k = gpu_cluster(xyz, 0.2, 1, xyz.shape[0])
    assert invariants.partition_problems(got) == []
    idx = oracle.Index(xyz, 0.2)
    sample = np.random.default_rng(3).choice(xyz.shape[0], 5000, replace=False)
    assert invariants.closure_problems(idx, got, sample) == []
    filt, kf = gpu_cluster(xyz, 0.2, 100, 5000000)
    assert invariants.filter_problems(filt, got, 100, 5000000) == []
    assert invariants.count_kept(filt) == kf


def test_column_index_modes():
    # each way of finding a neighbour column, checked against the oracle:
    # dense table (compact plane), hash table (sparse plane), binary search
    # (column key too wide for a hash slot)
    import torch

    import paper_2208_07678_amd as fec
    rng = np.random.default_rng(21)
    sparse = (rng.uniform(0, 400, size=(300, 3)) * np.array([1, 1, 0.01])).astype(np.float32)
    sparse = np.repeat(sparse, 20, axis=0) + rng.normal(0, 0.15, (6000, 3)).astype(np.float32)
    centres = rng.uniform(0, 100, size=(400, 3))
    wide = (np.repeat(centres, 8, axis=0) + rng.uniform(-3e-4, 3e-4, (3200, 3))).astype(np.float32)
    cases = [("compact", synth.random_cloud(20000, extent=(10, 10, 2), seed=5), 0.3, 1),
             ("sparse", sparse.astype(np.float32), 0.35, 2),
             ("wide", wide, 1e-3, 0)]
    for tag, x, d, mode in cases:
        say("column index", tag)
        ws = fec.new_workspace(x.shape[0], "cuda:0")
        got, k = gpu_cluster(x, d, 1, x.shape[0], workspace=ws)
        assert fec.workspace_stats(ws)["column_index"] == mode, tag
        want, wk = oracle.fec(x, d, 1, x.shape[0])
        assert np.array_equal(got, want), "%s: %s" % (tag, describe_mismatch(got, want))
        assert k == wk
    torch.cuda.synchronize()


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_labels_into_unaligned_buffer(offset):
    # the labels are first set to -1 with 16-byte stores when the caller's
    # buffer allows, word by word otherwise; only kept clusters are written
    # after.  A buffer at a 4-, 8- or 12-byte offset, with sentinels around
    # it that must stay untouched, and size windows that keep everything,
    # nothing, or some clusters.
    import torch

    import paper_2208_07678_amd as fec
    xyz = synth.blobs_cloud(n=5003, n_blobs=8, seed=4)
    n = xyz.shape[0]
    x = torch.from_numpy(xyz).cuda()
    for mn, mx in ((1, n), (n + 1, n + 5), (2, 600)):
        say("unaligned labels offset", offset, "window", mn, mx)
        buf = torch.full((n + 8,), 12345, dtype=torch.int32, device="cuda")
        lab = buf[offset:offset + n]
        fec.cluster_async(x, 0.5, mn, mx, labels=lab)
        torch.cuda.synchronize()
        got = buf.cpu().numpy()
        want, _ = oracle.fec(xyz, 0.5, mn, mx)
        assert np.array_equal(got[offset:offset + n], want)
        assert (got[:offset] == 12345).all() and (got[offset + n:] == 12345).all()


def _expected_passes(key_bits, rb):
    # the library's schedule: at 9-bit digits the passes after the first
    # four (36 bits) take 10 bits each; other widths are uniform
    if rb == 9 and key_bits > 36:
        return 4 + -(-(key_bits - 36) // 10)
    return -(-key_bits // rb)


def test_keys_of_many_radix_passes():
    # strips 4 km long at d = 2 mm: a 22-bit x field, for 4 to 6 radix
    # passes over about 50 tiles; 1 m across gives 42 key bits, 4 m 46 bits
    # (5 passes at 9-bit digits where uniform digits would take 6; with the
    # 18 index bits below it, the last digit reaches the word's top bit),
    # both one word per point, and 8 m 48 bits (keys and indices as pairs);
    # 20,000 clumps of 10 points each
    import paper_2208_07678_amd as fec

    rng = np.random.default_rng(21)
    ws = fec.new_workspace(200000, "cuda:0")
    try:
        for width in (1.0, 4.0, 8.0):
            centres = rng.uniform((0, 0, 0), (4000, width, width), size=(20000, 3))
            x = np.repeat(centres, 10, axis=0) + rng.uniform(-6e-4, 6e-4, size=(200000, 3))
            x = x.astype(np.float32)[rng.permutation(200000)]
            want, wk = oracle.fec(x, 2e-3, 1, 200000)
            for rb in (8, 9, 10, 11):
                fec.set_tuning(radix_bits=rb)
                say("case", "strip %g m wide, %d-bit digits" % (width, rb))
                got, k = gpu_cluster(x, 2e-3, 1, 200000, workspace=ws)
                st = fec.workspace_stats(ws)
                tag = "strip %g m, %d bits, stats %s" % (width, rb, st)
                assert np.array_equal(got, want), "%s: %s" % (tag, describe_mismatch(got, want))
                assert k == wk, tag
                assert st["key_bits"] == {1.0: 42, 4.0: 46, 8.0: 48}[width], tag
                assert st["radix_passes"] == _expected_passes(st["key_bits"], rb), tag
    finally:
        fec.set_tuning()
