"""GPU parity of the tile hooking mode (on-chip tiles of columns with links
between them): labels equal the CPU oracle's, bit for bit."""

import numpy as np
import pytest

import goldens
import oracle
import synth
from gpu_helpers import describe_mismatch, gpu_cluster, say

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def tile_mode():
    import paper_2208_07678_amd as fec
    prev = fec.set_hooking(fec.HOOK_TILES)
    yield
    fec.set_hooking(prev)


def _check(xyz, d, mn, mx, tag):
    say("tiles case", tag, "n=%d d=%g min=%d max=%d" % (xyz.shape[0], d, mn, mx))
    got, k = gpu_cluster(xyz, d, mn, mx)
    want, wk = oracle.fec(xyz, d, mn, mx)
    assert np.array_equal(got, want), "%s: %s" % (tag, describe_mismatch(got, want))
    assert k == wk, "%s: k gpu %d oracle %d" % (tag, k, wk)


def test_tiles_golden_fixtures():
    for name, xyz, d, mn, mx, k, labels in goldens.all_cases():
        _check(xyz, d, mn, mx, name)


def test_tiles_small_clouds():
    rng = np.random.default_rng(77)
    for i in range(60):
        n = int(rng.integers(1, 3000))
        ext = rng.uniform(0.5, 20.0, size=3)
        if i % 5 == 0:
            ext[2] = 0.0
        x = synth.random_cloud(n, extent=tuple(ext), seed=1000 + i)
        d = float(rng.uniform(0.05, 1.5))
        _check(x, d, 1, n, "small %d" % i)


def test_tiles_workloads():
    for name in ("blobs20k", "lidar120k"):
        xyz, d, mn, mx = synth.make_config(name)
        _check(xyz, d, mn, mx, name)
        _check(xyz, d, 1, xyz.shape[0], name + " unfiltered")


def test_tiles_map_prefix():
    xyz = synth.lidar_map(frames=list(range(6)))
    _check(xyz, 0.2, 100, 5000000, "map 6 frames")


def test_tiles_dense_patches_all_tiers():
    import torch

    import paper_2208_07678_amd as fec
    a = synth.blob_lattice(extent=(6.0, 6.0), spacing=0.235, pts_per_blob=34, layers=1, seed=21)
    b = synth.blob_lattice(extent=(2.0, 5.0), spacing=0.235, pts_per_blob=40, layers=3, seed=22,
                           origin=(8.0, 0.0, 0.0))
    c = synth.random_cloud(5000, extent=(12.0, 8.0, 1.0), seed=23, offset=(-1.0, -1.0, -0.2))
    x = np.concatenate([a, b, c])
    x = x[np.random.default_rng(24).permutation(x.shape[0])]
    _check(x, 0.2, 1, x.shape[0], "dense patches")
    _check(x, 0.2, 31, 200, "dense patches, filtered")
    t = torch.from_numpy(x).cuda()
    ws = fec.new_workspace(x.shape[0], "cuda:0")
    fec.cluster(t, 0.2, 1, x.shape[0], workspace=ws)
    st = fec.workspace_stats(ws)
    say(st)
    assert st["tiles"] > 0 and st["subtiles"] > 0 and st["cell_pass_subtiles"] > 0
    assert st["tile_edges"] > 0


def test_tiles_flat_and_line():
    x = synth.random_cloud(30000, extent=(30.0, 30.0, 0.0), seed=14)
    _check(x, 0.2, 1, 30000, "flat plane z=0")
    y = synth.chain_cloud(500, 0.3, axis=1)
    _check(y, 0.35, 1, 500, "line along y")
    z = synth.chain_cloud(500, 0.3, axis=0)
    _check(z, 0.35, 1, 500, "line along x")


def test_tiles_workspace_reuse():
    import paper_2208_07678_amd as fec
    big = synth.random_cloud(50000, extent=(20, 20, 5), seed=3)
    ws = fec.new_workspace(50000, "cuda:0")
    for n in (50000, 1000, 37, 50000, 20000):
        x = big[:n]
        say("tiles reuse n", n)
        got, k = gpu_cluster(x, 0.3, 1, n, workspace=ws)
        want, wk = oracle.fec(x, 0.3, 1, n)
        assert np.array_equal(got, want) and k == wk
