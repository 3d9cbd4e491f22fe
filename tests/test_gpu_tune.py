"""GPU: every launch configuration the autotuner may choose gives the
oracle's labels; the chosen one is cached."""

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import describe_mismatch, say

pytestmark = pytest.mark.gpu


def test_every_radix_width_and_block_size_gives_the_oracle_labels():
    # the sort's digit width and the hooking kernels' block size are
    # launch-time choices; each must reproduce the oracle's labels exactly
    # (the map prefix sorts 30+ key bits: 4 or 5 passes at 8 bits, 3 at 11)
    import torch

    import paper_2208_07678_amd as fec
    cases = [(synth.lidar_map(frames=[0, 1, 2, 3]), 0.2, 100, 5000000, "map 4 frames"),
             (synth.blobs_cloud(seed=21), 0.5, 10, 20000, "blobs20k")]
    try:
        for xyz, d, mn, mx, tag in cases:
            want, wk = oracle.fec(xyz, d, mn, mx)
            x = torch.from_numpy(xyz).to("cuda:0")
            for rb in (8, 9, 10, 11):
                for hb in (64, 128, 256):
                    say(tag, "radix bits", rb, "hook block", hb)
                    fec.set_tuning(0, 0, rb, hb)
                    labels, k = fec.cluster(x, d, mn, mx)
                    got = labels.cpu().numpy()
                    assert np.array_equal(got, want), (tag, rb, hb, describe_mismatch(got, want))
                    assert k == wk, (tag, rb, hb, k, wk)
    finally:
        fec.set_tuning(0, 0, 0, 0)


def test_autotune_shapes_agree_and_cache(tmp_path):
    import torch

    import paper_2208_07678_amd as fec
    from paper_2208_07678_amd import tune

    xyz, d, mn, mx = synth.make_config("lidar120k")
    x = torch.from_numpy(xyz).to("cuda:0")
    path = str(tmp_path / "tune.json")
    say("autotune lidar120k")
    try:
        res = tune.autotune(x, d, mn, mx, steps=2, path=path)   # raises if labels differ
        say("autotune", res)
        assert tune.lookup(tune._arch(x.device), x.shape[0], path) == tuple(res["best"])
        assert fec.get_tuning() == tuple(res["best"])
        labels, k = fec.cluster(x, d, mn, mx)
        want, wk = oracle.fec(xyz, d, mn, mx)
        got = labels.cpu().numpy()
        assert np.array_equal(got, want), describe_mismatch(got, want)
        assert k == wk
        assert tune.apply(x.shape[0], path=path) == tuple(res["best"])
    finally:
        fec.set_tuning(0, 0, 0, 0)
