"""GPU: the autotuner's launch shapes give identical labels; the chosen one is cached."""

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import describe_mismatch, say

pytestmark = pytest.mark.gpu


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
        fec.set_tuning(0, 0)
