"""GPU parity on the synthetic voxel-cluster sweeps (labels equal the oracle's)."""

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import describe_mismatch, gpu_cluster, say
from paper_2208_07678_amd.metrics import average_precision

pytestmark = pytest.mark.gpu

CASES = [("E1", 100, 10, 0), ("E1", 700, 100, 0), ("E1", 100, 500, 0), ("E2", 400, 200, 0),
         ("E3", 300, 200, 1), ("E3", 300, 200, 8), ("E3", 200, 200, 16)]


@pytest.mark.parametrize("exp,nc,m,sub", CASES)
def test_sweep_case_matches_oracle(exp, nc, m, sub):
    x, gt = synth.voxel_clusters(nc, m, subclusters=sub, seed=3)
    say("sweep", exp, nc, m, sub, "n=%d" % x.shape[0])
    got, k = gpu_cluster(x, synth.SWEEP_D, 1, x.shape[0])
    want, wk = oracle.fec(x, synth.SWEEP_D, 1, x.shape[0])
    assert np.array_equal(got, want), describe_mismatch(got, want)
    assert k == wk
    ap = average_precision(got, gt)
    if sub == 0:
        assert ap == 1.0 and k == nc
    else:
        assert ap > 0.9
