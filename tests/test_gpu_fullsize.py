"""GPU parity at the full 27,000,000-point map, in the configuration bench.py
times (same call, same workspace reuse): the oracle cannot cluster the whole
map in a test's time, so the labels are checked by properties that hold at
any size and by sampled exact comparisons with the oracle.

* partition and minimality of the unfiltered labelling;
* filter exactness (filtered == unfiltered with out-of-range sizes masked)
  and the kept count;
* closure on 20,000 sampled points: every neighbour within d of a sampled
  point carries its label (oracle kd-tree, exact binary32 predicate);
* exact components for 300 sampled points of clusters of at most 50,000
  points: the oracle's breadth-first component has the GPU cluster's size
  and smallest index;
* the same call repeated is bitwise identical.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import say
from oracle import invariants

pytestmark = pytest.mark.gpu


def test_map27m_full_size_sampled():
    import torch

    import paper_2208_07678_amd as fec
    xyz, d, mn, mx = synth.make_config("map27m")
    n = xyz.shape[0]
    say("map27m generated, n =", n)
    t = torch.from_numpy(xyz).cuda()
    ws = fec.new_workspace(n, t.device)
    unf_t, ku = fec.cluster(t, d, 1, n, workspace=ws)
    filt_t, kf = fec.cluster(t, d, mn, mx, workspace=ws)
    again_t, kf2 = fec.cluster(t, d, mn, mx, workspace=ws)
    torch.cuda.synchronize()
    unf, filt, again = unf_t.cpu().numpy(), filt_t.cpu().numpy(), again_t.cpu().numpy()
    say("gpu done: components", ku, "kept", kf)
    assert np.array_equal(filt, again) and kf == kf2
    assert invariants.partition_problems(unf) == []
    assert (unf >= 0).all() and ku == np.unique(unf).size
    assert invariants.filter_problems(filt, unf, mn, mx) == []
    assert invariants.count_kept(filt) == kf
    say("building the oracle index")
    idx = oracle.Index(xyz, d)
    rng = np.random.default_rng(2027)
    sample = rng.choice(n, 20000, replace=False)
    assert invariants.closure_problems(idx, unf, sample) == []
    sizes = np.bincount(unf, minlength=n)
    small = np.nonzero(sizes[unf] <= 50000)[0]
    seeds = rng.choice(small, 300, replace=False)
    for s in seeds:
        c, m = idx.component(int(s), 50000)
        assert (c, m) == (int(sizes[unf[s]]), int(unf[s])), "seed %d" % s
    # the giant ground component: its sampled members agree on one label
    giant = int(np.argmax(sizes))
    members = np.nonzero(unf == giant)[0]
    say("largest cluster", giant, "size", members.size)
    assert members.size > mx  # the max filter removes it (the map's ground)
    assert (filt[members] == -1).all()
