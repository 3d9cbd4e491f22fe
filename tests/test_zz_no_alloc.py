"""The no-allocation entry point (fec_cluster_noalloc, through the C ABI)
against the workspace form (fec_cluster_async) on the same inputs: labels
and counts equal, bit for bit, on two calls in a row, the second on a
smaller cloud (the static scratch array keeps the first call's contents).
"""

import ctypes

import numpy as np
import pytest

import synth
from gpu_helpers import describe_mismatch, say

pytestmark = pytest.mark.gpu


def _noalloc(lib, t, d, mn, mx, labels, k_out, stream):
    return lib.fec_cluster_noalloc(ctypes.c_void_p(t.data_ptr()), t.shape[0], ctypes.c_float(d),
                                   mn, mx, ctypes.c_void_p(labels.data_ptr()),
                                   ctypes.c_void_p(k_out.data_ptr()),
                                   ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_equals_workspace_form_two_calls():
    import torch

    import paper_2208_07678_amd as fec
    lib = fec.raw_lib()
    stream = torch.cuda.current_stream()
    cases = [
        (synth.make_config("lidar120k"), "lidar120k"),
        ((synth.blobs_cloud(n=9000, n_blobs=12, seed=31), 0.5, 10, 9000), "blobs 9k"),
    ]
    for (xyz, d, mn, mx), tag in cases:
        say("no-alloc case", tag, "n=%d" % xyz.shape[0])
        t = torch.from_numpy(xyz).cuda()
        want, wk = fec.cluster(t, d, mn, mx)
        labels = torch.full((xyz.shape[0],), 77, dtype=torch.int32, device="cuda")
        k_out = torch.full((1,), 77, dtype=torch.int32, device="cuda")
        rc = _noalloc(lib, t, d, mn, mx, labels, k_out, stream)
        assert rc == fec.FEC_OK, (tag, rc, lib.fec_last_error())
        torch.cuda.synchronize()
        got, gk = labels.cpu().numpy(), int(k_out.item())
        w = want.cpu().numpy()
        assert np.array_equal(got, w), "%s: %s" % (tag, describe_mismatch(got, w))
        assert gk == wk, (tag, gk, wk)


def test_noalloc_limits():
    import torch

    import paper_2208_07678_amd as fec
    lib = fec.raw_lib()
    stream = torch.cuda.current_stream()
    # the largest cloud it admits, then one point more (refused on the host)
    n = fec.NOALLOC_MAX_POINTS
    xyz = synth.random_cloud(n, extent=(60.0, 60.0, 3.0), seed=41)
    t = torch.from_numpy(xyz).cuda()
    say("no-alloc at its limit n=%d" % n)
    want, wk = fec.cluster(t, 0.3, 5, n)
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    k_out = torch.empty(1, dtype=torch.int32, device="cuda")
    assert _noalloc(lib, t, 0.3, 5, n, labels, k_out, stream) == fec.FEC_OK
    torch.cuda.synchronize()
    assert np.array_equal(labels.cpu().numpy(), want.cpu().numpy()) and int(k_out.item()) == wk
    big = torch.zeros((n + 1, 3), dtype=torch.float32, device="cuda")
    out = torch.full((n + 1,), 5, dtype=torch.int32, device="cuda")
    assert _noalloc(lib, big, 0.3, 1, 10, out, k_out, stream) == fec.FEC_EINVAL
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 5).all()
    # an empty cloud: k = 0, written on the stream
    empty = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    k_out.fill_(9)
    assert _noalloc(lib, empty, 0.3, 1, 10, out, k_out, stream) == fec.FEC_OK
    torch.cuda.synchronize()
    assert int(k_out.item()) == 0
