"""Error behaviour of the C ABI on the GPU (status codes, no output on error)."""

import ctypes

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_cluster, say

pytestmark = pytest.mark.gpu


def test_blocking_form_matches_async():
    import torch

    import oracle
    import paper_2208_07678_amd as fec
    lib = fec.raw_lib()
    xyz = synth.blobs_cloud(seed=4)
    t = torch.from_numpy(xyz).cuda()
    out = torch.full((xyz.shape[0],), 123, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    lib.fec_set_stream(None)
    k = lib.fec_cluster(ctypes.c_void_p(t.data_ptr()), xyz.shape[0], ctypes.c_float(0.5), 10,
                        20000, ctypes.c_void_p(out.data_ptr()))
    want, wk = oracle.fec(xyz, 0.5, 10, 20000)
    assert k == wk
    assert np.array_equal(out.cpu().numpy(), want)
    lib.fec_release()


def test_invalid_arguments_leave_output_untouched():
    import torch

    import paper_2208_07678_amd as fec
    x = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    out = torch.full((10,), 77, dtype=torch.int32, device="cuda")
    for d, mn, mx in ((0.0, 1, 5), (float("nan"), 1, 5), (1e-30, 1, 5), (0.5, 6, 5),
                      (float("inf"), 1, 5), (-1.0, 1, 5)):
        say("invalid", d, mn, mx)
        with pytest.raises(fec.FecError) as ei:
            fec.cluster(x, d, mn, mx, labels=out)
        assert ei.value.code == fec.FEC_EINVAL
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 77).all()


def test_range_error_for_huge_extent():
    import torch

    import paper_2208_07678_amd as fec
    x = np.array([[0, 0, 0], [3e37, 0, 0], [0, 3e37, 0], [0, 0, 3e37]], dtype=np.float32)
    t = torch.from_numpy(x).cuda()
    labels, k_out, _ = fec.cluster_async(t, 1.0, 1, 10)
    torch.cuda.synchronize()
    assert int(k_out.item()) == fec.FEC_ERANGE
    assert (labels.cpu().numpy() == -1).all()


def test_empty_and_single():
    got, k = gpu_cluster(np.zeros((0, 3), np.float32), 0.5, 1, 10)
    assert got.shape == (0,) and k == 0
    got, k = gpu_cluster(np.array([[1, 2, 3]], np.float32), 0.5, 1, 10)
    assert got.tolist() == [0] and k == 1
    got, k = gpu_cluster(np.array([[1, 2, 3]], np.float32), 0.5, 2, 10)
    assert got.tolist() == [-1] and k == 0


def test_workspace_stats_and_profile():
    import torch

    import paper_2208_07678_amd as fec
    xyz, d, mn, mx = synth.make_config("lidar120k")
    t = torch.from_numpy(xyz).cuda()
    ws = fec.new_workspace(xyz.shape[0], "cuda")
    fec.profile_reset()
    fec.profile_enable()
    fec.cluster(t, d, mn, mx, workspace=ws)
    prof = fec.profile_read()
    fec.profile_enable([])
    st = fec.workspace_stats(ws)
    say(st)
    say(prof)
    assert st["n"] == xyz.shape[0] and st["finite_points"] == xyz.shape[0]
    assert 0 < st["cells"] <= xyz.shape[0] and st["status"] == 0
    # the near shell launches only its small-table form when the cloud has
    # fewer points than the split threshold (131,072), both forms otherwise
    # (the one not meant for the table returns at once)
    assert xyz.shape[0] < 131072
    assert prof["hook_near"][1] == 1 and prof["hook_near"][0] > 0
    assert prof["hook_far"][1] == 1


def test_library_first_then_torch_in_fresh_process():
    # the binding loads its library before torch has touched the GPU (one HIP
    # runtime in the process either way)
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2208_07678_amd as fec\n"
        "print(fec.version())\n"
        "import numpy as np, torch\n"
        "x = torch.tensor([[0, 0, 0], [0.5, 0, 0], [5, 5, 5]], dtype=torch.float32).cuda()\n"
        "labels, k = fec.cluster(x, 1.0, 1, 10)\n"
        "print(labels.cpu().tolist(), k)\n" % root)
    say("fresh process")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "[0, 0, 2] 2"


def test_empty_call_writes_its_count_on_the_stream_and_captures():
    # n == 0 enqueues one kernel that writes k = 0 (no host copy, no
    # synchronisation), so even the empty call can be captured in a graph
    import torch

    import paper_2208_07678_amd as fec
    dev = torch.device("cuda:0")
    empty = torch.zeros((0, 3), dtype=torch.float32, device=dev)
    labels = torch.empty(0, dtype=torch.int32, device=dev)
    k_out = torch.full((1,), 9, dtype=torch.int32, device=dev)
    ws = fec.new_workspace(0, dev)
    fec.cluster_async(empty, 0.5, 1, 10, labels=labels, k_out=k_out, workspace=ws)
    torch.cuda.synchronize()
    assert int(k_out.item()) == 0
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fec.cluster_async(empty, 0.5, 1, 10, labels=labels, k_out=k_out, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    say("graph capture of an empty call")
    with torch.cuda.graph(graph):
        fec.cluster_async(empty, 0.5, 1, 10, labels=labels, k_out=k_out, workspace=ws)
    torch.cuda.synchronize()
    for r in range(3):
        k_out.fill_(9)
        torch.cuda.synchronize()
        say("graph replay", r)
        graph.replay()
        torch.cuda.synchronize()
        assert int(k_out.item()) == 0, r
