"""GPU parity of the batched form (fec_cluster_batch_async through the C ABI).

Every frame of a batch must get exactly the labels (frame-local) and kept
count that the oracle gives for that frame alone, and that the single-cloud
entry point gives for it alone.  Integer labels: exact equality.
"""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import describe_mismatch, gpu_cluster, say

pytestmark = pytest.mark.gpu

FEC_EINVAL, FEC_ERANGE = -1, -2


def _run_batch(frames, ds, mins, maxs, offsets=None):
    import torch

    import paper_2208_07678_amd as fec

    host = [np.ascontiguousarray(f, dtype=np.float32).reshape(-1, 3) for f in frames]
    allx = np.concatenate(host, 0) if host else np.zeros((0, 3), np.float32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum([h.shape[0] for h in host])]).astype(np.int64)
    xyz = torch.from_numpy(allx).to("cuda:0")
    labels, ks = fec.cluster_batch(xyz, torch.from_numpy(np.asarray(offsets, np.int64)),
                                   list(ds), list(mins), list(maxs))
    torch.cuda.synchronize()
    return labels.cpu().numpy(), ks, offsets


def _oracle_all(frames, ds, mins, maxs):
    """The oracle on every frame alone (threads: the oracle's C calls release the GIL)."""
    def one(b):
        return oracle.fec(frames[b], ds[b], mins[b], maxs[b])
    with ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(one, range(len(frames))))


def _check_batch(frames, ds, mins, maxs, tag, alone=True):
    say("batch", tag, "frames=%d n=%d" % (len(frames), sum(len(f) for f in frames)))
    got, ks, offs = _run_batch(frames, ds, mins, maxs)
    want = _oracle_all(frames, ds, mins, maxs)
    for b, (wl, wk) in enumerate(want):
        gl = got[offs[b]:offs[b + 1]]
        assert np.array_equal(gl, wl), "%s frame %d: %s" % (tag, b, describe_mismatch(gl, wl))
        assert ks[b] == wk, "%s frame %d: k batch %d oracle %d" % (tag, b, ks[b], wk)
        if alone and len(frames[b]) > 0:
            al, ak = gpu_cluster(frames[b], ds[b], mins[b], maxs[b])
            assert np.array_equal(gl, al), "%s frame %d vs alone: %s" % (
                tag, b, describe_mismatch(gl, al))
            assert ak == ks[b]
    return got, ks


def _small_frame(rng, seed):
    kind = seed % 5
    n = int(rng.integers(1, 2500))
    if kind == 0:
        x = synth.random_cloud(n, extent=(6, 6, 2), seed=seed)
        d = float(rng.uniform(0.1, 0.8))
    elif kind == 1:
        c = rng.uniform(0, 20, size=(int(rng.integers(1, 10)), 3))
        x = (c[rng.integers(0, c.shape[0], n)] + rng.normal(0, 0.5, (n, 3))).astype(np.float32)
        d = float(rng.uniform(0.1, 0.6))
    elif kind == 2:
        d = float(rng.choice([0.5, 0.35, 0.2]))
        x = synth.near_threshold_cloud(max(1, n // 2), d, seed=seed, spread=4.0)
    elif kind == 3:
        x = synth.random_cloud(n, extent=(2, 2, 2), seed=seed, offset=(-900, 300, 5))
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


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_small_batches_match_oracle_and_alone(seed):
    rng = np.random.default_rng(1000 + seed)
    nf = int(rng.integers(2, 24))
    parts = [_small_frame(rng, 50 * seed + b) for b in range(nf)]
    frames, ds, mins, maxs = (list(t) for t in zip(*parts))
    _check_batch(frames, ds, mins, maxs, "small seed %d" % seed)


def test_one_frame_batch_equals_single_call():
    x = synth.blobs_cloud(n=20000, seed=1)
    _check_batch([x], [0.5], [10], [20000], "one frame")


def test_many_tiny_frames():
    # more frames than one block of the planning kernel plans at once
    rng = np.random.default_rng(7)
    frames, ds, mins, maxs = [], [], [], []
    for b in range(700):
        n = int(rng.integers(0, 40))
        frames.append(synth.random_cloud(n, extent=(1.5, 1.5, 1.5), seed=b) if n else
                      np.zeros((0, 3), np.float32))
        ds.append(float(rng.choice([0.2, 0.35, 0.5])))
        mins.append(int(rng.integers(0, 4)))
        maxs.append(int(rng.integers(4, 50)))
    _check_batch(frames, ds, mins, maxs, "700 tiny frames", alone=False)


def test_refused_frames_do_not_disturb_others():
    base = [synth.random_cloud(500 + 100 * b, extent=(4, 4, 1), seed=b) for b in range(6)]
    far = synth.random_cloud(50, extent=(1, 1, 1), seed=9)
    far[0] = (-3e37, 0, 0)
    far[1] = (3e37, 0, 0)   # extent / cell side >= 2^31: out of range
    frames = [base[0], base[1], base[2], far, base[3], base[4], base[5], base[0]]
    ds = [0.3, float("nan"), 0.0, 0.3, -0.5, 0.3, 1e-30, 0.3]
    mins = [1, 1, 1, 1, 1, 9, 1, 1]
    maxs = [100, 100, 100, 100, 100, 5, 100, 100]   # frame 5: min > max
    say("batch refused frames")
    got, ks, offs = _run_batch(frames, ds, mins, maxs)
    expect_status = {1: FEC_EINVAL, 2: FEC_EINVAL, 3: FEC_ERANGE, 4: FEC_EINVAL, 5: FEC_EINVAL,
                     6: FEC_EINVAL}
    for b in range(len(frames)):
        gl = got[offs[b]:offs[b + 1]]
        if b in expect_status:
            assert ks[b] == expect_status[b], (b, ks[b])
            assert (gl == -1).all(), b
        else:
            wl, wk = oracle.fec(frames[b], ds[b], mins[b], maxs[b])
            assert np.array_equal(gl, wl), "frame %d: %s" % (b, describe_mismatch(gl, wl))
            assert ks[b] == wk


def test_empty_and_nonfinite_frames():
    rng = np.random.default_rng(3)
    nanf = np.full((30, 3), np.nan, np.float32)
    mixed = synth.random_cloud(300, extent=(2, 2, 2), seed=4)
    mixed[::7, 1] = np.inf
    frames = [np.zeros((0, 3), np.float32), mixed, np.zeros((0, 3), np.float32), nanf,
              synth.random_cloud(1, seed=1), np.zeros((0, 3), np.float32)]
    ds = [0.4, 0.4, 0.2, 0.3, 0.3, 0.5]
    mins = [1, 1, 1, 1, 2, 1]
    maxs = [10, 10, 10, 10, 10, 10]
    _check_batch(frames, ds, mins, maxs, "empty/non-finite")
    # singletons of non-finite points are kept when min_size <= 1
    _check_batch([nanf, mixed], [0.3, 0.3], [0, 0], [1, 1], "non-finite singletons")
    del rng


def test_all_frames_empty():
    got, ks, _ = _run_batch([np.zeros((0, 3), np.float32)] * 3, [0.3, 0.0, 0.3], [1] * 3,
                            [5] * 3)
    assert got.size == 0 and ks == [0, FEC_EINVAL, 0]


def test_offsets_not_a_partition_refuse_the_batch():
    frames = [synth.random_cloud(100, seed=b) for b in range(3)]
    for offs in ([0, 150, 100, 300], [1, 100, 200, 300], [0, 100, 200, 299]):
        say("bad offsets", offs)
        got, ks, _ = _run_batch(frames, [0.3] * 3, [1] * 3, [100] * 3, offsets=offs)
        assert ks == [FEC_EINVAL] * 3, (offs, ks)
        assert (got == -1).all()


def test_batch64_workload_matches_oracle_and_alone():
    frames, ds, mn, mx = synth.make_batch_config("batch64")
    got, ks = _check_batch(frames, ds, [mn] * len(frames), [mx] * len(frames), "batch64")
    assert sum(ks) > 0


def test_batch_is_repeatable_and_reuses_workspace():
    import torch

    import paper_2208_07678_amd as fec

    frames, ds, mn, mx = synth.make_batch_config("batch64", n_frames=12, seed=11)
    xyz, offs = fec.pack_frames([torch.from_numpy(f).to("cuda:0") for f in frames])
    ws = fec.new_batch_workspace(xyz.shape[0], len(frames), xyz.device)
    say("batch repeat")
    l1, k1 = fec.cluster_batch(xyz, offs, ds, mn, mx, workspace=ws)
    l1 = l1.cpu().numpy()
    # a smaller batch through the same workspace, then the first again
    l2, k2 = fec.cluster_batch(xyz[: int(offs[5])].contiguous(), offs[:6], ds[:5], mn, mx,
                               workspace=ws)
    assert np.array_equal(l2.cpu().numpy(), l1[: int(offs[5])]) and k2 == k1[:5]
    l3, k3 = fec.cluster_batch(xyz, offs, ds, mn, mx, workspace=ws)
    assert np.array_equal(l3.cpu().numpy(), l1) and k3 == k1


def test_batch_call_captured_in_a_graph_replays_exactly():
    # the batched call enqueues kernels only (no memset, no sync, no host
    # read), so it can be captured once and replayed on new point data of
    # the same sizes; every replay, with eager work in between, must equal
    # an eager call
    import torch

    import paper_2208_07678_amd as fec

    frames, ds, mn, mx = synth.make_batch_config("batch64", n_frames=10, seed=12)
    dev = torch.device("cuda:0")
    xyz, offs = fec.pack_frames([torch.from_numpy(f).to(dev) for f in frames])
    nf = len(frames)
    n = xyz.shape[0]
    d_t = torch.tensor(ds, dtype=torch.float32, device=dev)
    lo_t = torch.full((nf,), mn, dtype=torch.int32, device=dev)
    hi_t = torch.full((nf,), mx, dtype=torch.int32, device=dev)
    static_x = xyz.clone()
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    k_out = torch.empty(nf, dtype=torch.int32, device=dev)
    ws = fec.new_batch_workspace(n, nf, dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fec.cluster_batch_async(static_x, offs, d_t, lo_t, hi_t, labels=labels, k_out=k_out,
                                workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    say("graph capture")
    with torch.cuda.graph(graph):
        fec.cluster_batch_async(static_x, offs, d_t, lo_t, hi_t, labels=labels, k_out=k_out,
                                workspace=ws)
    torch.cuda.synchronize()
    gen = torch.Generator(device="cpu").manual_seed(5)
    for r in range(4):
        shift = (torch.rand((n, 3), generator=gen) * 0.05).to(dev)
        newx = (xyz + shift).contiguous()
        static_x.copy_(newx)
        say("graph replay", r)
        graph.replay()
        torch.cuda.synchronize()
        got, gk = labels.cpu().numpy(), k_out.cpu().tolist()
        want, wk = fec.cluster_batch(newx, offs, ds, mn, mx)
        torch.cuda.synchronize()
        assert np.array_equal(got, want.cpu().numpy()), "replay %d" % r
        assert gk == wk, (r, gk, wk)


def test_batch_with_a_wide_frame_uses_pairs_and_search():
    # one frame at d = 1 mm over 100 m: the stacked key no longer fits beside
    # the point index (pair mode) and the column key is too wide for a hash
    # slot (binary search); the other frames must not notice
    import paper_2208_07678_amd as fec
    import torch

    rng = np.random.default_rng(8)
    centres = rng.uniform(0, 100, size=(300, 3))
    wide = (np.repeat(centres, 10, axis=0) + rng.uniform(-3e-4, 3e-4, size=(3000, 3)))
    wide = wide.astype(np.float32)[rng.permutation(3000)]
    frames = [synth.blobs_cloud(n=4000, n_blobs=8, seed=5), wide,
              synth.random_cloud(2000, extent=(5, 5, 1), seed=6)]
    ds, mins, maxs = [0.4, 1e-3, 0.3], [1, 1, 2], [4000, 3000, 2000]
    _check_batch(frames, ds, mins, maxs, "wide frame")
    xyz, offs = fec.pack_frames([torch.from_numpy(f).to("cuda:0") for f in frames])
    ws = fec.new_batch_workspace(xyz.shape[0], 3, xyz.device)
    fec.cluster_batch(xyz, offs, ds, mins, maxs, workspace=ws)
    st = fec.workspace_stats(ws)
    assert st["key_bits"] + 13 > 64 and st["column_index"] == 0, st
