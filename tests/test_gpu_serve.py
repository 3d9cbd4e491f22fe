"""GPU tests of the serving engine (fec_server_* through the C ABI).

Each request's labels and count must equal the single-cloud call on that
cloud alone and the oracle's, whatever it was batched with: tolerance 0.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import describe_mismatch, gpu_cluster, say

pytestmark = pytest.mark.gpu

FEC_EINVAL, FEC_ENOMEM = -1, -3


def _requests(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 4
        if kind == 0:
            n = int(rng.integers(0, 3000))
            x = synth.random_cloud(n, extent=(5, 5, 2), seed=seed * 1000 + i)
        elif kind == 1:
            x = synth.lidar_frame(n=int(rng.integers(5000, 60000)), seed=seed * 1000 + i)
        elif kind == 2:
            n = int(rng.integers(1, 2000))
            c = rng.uniform(0, 15, size=(int(rng.integers(1, 8)), 3))
            x = (c[rng.integers(0, c.shape[0], n)] + rng.normal(0, 0.4, (n, 3))).astype(np.float32)
        else:
            x = synth.random_cloud(int(rng.integers(1, 500)), extent=(1, 1, 1), seed=i)
            x[::5, 0] = np.nan
        d = float(rng.choice([0.2, 0.35, 0.5]))
        mn = int(rng.integers(0, 30))
        mx = int(rng.integers(mn, max(mn, x.shape[0]) + 5))
        out.append((np.ascontiguousarray(x, dtype=np.float32), d, mn, max(mn, mx)))
    return out


def _server(budget_mb=256, nslots=2, frames=8):
    import paper_2208_07678_amd as fec
    return fec.Server(budget_mb << 20, nslots=nslots, slot_frames=frames)


def test_mix_equals_alone_and_oracle():
    import torch
    reqs = _requests(1, 40)
    srv = _server()
    say("server slot points", srv.slot_points)
    tensors = [torch.from_numpy(x).to("cuda:0") for x, _, _, _ in reqs]
    tickets = [srv.submit(t, d, mn, mx) for t, (_, d, mn, mx) in zip(tensors, reqs)]
    done = {t: (lab, k) for t, lab, k, _ in srv.drain()}
    st = srv.stats()
    say("server stats", st)
    assert st["completed"] == len(reqs) and st["batches"] < len(reqs)
    for i, (x, d, mn, mx) in enumerate(reqs):
        lab, k = done[tickets[i]]
        got = lab.cpu().numpy()
        alone, ka = gpu_cluster(x, d, mn, mx) if x.shape[0] else (np.zeros(0, np.int32), 0)
        assert np.array_equal(got, alone), "request %d: %s" % (i, describe_mismatch(got, alone))
        assert k == ka, (i, k, ka)
        want, wk = oracle.fec(x, d, mn, mx)
        assert np.array_equal(got, want), "request %d: %s" % (i, describe_mismatch(got, want))
        assert k == wk, (i, k, wk)
    srv.close()


def test_batch_refused_as_a_whole_reruns_each_request_alone():
    # Three 2-point requests, each 10^6 m long along its own axis with d = 1 mm:
    # alone each grid key has about 31 bits; stacked into one batch the key
    # needs about 93, so the batch is refused (FEC_ERANGE) as a whole.  The
    # engine re-runs each request alone, where it gets its own result.
    import torch
    reqs = []
    for ax in range(3):
        x = np.zeros((2, 3), dtype=np.float32)
        x[1, ax] = 1.0e6
        reqs.append(x)
    srv = _server(budget_mb=64, nslots=1, frames=8)
    ts = [torch.from_numpy(x).to("cuda:0") for x in reqs]
    tickets = [srv.submit(t, 1e-3, 1, 10) for t in ts]
    done = {t: (lab, k) for t, lab, k, _ in srv.drain()}
    st = srv.stats()
    say("server stats", st)
    assert st["requeued"] == 3 and st["completed"] == 3
    for i, x in enumerate(reqs):
        lab, k = done[tickets[i]]
        got = lab.cpu().numpy()
        alone, ka = gpu_cluster(x, 1e-3, 1, 10)
        want, wk = oracle.fec(x, 1e-3, 1, 10)
        assert np.array_equal(got, alone) and k == ka, (i, got, alone, k, ka)
        assert np.array_equal(got, want) and k == wk == 2, (i, got, want, k, wk)
    srv.close()


def test_arrivals_while_batches_run():
    # requests submitted while earlier batches are on the device join the
    # next free slot; several batches are in flight at once
    import torch
    frames = [synth.lidar_frame(n=40000 + 5000 * i, seed=70 + i) for i in range(24)]
    ts = [torch.from_numpy(f).to("cuda:0") for f in frames]
    srv = _server(budget_mb=512, nslots=3, frames=4)
    results = {}
    for i, t in enumerate(ts):
        srv.submit(t, 0.35, 20, 10**9)
        srv.pump()
        for tk, lab, k, _ in srv.poll():
            results[tk] = (lab, k)
    for tk, lab, k, _ in srv.drain():
        results[tk] = (lab, k)
    st = srv.stats()
    say("server stats", st)
    assert st["completed"] == 24 and st["max_in_flight"] >= 2
    for i, f in enumerate(frames):
        alone, ka = gpu_cluster(f, 0.35, 20, 10**9)
        lab, k = results[i]
        assert np.array_equal(lab.cpu().numpy(), alone) and k == ka, i
    srv.close()


def test_pump_for_retires_as_batches_finish():
    # a client that admits requests at known times waits with pump_for:
    # every request completes, with the labels of its single call
    import torch
    frames = [synth.lidar_frame(n=8000 + 3000 * i, seed=90 + i) for i in range(6)]
    ts = [torch.from_numpy(f).to("cuda:0") for f in frames]
    srv = _server(budget_mb=256, nslots=2, frames=4)
    results = {}
    for i, t in enumerate(ts):
        srv.submit(t, 0.35, 20, 10**9)
        srv.pump()
        srv.pump_for(200)
        for tk, lab, k, _ in srv.poll():
            results[tk] = (lab, k)
    for _ in range(10000):
        if len(results) == len(ts):
            break
        srv.pump_for(1000)
        for tk, lab, k, _ in srv.poll():
            results[tk] = (lab, k)
    assert len(results) == len(ts)
    for i, f in enumerate(frames):
        want, wk = oracle.fec(f, 0.35, 20, 10**9)
        lab, k = results[i]
        assert np.array_equal(lab.cpu().numpy(), want) and k == wk, i
    srv.close()


def test_admission_limits_and_argument_checks():
    import torch

    import paper_2208_07678_amd as fec
    srv = _server(budget_mb=8, nslots=1, frames=2)
    cap = srv.slot_points
    say("slot points", cap)
    assert cap > 1000
    big = torch.zeros((cap + 1, 3), dtype=torch.float32, device="cuda:0")
    with pytest.raises(fec.FecError) as e:
        srv.submit(big, 0.3)
    assert e.value.code == FEC_ENOMEM
    small = torch.from_numpy(synth.random_cloud(100, seed=3)).to("cuda:0")
    for bad in (dict(d=0.0), dict(d=float("nan")), dict(d=0.3, min_size=5, max_size=4)):
        with pytest.raises(fec.FecError) as e:
            srv.submit(small, **bad)
        assert e.value.code == FEC_EINVAL
    # a full slot: requests beyond its points wait for the next batch
    half = torch.from_numpy(synth.random_cloud(cap // 2 + 1, extent=(20, 20, 2), seed=4)).to(
        "cuda:0")
    t1 = srv.submit(half, 0.3)
    t2 = srv.submit(half, 0.3)
    t3 = srv.submit(torch.zeros((0, 3), dtype=torch.float32, device="cuda:0"), 0.3)
    done = {t: (lab, k) for t, lab, k, _ in srv.drain()}
    assert srv.stats()["batches"] >= 2
    alone, ka = gpu_cluster(half.cpu().numpy(), 0.3, 1, 2**31 - 1)
    for t in (t1, t2):
        assert np.array_equal(done[t][0].cpu().numpy(), alone) and done[t][1] == ka
    assert done[t3][1] == 0 and done[t3][0].numel() == 0
    srv.close()
