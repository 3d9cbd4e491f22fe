"""Throughput of fixed-radius Euclidean clustering on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload map27m]

A step is one whole clustering call (grid build, sort, hooking, labels) on
one resident cloud: the 27,000,000-point map of 200 simulated 64-beam LiDAR
frames along a 2 km random walk, d = 0.2 m, sizes 100..5,000,000 (the
synthetic stand-in for the paper's accumulated KITTI sequence).  Inputs are
in HBM before timing starts.  Prints one JSON line.

The dominant kernel is timed live with HIP events recorded on the launch
stream by the library; its algorithmic bytes per launch over its average
duration give the roofline fraction against the 8 TB/s HBM peak.  The CPU
oracle, single-threaded, clusters the same whole map once.  The same line
carries the batched form on 64 frames (frames/s against 64 plain calls, and
graph replay) and the serving engine on the Poisson request trace (saturated
frames/s, p50/p99 latency at 400 requests/s against plain FIFO calls).
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per point of each stage: the bytes the stage must
# move at minimum, per the path's byte model (the design notes derive each).
ALG_BYTES_PER_POINT = {
    "bbox": 12.0,        # read xyz
    "keys": 12.0 + 8.0,  # read xyz, write packed key
    "sort_hist": 8.0,     # read one 8-byte packed key per pass
    "sort_scatter": 16.0,  # read + write one 8-byte packed key per pass
    "gather": 8.0 + 12.0 + 16.0 + 4.0,  # read key, read xyz, write float4 + index
    "cells": 8.0,        # the cell table: sorted keys read once, cell starts and keys written
    # hooking: every point read once (16) plus parent initialisation and
    # unions (12); the far shell visits only the cells outside the giant
    # component, so its share is scaled by work cells / cells, and so is the
    # near shell's when it runs on the sampled links' work list
    "hook_near": 28.0,
    "hook_far": 28.0,
    "final_labels": 4.0,  # write every label once (-1 pass); kept clusters' labels again
}
# Stages whose work is per cell, not per point: bytes per cell.
ALG_BYTES_PER_CELL = {
    # the sampling links: each cell's key, point range, parent and first
    # point read once (8 + 4 + 4 + 16)
    "sample": 32.0,
}


def alg_bytes_per_point(stage: str, stats: dict, n: int) -> float:
    """The byte model of `stage` per point of the cloud, for the call whose
    workspace statistics are `stats` (the work lists scale the shells)."""
    cells = max(stats.get("cells") or 1, 1)
    if stage in ALG_BYTES_PER_CELL:
        return ALG_BYTES_PER_CELL[stage] * cells / max(n, 1)
    bpp = ALG_BYTES_PER_POINT.get(stage, 16.0)
    if stage == "hook_far":
        bpp *= (stats.get("work_cells") or 0) / cells
    elif stage == "hook_near" and (stats.get("near_work_cells") or 0) > 0:
        bpp *= stats["near_work_cells"] / cells
    return bpp
# The whole path per point (survey byte model of the specified pipeline with
# 64-bit keys): the figure the path's algorithmic HBM fraction is taken on.
PATH_ALG_BYTES_PER_POINT = 260.0
# What bounds each stage in practice (the roof is HBM for all of them).
LIMITER = {
    "hook_near": "latency: chains of dependent loads and device-scope compare-and-swap",
    "hook_far": "latency: chains of dependent loads and device-scope compare-and-swap",
    "sample": "latency: dependent loads and device-scope compare-and-swap",
    "runs": "latency: dependent loads",
}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(frames: int, runs: int = 3, xyz=None):
    """The oracle, single-threaded and pinned to one core, on the first
    ``frames`` frames of the map (all 200: the whole map, ``xyz`` when given):
    median of ``runs`` runs."""
    import numpy as np  # noqa: F401

    import oracle
    import synth
    if xyz is None or frames < 200:
        xyz = synth.lidar_map(frames=list(range(frames)))
    pinned = None
    try:
        allowed = sorted(os.sched_getaffinity(0))
        pinned = allowed[0]
        os.sched_setaffinity(0, {pinned})
    except (AttributeError, OSError):
        allowed = None
    times = []
    try:
        for _ in range(runs):
            t0 = time.perf_counter()
            _, k = oracle.fec(xyz, 0.2, 100, 5000000)
            times.append(time.perf_counter() - t0)
    finally:
        if allowed is not None:
            os.sched_setaffinity(0, set(allowed))
    dt = sorted(times)[len(times) // 2]
    return {
        "value": xyz.shape[0] / dt,
        "unit": "points/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "%s (%d points), d=0.2, sizes 100..5e6; "
                  "single-threaded C++ (Alg. 1 over a kd-tree) pinned to core %s, %s %.2f s, "
                  "host %s, %d cores available" % (
                      "the whole map" if frames >= 200 else
                      "first %d of 200 frames of the map" % frames, xyz.shape[0], pinned,
                      "median of %d runs" % runs if runs > 1 else "one run", dt, _cpu_model(),
                      os.cpu_count() or 0),
        "seconds": dt,
        "clusters": k,
    }


def copy_probe(nbytes: int) -> None:
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 3}), flush=True)


def _source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in ("fec_device.hip", "fec_internal.h"):
        with open(os.path.join(ROOT, "paper_2208_07678_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic_record(workload: str):
    """The committed counter summary of `workload`, while the kernel sources
    are the ones it was taken with; None otherwise (counters are per
    workload: one cloud's bytes say nothing of another's)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("source_sha256") != _source_digest():
        return None
    return rec


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary, or None (see _traffic_record)."""
    rec = _traffic_record(workload)
    k = None if rec is None else rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def path_traffic(workload: str, passes: int):
    """Measured HBM bytes of one whole call on `workload` (every kernel, the
    sort's kernels once per pass), or None (see _traffic_record)."""
    rec = _traffic_record(workload)
    if rec is None:
        return None
    tot = 0
    for st, k in rec.get("kernels", {}).items():
        # sort stages: per working pass; the others per launch, or per call
        # where a call launches them more than once
        mult = passes if st.startswith("sort") else 1
        tot += k["hbm_bytes_per_launch"] * mult
    return tot


def bench_batch(args) -> None:
    print(json.dumps(batch_result(args)), flush=True)


def batch_result(args) -> dict:
    """Frames/s of the batched form on the 64-frame batch, beside 64 plain
    per-frame calls on the same resident frames."""
    import torch

    import paper_2208_07678_amd as fec
    import synth

    t_gen = time.perf_counter()
    frames, ds, mn, mx = synth.make_batch_config("batch64")
    t_gen = time.perf_counter() - t_gen
    nf = len(frames)
    dev = torch.device("cuda:0")
    xs = [torch.from_numpy(f).to(dev) for f in frames]
    xyz, offs = fec.pack_frames(xs)
    n = xyz.shape[0]
    print("bench: workload batch64 %d frames n=%d generated in %.1f s" % (nf, n, t_gen),
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    kdev = torch.empty(nf, dtype=torch.int32, device=dev)
    ws = fec.new_batch_workspace(n, nf, dev)
    d_t = torch.tensor(ds, dtype=torch.float32, device=dev)
    lo_t = torch.full((nf,), mn, dtype=torch.int32, device=dev)
    hi_t = torch.full((nf,), mx, dtype=torch.int32, device=dev)

    def step():
        fec.cluster_batch_async(xyz, offs, d_t, lo_t, hi_t, labels=labels, k_out=kdev,
                                workspace=ws, stream=stream)

    # the same frames, one plain call each (labels into the same buffer)
    seq_ws = fec.new_workspace(max(int(t.shape[0]) for t in xs), dev)
    seq_k = torch.empty(nf, dtype=torch.int32, device=dev)
    bounds = [int(v) for v in offs.cpu().tolist()]
    seq_labels = [labels[bounds[b]:bounds[b + 1]] for b in range(nf)]

    def step_seq():
        for b in range(nf):
            fec.cluster_async(xs[b], ds[b], mn, mx, labels=seq_labels[b], k_out=seq_k[b:b + 1],
                              workspace=seq_ws, stream=stream)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    for _ in range(args.warmup):
        step_seq()
    torch.cuda.synchronize()
    ks_seq = seq_k.cpu().tolist()
    labels_seq = labels.clone()
    seq_ms = timed(step_seq, args.steps)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ks = kdev.cpu().tolist()
    if min(ks) < 0:
        raise SystemExit("bench: device status %s" % ks)
    if ks != ks_seq or not torch.equal(labels, labels_seq):
        raise SystemExit("bench: batched and per-frame results differ")

    # the same call captured once in a graph and replayed (kernels only)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fec.cluster_batch_async(xyz, offs, d_t, lo_t, hi_t, labels=labels, k_out=kdev,
                                workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fec.cluster_batch_async(xyz, offs, d_t, lo_t, hi_t, labels=labels, k_out=kdev,
                                workspace=ws)
    graph.replay()
    torch.cuda.synchronize()
    if kdev.cpu().tolist() != ks or not torch.equal(labels, labels_seq):
        raise SystemExit("bench: graph replay differs from the eager call")
    graph_ms = timed(graph.replay, args.steps)

    fec.profile_reset()
    fec.profile_enable()
    step()
    torch.cuda.synchronize()
    prof_all = fec.profile_read()
    fec.profile_reset()
    dominant = max(prof_all, key=lambda s: prof_all[s][0])
    fec.profile_enable([dominant])
    ms_per_step = timed(step, args.steps)
    dom_ms, dom_launches = fec.profile_read()[dominant]
    fec.profile_enable([])
    # per working launch (see the map bench: the hooking stages launch two
    # forms of which one returns at once; sort stages once per pass)
    dst = fec.workspace_stats(ws)
    work_launches = (dst.get("radix_passes") or 1) if dominant.startswith("sort") else 1
    avg_launch_ms = dom_ms / args.steps / work_launches
    bytes_per_launch = alg_bytes_per_point(dominant, dst, n) * n
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    out = {
        "metric": "frames/s clustered (64-frame batch)",
        "value": nf / (ms_per_step * 1e-3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch64", "frames": nf, "n_points": n,
                   "d_values": sorted(set(ds)), "min_size": mn, "max_size": mx,
                   "clusters_kept": int(sum(ks))},
        "sequential": {"ms_per_batch": seq_ms, "frames_per_s": nf / (seq_ms * 1e-3),
                       "speedup": seq_ms / ms_per_step},
        "graph_replay": {"ms_per_batch": graph_ms, "frames_per_s": nf / (graph_ms * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dominant,
                     "avg_launch_ms": avg_launch_ms, "alg_bytes_per_launch": bytes_per_launch},
        "cpu_baseline": None,
    }
    if args.stages:
        out["stage_ms_per_call"] = {s: round(v[0], 4) for s, v in prof_all.items()}
    return out


def bench_serve(args) -> None:
    print(json.dumps(serve_result(args)), flush=True)


def serve_result(args) -> dict:
    """The serving engine on a Poisson request stream, beside plain
    per-request FIFO calls on the same trace: latency percentiles at the
    stream's rate, and frames/s with every request available at once
    (saturated)."""
    import numpy as np
    import torch

    import paper_2208_07678_amd as fec
    import synth

    t_gen = time.perf_counter()
    frames, arrivals, frame_of, d_of = synth.serve_trace(n_requests=args.requests,
                                                         rate=args.rate, pool=args.pool)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    pool = [torch.from_numpy(f).to(dev) for f in frames]
    nreq = len(arrivals)
    sizes = np.array([pool[int(f)].shape[0] for f in frame_of])
    max_n = max(int(t.shape[0]) for t in pool)
    mn, mx = 20, 2**31 - 1
    ring_n = 1024   # label buffers in flight at most
    ring = torch.empty((ring_n, max_n), dtype=torch.int32, device=dev)
    print("bench: serve trace %d requests, pool %d frames (mean %.0f points), generated in "
          "%.1f s" % (nreq, len(pool), sizes.mean(), t_gen), file=sys.stderr, flush=True)

    def run_engine(times):
        srv = fec.Server(args.serve_budget_gb << 30, nslots=args.slots,
                         slot_frames=args.slot_frames)
        lat = np.zeros(nreq)
        ks = np.zeros(nreq, dtype=np.int64)
        i = done = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done < nreq:
            now = time.perf_counter() - t0
            moved = 0
            while i < nreq and times[i] <= now and i - done < ring_n:
                t = pool[int(frame_of[i])]
                srv.submit(t, float(d_of[i]), mn, mx, labels=ring[i % ring_n, :t.shape[0]])
                i += 1
                moved += 1
            moved += srv.pump()
            for tk, _, k, _ in srv.poll():
                lat[tk] = time.perf_counter() - t0 - times[tk]
                ks[tk] = k
                done += 1
                moved += 1
            if not moved:
                if i >= nreq or i - done >= ring_n:
                    srv.pump(wait=True)
                else:
                    # watch the batches in flight until the next arrival is
                    # due (the engine spins on their events: a completion is
                    # seen at once, not after a sleep of this loop)
                    left_us = (times[i] - (time.perf_counter() - t0)) * 1e6
                    if left_us > 5:
                        srv.pump_for(int(left_us))
        elapsed = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return lat, ks, elapsed, st

    def run_plain(times):
        ws = fec.new_workspace(max_n, dev)
        kall = torch.empty(nreq, dtype=torch.int32, device=dev)
        stream = torch.cuda.current_stream(dev)
        lat = np.zeros(nreq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nreq):
            while time.perf_counter() - t0 < times[i]:
                pass
            t = pool[int(frame_of[i])]
            fec.cluster_async(t, float(d_of[i]), mn, mx, labels=ring[i % ring_n, :t.shape[0]],
                              k_out=kall[i:i + 1], workspace=ws, stream=stream)
            stream.synchronize()
            lat[i] = time.perf_counter() - t0 - times[i]
        elapsed = time.perf_counter() - t0
        return lat, kall.cpu().numpy().astype(np.int64), elapsed

    def pct(v, q):
        return float(np.percentile(v, q) * 1e3)

    zero = np.zeros(nreq)
    run_engine(zero)  # warm-up
    s_lat, s_ks, s_el, s_st = run_engine(zero)
    p_lat0, p_ks0, p_el0 = run_plain(zero)
    if not np.array_equal(s_ks, p_ks0):
        raise SystemExit("bench: served and plain kept counts differ")
    e_lat, e_ks, e_el, e_st = run_engine(arrivals)
    p_lat, p_ks, p_el = run_plain(arrivals)
    if not (np.array_equal(e_ks, p_ks) and np.array_equal(e_ks, s_ks)):
        raise SystemExit("bench: served and plain kept counts differ")
    out = {
        "metric": "frames/s served (continuous batching, saturated) with p50/p99 latency at "
                  "%g requests/s" % args.rate,
        "value": nreq / s_el,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": nreq,
        "warmup": 1,
        "ms_per_step": s_el * 1e3 / nreq,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serve", "requests": nreq, "rate_per_s": args.rate,
                   "pool_frames": len(pool), "mean_points": float(sizes.mean()),
                   "d_values": sorted(set(float(v) for v in d_of)), "min_size": mn,
                   "max_size": mx, "slots": args.slots, "slot_frames": args.slot_frames,
                   "slot_points": s_st["slot_points"]},
        "saturated": {"served_frames_per_s": nreq / s_el, "plain_frames_per_s": nreq / p_el0,
                      "speedup": p_el0 / s_el, "batches": s_st["batches"],
                      "max_batch_frames": s_st["max_batch_frames"],
                      "max_in_flight": s_st["max_in_flight"]},
        "poisson": {"served": {"frames_per_s": nreq / e_el, "p50_ms": pct(e_lat, 50),
                               "p99_ms": pct(e_lat, 99), "batches": e_st["batches"],
                               "max_batch_frames": e_st["max_batch_frames"],
                               "max_in_flight": e_st["max_in_flight"]},
                    "plain_fifo": {"frames_per_s": nreq / p_el, "p50_ms": pct(p_lat, 50),
                                   "p99_ms": pct(p_lat, 99)}},
        "roofline": None,
        "cpu_baseline": None,
    }
    return out


def bench_sweep(args) -> None:
    """The paper's synthetic sweeps (voxel clusters): time per call and AP of
    Eq. (2) against the generator's ground truth for every configuration, the
    oracle timed beside it where the cloud has at most 400,000 points (one
    JSON line)."""
    import numpy as np
    import torch

    import paper_2208_07678_amd as fec
    import synth
    from paper_2208_07678_amd.metrics import average_precision

    dev = torch.device("cuda:0")
    d = synth.SWEEP_D
    rows = []
    for exp, nc, m, sub in synth.SWEEPS:
        xyz, gt = synth.voxel_clusters(nc, m, subclusters=sub, seed=7)
        n = xyz.shape[0]
        x = torch.from_numpy(xyz).to(dev)
        labels = torch.empty(n, dtype=torch.int32, device=dev)
        kdev = torch.empty(1, dtype=torch.int32, device=dev)
        ws = fec.new_workspace(n, dev)
        stream = torch.cuda.current_stream(dev)
        for _ in range(2):
            fec.cluster_async(x, d, 1, n, labels=labels, k_out=kdev, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fec.cluster_async(x, d, 1, n, labels=labels, k_out=kdev, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        lab = labels.cpu().numpy()
        row = {"experiment": exp, "clusters": nc, "density": m, "subclusters": sub, "n": n,
               "gpu_ms": ms, "points_per_s": n / (ms * 1e-3), "kept": int(kdev.item()),
               "ap": average_precision(lab, gt)}
        if args.cpu_frames > 0 and n <= 400000 and exp.startswith(("E2", "E3")):
            import oracle
            t0 = time.perf_counter()
            want, _ = oracle.fec(xyz, d, 1, n)
            row["oracle_s"] = time.perf_counter() - t0
            row["oracle_equal"] = bool(np.array_equal(want, lab))
        rows.append(row)
        print("bench: %s clusters=%d density=%d sub=%d n=%d %.3f ms AP %.4f" % (
            exp, nc, m, sub, n, ms, row["ap"]), file=sys.stderr, flush=True)
    big = max(rows, key=lambda r: r["n"])
    out = {
        "metric": "points/s on the synthetic voxel-cluster sweeps (largest configuration)",
        "value": big["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 2,
        "ms_per_step": big["gpu_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sweep", "d": d, "voxel": 1.0, "configs": len(rows)},
        "sweep": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_scale(args) -> None:
    """Single-cloud calls on growing prefixes of the map (1 to 200 frames):
    time per call and points/s, from the latency-bound to the throughput-bound
    regime (one JSON line)."""
    import numpy as np
    import torch

    import paper_2208_07678_amd as fec
    import synth

    xyz_all, d, mn, mx = synth.make_config("map27m")
    per = xyz_all.shape[0] // 200
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    rows = []
    for frames in (1, 2, 5, 10, 20, 50, 100, 200):
        n = frames * per
        x = torch.from_numpy(np.ascontiguousarray(xyz_all[:n])).to(dev)
        labels = torch.empty(n, dtype=torch.int32, device=dev)
        kdev = torch.empty(1, dtype=torch.int32, device=dev)
        ws = fec.new_workspace(n, dev)
        for _ in range(2):
            fec.cluster_async(x, d, mn, mx, labels=labels, k_out=kdev, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fec.cluster_async(x, d, mn, mx, labels=labels, k_out=kdev, workspace=ws, stream=stream)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        rows.append({"frames": frames, "n": n, "ms_median": ms, "points_per_s": n / (ms * 1e-3),
                     "kept": int(kdev.item())})
        print("bench: %d frames n=%d %.3f ms" % (frames, n, ms), file=sys.stderr, flush=True)
        del x, labels, ws
    big = rows[-1]
    out = {
        "metric": "points/s clustered on map prefixes (largest = the whole map)",
        "value": big["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 2,
        "ms_per_step": big["ms_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "scale", "d": d, "min_size": mn, "max_size": mx},
        "scale": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="map27m",
                    choices=["map27m", "lidar120k", "blobs20k", "batch64", "serve", "sweep",
                             "scale"])
    ap.add_argument("--requests", type=int, default=10000, help="serve: requests in the trace")
    ap.add_argument("--rate", type=float, default=400.0, help="serve: Poisson arrivals per s")
    ap.add_argument("--pool", type=int, default=512, help="serve: distinct frames in the pool")
    ap.add_argument("--slots", type=int, default=2, help="serve: batch slots")
    ap.add_argument("--slot-frames", type=int, default=64, help="serve: requests per batch")
    ap.add_argument("--serve-budget-gb", type=int, default=16, help="serve: HBM budget")
    ap.add_argument("--cpu-frames", type=int, default=200,
                    help="map frames in the CPU-baseline sample (200 = the whole map, one run; "
                         "0 = skip)")
    ap.add_argument("--extras", type=int, default=1,
                    help="map27m: also run the batch64 and serve workloads into the same line "
                         "(0 = map only)")
    ap.add_argument("--stages", action="store_true", help="also print a per-stage breakdown")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shape with the autotuner before timing")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES, three times (the "
                         "known-size reference for scaling HBM byte counters), then exit")
    args = ap.parse_args()
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py: the clustering runs on one GPU; --gpus %d is not supported "
              "(splitting the map into slabs over several GPUs is described, not implemented)"
              % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "scale":
        bench_scale(args)
        return

    import numpy as np  # noqa: F401
    import synth

    t_gen = time.perf_counter()
    xyz, d, mn, mx = synth.make_config(args.workload)
    t_gen = time.perf_counter() - t_gen
    print("bench: workload %s n=%d generated in %.1f s" % (args.workload, xyz.shape[0], t_gen),
          file=sys.stderr, flush=True)

    import torch

    import paper_2208_07678_amd as fec

    dev = torch.device("cuda:0")
    x = torch.from_numpy(xyz).to(dev)
    n = x.shape[0]
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    kdev = torch.empty(1, dtype=torch.int32, device=dev)
    ws = fec.new_workspace(n, dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        fec.cluster_async(x, d, mn, mx, labels=labels, k_out=kdev, workspace=ws, stream=stream)

    tuned = None
    if args.autotune:
        from paper_2208_07678_amd import tune
        tuned = tune.autotune(x, d, mn, mx, steps=3)
        print("bench: autotune %s" % json.dumps(tuned), file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    k = int(kdev.item())
    if k < 0:
        raise SystemExit("bench: device status %d" % k)

    # one profiled call with every stage timed, to find the dominant kernel
    fec.profile_reset()
    fec.profile_enable()
    step()
    torch.cuda.synchronize()
    prof_all = fec.profile_read()
    fec.profile_reset()
    per_launch = {s: (ms / c if c else 0.0, ms, c) for s, (ms, c) in prof_all.items()}
    dominant = max(prof_all, key=lambda s: prof_all[s][0])
    stats = fec.workspace_stats(ws)

    # timed region: only the dominant stage carries events
    fec.profile_enable([dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_ms, dom_launches = fec.profile_read()[dominant]
    fec.profile_enable([])
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3)

    # per-call times (events on the stream, outside the timed region), and
    # the blocking form's wall time
    import numpy as np
    per_call = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step()
        e1.record(stream)
        e1.synchronize()
        per_call.append(e0.elapsed_time(e1))
    blocking = []
    for _ in range(3):
        b0 = time.perf_counter()
        fec.cluster(x, d, mn, mx, workspace=ws, labels=labels)
        blocking.append((time.perf_counter() - b0) * 1e3)
    call_ms = {"median": float(np.median(per_call)), "p99": float(np.percentile(per_call, 99)),
               "blocking_median": float(np.median(blocking))}
    # whole path: the algorithmic fraction (path byte model over the call
    # time) and, while the committed counter summary matches the sources,
    # the measured HBM bytes of one call over the call's median event time
    # (the stage events of the profiled call add their own gaps, so their
    # sum is reported only as a breakdown)
    kernel_ms = sum(v[0] for v in prof_all.values())
    tb = path_traffic(args.workload, stats.get("radix_passes") or 0)
    call_s = call_ms["median"] * 1e-3
    path = {"alg_bytes_per_point": PATH_ALG_BYTES_PER_POINT,
            "alg_GBps": PATH_ALG_BYTES_PER_POINT * n / (ms_per_step * 1e-3) / 1e9,
            "alg_frac": PATH_ALG_BYTES_PER_POINT * n / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "hbm_bytes": tb,
            "hbm_GBps": None if tb is None else tb / call_s / 1e9,
            "frac": None if tb is None else tb / call_s / 1e9 / HBM_PEAK_GBS,
            "stage_event_ms_sum": kernel_ms}

    # The stage's time per call covers all its launches: the sort stages run
    # once per radix pass (passes beyond the key's width return at once), the
    # two hooking stages on clouds of 131,072 points or more launch a
    # large-table and a small-table form of which one returns at once.  Per working launch: the stage time per call over
    # the working launches.
    passes = stats.get("radix_passes") or 0
    work_launches = passes if dominant.startswith("sort") else 1
    avg_launch_ms = dom_ms / args.steps / max(work_launches, 1)
    # stages without a per-point byte model are reported against HBM with the
    # bytes of their cells' points read once (a lower bound)
    bpp = alg_bytes_per_point(dominant, stats, n)
    bytes_per_launch = bpp * n
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload, dominant),
                "kernel": dominant, "limiter": LIMITER.get(dominant, "hbm bandwidth"),
                "avg_launch_ms": avg_launch_ms,
                "launches_per_step": dom_launches / args.steps,
                "working_launches_per_step": work_launches,
                "alg_bytes_per_point": bpp, "alg_bytes_per_launch": bytes_per_launch}

    extras = {}
    if args.extras and args.workload == "map27m":
        del x, labels, ws
        torch.cuda.empty_cache()
        b = batch_result(args)
        extras["batch64"] = {"frames_per_s": b["value"], "ms_per_batch": b["ms_per_step"],
                             "frames": b["config"]["frames"], "n_points": b["config"]["n_points"],
                             "plain_calls": b["sequential"], "graph_replay": b["graph_replay"],
                             "dominant_kernel": b["roofline"]["kernel"]}
        sv = serve_result(args)
        extras["serve"] = {"config": sv["config"], "saturated": sv["saturated"],
                           "poisson": sv["poisson"]}

    cpu = None
    if args.cpu_frames > 0 and args.workload == "map27m":
        print("bench: CPU oracle on %d frames ..." % args.cpu_frames, file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.cpu_frames, runs=1 if args.cpu_frames >= 200 else 3, xyz=xyz)

    out = {
        "metric": "points/s clustered (27M-pt map, % HBM peak)",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_points": n, "d": d, "min_size": mn,
                   "max_size": mx, "clusters_kept": k, "cells": stats.get("cells"),
                   "max_points_per_cell": stats.get("max_points_per_cell"),
                   "mean_points_per_cell": n / max(stats.get("cells") or 1, 1),
                   "radix_passes": stats.get("radix_passes"),
                   "work_cells": stats.get("work_cells"),
                   "near_work_cells": stats.get("near_work_cells"),
                   "launch_config": dict(zip(("cell_blocks", "stream_blocks", "radix_bits", "hook_block", "near_sampling"), fec.get_tuning())),
                   "autotuned": tuned is not None},
        "roofline": roofline,
        "call_ms": call_ms,
        "path": path,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    if args.stages:
        out["stage_ms_per_call"] = {s: round(v[1], 4) for s, v in per_launch.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
