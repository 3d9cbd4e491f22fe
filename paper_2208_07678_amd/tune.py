"""Autotuner for the launch shape of the clustering kernels.

The per-cell kernels (near and far shells, compression, finalize) and the
per-point streaming kernels are grid-stride loops; how many blocks they are
launched with changes how work spreads over the chip's 256 CUs, not the
result.  ``autotune`` times a set of candidate shapes on a representative
cloud and keeps the fastest; the choice is cached in a JSON file keyed by
GPU architecture and size bucket (log2 of the point count), and ``apply``
sets the cached shape for a coming call.

    from paper_2208_07678_amd import tune
    best = tune.autotune(xyz, d, min_size, max_size)   # measures, caches
    tune.apply(n)                                       # later: cached shape

Cache file: ``$FEC_TUNE_CACHE``, else ``~/.cache/fec_mi355x_tune.json``.
"""

from __future__ import annotations

import json
import math
import os
import time

from . import cluster_async, get_tuning, new_workspace, set_tuning

CANDIDATES = [(c, s) for c in (1024, 2048, 4096, 8192, 16384) for s in (2048, 4096, 8192)]


def cache_path() -> str:
    return os.environ.get("FEC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "fec_mi355x_tune.json"))


def bucket(n: int) -> int:
    return max(0, int(math.log2(max(int(n), 1))))


def _arch(device) -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _key(arch: str, n: int) -> str:
    return "%s/%d" % (arch, bucket(n))


def record(arch: str, n: int, shape, ms: float, path: str | None = None) -> None:
    """Stores the chosen shape for (arch, size bucket of n)."""
    path = path or cache_path()
    c = _load_cache(path)
    c[_key(arch, n)] = {"cell_blocks": int(shape[0]), "stream_blocks": int(shape[1]),
                        "ms": float(ms), "n": int(n)}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(arch: str, n: int, path: str | None = None):
    """The cached (cell_blocks, stream_blocks) for (arch, size bucket of n), or None."""
    e = _load_cache(path or cache_path()).get(_key(arch, n))
    return None if e is None else (int(e["cell_blocks"]), int(e["stream_blocks"]))


def apply(n: int, device="cuda:0", path: str | None = None) -> tuple[int, int]:
    """Sets the cached shape for n points (the defaults when none is cached)."""
    shape = lookup(_arch(device), n, path)
    if shape is None:
        set_tuning(0, 0)
    else:
        set_tuning(*shape)
    return get_tuning()


def autotune(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1,
             candidates=None, steps: int = 5, path: str | None = None, timer=None) -> dict:
    """Times every candidate shape on ``xyz`` (a CUDA float32 [n, 3] tensor),
    checks that all give the same labels, caches and applies the fastest.

    Returns {"best": (cell_blocks, stream_blocks), "ms": {shape: ms}}.
    ``timer(fn, steps)`` may replace the wall-clock timing (for tests).
    """
    import torch

    cands = list(candidates or CANDIDATES)
    n = int(xyz.shape[0])
    dev = xyz.device
    ws = new_workspace(n, dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    k_out = torch.empty(1, dtype=torch.int32, device=dev)

    def call():
        cluster_async(xyz, d, min_size, max_size, labels=labels, k_out=k_out, workspace=ws)

    def wall(fn, k):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    timer = timer or wall
    saved = get_tuning()
    times = {}
    ref = None
    try:
        for shape in cands:
            set_tuning(*shape)
            times[tuple(shape)] = timer(call, steps)
            torch.cuda.synchronize()
            got = labels.clone()
            if ref is None:
                ref = got
            elif not torch.equal(ref, got):
                raise RuntimeError("labels depend on the launch shape %s" % (shape,))
    finally:
        set_tuning(*saved)
    best = min(times, key=times.get)
    record(_arch(dev), n, best, times[best], path)
    set_tuning(*best)
    return {"best": best, "ms": {"%d/%d" % k: v for k, v in times.items()}}
