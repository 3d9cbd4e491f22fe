"""Autotuner for the launch configuration of the clustering kernels.

Five knobs change how the work is laid out on the chip, never the result:

* ``cell_blocks``   -- blocks of the per-cell grid-stride kernels (near and
  far shells, compression, finalize);
* ``stream_blocks`` -- blocks of the per-point streaming kernel that clears
  the labels;
* ``radix_bits``    -- bits per radix-sort pass (8 to 11: fewer passes over
  larger per-tile tables);
* ``hook_block``    -- threads per block of the hooking kernels (64, 128,
  256);
* ``near_sampling`` -- sampled links before the near shell, which then runs
  only outside the giant component they form: 0 by cloud size (2^23 points
  or more; in a batch, the average frame's), 1 on, 2 off.

``autotune`` times candidate configurations on a representative cloud, checks
that all give the same labels, and keeps the fastest: by default a coordinate
search (each knob over its values with the others at the best so far, in the
order near_sampling, radix_bits, hook_block, cell_blocks, stream_blocks), or every
configuration of an explicit candidate list.  The choice is cached in a JSON
file keyed by GPU architecture and size bucket (log2 of the point count), and
``apply`` sets the cached configuration for a coming call.

    from paper_2208_07678_amd import tune
    best = tune.autotune(xyz, d, min_size, max_size)   # measures, caches
    tune.apply(n)                                       # later: cached choice

Cache file: ``$FEC_TUNE_CACHE``, else ``~/.cache/fec_mi355x_tune.json``.
"""

from __future__ import annotations

import json
import math
import os
import time

from . import cluster_async, get_tuning, new_workspace, set_tuning

KNOBS = ("cell_blocks", "stream_blocks", "radix_bits", "hook_block", "near_sampling")
VALUES = {
    "cell_blocks": (1024, 2048, 4096, 8192, 16384),
    "stream_blocks": (2048, 4096, 8192),
    "radix_bits": (8, 9, 10, 11),
    "hook_block": (64, 128, 256),
    "near_sampling": (1, 2),
}
SEARCH_ORDER = ("near_sampling", "radix_bits", "hook_block", "cell_blocks", "stream_blocks")
DEFAULT = (4096, 4096, 9, 256, 0)


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


def _full(cfg) -> tuple:
    """A configuration as all five knobs (missing trailing knobs: defaults)."""
    cfg = tuple(int(v) for v in cfg)
    return cfg + DEFAULT[len(cfg):]


def record(arch: str, n: int, cfg, ms: float, path: str | None = None) -> None:
    """Stores the chosen configuration for (arch, size bucket of n)."""
    path = path or cache_path()
    c = _load_cache(path)
    e = dict(zip(KNOBS, _full(cfg)))
    e.update({"ms": float(ms), "n": int(n)})
    c[_key(arch, n)] = e
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(arch: str, n: int, path: str | None = None):
    """The cached configuration (five knobs) for (arch, size bucket of n), or None."""
    e = _load_cache(path or cache_path()).get(_key(arch, n))
    if e is None:
        return None
    return tuple(int(e.get(k, d)) for k, d in zip(KNOBS, DEFAULT))


def apply(n: int, device="cuda:0", path: str | None = None) -> tuple:
    """Sets the cached configuration for n points (the defaults when none is cached)."""
    cfg = lookup(_arch(device), n, path)
    set_tuning(*(cfg or (0, 0, 0, 0, 0)))
    return get_tuning()


def _label(cfg) -> str:
    return "/".join(str(v) for v in cfg)


def autotune(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1,
             candidates=None, steps: int = 5, path: str | None = None, timer=None) -> dict:
    """Times candidate configurations on ``xyz`` (a CUDA float32 [n, 3]
    tensor), checks that all give the same labels, caches and applies the
    fastest.

    ``candidates``: explicit configurations (tuples of up to five knobs,
    missing ones at their defaults), all timed; None: the coordinate search.
    Returns {"best": five knobs, "ms": {"c/s/r/h/s": ms}}.  ``timer(fn, steps)``
    may replace the wall-clock timing (for tests).
    """
    import torch

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
    ref = [None]

    def measure(cfg):
        cfg = _full(cfg)
        if cfg in times:
            return times[cfg]
        set_tuning(*cfg)
        times[cfg] = timer(call, steps)
        torch.cuda.synchronize()
        got = labels.clone()
        if ref[0] is None:
            ref[0] = got
        elif not torch.equal(ref[0], got):
            raise RuntimeError("labels depend on the launch configuration %s" % (cfg,))
        return times[cfg]

    try:
        if candidates is not None:
            for cfg in candidates:
                measure(cfg)
            best = min(times, key=times.get)
        else:
            best = DEFAULT
            measure(best)
            for knob in SEARCH_ORDER:
                i = KNOBS.index(knob)
                for v in VALUES[knob]:
                    cfg = best[:i] + (v,) + best[i + 1:]
                    measure(cfg)
                best = min((c for c in times
                            if all(c[j] == best[j] for j in range(len(KNOBS)) if j != i)),
                           key=times.get)
    finally:
        set_tuning(*saved)
    record(_arch(dev), n, best, times[best], path)
    set_tuning(*best)
    return {"best": best, "ms": {_label(k): v for k, v in times.items()}}
