"""MI355X (gfx950) fixed-radius Euclidean clustering -- Python binding.

Thin ctypes layer over the C ABI declared in include/fec.h and implemented by
the in-tree HIP library ``libfec_hip.so`` (built by
``python -m paper_2208_07678_amd.build``).  PyTorch only provides device
memory and the current stream; every step of the clustering runs in the HIP
kernels.  There is no CPU fallback: every entry point raises when the built
library is missing, and tensors must live on the GPU.

    labels, k = paper_2208_07678_amd.cluster(xyz, d, min_size, max_size)
    labels, k = paper_2208_07678_amd.cluster_batch(xyz_all, offsets, d, min_size, max_size)

``xyz`` is a contiguous float32 CUDA tensor [n, 3]; ``labels`` is an int32
CUDA tensor [n] with the smallest point index of each kept cluster, -1 for
points of clusters whose size is outside [min_size, max_size].
"""

from __future__ import annotations

import ctypes
import os

__all__ = [
    "cluster", "cluster_async", "cluster_noalloc", "workspace_bytes", "workspace_stats",
    "FecError", "NOALLOC_MAX_POINTS",
    "cluster_batch", "cluster_batch_async", "batch_workspace_bytes", "pack_frames", "Server",
    "profile_enable", "profile_read", "profile_reset", "stage_names", "lib_path",
    "FEC_OK", "FEC_EINVAL", "FEC_ERANGE", "FEC_ENOMEM", "FEC_EDEVICE",
]

FEC_OK = 0
FEC_EINVAL = -1
FEC_ERANGE = -2
FEC_ENOMEM = -3
FEC_EDEVICE = -4
NOALLOC_MAX_POINTS = 524288  # FEC_NOALLOC_MAX_POINTS of include/fec.h

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libfec_hip.so")

_lib = None


def _load():
    """Loads the HIP library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise ImportError(
            "paper_2208_07678_amd: HIP library %s is missing; build it with "
            "'python -m paper_2208_07678_amd.build'" % lib_path)
    # torch ships its own HIP runtime under the same soname; loading it first
    # makes this library bind to that one, so the process has one runtime
    # (two would each try to own the device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(lib_path)
    i32, i64, f32, vp, u64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p,
                              ctypes.c_uint64)
    sigs = {
        "fec_cluster": ([vp, i64, f32, i32, i32, vp], i32),
        "fec_workspace_bytes": ([i64], ctypes.c_size_t),
        "fec_cluster_async": ([vp, i64, f32, i32, i32, vp, vp, vp, ctypes.c_size_t, vp], i32),
        "fec_cluster_noalloc": ([vp, i64, f32, i32, i32, vp, vp, vp], i32),
        "fec_cluster_batch_async": ([vp, i64, i32, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t,
                                     vp], i32),
        "fec_batch_workspace_bytes": ([i64, i32], ctypes.c_size_t),
        "fec_server_slot_bytes": ([i64, i32], ctypes.c_size_t),
        "fec_tuning_set": ([i32, i32, i32, i32, i32], i32),
        "fec_tuning_get": ([vp, vp, vp, vp, vp], i32),
        "fec_server_create": ([ctypes.c_size_t, i32, i32, vp], i32),
        "fec_server_slot_points": ([vp], i64),
        "fec_server_submit": ([vp, vp, i64, f32, i32, i32, vp, vp], i32),
        "fec_server_pump": ([vp, i32], i32),
        "fec_server_pump_for": ([vp, i64], i32),
        "fec_server_poll": ([vp, vp, vp, vp, i32], i32),
        "fec_server_stats": ([vp, vp, i32], i32),
        "fec_server_destroy": ([vp], None),
        "fec_set_stream": ([vp], i32),
        "fec_release": ([], None),
        "fec_last_error": ([], ctypes.c_char_p),
        "fec_version": ([], ctypes.c_char_p),
        "fec_workspace_stats": ([vp, vp, vp, i32], i32),
        "fec_profile_enable": ([u64], i32),
        "fec_profile_read": ([vp, vp, i32], i32),
        "fec_profile_reset": ([], None),
        "fec_stage_count": ([], i32),
        "fec_stage_name": ([i32], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


EXPORTED = [
    "fec_cluster", "fec_workspace_bytes", "fec_cluster_async", "fec_cluster_noalloc",
    "fec_set_stream", "fec_release",
    "fec_cluster_batch_async", "fec_batch_workspace_bytes", "fec_server_slot_bytes",
    "fec_server_create", "fec_server_slot_points", "fec_server_submit", "fec_server_pump",
    "fec_server_pump_for",
    "fec_server_poll", "fec_server_stats", "fec_server_destroy", "fec_tuning_set",
    "fec_tuning_get",
    "fec_last_error", "fec_version", "fec_workspace_stats", "fec_profile_enable",
    "fec_profile_read", "fec_profile_reset", "fec_stage_count", "fec_stage_name",
]

STATS_FIELDS = ["n", "finite_points", "cells", "columns", "key_bits", "radix_passes",
                "grid_x", "grid_y", "grid_z", "max_points_per_cell", "status",
                "work_cells", "giant_root"] + ["counter%d" % i for i in range(8)] + [
                "column_index", "near_work_cells"]


class FecError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("FEC error %d: %s" % (code, msg))
        self.code = code


def _raise(code: int):
    raise FecError(code, (_load().fec_last_error() or b"").decode())


def version() -> str:
    return _load().fec_version().decode()


def workspace_bytes(n: int) -> int:
    return int(_load().fec_workspace_bytes(int(n)))


def _torch():
    import torch
    return torch


def _check_xyz(xyz):
    torch = _torch()
    if not isinstance(xyz, torch.Tensor):
        raise TypeError("xyz must be a torch tensor on a GPU")
    if xyz.device.type != "cuda":
        raise ValueError("xyz must be on a GPU (got %s); there is no CPU path" % xyz.device)
    if xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3:
        raise ValueError("xyz must be float32 [n, 3]")
    if not xyz.is_contiguous():
        raise ValueError("xyz must be contiguous")


def new_workspace(n: int, device):
    """A device workspace (uint8 tensor) large enough for n points."""
    torch = _torch()
    nb = max(workspace_bytes(n), 256)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=device)
    return ws


def _aligned_ptr(ws) -> tuple[int, int]:
    p = ws.data_ptr()
    a = (p + 255) // 256 * 256
    return a, ws.numel() - (a - p)


def cluster_async(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1, *,
                  labels=None, k_out=None, workspace=None, stream=None):
    """Enqueues the clustering on the current (or given) stream.

    Returns (labels, k_out, workspace): labels int32 [n] and k_out int32 [1]
    are device tensors written when the stream reaches the work.
    """
    torch = _torch()
    _check_xyz(xyz)
    n = xyz.shape[0]
    dev = xyz.device
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    if k_out is None:
        k_out = torch.empty(1, dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = new_workspace(n, dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    wptr, wbytes = _aligned_ptr(workspace)
    with torch.cuda.device(dev):
        rc = _load().fec_cluster_async(ctypes.c_void_p(xyz.data_ptr()), n, float(d), int(min_size),
                                    int(max_size), ctypes.c_void_p(labels.data_ptr()),
                                    ctypes.c_void_p(k_out.data_ptr()), ctypes.c_void_p(wptr),
                                    wbytes, ctypes.c_void_p(stream.cuda_stream))
    if rc != FEC_OK:
        _raise(rc)
    return labels, k_out, workspace


def cluster(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1, *,
            workspace=None, labels=None, stream=None):
    """Clusters xyz; returns (labels int32 CUDA tensor [n], kept cluster count)."""
    labels, k_out, _ = cluster_async(xyz, d, min_size, max_size, labels=labels,
                                     workspace=workspace, stream=stream)
    k = int(k_out.item())
    if k < 0:
        raise FecError(k, "device-side status %d" % k)
    return labels, k


def cluster_noalloc(xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1, *,
                    labels, k_out, stream=None):
    """Enqueues the clustering with the library's static scratch array as its
    workspace (fec_cluster_noalloc): nothing is allocated, so ``labels``
    (int32 [n]) and ``k_out`` (int32 [1]) are the caller's device tensors.
    At most NOALLOC_MAX_POINTS points; calls that overlap on one GPU race."""
    torch = _torch()
    _check_xyz(xyz)
    n = xyz.shape[0]
    dev = xyz.device
    for name, t in (("labels", labels), ("k_out", k_out)):
        if (not isinstance(t, torch.Tensor) or t.device != dev or t.dtype != torch.int32
                or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous int32 tensor on %s" % (name, dev))
    if labels.numel() < n or k_out.numel() < 1:
        raise ValueError("labels needs %d entries and k_out one" % n)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc = _load().fec_cluster_noalloc(ctypes.c_void_p(xyz.data_ptr()), n, float(d),
                                         int(min_size), int(max_size),
                                         ctypes.c_void_p(labels.data_ptr()),
                                         ctypes.c_void_p(k_out.data_ptr()),
                                         ctypes.c_void_p(stream.cuda_stream))
    if rc != FEC_OK:
        _raise(rc)
    return labels, k_out


def set_tuning(cell_blocks: int = 0, stream_blocks: int = 0, radix_bits: int = 0,
               hook_block: int = 0, near_sampling: int = 0) -> None:
    """Launch configuration of later calls (0 = a knob's default): grid sizes
    of the per-cell and streaming kernels, radix-sort digit width, block size
    of the hooking kernels, sampling links before the near shell (0 by cloud
    size, 1 on, 2 off); see ``paper_2208_07678_amd.tune``."""
    rc = _load().fec_tuning_set(int(cell_blocks), int(stream_blocks), int(radix_bits),
                                int(hook_block), int(near_sampling))
    if rc != FEC_OK:
        _raise(rc)


def get_tuning() -> tuple[int, int, int, int, int]:
    """(cell_blocks, stream_blocks, radix_bits, hook_block, near_sampling) in force."""
    v = [ctypes.c_int32() for _ in range(5)]
    _load().fec_tuning_get(*[ctypes.byref(x) for x in v])
    return tuple(int(x.value) for x in v)


def batch_workspace_bytes(n_total: int, nframes: int) -> int:
    return int(_load().fec_batch_workspace_bytes(int(n_total), int(nframes)))


def new_batch_workspace(n_total: int, nframes: int, device):
    """A device workspace (uint8 tensor) for a batch of n_total points in nframes frames."""
    torch = _torch()
    nb = batch_workspace_bytes(n_total, nframes)
    if nb <= 0:
        raise ValueError("bad batch sizes n_total=%d nframes=%d" % (n_total, nframes))
    return torch.empty(nb + 256, dtype=torch.uint8, device=device)


def _per_frame(v, nframes: int, dtype, dev):
    """A device tensor [nframes] from a scalar, a sequence or a tensor."""
    torch = _torch()
    if isinstance(v, torch.Tensor):
        t = v.to(device=dev, dtype=dtype).reshape(-1)
    else:
        if isinstance(v, (int, float)):
            v = [v] * nframes
        t = torch.tensor(list(v), dtype=dtype, device=dev)
    if t.numel() != nframes:
        raise ValueError("per-frame argument has %d values for %d frames" % (t.numel(), nframes))
    return t.contiguous()


def pack_frames(frames):
    """Concatenates a list of float32 CUDA tensors [n_f, 3] into (xyz [sum n_f, 3], offsets).

    offsets is an int64 CUDA tensor [len(frames) + 1].
    """
    torch = _torch()
    if not frames:
        raise ValueError("no frames")
    for t in frames:
        _check_xyz(t)
    dev = frames[0].device
    sizes = [int(t.shape[0]) for t in frames]
    offs = [0]
    for k in sizes:
        offs.append(offs[-1] + k)
    xyz = torch.cat(frames, 0) if len(frames) > 1 else frames[0]
    return xyz.contiguous(), torch.tensor(offs, dtype=torch.int64, device=dev)


def cluster_batch_async(xyz, offsets, d, min_size=1, max_size=2**31 - 1, *, labels=None,
                        k_out=None, workspace=None, stream=None):
    """Enqueues the clustering of a batch of frames (see fec_cluster_batch_async).

    xyz float32 CUDA [n_total, 3]; offsets int64 [nframes + 1] (CUDA tensor, or
    a sequence copied to the device); d, min_size, max_size per frame (scalar,
    sequence or tensor).  Returns (labels int32 [n_total] frame-local,
    k_out int32 [nframes], workspace) written when the stream gets there.
    """
    torch = _torch()
    _check_xyz(xyz)
    dev = xyz.device
    n = xyz.shape[0]
    if isinstance(offsets, torch.Tensor):
        offs = offsets.to(device=dev, dtype=torch.int64).contiguous()
    else:
        offs = torch.tensor(list(offsets), dtype=torch.int64, device=dev)
    nframes = offs.numel() - 1
    if nframes < 1:
        raise ValueError("offsets needs at least two entries")
    d_t = _per_frame(d, nframes, torch.float32, dev)
    lo_t = _per_frame(min_size, nframes, torch.int32, dev)
    hi_t = _per_frame(max_size, nframes, torch.int32, dev)
    # argument tensors made here (not the caller's) must outlive the launch
    made = [t for t, src in ((offs, offsets), (d_t, d), (lo_t, min_size), (hi_t, max_size))
            if t is not src]
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=dev)
    if k_out is None:
        k_out = torch.empty(nframes, dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = new_batch_workspace(n, nframes, dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    wptr, wbytes = _aligned_ptr(workspace)
    with torch.cuda.device(dev):
        rc = _load().fec_cluster_batch_async(
            ctypes.c_void_p(xyz.data_ptr()), n, nframes, ctypes.c_void_p(offs.data_ptr()),
            ctypes.c_void_p(d_t.data_ptr()), ctypes.c_void_p(lo_t.data_ptr()),
            ctypes.c_void_p(hi_t.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
            ctypes.c_void_p(k_out.data_ptr()), ctypes.c_void_p(wptr), wbytes,
            ctypes.c_void_p(stream.cuda_stream))
    if rc != FEC_OK:
        _raise(rc)
    for t in made:
        t.record_stream(stream)
    return labels, k_out, workspace


def cluster_batch(xyz, offsets, d, min_size=1, max_size=2**31 - 1, *, workspace=None,
                  labels=None, stream=None):
    """Clusters a batch of frames; returns (frame-local labels [n_total], k per frame list).

    A frame whose arguments are refused reports its negative FEC_* status in
    the list instead of a count (its labels are -1).
    """
    labels, k_out, _ = cluster_batch_async(xyz, offsets, d, min_size, max_size, labels=labels,
                                           workspace=workspace, stream=stream)
    return labels, [int(v) for v in k_out.cpu().tolist()]


SERVER_STATS_FIELDS = ["submitted", "completed", "batches", "queued", "slots_busy",
                       "max_batch_frames", "max_in_flight", "slot_points", "slot_bytes",
                       "requeued"]


class Server:
    """Continuous-batching engine over the C ABI (fec_server_*).

    ``submit`` queues a CUDA float32 [n, 3] cloud (kept referenced until its
    request completes) and returns its ticket; ``pump`` retires finished
    batches and launches queued requests into free slots; ``poll`` returns the
    completed requests as (ticket, labels tensor, k, latency ms).
    """

    def __init__(self, hbm_budget: int, nslots: int = 2, slot_frames: int = 64):
        lib = _load()
        h = ctypes.c_void_p()
        rc = lib.fec_server_create(int(hbm_budget), int(nslots), int(slot_frames),
                                   ctypes.byref(h))
        if rc != FEC_OK:
            raise FecError(rc, "fec_server_create failed")
        self._h = h
        self._live = {}   # ticket -> (xyz, labels) kept alive until done
        self._cap = 4096  # poll buffers, allocated once
        self._tk = (ctypes.c_int64 * self._cap)()
        self._kk = (ctypes.c_int32 * self._cap)()
        self._lat = (ctypes.c_double * self._cap)()

    @property
    def slot_points(self) -> int:
        return int(_load().fec_server_slot_points(self._h))

    def submit(self, xyz, d: float, min_size: int = 1, max_size: int = 2**31 - 1,
               labels=None) -> int:
        torch = _torch()
        _check_xyz(xyz)
        n = xyz.shape[0]
        if labels is None:
            labels = torch.empty(n, dtype=torch.int32, device=xyz.device)
        t = ctypes.c_int64()
        rc = _load().fec_server_submit(self._h, ctypes.c_void_p(xyz.data_ptr()), n, float(d),
                                       int(min_size), int(max_size),
                                       ctypes.c_void_p(labels.data_ptr()), ctypes.byref(t))
        if rc != FEC_OK:
            raise FecError(rc, "submit refused (n=%d, d=%g, min=%d, max=%d)"
                           % (n, d, min_size, max_size))
        self._live[t.value] = (xyz, labels)
        return t.value

    def pump(self, wait: bool = False) -> int:
        rc = _load().fec_server_pump(self._h, 1 if wait else 0)
        if rc < 0:
            raise FecError(rc, "fec_server_pump failed")
        return rc

    def pump_for(self, max_wait_us: int) -> int:
        """pump(); when nothing completed, watch the batches in flight for up
        to max_wait_us microseconds and retire the first that finishes."""
        rc = _load().fec_server_pump_for(self._h, max(0, int(max_wait_us)))
        if rc < 0:
            raise FecError(rc, "fec_server_pump_for failed")
        return rc

    def poll(self, max_items: int = 4096):
        max_items = min(int(max_items), self._cap)
        tk, kk, lat = self._tk, self._kk, self._lat
        c = _load().fec_server_poll(self._h, tk, kk, lat, max_items)
        out = []
        for i in range(c):
            _, labels = self._live.pop(int(tk[i]))
            out.append((int(tk[i]), labels, int(kk[i]), float(lat[i])))
        return out

    def stats(self) -> dict:
        out = (ctypes.c_int64 * len(SERVER_STATS_FIELDS))()
        c = _load().fec_server_stats(self._h, out, len(SERVER_STATS_FIELDS))
        return {k: int(out[i]) for i, k in enumerate(SERVER_STATS_FIELDS[:c])}

    def drain(self):
        """Pumps until every submitted request has completed; returns poll()."""
        done = []
        while True:
            st = self.stats()
            if st["completed"] >= st["submitted"]:
                break
            self.pump(wait=True)
            done += self.poll()
        return done + self.poll()

    def close(self):
        if self._h:
            _load().fec_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_stats(workspace, stream=None) -> dict:
    """Diagnostics of the last call that used ``workspace``."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(workspace.device)
    out = (ctypes.c_int64 * len(STATS_FIELDS))()
    wptr, _ = _aligned_ptr(workspace)
    rc = _load().fec_workspace_stats(ctypes.c_void_p(wptr), ctypes.c_void_p(stream.cuda_stream),
                                  out, len(STATS_FIELDS))
    if rc < 0:
        _raise(rc)
    return {k: int(out[i]) for i, k in enumerate(STATS_FIELDS[:rc])}


def stage_names() -> list[str]:
    return [_load().fec_stage_name(i).decode() for i in range(_load().fec_stage_count())]


def profile_enable(stages=None) -> None:
    """Time the named stages (all when None) with HIP events; [] turns timing off."""
    names = stage_names()
    if stages is None:
        mask = (1 << len(names)) - 1
    else:
        mask = 0
        for s in stages:
            mask |= 1 << names.index(s)
    _load().fec_profile_enable(mask)


def profile_read() -> dict:
    """{stage: (total ms, timed launches)} accumulated since the last reset."""
    ns = _load().fec_stage_count()
    ms = (ctypes.c_double * ns)()
    cnt = (ctypes.c_int64 * ns)()
    _load().fec_profile_read(ms, cnt, ns)
    names = stage_names()
    return {names[i]: (float(ms[i]), int(cnt[i])) for i in range(ns)}


def profile_reset() -> None:
    _load().fec_profile_reset()


def raw_lib():
    """The loaded ctypes library (for ABI tests)."""
    return _load()
