"""The C ABI library loads on the CPU host and exports what include/fec.h declares.

No compute call is made here (no GPU); only host-side entry points that do
not touch a device: argument checks, workspace sizing, names.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fec.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fec_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def fec():
    import paper_2208_07678_amd as fec
    if not os.path.exists(fec.lib_path):
        pytest.fail("HIP library not built: run python -m paper_2208_07678_amd.build")
    fec._load()
    return fec


def test_every_declared_symbol_is_exported(fec):
    names = _declared()
    assert len(names) >= 10
    lib = fec.raw_lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(fec.EXPORTED) == names


def test_workspace_bytes_linear(fec):
    assert fec.workspace_bytes(0) == 0
    assert fec.workspace_bytes(-5) == 0
    a, b = fec.workspace_bytes(1_000_000), fec.workspace_bytes(2_000_000)
    assert 60 * 1_000_000 < a < 200 * 1_000_000, a
    assert b > a


def test_stage_names(fec):
    names = fec.stage_names()
    assert "hook_near" in names and "sort_scatter" in names and len(names) == len(set(names))


def test_host_side_argument_checks(fec):
    lib = fec.raw_lib()
    buf = ctypes.c_void_p(0x1000)   # never dereferenced: checks fail first
    ws = ctypes.c_void_p(0x100000)
    cases = [
        (-1, 0.5, 1, 5), (2**31, 0.5, 1, 5), (10, 0.0, 1, 5), (10, -1.0, 1, 5),
        (10, float("nan"), 1, 5), (10, float("inf"), 1, 5), (10, 1e-30, 1, 5), (10, 0.5, 6, 5),
    ]
    for n, d, mn, mx in cases:
        rc = lib.fec_cluster_async(buf, n, ctypes.c_float(d), mn, mx, buf, None, ws, 1 << 40, None)
        assert rc == fec.FEC_EINVAL, (n, d, mn, mx)
        assert lib.fec_last_error()
    # null pointers with n > 0
    rc = lib.fec_cluster_async(None, 10, ctypes.c_float(0.5), 1, 5, buf, None, ws, 1 << 40, None)
    assert rc == fec.FEC_EINVAL
    # workspace too small / misaligned
    rc = lib.fec_cluster_async(buf, 10, ctypes.c_float(0.5), 1, 5, buf, None, ws, 16, None)
    assert rc == fec.FEC_EINVAL
    rc = lib.fec_cluster_async(buf, 10, ctypes.c_float(0.5), 1, 5, buf, None,
                               ctypes.c_void_p(0x100001), 1 << 40, None)
    assert rc == fec.FEC_EINVAL
    # n == 0 with no k_out: nothing to do, no device touched
    rc = lib.fec_cluster_async(None, 0, ctypes.c_float(0.5), 1, 5, None, None, None, 0, None)
    assert rc == fec.FEC_OK


def test_noalloc_host_side_checks(fec):
    # the no-allocation form's size limit and argument checks come before
    # any device call (that its scratch array holds the workspace of the
    # largest call it admits is a static_assert of the library's build; that
    # workspace keeps a smaller dense column index than fec_workspace_bytes
    # sizes for the other entry points)
    lib = fec.raw_lib()
    buf = ctypes.c_void_p(0x1000)   # never dereferenced: checks fail first
    hdr = open(HEADER).read()
    lim = int(re.search(r"#define FEC_NOALLOC_MAX_POINTS (\d+)", hdr).group(1))
    sb = re.search(r"#define FEC_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", hdr)
    scratch = int(sb.group(1)) << int(sb.group(2))
    assert lim == fec.NOALLOC_MAX_POINTS
    assert 0 < lim * 64 <= scratch
    for n, d, mn, mx in [(lim + 1, 0.5, 1, 5), (-1, 0.5, 1, 5), (10, 0.0, 1, 5),
                         (10, float("nan"), 1, 5), (10, 0.5, 6, 5)]:
        rc = lib.fec_cluster_noalloc(buf, n, ctypes.c_float(d), mn, mx, buf, None, None)
        assert rc == fec.FEC_EINVAL, (n, d, mn, mx)
        assert lib.fec_last_error()
    rc = lib.fec_cluster_noalloc(None, 10, ctypes.c_float(0.5), 1, 5, buf, None, None)
    assert rc == fec.FEC_EINVAL
    # n == 0 with no k_out: nothing to do, no device touched
    assert lib.fec_cluster_noalloc(None, 0, ctypes.c_float(0.5), 1, 5, None, None, None) == 0


def test_cpu_tensors_are_refused(fec):
    import torch
    with pytest.raises(ValueError):
        fec.cluster(torch.zeros((4, 3)), 0.5)


def test_batch_host_side_argument_checks(fec):
    lib = fec.raw_lib()
    buf = ctypes.c_void_p(0x1000)   # never dereferenced: checks fail first
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40

    def call(xyz, n, nf, offs, d, lo, hi, labels, k, w, wb):
        return lib.fec_cluster_batch_async(xyz, n, nf, offs, d, lo, hi, labels, k, w, wb, None)

    assert call(buf, -1, 2, buf, buf, buf, buf, buf, buf, ws, big) == fec.FEC_EINVAL
    assert call(buf, 2**31, 2, buf, buf, buf, buf, buf, buf, ws, big) == fec.FEC_EINVAL
    assert call(buf, 10, 0, buf, buf, buf, buf, buf, buf, ws, big) == fec.FEC_EINVAL
    assert call(buf, 10, 65537, buf, buf, buf, buf, buf, buf, ws, big) == fec.FEC_EINVAL
    for miss in range(5):   # offsets, d, min_size, max_size, k_out
        a = [buf] * 5
        a[miss] = None
        assert call(buf, 10, 2, a[0], a[1], a[2], a[3], buf, a[4], ws, big) == fec.FEC_EINVAL
    assert call(None, 10, 2, buf, buf, buf, buf, buf, buf, ws, big) == fec.FEC_EINVAL
    assert call(buf, 10, 2, buf, buf, buf, buf, None, buf, ws, big) == fec.FEC_EINVAL
    assert call(buf, 10, 2, buf, buf, buf, buf, buf, buf, ws, 16) == fec.FEC_EINVAL
    assert call(buf, 10, 2, buf, buf, buf, buf, buf, buf, ctypes.c_void_p(0x100001),
                big) == fec.FEC_EINVAL
    assert lib.fec_last_error()


def test_batch_workspace_bytes(fec):
    assert fec.batch_workspace_bytes(1000, 0) == 0
    assert fec.batch_workspace_bytes(-1, 3) == 0
    a = fec.batch_workspace_bytes(1_000_000, 1)
    b = fec.batch_workspace_bytes(1_000_000, 64)
    # one frame: the single-cloud layout; frames add a frame table and a
    # frame id per cell
    assert a == fec.workspace_bytes(1_000_000)
    assert a < b < a + 8 * 1_000_000
    assert fec.batch_workspace_bytes(0, 5) > 0


def test_server_host_side_checks(fec):
    lib = fec.raw_lib()
    h = ctypes.c_void_p()
    assert lib.fec_server_create(1 << 30, 0, 8, ctypes.byref(h)) == fec.FEC_EINVAL
    assert lib.fec_server_create(1 << 30, 65, 8, ctypes.byref(h)) == fec.FEC_EINVAL
    assert lib.fec_server_create(1 << 30, 2, 0, ctypes.byref(h)) == fec.FEC_EINVAL
    assert lib.fec_server_create(1 << 30, 2, 1025, ctypes.byref(h)) == fec.FEC_EINVAL
    assert lib.fec_server_create(1 << 30, 2, 8, None) == fec.FEC_EINVAL
    t = ctypes.c_int64()
    assert lib.fec_server_submit(None, None, 0, ctypes.c_float(0.3), 1, 2, None,
                                 ctypes.byref(t)) == fec.FEC_EINVAL
    assert lib.fec_server_pump(None, 0) == fec.FEC_EINVAL
    assert lib.fec_server_poll(None, None, None, None, 4) == fec.FEC_EINVAL
    assert lib.fec_server_slot_points(None) == 0
    lib.fec_server_destroy(None)
    # slot footprint: linear in points, grows with frames
    a, b = fec.raw_lib().fec_server_slot_bytes(1_000_000, 64), lib.fec_server_slot_bytes(
        2_000_000, 64)
    assert 0 < a < b and lib.fec_server_slot_bytes(0, 8) == 0
    assert lib.fec_server_slot_bytes(1000, 1025) == 0


def test_tuning_knobs_and_cache(fec, tmp_path):
    from paper_2208_07678_amd import tune
    assert fec.get_tuning() == tune.DEFAULT == (4096, 4096, 9, 256, 0)
    fec.set_tuning(1024, 8192, 9, 128, 2)
    assert fec.get_tuning() == (1024, 8192, 9, 128, 2)
    fec.set_tuning(1024, 8192)          # the other knobs back to their defaults
    assert fec.get_tuning() == (1024, 8192, 9, 256, 0)
    for bad in [(-1, 0), (0, 1 << 21), (0, 0, 7), (0, 0, 12), (0, 0, 0, 96), (0, 0, 0, 512),
                (0, 0, 0, 0, -1), (0, 0, 0, 0, 3)]:
        with pytest.raises(fec.FecError):
            fec.set_tuning(*bad)
    fec.set_tuning(0, 0, 0, 0, 0)
    assert fec.get_tuning() == (4096, 4096, 9, 256, 0)
    # cache round trip, keyed by arch and size bucket
    p = str(tmp_path / "tune.json")
    assert tune.lookup("gfx950", 27_000_000, p) is None
    tune.record("gfx950", 27_000_000, (2048, 8192, 9, 128, 1), 6.1, p)
    assert tune.lookup("gfx950", 20_000_000, p) == (2048, 8192, 9, 128, 1)  # same bucket (2^24)
    tune.record("gfx950", 1000, (2048, 8192), 0.2, p)   # knobs not given: defaults
    assert tune.lookup("gfx950", 1000, p) == (2048, 8192, 9, 256, 0)
    assert tune.lookup("gfx950", 40_000_000, p) is None            # next bucket
    assert tune.lookup("gfx942", 27_000_000, p) is None
    assert tune.bucket(1) == 0 and tune.bucket(4096) == 12
