"""The GPU library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU, no GPU touched).

The library is built a second time with the sanitizers on its host code
only (`-Xarch_host -fsanitize=...`; device code is built as usual) and
loaded in a child process that preloads clang's sanitizer runtime.  The
child drives every entry point along paths that end before any GPU call:
workspace sizes, argument checks of the single, batched and no-allocation
forms, the serving engine's argument checks, the launch knobs, the stage
names and the error strings.  Any sanitizer finding aborts the child.
"""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import ctypes, sys
lib = ctypes.CDLL(sys.argv[1])
i32, i64, f32, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t
sig = {
    "fec_workspace_bytes": ([i64], sz), "fec_batch_workspace_bytes": ([i64, i32], sz),
    "fec_server_slot_bytes": ([i64, i32], sz),
    "fec_cluster_async": ([vp, i64, f32, i32, i32, vp, vp, vp, sz, vp], i32),
    "fec_cluster_noalloc": ([vp, i64, f32, i32, i32, vp, vp, vp], i32),
    "fec_cluster_batch_async": ([vp, i64, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp], i32),
    "fec_tuning_set": ([i32, i32, i32, i32, i32], i32), "fec_tuning_get": ([vp, vp, vp, vp, vp], i32),
    "fec_server_create": ([sz, i32, i32, vp], i32), "fec_server_slot_points": ([vp], i64),
    "fec_server_submit": ([vp, vp, i64, f32, i32, i32, vp, vp], i32),
    "fec_server_pump": ([vp, i32], i32), "fec_server_poll": ([vp, vp, vp, vp, i32], i32),
    "fec_server_destroy": ([vp], None), "fec_workspace_stats": ([vp, vp, vp, i32], i32),
    "fec_last_error": ([], ctypes.c_char_p), "fec_version": ([], ctypes.c_char_p),
    "fec_stage_count": ([], i32), "fec_stage_name": ([i32], ctypes.c_char_p),
}
for k, (a, r) in sig.items():
    f = getattr(lib, k); f.argtypes = a; f.restype = r
EINVAL = -1
assert lib.fec_workspace_bytes(0) == 0 and lib.fec_workspace_bytes(-3) == 0
for n in (1, 4095, 4096, 4097, 10**6, 27 * 10**6):
    assert lib.fec_workspace_bytes(n) > 0
assert lib.fec_batch_workspace_bytes(10**6, 64) > lib.fec_batch_workspace_bytes(10**6, 1) > 0
assert lib.fec_batch_workspace_bytes(1000, 0) == 0
assert lib.fec_server_slot_bytes(10**6, 64) > 0 and lib.fec_server_slot_bytes(1000, 1025) == 0
buf = vp(0x1000)   # never dereferenced: every call below fails its checks first
for n, d, mn, mx in [(-1, .5, 1, 5), (10, 0., 1, 5), (10, float("nan"), 1, 5),
                     (10, float("inf"), 1, 5), (10, .5, 6, 5), (10, -1., 1, 5)]:
    assert lib.fec_cluster_async(buf, n, d, mn, mx, buf, None, buf, 1 << 40, None) == EINVAL
    assert lib.fec_last_error()
    assert lib.fec_cluster_noalloc(buf, n, d, mn, mx, buf, None, None) == EINVAL
assert lib.fec_cluster_async(None, 10, .5, 1, 5, buf, None, buf, 1 << 40, None) == EINVAL
assert lib.fec_cluster_async(buf, 10, .5, 1, 5, buf, None, buf, 16, None) == EINVAL
assert lib.fec_cluster_async(buf, 10, .5, 1, 5, buf, None, vp(0x1001), 1 << 40, None) == EINVAL
assert lib.fec_cluster_async(None, 0, .5, 1, 5, None, None, None, 0, None) == 0
assert lib.fec_cluster_noalloc(buf, 524289, .5, 1, 5, buf, None, None) == EINVAL
assert lib.fec_cluster_noalloc(None, 0, .5, 1, 5, None, None, None) == 0
assert lib.fec_cluster_batch_async(buf, 10, 0, buf, buf, buf, buf, buf, buf, buf, 1 << 40, None) == EINVAL
assert lib.fec_cluster_batch_async(buf, -1, 2, buf, buf, buf, buf, buf, buf, buf, 1 << 40, None) == EINVAL
h = vp()
for slots, frames in [(0, 8), (65, 8), (2, 0), (2, 1025)]:
    assert lib.fec_server_create(1 << 30, slots, frames, ctypes.byref(h)) == EINVAL
assert lib.fec_server_create(1 << 30, 2, 8, None) == EINVAL
assert lib.fec_server_submit(None, None, 0, .3, 1, 2, None, None) == EINVAL
assert lib.fec_server_pump(None, 0) == EINVAL and lib.fec_server_poll(None, None, None, None, 4) == EINVAL
assert lib.fec_server_slot_points(None) == 0
lib.fec_server_destroy(None)
v = [i32() for _ in range(5)]
assert lib.fec_tuning_set(1024, 8192, 10, 128, 2) == 0
lib.fec_tuning_get(*[ctypes.byref(x) for x in v])
assert [x.value for x in v] == [1024, 8192, 10, 128, 2]
for bad in [(-1, 0, 0, 0, 0), (0, 1 << 21, 0, 0, 0), (0, 0, 7, 0, 0), (0, 0, 0, 96, 0), (0, 0, 0, 0, 3)]:
    assert lib.fec_tuning_set(*bad) == EINVAL
assert lib.fec_tuning_set(0, 0, 0, 0, 0) == 0
assert lib.fec_workspace_stats(None, None, None, 4) == EINVAL
assert lib.fec_version()
names = [lib.fec_stage_name(i) for i in range(lib.fec_stage_count())]
assert all(names) and len(set(names)) == len(names) and lib.fec_stage_name(999) == b""
print("host checks ok")
'''


def _runtime():
    c = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return c[-1] if c else None


@pytest.mark.timeout(900)
def test_host_code_under_sanitizers(tmp_path):
    rt = _runtime()
    if rt is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no hipcc or no clang sanitizer runtime")
    sys.path.insert(0, ROOT)
    from paper_2208_07678_amd import build as B
    lib = str(tmp_path / "libfec_san.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-shared-libsan"]
    subprocess.run([B.HIPCC, *B.FLAGS, *san, "-o", lib, *B.SOURCES], check=True,
                   capture_output=True)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD, lib], capture_output=True, text=True,
                       env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host checks ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
