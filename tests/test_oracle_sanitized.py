"""The oracle's C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle is built a second time with -fsanitize=address,undefined (any
finding aborts) and run in a child process that preloads the sanitizer
runtime.  It clusters small clouds of every kind the oracle's pins use
(random, clumped, chains, non-finite points, duplicates, wide extents), with
size filters, the raw Alg. 1 values and the kd-tree queries, and its labels
must equal the regular build's.
"""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
oracle._LIB = sys.argv[2]
oracle._lib = None
cases = json.loads(sys.stdin.read())
out = []
for c in cases:
    xyz = np.asarray(c["xyz"], dtype=np.float32).reshape(-1, 3)
    lab, k = oracle.fec(xyz, c["d"], c["mn"], c["mx"])
    f, kf, u, nc = oracle.fec_both(xyz, c["d"], c["mn"], c["mx"])
    raw = oracle.fec_raw(xyz, c["d"], steps=xyz.shape[0] // 2)
    capped, _ = oracle.fec(xyz, c["d"], 1, xyz.shape[0] + 1, th_max=3)
    skip, _ = oracle.fec(xyz, c["d"], 1, xyz.shape[0] + 1, flags=oracle.SKIP_LABELLED)
    ix = oracle.Index(xyz, c["d"])
    nbrs = [ix.neighbors(i).tolist() for i in range(min(20, xyz.shape[0]))]
    comp = ix.component(0, 50) if xyz.shape[0] else None
    viol = ix.closure_violations(lab, np.arange(xyz.shape[0]))
    ix.close()
    out.append({"lab": lab.tolist(), "k": k, "f": f.tolist(), "kf": kf, "u": u.tolist(), "nc": nc,
                "raw": raw.tolist(), "capped": capped.tolist(), "skip": skip.tolist(),
                "nbrs": nbrs, "comp": list(comp) if comp else None, "viol": viol})
print(json.dumps(out))
'''


def _cases():
    rng = np.random.default_rng(5)
    cases = []
    for seed in range(6):
        n = int(rng.integers(50, 600))
        kind = seed % 3
        if kind == 0:
            x = rng.uniform(0, 4, size=(n, 3))
        elif kind == 1:
            c = rng.uniform(0, 10, size=(5, 3))
            x = c[rng.integers(0, 5, n)] + rng.normal(0, 0.3, (n, 3))
        else:
            x = np.zeros((n, 3))
            x[:, int(rng.integers(0, 3))] = np.arange(n) * 0.2
        x = x.astype(np.float32)
        if seed == 4:   # non-finite points and exact duplicates
            x[::7] = np.nan
            x[1::11, 2] = np.inf
            x[2::13] = x[3::13][: len(x[2::13])]
        cases.append({"xyz": x.ravel().tolist(), "d": float(rng.uniform(0.15, 0.6)),
                      "mn": int(rng.integers(0, 4)), "mx": int(rng.integers(5, n + 2))})
    wide = (rng.uniform(0, 1e5, size=(200, 3))).astype(np.float32)   # sparse, wide extent
    cases.append({"xyz": wide.ravel().tolist(), "d": 1e-2, "mn": 1, "mx": 200})
    cases.append({"xyz": [], "d": 0.5, "mn": 1, "mx": 5})            # empty cloud
    return cases


@pytest.mark.timeout(600)
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-fPIC", "-shared", "-o", lib,
                    os.path.join(ROOT, "oracle", "fec_oracle.cpp")], check=True)
    cases = _cases()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, lib], input=json.dumps(cases),
                       capture_output=True, text=True, env=env, timeout=540)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert len(got) == len(cases)
    for c, g in zip(cases, got):
        xyz = np.asarray(c["xyz"], dtype=np.float32).reshape(-1, 3)
        lab, k = oracle.fec(xyz, c["d"], c["mn"], c["mx"])
        assert g["lab"] == lab.tolist() and g["k"] == k
        f, kf, u, nc = oracle.fec_both(xyz, c["d"], c["mn"], c["mx"])
        assert g["f"] == f.tolist() and g["u"] == u.tolist() and g["nc"] == nc
        assert g["raw"] == oracle.fec_raw(xyz, c["d"], steps=xyz.shape[0] // 2).tolist()
        assert g["viol"] == 0
