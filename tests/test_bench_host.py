"""Host logic of bench.py that needs no GPU: measured traffic is used only for
the workload its counters were taken on and only while the kernel sources
are the ones they were taken with; the whole-path sum counts the sort's
kernels once per pass; more than one GPU is refused before anything runs."""

import json
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tree(tmp_path, record):
    """A copy of the two kernel sources and a counter record under tmp_path."""
    src = os.path.join(ROOT, "paper_2208_07678_amd", "csrc")
    dst = tmp_path / "paper_2208_07678_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in ("fec_device.hip", "fec_internal.h"):
        shutil.copy(os.path.join(src, name), dst / name)
    (tmp_path / "profiles").mkdir()
    with open(tmp_path / "profiles" / ("traffic_%s.json" % record["workload"]), "w") as f:
        json.dump(record, f)
    return dst


def _record(workload, digest):
    k = lambda b: {"kernel": "k", "fetch_bytes_per_launch": b, "write_bytes_per_launch": 0,
                   "hbm_bytes_per_launch": b}
    return {"workload": workload, "source_sha256": digest,
            "kernels": {"hook_near": k(100), "sort_hist": k(10), "sort_scatter": k(20),
                        "compress": k(3), "gather": k(7)}}


def test_traffic_only_for_its_workload_and_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    csrc = _tree(tmp_path, _record("map27m", "0" * 64))
    digest = bench._source_digest()
    with open(tmp_path / "profiles" / "traffic_map27m.json", "w") as f:
        json.dump(_record("map27m", digest), f)
    assert bench.measured_traffic("map27m", "hook_near") == 100
    assert bench.measured_traffic("map27m", "no_such_stage") is None
    # another workload has no counters of its own
    assert bench.measured_traffic("lidar120k", "hook_near") is None
    assert bench.path_traffic("lidar120k", 5) is None
    # sort kernels once per pass, the rest once (kernels launched several
    # times per call are recorded per call)
    assert bench.path_traffic("map27m", 5) == 100 + 5 * (10 + 20) + 3 + 7
    # a record filed under one name but taken on another workload
    with open(tmp_path / "profiles" / "traffic_batch64.json", "w") as f:
        json.dump(_record("map27m", digest), f)
    assert bench.measured_traffic("batch64", "hook_near") is None
    # kernel sources changed since the counters were taken
    with open(csrc / "fec_internal.h", "a") as f:
        f.write("\n")
    assert bench.measured_traffic("map27m", "hook_near") is None
    assert bench.path_traffic("map27m", 5) is None


def test_committed_record_names_its_workload():
    with open(os.path.join(ROOT, "profiles", "traffic_map27m.json")) as f:
        rec = json.load(f)
    assert rec["workload"] == "map27m"
    assert len(rec["source_sha256"]) == 64
    for st, k in rec["kernels"].items():
        # each of the three is rounded to whole bytes on its own
        total = k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
        assert abs(k["hbm_bytes_per_launch"] - total) <= 1, st


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_models_follow_the_work_lists():
    n = 1000
    st = {"cells": 400, "work_cells": 100, "near_work_cells": 0}
    assert bench.alg_bytes_per_point("gather", st, n) == 40.0
    assert bench.alg_bytes_per_point("hook_near", st, n) == 28.0
    assert bench.alg_bytes_per_point("hook_far", st, n) == 28.0 * 100 / 400
    # the near shell on the sampled links' work list
    st["near_work_cells"] = 200
    assert bench.alg_bytes_per_point("hook_near", st, n) == 28.0 * 200 / 400
    # the sampling links: per cell
    assert bench.alg_bytes_per_point("sample", st, n) == 32.0 * 400 / 1000
    assert bench.alg_bytes_per_point("no_model", st, n) == 16.0
