"""Helpers shared by the GPU tests: run the HIP path, compare with the oracle."""

from __future__ import annotations

import sys

import numpy as np


def say(*a):
    """Progress line, flushed before each GPU step so a failing case is named."""
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_cluster(xyz: np.ndarray, d: float, mn: int, mx: int, workspace=None):
    import torch

    import paper_2208_07678_amd as fec

    t = torch.from_numpy(np.ascontiguousarray(xyz, dtype=np.float32)).to("cuda:0")
    labels, k = fec.cluster(t, d, mn, mx, workspace=workspace)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), k


def describe_mismatch(got: np.ndarray, want: np.ndarray) -> str:
    bad = np.nonzero(got != want)[0]
    if bad.size == 0:
        return "equal"
    i = int(bad[0])
    return "%d of %d labels differ; first at %d: gpu %d oracle %d" % (
        bad.size, got.size, i, int(got[i]), int(want[i]))
