"""Builds the HIP library for gfx950 in-tree: paper_2208_07678_amd/libfec_hip.so.

    python -m paper_2208_07678_amd.build

Flags: no floating-point contraction (the edge test must round every
operation), no packed-FP32 instructions, IEEE denormals (the default).
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfec_hip.so")
SOURCES = [os.path.join(CSRC, "fec_device.hip"), os.path.join(CSRC, "fec_api.hip"),
           os.path.join(CSRC, "fec_serve.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def asm(out_dir: str) -> list[str]:
    """Writes the gfx950 assembly of the device code (for inspection)."""
    os.makedirs(out_dir, exist_ok=True)
    outs = []
    for src in SOURCES[:1]:
        out = os.path.join(out_dir, os.path.basename(src) + ".s")
        subprocess.run([HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC")],
                        "--cuda-device-only", "-S", "-o", out, src], check=True)
        outs.append(out)
    return outs


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
