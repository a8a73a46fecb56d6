"""Build libfvrk3.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2402_05193_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfvrk3.so")
SOURCES = ["fv_stage.hip", "fv_aux.hip", "fv_adjoint.hip", "fv_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from forming packed FP32 VALU operations
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fused multiply-adds only where one source expression has the a*b+c form:
    # the arithmetic then follows the source, identical in every kernel that
    # inlines the same device code (single-problem and batched launches)
    "-ffp-contract=on",
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    out = out or LIB
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *(extra or []), "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
