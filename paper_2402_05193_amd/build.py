"""Build libfvrk3.so (HIP, gfx950) in-tree with hipcc, and the same sources with a
second tile shape (libfvrk3_tile32x8.so) for the tile-race check of the tests.

Usage: python -m paper_2402_05193_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfvrk3.so")
# The stage kernels with 32 x 8 cells per workgroup and 320 threads (the product's are
# 16 x 16 and 256): every x/y task list, the halo and ring assignments and the z chunks
# map to threads differently, while each cell's arithmetic does not depend on the tiling,
# so results equal bitwise to the product's unless the LDS plane or the face buffers race.
LIB_TILE = os.path.join(HERE, "libfvrk3_tile32x8.so")
TILE_VARIANT = ("-DTILE_BX=32", "-DTILE_BY=8", "-DTILE_NT=320")
# (source, defines, extra options): the stage kernels compile per precision, model and
# reconstruction (0 primitive WENO5-Z, 1 characteristic WENO5-Z, 2 primitive TENO6-A,
# 3 characteristic TENO6-A) so that the units build in parallel and each family gets
# its own code-generation options
# The iterative occupancy-driven instruction scheduler: measured faster for the
# primitive WENO5-Z kernels of the single-phase models (NS 256^3 FP64 2.40 -> 2.34 ms
# per stage, FP32 1.36 -> 1.32, Euler 1.76 -> 1.73, with sixth-order viscous fluxes
# 3.96 -> 3.80), slower for the characteristic ones (3.01 -> 3.81 ms) and the
# five-equation model (0.92 -> 0.95 ms), equal for TENO6-A.
SCHED_OCC = ("-mllvm", "-amdgpu-sched-strategy=iterative-maxocc")
UNITS = [("fv_stage_inst.hip", (f"-DFV_REAL={r}", f"-DFV_MODEL={m}", f"-DFV_REC={rec}"),
          SCHED_OCC if (m != "DIM" and rec == 0) else ())
         for r in ("double", "float") for m in ("NS", "EULER", "DIM") for rec in range(4)] + [
    (src, (), ()) for src in ("fv_stage_launch.hip", "fv_visc6.hip", "fv_aux.hip", "fv_adjoint.hip", "fv_api.hip")]
SOURCES = sorted({u[0] for u in UNITS})
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep the compiler from forming packed FP32 VALU operations
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fused multiply-adds only where one source expression has the a*b+c form:
    # the arithmetic then follows the source, identical in every kernel that
    # inlines the same device code (single-problem and batched launches)
    "-ffp-contract=on",
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None,
          jobs: int | None = None) -> str:
    """Compile every unit to an object (in parallel), then link the shared library."""
    out = out or LIB
    objdir = out + ".objs"
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1, 8))
    cmds = []
    for src, defs, opts in UNITS:
        tag = "".join(d.split("=")[1][0].lower() for d in defs)
        obj = os.path.join(objdir, os.path.splitext(src)[0] + (f"_{tag}" if tag else "") + ".o")
        cmds.append((obj, [HIPCC, *FLAGS, *opts, *(extra or []), *defs, "-c", os.path.join(CSRC, src), "-o", obj]))
    pending = list(cmds)
    running = []
    failed = []
    while pending or running:
        while pending and len(running) < jobs:
            obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((obj, subprocess.Popen(cmd)))
        obj, proc = running.pop(0)
        if proc.wait() != 0:
            failed.append(obj)
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc ({', '.join(os.path.basename(f) for f in failed)})")
    tmp = out + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for o, _ in cmds]]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, out)
    return out


def build_tile_variant(verbose: bool = False) -> str:
    """The second tile shape (LIB_TILE)."""
    return build(verbose=verbose, extra=list(TILE_VARIANT), out=LIB_TILE)


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
    if not sys.argv[1:]:
        build_tile_variant(verbose=True)
