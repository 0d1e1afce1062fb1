"""Build the HIP library (gfx950) in-tree: paper_2306_04467_amd/libgks.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgks.so")
SOURCES = ["gks_api.hip", "mesh_setup.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary vector registers: the fused indicator then adds no
    # accumulation registers to the reconstruction's budget (7 instead of 5 waves per SIMD in FP32)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


# the checked build: every index the kernels read from a mesh table is tested (gks_debug_bounds)
LIB_CHECKED = os.path.join(HERE, "libgks_checked.so")


def _compile(out: str, extra, verbose: bool):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-o", out + ".tmp", *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    return cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def build(verbose: bool = False) -> str:
    """Compile the library and its checked build (in parallel); returns the library's path."""
    jobs = [(LIB, _compile(LIB, [], verbose)), (LIB_CHECKED, _compile(LIB_CHECKED, ["-DGKS_CHECKED"], verbose))]
    for out, (cmd, proc) in jobs:
        _, err = proc.communicate()
        if proc.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + err)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
