"""Compile the HIP library libsr.so for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsr.so")
SOURCES = [os.path.join(CSRC, "sr_kernels.hip"), os.path.join(CSRC, "sr_blocks.hip"),
           os.path.join(CSRC, "sr_centres.hip"), os.path.join(CSRC, "sr_pk.hip"),
           os.path.join(CSRC, "sr_static.hip"),
           os.path.join(CSRC, "sr_api.cpp")]
LIBS = ["-L/opt/rocm/lib", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib"]
ARCH = os.environ.get("SR_OFFLOAD_ARCH", "gfx950")

# -packed-fp32-ops: keep the compiler from forming packed float32 arithmetic.
# -ffp-contract=off: no implicit fused multiply-add; the kernels call fmaf
# where they want one, and the binning rule is specified without it.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def build(verbose: bool = False, extra=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPFLAGS, *(extra or []), "-I", INCLUDE, "-I", CSRC, "-shared", "-o", tmp,
           *SOURCES, *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
