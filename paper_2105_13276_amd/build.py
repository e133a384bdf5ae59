"""Build libdmr.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2105_13276_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = [os.path.join(PKG, "csrc", f) for f in ("dmr_kernels.hip", "dmr_adjoint.hip", "dmr_api.hip")]
LIB = os.path.join(PKG, "libdmr.so")
ARCH = os.environ.get("DMR_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    "-fno-gpu-flush-denormals-to-zero",
    # contract only a*b+c written in one expression, so that every
    # instantiation of a kernel body rounds identically
    "-ffp-contract=on",
    # keep the compiler from emitting packed fp32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + ["-I", os.path.join(ROOT, "include"),
                             "-I", os.path.join(PKG, "csrc"), "-o", tmp] + SRC
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
