"""Compile the gfx950 HIP library ``libgfix.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgfix.so")
SOURCES = ["gf_kernels.hip", "gf_heatbath.hip", "gf_runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    # no packed-FP32 instructions anywhere (they are not used deliberately)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a multiply-add is fused only where one source expression holds it, so
    # every inlined copy of a helper rounds alike (a link recomputed by a
    # neighbouring work-group equals the one its owner stores)
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
