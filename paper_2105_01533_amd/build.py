"""Build libsparsesim.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsparsesim.so")
SOURCES = ["sim_api.hip", "sim_kernels.hip", "mono_bitslice.hip", "run_compiler.hip", "batch_kernels.hip", "serve.hip",
           "commute.hip", "pauli.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",                      # no fused multiply-add: fixed rounding
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Branches on wave-uniform values (the fused pass's per-group dispatch)
    # stay plain scalar branches instead of being rewritten as exec-masked
    # flow blocks.
    "-mllvm", "-structurizecfg-skip-uniform-regions",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
