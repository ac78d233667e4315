"""Build libsparsesim.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsparsesim.so")
SOURCES = ["sim_api.hip", "sim_kernels.hip", "mono_bitslice.hip", "mono_regplane.hip", "run_compiler.hip", "batch_kernels.hip", "serve.hip",
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
    # The register-plane pass clobbers M0 and names reserved VGPRs in inline
    # assembly on purpose (the compiler never allocates them).
    "-Wno-inline-asm",
]


# The register-plane pass keeps its bit-planes in VGPRs v80 and above, which
# only its inline assembly may touch (the compiler is capped below v80), and
# its assembly changes M0.  After every build the pass's own gfx950 assembly
# is checked: no compiler-generated instruction may name v80 or above or M0,
# and no kernel may spill to scratch.
REGPLANE_SRC = "mono_regplane.hip"
RESERVED_VGPR = 80


def check_regplane_asm(text: str) -> list[str]:
    import re

    bad, in_asm = [], False
    for ln in text.split("\n"):
        if ";;#ASMSTART" in ln:
            in_asm = True
            continue
        if ";;#ASMEND" in ln:
            in_asm = False
            continue
        m = re.match(r"; ScratchSize: (\d+)", ln.strip())
        if m and int(m.group(1)):
            bad.append("scratch use: " + ln.strip())
        body = ln.strip()
        if in_asm or not ln.startswith("\t") or body.startswith((";", ".")):
            continue
        if re.search(r"\bm0\b", body):
            bad.append("M0 use: " + body)
        for r in re.finditer(r"\bv\[?(\d+)(?::(\d+))?\]?", body):
            if int(r.group(2) or r.group(1)) >= RESERVED_VGPR:
                bad.append("reserved VGPR: " + body)
    return bad


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    asm = LIB + ".regplane.s"
    subprocess.check_call([HIPCC, *[f for f in FLAGS if f not in ("-fPIC", "-shared")], "--offload-device-only", "-S",
                           "-o", asm, os.path.join(CSRC, REGPLANE_SRC)], stderr=subprocess.DEVNULL)
    with open(asm) as f:
        bad = check_regplane_asm(f.read())
    os.remove(asm)
    if bad:
        os.remove(tmp)
        raise RuntimeError("register-plane pass: compiler code touches its reserved registers:\n" + "\n".join(bad[:20]))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
