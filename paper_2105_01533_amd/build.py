"""Build libsparsesim.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsparsesim.so")
SOURCES = ["sim_api.hip", "sim_kernels.hip", "mono_bitslice.hip", "mono_regplane.hip", "run_compiler.hip", "batch_kernels.hip",
           "serve.hip", "commute.hip", "pauli.hip", "state_copy.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
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
REGPLANE_SRCS = ["mono_regplane.hip"]
# Per-source extra flags (none at present).
EXTRA_FLAGS: dict[str, list[str]] = {}
RESERVED_VGPR = 80


def check_regplane_asm(text: str, regplane_only: str | None = None) -> list[str]:
    """Lines of compiler-generated code (outside inline assembly) that name
    v80 or above or M0, and nonzero scratch sizes; with regplane_only, only
    inside functions whose (mangled) symbol contains that string."""
    import re

    bad, in_asm = [], False
    keep = regplane_only is None
    for ln in text.split("\n"):
        m = re.match(r"^(\S+):\s*(;.*)?$", ln)
        if m and not m.group(1).startswith(".") and not m.group(1)[0].isdigit() and regplane_only is not None:
            keep = regplane_only in m.group(1)
        if not keep:
            continue
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


def _compile_cmd(src: str, out: str, *extra: str) -> list[str]:
    return [HIPCC, *FLAGS, *EXTRA_FLAGS.get(src, []), *extra, "-o", out, os.path.join(CSRC, src)]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    jobs = int(os.environ.get("MAX_JOBS", "0") or 0) or min(8, os.cpu_count() or 1)
    pending = list(zip(SOURCES, objs))
    running: list[tuple[str, subprocess.Popen]] = []
    failed = []
    while pending or running:
        while pending and len(running) < jobs:
            src, obj = pending.pop(0)
            cmd = _compile_cmd(src, obj, "-c")
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((src, subprocess.Popen(cmd)))
        src, proc = running.pop(0)
        if proc.wait() != 0:
            failed.append(src)
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc -c " + " ".join(failed))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    bad = []
    for src in REGPLANE_SRCS:
        asm = os.path.join(objdir, src.replace(".hip", ".s"))
        subprocess.check_call([*(c for c in _compile_cmd(src, asm) if c != "-fPIC"), "--offload-device-only", "-S"],
                              stderr=subprocess.DEVNULL)
        with open(asm) as f:
            bad += [f"{src}: {b}" for b in check_regplane_asm(f.read())]
        os.remove(asm)
    if bad:
        os.remove(tmp)
        raise RuntimeError("register-plane pass: compiler code touches its reserved registers:\n" + "\n".join(bad[:20]))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
