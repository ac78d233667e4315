"""Host-side checks of the bit-sliced passes' op schedulers: RunCompiler::group
(LDS-plane kernel, bs_group_check.cpp) and RunCompiler::schedule
(register-plane kernel, rp_program_check.cpp).  Random phase/permutation op
lists are scheduled, replayed with the kernel's semantics on random bit planes
and compared with one-by-one application in the original order.  No GPU
needed: the harnesses are built for the host only.  Also checks the build's
guard on the register-plane kernel's assembly."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("bsc") / "bs_group_check")
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17", "-o", exe,
           os.path.join(HERE, "bs_group_check.cpp"),
           os.path.join(ROOT, "paper_2105_01533_amd", "csrc", "run_compiler.hip")]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def test_grouped_ops_match_sequential(harness):
    r = subprocess.run([harness, "400"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr


@pytest.fixture(scope="module")
def rp_harness(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rpc") / "rp_program_check")
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17", "-o", exe,
           os.path.join(HERE, "rp_program_check.cpp"),
           os.path.join(ROOT, "paper_2105_01533_amd", "csrc", "run_compiler.hip")]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def test_register_plane_programs_match_sequential(rp_harness):
    r = subprocess.run([rp_harness, "400"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr


def test_regplane_asm_guard():
    """The build rejects compiler code that names a reserved VGPR or M0, or
    spills, in the register-plane kernel, and accepts the same registers
    inside inline assembly."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2105_01533_amd.build import check_regplane_asm

    ok = "\t;;#ASMSTART\n\tv_xor_b32 v100, v100, v86\n\ts_set_gpr_idx_on s4, gpr_idx(SRC0)\n\t;;#ASMEND\n" \
         "\tv_add_u32_e32 v1, v2, v79\n; ScratchSize: 0\n"
    assert check_regplane_asm(ok) == []
    assert check_regplane_asm("\tv_mov_b32_e32 v80, v1\n")
    assert check_regplane_asm("\tglobal_load_dwordx4 v[78:81], v2, s[0:1]\n")
    assert check_regplane_asm("\ts_mov_b32 m0, s4\n")
    assert check_regplane_asm("; ScratchSize: 16\n")
