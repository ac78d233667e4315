"""Host-side check of the bit-sliced pass's op scheduler (RunCompiler::group):
random phase/permutation op lists are grouped, replayed with the kernel's group
semantics on random bit planes and compared with one-by-one application in the
original order (bs_group_check.cpp).  No GPU needed: the harness is built for
the host only."""
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
