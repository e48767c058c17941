"""Host-side logic of the library checked on the CPU (no GPU calls)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_freeze_decision_and_workspace_layout(tmp_path):
    """The precision-freeze decision (bitwise by default, else at most
    max_slots messages changed by at most max_rel each; 64-bit counts) and
    the workspace layout (256-byte aligned rows, planes and regions, the
    plane skew, disjoint regions)."""
    from paper_2404_12968_amd import build as B
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_logic_check")
    cmd = [B.HIPCC, f"--offload-arch={B.ARCH}", "-std=c++17",
           "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2404_12968_amd", "csrc"),
           os.path.join(ROOT, "tests", "host_logic_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
