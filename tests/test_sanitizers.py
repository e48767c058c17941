"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the C oracle, driven through every entry point by tests/oracle_check.c, and
the library's host-side logic (tests/host_logic_check.cpp: freeze decision,
held state after a divergence, workspace layout).  Device code is not
instrumented; the sanitizer flags apply to the host compilation only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=SAN_ENV)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr


def test_oracle_c_is_clean_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "gabp_oracle.c"),
           os.path.join(ROOT, "tests", "oracle_check.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    _run(exe)


def test_host_logic_is_clean_under_asan_and_ubsan(tmp_path):
    from paper_2404_12968_amd import build as B
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_logic_check")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [B.HIPCC, f"--offload-arch={B.ARCH}", "-std=c++17", "-g", "-O1"] + host_san + [
        "-I" + os.path.join(ROOT, "include"),
        "-I" + os.path.join(ROOT, "paper_2404_12968_amd", "csrc"),
        os.path.join(ROOT, "tests", "host_logic_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    _run(exe)
