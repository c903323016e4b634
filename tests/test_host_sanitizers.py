"""The host-side moment-matrix builder under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): tests/host/dvm_host_check.cpp drives paper_1411_6697_amd/csrc/dvm_host.cpp for
the velocity sets of the paper's runs and a degenerate one; any memory error or undefined
behaviour aborts the driver."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1411_6697_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_moment_matrix_builder_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "dvm_host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "host", "dvm_host_check.cpp"),
           os.path.join(CSRC, "dvm_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
