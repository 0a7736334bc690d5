"""The library's host runtime built as plain C++ against a stub of the HIP API and run
under AddressSanitizer + UndefinedBehaviorSanitizer (tests/host_check.cpp): argument
validation, the chunked launch schedule and output binding of rd_step, the stop-decision
state machine (the same decide() the kernels call), serving admission / batching /
retirement, the adaptive step rule and context teardown (no leaks).  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = shutil.which("g++") or shutil.which("clang++")


@pytest.mark.skipif(CXX is None, reason="no host C++ compiler")
def test_runtime_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "tests", "hoststub"),
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2305_03945_amd", "csrc"),
           os.path.join(ROOT, "tests", "host_check.cpp"),
           os.path.join(ROOT, "paper_2305_03945_amd", "csrc", "runtime.cpp"), "-o", exe]
    b = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert b.returncode == 0, b.stdout
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "host checks passed" in r.stdout, r.stdout
