"""The library's host C++ (problem assembly, KL expansion, block cyclic
reduction factor, convection values, checkpoint files) built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on the Table 6.1
mesh; the run must be clean and its self-checks must pass."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_06785_amd", "csrc")

pytestmark = pytest.mark.slow


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_code_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "host_check.cpp"), os.path.join(CSRC, "host_setup.cpp"),
           os.path.join(CSRC, "checkpoint.cpp"), "-pthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "0 failures" in r.stdout
