"""The host-only parts of the library (instance compiler, width-set
planner) built with AddressSanitizer and UndefinedBehaviorSanitizer by g++
and driven by tests/sanitize/host_harness.cpp: valid and malformed
instances, planner bounds, and seeded random instances.  No GPU, no HIP."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_12037_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_compiler_and_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_harness")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", f"-I{ROOT}",
           os.path.join(ROOT, "tests", "sanitize", "host_harness.cpp"),
           os.path.join(CSRC, "compile.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host harness ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
