"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the FP64 oracle and the library's host planner, each built with the
host compiler into a small test program (tests/sanitize/) and run.  Memory
errors, leaks and undefined behaviour end the program with a report."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def run(cmd, **kw):
    return subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    b = run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"),
             "-lm", "-o", exe])
    assert b.returncode == 0, b.stdout
    r = run([exe], env=ENV, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failures" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="g++ or the HIP runtime library not available")
def test_host_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_san")
    csrc = os.path.join(ROOT, "paper_2602_11709_amd", "csrc")
    b = run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__=1", "-I/opt/rocm/include", "-I", csrc,
             os.path.join(csrc, "api.cpp"), os.path.join(ROOT, "tests", "sanitize", "launch_stubs.cpp"),
             os.path.join(ROOT, "tests", "sanitize", "planner_main.cpp"), "-L/opt/rocm/lib", "-lamdhip64",
             "-Wl,-rpath,/opt/rocm/lib", "-lpthread", "-o", exe])
    assert b.returncode == 0, b.stdout
    r = run([exe], env=ENV, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failures" in r.stdout
