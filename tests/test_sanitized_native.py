"""The C oracle and the library's host-side planning, built with the address
and undefined-behaviour sanitizers and run on the CPU.

Two small programs under tests/native/ drive them: one runs every entry point
of oracle/fcref.c on random instances (and checks that projected rows lie on
the simplex and that the structured loss equals the double-sum definition),
the other checks the row-pointer validation, the long-row plan of the sparse
product and the fused kernel's grid rule (paper_2506_04045_amd/csrc/fc_host.hpp).
Any sanitizer report ends the program with a non-zero status.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(exe):
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    return res.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["gcc", "-std=c99", "-fopenmp", *SAN,
                           os.path.join(NATIVE, "oracle_check.c"),
                           os.path.join(ROOT, "oracle", "fcref.c"), "-lm", "-o", exe])
    assert "all checks passed" in _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_logic_check")
    subprocess.check_call(["g++", "-std=c++17", *SAN,
                           "-I", os.path.join(ROOT, "paper_2506_04045_amd", "csrc"),
                           os.path.join(NATIVE, "host_logic_check.cpp"), "-o", exe])
    assert "all checks passed" in _run(exe)
