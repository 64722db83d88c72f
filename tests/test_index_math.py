"""The kernels' index arithmetic (csrc/index_math.h: split-range plan, supertile keys and
masks, level-2 chunk bounds, backward pair slots) replayed on the host against brute-force
enumerations, built with the address and undefined-behaviour sanitizers (g++, CPU only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "index_math_check.cpp")
CSRC = os.path.join(ROOT, "paper_2603_11531_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_index_arithmetic_under_sanitizers(tmp_path):
    exe = tmp_path / "index_math_check"
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-I", CSRC, SRC, "-o", str(exe)]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the sanitizer runtime need not be the first library in the process
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
