"""Host integer phases under AddressSanitizer and UBSan (CPU only).

Compiles the host planning code (octree, partition, orderings, symbolic
fill) with the driver tests/host/plan_sanitize.cpp using g++ with
-fsanitize=address,undefined, and runs it: any out-of-bounds access, leak
or undefined behaviour on the awkward inputs it generates fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_13483_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_plan_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "plan_sanitize"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I" + CSRC, os.path.join(CSRC, "plan.cpp"),
           os.path.join(ROOT, "tests", "host", "plan_sanitize.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    # verify_asan_link_order=0: the sanitizer runtime need not come first
    # when the environment preloads another library
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "ok:" in p.stdout
