"""The host-side model build under AddressSanitizer and UndefinedBehaviorSanitizer.

Compiles host_model.cpp (pure C++, no HIP) with a small driver that feeds it
valid meshes (10 x 10 and 150 x 150 grids, self-collision on), malformed ones
(indices out of range, non-finite positions, zero masses, negative weights,
bad mesh obstacles, bad edges) and checks the documented return codes; the
sanitizers abort on any memory error or undefined behaviour.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_05306_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_model_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "host_model.cpp"), os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "failures: 0" in r.stdout
