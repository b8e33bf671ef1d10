"""Host-only checks of the serving scheduler core (ring arenas, launch
planning, the admission / launch / retire pipeline) against a fake executor:
tests/serve_core_check.cpp, built here with g++ and the host sanitizers."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_serve_core_with_fake_executor(tmp_path):
    exe = tmp_path / "serve_core_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "paper_1208_0277_amd", "csrc"),
           os.path.join(ROOT, "tests", "serve_core_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=240)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "ALL OK" in r.stdout
