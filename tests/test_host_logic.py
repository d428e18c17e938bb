"""Host-side native logic on the CPU: the budget arena of the runtime,
compiled with g++ from its header and exercised by a randomised test."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena(tmp_path):
    exe = str(tmp_path / "arena_test")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-I", os.path.join(ROOT, "paper_2008_03095_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "arena_test.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "arena ok" in r.stdout
