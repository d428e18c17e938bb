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


def _run_sanitized(cmd, exe):
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena_under_sanitizers(tmp_path):
    """The arena again, built with AddressSanitizer and UndefinedBehaviorSanitizer."""
    exe = str(tmp_path / "arena_san")
    r = _run_sanitized(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                        "-I", os.path.join(ROOT, "paper_2008_03095_amd", "csrc"),
                        os.path.join(ROOT, "tests", "cpp", "arena_test.cpp"), "-o", exe], exe)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "arena ok" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    """Every oracle entry point on small random graphs, built with
    AddressSanitizer and UndefinedBehaviorSanitizer (no ctypes: a C driver
    linked with oracle.c), with the results cross-checked."""
    exe = str(tmp_path / "oracle_san")
    r = _run_sanitized(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                        os.path.join(ROOT, "tests", "cpp", "oracle_san.c"), os.path.join(ROOT, "oracle", "oracle.c"),
                        "-o", exe, "-lpthread", "-lm"], exe)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle sanitizer run ok" in r.stdout
