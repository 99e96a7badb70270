"""Host code built with AddressSanitizer and UndefinedBehaviorSanitizer (no
GPU): the CPU oracle, driven through every entry point on small lattices of
all three models, and the serving arena allocator's randomised check.  Any
invalid access, leak or undefined operation makes the run fail."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1612_08312_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("compiler has no sanitizer runtime")
    assert r.returncode == 0, r.stderr


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _build(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-o", exe, os.path.join(ROOT, "oracle", "pyro_oracle.c"),
            os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-lm"])
    out = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "oracle sanitize ok" in out.stdout
    assert "runtime error" not in out.stderr


def test_arena_under_sanitizers(tmp_path):
    exe = str(tmp_path / "arena_san")
    _build(["g++", "-std=c++17", *SAN, "-I", CSRC, os.path.join(ROOT, "tests", "arena_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "arena ok" in out.stdout
    assert "runtime error" not in out.stderr
