"""Sanitizer builds, CPU only: the FP64 oracle and the C ABI's host-side
argument checks, each compiled with AddressSanitizer and
UndefinedBehaviorSanitizer and run over every entry point or check
(tests/sanitize/).  No device code is built or run."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def run(exe, **env):
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, **env))
    out = p.stdout + p.stderr
    assert p.returncode == 0 and "ERROR: AddressSanitizer" not in out and \
        "runtime error" not in out, out[-3000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_run")
    subprocess.check_call(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off",
                           os.path.join(ROOT, "tests", "sanitize", "oracle_run.c"),
                           "-o", exe, "-lm"])
    assert "ok" in run(exe, OMP_NUM_THREADS="2")


def test_host_argument_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-Wall",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2306_09537_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
                           "-o", exe])
    assert "ok (0 failures)" in run(exe)
