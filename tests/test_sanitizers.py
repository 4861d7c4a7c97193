"""The host-side code (the GPU library's canonicalisation, bound check, packing and schedules, and
the oracle) built with the address and undefined-behaviour sanitizers and driven over fixtures
that reach its edges (no GPU; host compilers only)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe, tmp_path):
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stderr[-4000:]


def test_host_preparation_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_host")
    cmd = ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize_host.cpp"),
           os.path.join(ROOT, "paper_2511_17245_amd", "csrc", "sa_host.cpp"), "-o", exe]
    _run(cmd, exe, tmp_path)


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    cmd = ["gcc", "-std=gnu11", *SAN, "-ffp-contract=off", "-pthread",
           os.path.join(ROOT, "tests", "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "sa_oracle.c"),
           "-o", exe, "-lm"]
    _run(cmd, exe, tmp_path)
