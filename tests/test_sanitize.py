"""The host-side code under AddressSanitizer and UBSan (no device involved).

Two programs are built with the host compilers and run:
  * tests/native/host_checks.cpp with the library's host logic
    (paper_2311_05038_amd/csrc/fd_host.cpp: grid and shot validation,
    buffer layouts, the stability check, damping profiles, the kernel
    arguments of a shot on whole grids and z-slabs), over ordinary, edge and
    hostile inputs (sizes near 2^30 and INT64_MAX, overflowing receiver
    arrays, slabs off the grid);
  * tests/native/oracle_checks.c with the oracle (oracle/fd_oracle.c), every
    entry point over small grids and edge cases.
Any out-of-bounds access, leak, signed overflow or other undefined
behaviour aborts the program (-fno-sanitize-recover=all)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _run(cmd_build, exe, tmp_path):
    subprocess.run(cmd_build, check=True, cwd=tmp_path, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], cwd=tmp_path, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    out = _run(["g++", "-std=c++17", "-Wall", "-Wextra"] + SAN +
               [os.path.join(ROOT, "tests", "native", "host_checks.cpp"),
                os.path.join(ROOT, "paper_2311_05038_amd", "csrc", "fd_host.cpp"), "-o", exe],
               exe, tmp_path)
    assert "host checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    out = _run(["gcc", "-std=c11", "-Wall", "-Wextra", "-fopenmp"] + SAN +
               [os.path.join(ROOT, "tests", "native", "oracle_checks.c"),
                os.path.join(ROOT, "oracle", "fd_oracle.c"), "-o", exe, "-lm"],
               exe, tmp_path)
    assert "oracle checks passed" in out
