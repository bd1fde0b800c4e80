"""Host check of the multiply-and-shift integer division (``csrc/fastdiv.h``)
that the kernels use for site coordinates and the tile traversal: the header
is compiled with the host compiler into a small driver that compares every
quotient and remainder with the C++ operators over edge and random cases."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_07557_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "native", "fastdiv_check.cpp")


def test_fastdiv_matches_integer_division(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "fastdiv_check")
    # the header's __host__ __device__ qualifiers mean nothing to a host compiler
    subprocess.run([cxx, "-O2", "-std=c++17", "-D__host__=", "-D__device__=",
                    "-D__forceinline__=inline", "-I", CSRC, DRIVER, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout
    checks = int(r.stdout.split()[1])
    assert checks > 500_000
