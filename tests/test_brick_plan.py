"""Host check of the hop kernels' tile traversal (``csrc/hop_common.h``):
the plans built for both-parity and even-odd launches, t-region launches and
the plain order visit every tile of a half lattice exactly once, the y-bands
of both-parity plans are whole rows within the band budget, and the band
counts are the ones the kernels were measured with (48^3x96: six FP64, three
FP32; 32^4: two FP64; none for binary16, for two-plane z-groups or for
even-odd launches).  The driver includes the library's headers and runs on
the host only (no GPU call)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_07557_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "native", "brick_check.hip")


def test_traversal_plans_visit_every_tile_once(tmp_path):
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and shutil.which(hipcc) is None:
        pytest.skip("no hipcc")
    exe = str(tmp_path / "brick_check")
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC, DRIVER,
                    "-o", exe], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    last = r.stdout.strip().splitlines()[-1].split()
    assert last[0] == "cases" and last[2] == "bad" and last[3] == "0", r.stdout
    assert int(last[1]) >= 50
