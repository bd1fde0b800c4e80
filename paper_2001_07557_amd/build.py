"""Build liblqcd.so (HIP, gfx950) in-tree.

Every ``csrc/*.hip`` translation unit is compiled with hipcc for gfx950 and
linked into ``paper_2001_07557_amd/liblqcd.so``.  Packed FP32 instructions
are disabled for all device code.  Run ``python -m paper_2001_07557_amd.build``
or call :func:`build`.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblqcd.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build liblqcd.so")


COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, verbose: bool, out_dir: str, defines) -> str:
    obj = os.path.join(out_dir, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc(), *COMMON, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines:
            print("\n".join(lines), file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int = 8, defines=(), lib_path: str = LIB,
          out_dir: str = OUT_DIR) -> str:
    """Compile every HIP source and link liblqcd.so; returns the library path.

    `defines` (NAME=VALUE strings) select kernel-shape options of the sources;
    the defaults in the sources are the shipped configuration."""
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, out_dir, defines), srcs))
    tmp = lib_path + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="build liblqcd.so for gfx950")
    ap.add_argument("-D", dest="defines", action="append", default=[],
                    help="NAME=VALUE kernel option (ablation builds)")
    ap.add_argument("--out", default=None, help="directory for an ablation build "
                    "(default: the in-tree library)")
    a = ap.parse_args()
    if a.out:
        print(build(verbose=True, defines=a.defines, lib_path=os.path.join(a.out, "liblqcd.so"),
                    out_dir=os.path.join(a.out, "obj")))
    else:
        print(build(verbose=True, defines=a.defines))
