"""Build libcsot.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

Every source under csrc/ goes into one shared library next to this file.  Packed-FP32 VALU
instructions are disabled for device code (the host pass warns that it does not know the
feature; that warning is harmless).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcsot.so")
ARCH = os.environ.get("CSOT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    srcs += sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")))
    return srcs


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source into libcsot.so; returns the library path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libcsot.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
