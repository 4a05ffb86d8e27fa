"""Build ``libpotato.so`` (the C ABI of include/potato.h) for gfx950 with hipcc.

The library is built in-tree, next to this file, so the binding finds it
without any install step.  hipcc cross-compiles without a GPU present.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpotato.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "collide.hip", "abi.hip", "pipeline.hip")]
ARCH = os.environ.get("POTATO_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for every HIP translation unit; the
# compiler otherwise forms them from plain float code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


# roctx ranges name each entry point in marker traces.
LIBS = ["-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC or install ROCm)")


def build_library(verbose: bool = False) -> str:
    """Compile the sources into libpotato.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-I", INCLUDE, *SOURCES, *LIBS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpotato.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
