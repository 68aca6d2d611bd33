"""Build libnek.so in-tree for gfx950 with hipcc.

    python -m paper_2405_11065_amd.build

Every HIP translation unit is compiled for gfx950 only, with packed-FP32
instructions disabled, and the resulting device code is scanned for stores
through the scalar data cache (the build fails if any appear).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libnek.so")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
SOURCES = [os.path.join(CSRC, "nek_lib.hip"), os.path.join(CSRC, "nek_setup.cpp")]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: libnek needs ROCm's hipcc to build")


def build(verbose: bool = False) -> str:
    """Compile libnek.so (always recompiles) and check its device code."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-shared", "-o", tmp, *SOURCES, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    check = os.path.join(PKG, "isa_check.py")
    if os.path.exists(check):
        sys.path.insert(0, PKG)
        try:
            import isa_check  # noqa: E402
            isa_check.check_sources(hipcc(), HIP_FLAGS + ["-I", INCLUDE, "-I", CSRC],
                                    [s for s in SOURCES if s.endswith(".hip")])
        finally:
            sys.path.pop(0)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
