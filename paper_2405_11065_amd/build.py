"""Build libnek.so in-tree for gfx950 with hipcc.

    python -m paper_2405_11065_amd.build

Every HIP translation unit (the order-independent driver and one unit per
polynomial order) is compiled for gfx950 only, with packed-FP32 instructions
disabled, in parallel; the device assembly kept from the compile is scanned
for stores through the scalar data cache (the build fails if any appear).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libnek.so")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    hip = [os.path.join(CSRC, f) for f in ("nek_lib.hip", "nek_batch.hip", "nek_mlp.hip", "nek_x0.hip")] + sorted(glob.glob(os.path.join(CSRC, "nek_np[0-9][0-9].hip")))
    return hip, [os.path.join(CSRC, "nek_setup.cpp")]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: libnek needs ROCm's hipcc to build")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", "-o", obj, src]
    if src.endswith(".hip"):
        cmd.insert(1, "-save-temps=obj")
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=BUILD, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile libnek.so (always recompiles) and check its device code."""
    os.makedirs(BUILD, exist_ok=True)
    for f in glob.glob(os.path.join(BUILD, "*")):
        os.remove(f)
    hip, cpp = sources()
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), hip + cpp))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc(), f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    check = os.path.join(PKG, "isa_check.py")
    if os.path.exists(check):
        sys.path.insert(0, PKG)
        try:
            import isa_check  # noqa: E402
            isa_check.check_dir(BUILD)
        finally:
            sys.path.pop(0)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
