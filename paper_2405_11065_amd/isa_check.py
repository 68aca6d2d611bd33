"""Build-time scan of libnek's gfx950 device assembly.

Fails the build when the device code writes through the scalar data cache
(scalar stores, scalar atomics, scalar-cache write-back or discard): all
device writes in libnek must be vector stores.  Also reports each kernel's
register, spill and LDS figures.  Runs on the build host only.
"""
from __future__ import annotations

import os
import re
import subprocess
import tempfile

FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic|s_dcache_wb|s_dcache_discard)", re.M)


def device_asm(hipcc: str, flags: list[str], src: str) -> str:
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "dev.s")
        subprocess.check_call([hipcc, *flags, "--cuda-device-only", "-S", "-o", out, src])
        with open(out) as fh:
            return fh.read()


def kernel_stats(asm: str):
    stats = {}
    for m in re.finditer(r"\.name:\s+(\S+)\n(.*?)(?=\n\s+- \.|\Z)", asm, re.S):
        body = m.group(2)
        def f(key):
            mm = re.search(r"\." + key + r":\s+(\d+)", body)
            return int(mm.group(1)) if mm else None
        stats[m.group(1)] = dict(vgpr=f("vgpr_count"), sgpr=f("sgpr_count"), spill=f("vgpr_spill_count"),
                                 lds=f("group_segment_fixed_size"), agpr=f("agpr_count"))
    return stats


def check_dir(build_dir: str, report: bool = False):
    """Scan the gfx950 device assembly that the compile kept in build_dir."""
    files = sorted(f for f in os.listdir(build_dir) if f.endswith(".s") and "amdgcn" in f)
    if not files:
        raise RuntimeError("no device assembly found to check")
    for f in files:
        asm = open(os.path.join(build_dir, f)).read()
        bad = FORBIDDEN.findall(asm)
        if bad:
            raise RuntimeError(f"{f}: device code writes through the scalar cache: {sorted(set(bad))}")
        if report:
            for name, st in sorted(kernel_stats(asm).items()):
                print(f"{st['vgpr']!s:>4} vgpr {st['sgpr']!s:>4} sgpr {st['spill']!s:>4} spill {st['lds']!s:>6} lds  {name}")


def check_sources(hipcc: str, flags: list[str], sources: list[str], report: bool = False):
    for src in sources:
        asm = device_asm(hipcc, flags, src)
        bad = FORBIDDEN.findall(asm)
        if bad:
            raise RuntimeError(f"{os.path.basename(src)}: device code writes through the scalar cache: {sorted(set(bad))}")
        if report:
            for name, st in sorted(kernel_stats(asm).items()):
                print(f"{st['vgpr']!s:>4} vgpr {st['agpr']!s:>4} agpr {st['sgpr']!s:>4} sgpr {st['spill']!s:>4} spill "
                      f"{st['lds']!s:>6} lds  {name}")


if __name__ == "__main__":
    check_dir(os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build"), report=True)
