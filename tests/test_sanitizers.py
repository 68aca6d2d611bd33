"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code.

tests/sanitize/host_driver.c calls every nek_host_* set-up routine of libnek
(csrc/nek_setup.cpp) and every routine of the oracle (nek_oracle.c,
nek_vprec.c) on box meshes of orders 1..15, each output buffer allocated at
exactly the size its header states.  Built with gcc/g++ (host code only; no
GPU code is involved) under -fsanitize=address,undefined with recovery off,
it must run to the end with no report and every cross-check agreeing.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="no host compiler")
def test_host_code_under_asan_ubsan(tmp_path):
    inc = os.path.join(ROOT, "include")
    objs = []
    for src, lang in [("tests/sanitize/host_driver.c", "c"), ("oracle/nek_oracle.c", "c"),
                      ("oracle/nek_vprec.c", "c"), ("paper_2405_11065_amd/csrc/nek_setup.cpp", "c++")]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cc = ["gcc", "-std=c11", "-ffp-contract=off"] if lang == "c" else ["g++", "-std=c++17"]
        _compile(cc + SAN + ["-I", inc, "-c", os.path.join(ROOT, src), "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    _compile(["g++", "-fsanitize=address,undefined"] + objs + ["-o", exe, "-lm", "-pthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert "all host checks passed" in r.stdout
