"""nek_ax_noalloc (the operator entry point that allocates nothing) against
nek_ax, through the C ABI.

Both run the same kernels in the same configuration, so the outputs must be
bit-identical; FP64 is also checked against the oracle's assembled operator
(1e-12, max-norm relative).  Two calls in a row share the library's static
scratch: the first on a larger mesh, the second on a smaller one, so the
second call finds the first call's data beyond its own range and must not
read it.  A vector larger than the scratch is refused with NEK_E_SCRATCH,
and a precision whose factor copy does not exist yet with NEK_E_ARG.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11065_amd import nek, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nek.load()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16g"])
def test_noalloc_matches_nek_ax_twice(prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    for nel, N, seed in (((6, 5, 4), 9, 11), ((3, 2, 2), 7, 12)):   # larger, then smaller
        vtx = synth.box_vertices(nel, perturb=0.1, seed=seed)
        _case(f"nek_ax_noalloc {prec} nel={nel} N={N}")
        ctx = nek.Context(nel, N, vtx=vtx, prec=prec)
        u = torch.from_numpy(synth.uniform_load(ctx.nl, seed)).to(device="cuda", dtype=dt)
        w_ref = ctx.ax(u)
        w = torch.full_like(u, float("nan"))
        ctx.ax_noalloc(u, w)
        a, b = host(w), host(w_ref)
        print(f"  identical entries {np.mean(a == b):.6f}", flush=True)
        assert np.array_equal(a, b)
        if prec == "fp64":
            P = oracle.Problem(N, nel, vtx)
            ref = P.A(host(u))
            err = float(np.abs(a - ref).max() / np.abs(ref).max())
            print(f"  vs oracle {err:.2e}", flush=True)
            assert err <= 1e-12
        ctx.close()


def test_noalloc_limits():
    _case("nek_ax_noalloc: FP64 vector of 9.26 M points (74 MB > 32 MiB)")
    ctx = nek.Context((21, 21, 21), 9)
    u = torch.zeros(ctx.nl, dtype=torch.float64, device="cuda")
    w = torch.empty_like(u)
    with pytest.raises(nek.NekError) as ei:
        ctx.ax_noalloc(u, w)
    assert ei.value.status == nek.NEK_E_SCRATCH
    ctx.close()
    _case("nek_ax_noalloc: FP32 on an FP64 context without the FP32 factor copy")
    ctx = nek.Context((2, 2, 2), 5, prec="fp64")
    u = torch.zeros(ctx.nl, dtype=torch.float32, device="cuda")
    with pytest.raises(nek.NekError) as ei:
        ctx.ax_noalloc(u, torch.empty_like(u))
    assert ei.value.status == nek.NEK_E_ARG
    ctx.set_prec("fp32")   # builds the copy; then the call runs
    ctx.ax_noalloc(u, torch.empty_like(u))
    torch.cuda.synchronize()
    ctx.close()
