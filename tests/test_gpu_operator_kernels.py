"""The two kernels of the plain operator pass (nek_set_operator_kernel):
the D contractions of local_grad3 / local_grad3_t on the matrix cores
against the oracle, at the orders where the choice between matrix cores and
vector ALUs was measured (N + 1 = 8, 10, 12) and at low orders:

  * FP64 nek_ax_local and nek_ax within 1e-12 of the oracle (max-norm,
    relative), FP32 within 2e-6, as the vector-ALU kernel;
  * BF16-stored factors: within 1e-6 of the vector-ALU kernel's result with
    the same factors (the two differ only in summation order);
  * every element walked by a persistent workgroup of several elements;
  * the choice refused above N + 1 = 12.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11065_amd import nek, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nek.load()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("N,nel", [(2, (3, 2, 2)), (4, (2, 3, 2)), (7, (4, 3, 3)), (9, (3, 4, 2)), (11, (2, 3, 3))])
def test_mfma_operator_matches_oracle(N, nel):
    vtx = synth.box_vertices(nel, perturb=0.1, seed=50 + N)
    P = oracle.Problem(N, nel, vtx)
    u = synth.uniform_load(P.nl, 200 + N) - 0.5
    ref, refA = P.ax_local(u), P.A(u)
    ctx = nek.Context(nel, N, vtx=vtx, prec="fp64")
    print(f"[case] operator kernels N={N} nel={nel}", flush=True)
    ctx.set_operator_kernel("mfma")
    e64 = relmax(host(ctx.ax_local(dev(u))), ref)
    a64 = relmax(host(ctx.ax(dev(u))), refA)
    u32 = dev(u, torch.float32)
    ctx.set_prec("fp32")
    e32 = relmax(host(ctx.ax_local(u32)).astype(np.float64), ref)
    a32 = relmax(host(ctx.ax(u32)).astype(np.float64), refA)
    ctx.set_prec("bf16g")
    m16 = host(ctx.ax_local(u32)).astype(np.float64)
    ctx.set_operator_kernel("valu")
    v16 = host(ctx.ax_local(u32)).astype(np.float64)
    e16 = relmax(m16, v16)
    print(f"  fp64 {e64:.2e} (assembled {a64:.2e})  fp32 {e32:.2e} (assembled {a32:.2e})  bf16-g vs valu {e16:.2e}")
    assert e64 <= 1e-12 and a64 <= 1e-12
    assert e32 <= 2e-6 and a32 <= 2e-6
    assert e16 <= 1e-6
    ctx.close()


def test_mfma_operator_refused_above_twelve_points():
    ctx = nek.Context((1, 1, 1), 12)
    with pytest.raises(nek.NekError) as ei:
        ctx.set_operator_kernel("mfma")
    assert ei.value.status == nek.NEK_E_ARG
    ctx.close()
