"""GPU parity of the in-kernel geometric factors (nek_set_geometry with
NEK_GSRC_TRILINEAR) against the FP64 CPU oracle, through the C ABI.

The kernels recompute G = w det(J) J^-1 J^-T per point from each element's
trilinear map; the oracle forms J by GLL differentiation of the mapped nodes
(Sect. 4.1, Fig. 2: g1..g6 of ax_e).  Both are exact for trilinear elements,
so the operators agree to rounding: FP64 within the stored-factor bound
(1e-12, max-norm relative), FP32 within 2e-6, as for the stored FP32 copy.
Solves are checked as the stored-factor ones: the oracle's true FP64
residual on the GPU's x and the iteration count within 1 of the oracle's.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11065_amd import nek, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MESHES = [(1, (2, 2, 2)), (2, (1, 1, 1)), (2, (3, 1, 2)), (3, (2, 3, 2)), (4, (3, 5, 2)), (5, (2, 2, 3)),
          (7, (4, 4, 4)), (9, (3, 2, 1)), (11, (2, 1, 2)), (12, (1, 2, 2)), (15, (1, 2, 1))]


def _case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nek.load()   # raises when libnek.so is missing: no fallback


def make(N, nel, perturb=0.1, seed=7, hi=None, prec="fp64", **kw):
    vtx = synth.box_vertices(nel, hi=hi, perturb=perturb, seed=seed)
    _case(f"setup N={N} nel={nel} perturb={perturb} prec={prec} geometry=trilinear")
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec, **kw)
    ctx.set_geometry("trilinear")
    return ctx, oracle.Problem(N, nel, vtx)


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("N,nel", MESHES)
def test_ax_fp64_trilinear(N, nel):
    ctx, P = make(N, nel)
    u = synth.uniform_load(P.nl, 200 + N) - 0.5
    _case(f"nek_ax_local / nek_ax fp64 trilinear N={N}")
    e1 = relmax(host(ctx.ax_local(dev(u))), P.ax_local(u))
    e2 = relmax(host(ctx.ax(dev(u))), P.A(u))
    print(f"  ax_local err {e1:.2e}  ax err {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12
    ctx.close()


@pytest.mark.parametrize("N,nel", [(1, (3, 2, 2)), (3, (2, 2, 3)), (5, (2, 3, 2)), (7, (4, 4, 4)), (9, (3, 2, 2)),
                                   (11, (2, 3, 2)), (12, (2, 1, 2)), (15, (1, 2, 1))])
def test_ax_fp32_trilinear(N, nel):
    ctx, P = make(N, nel, prec="fp32")
    u = synth.uniform_load(P.nl, 3) - 0.5
    u32 = dev(u, torch.float32)
    _case(f"nek_ax_local / nek_ax fp32 trilinear N={N}")
    e1 = relmax(host(ctx.ax_local(u32)).astype(np.float64), P.ax_local(u))
    e2 = relmax(host(ctx.ax(u32)).astype(np.float64), P.A(u))
    print(f"  fp32 ax_local err {e1:.2e}  ax err {e2:.2e}")
    assert e1 <= 2e-6 and e2 <= 2e-6
    ctx.close()


def test_geometry_switch_and_arguments():
    """Stored factors come back bit-identical after a trilinear call; unknown
    modes are refused; BF16-g keeps its stored factors."""
    ctx, P = make(7, (3, 2, 2))
    u = dev(synth.uniform_load(P.nl, 9) - 0.5)
    ctx.set_geometry("stored")
    a = host(ctx.ax(u))
    ctx.set_geometry("trilinear")
    t = host(ctx.ax(u))
    ctx.set_geometry("stored")
    b = host(ctx.ax(u))
    assert np.array_equal(a, b)
    print(f"  stored vs trilinear {relmax(t, a):.2e}")
    assert relmax(t, a) <= 1e-12
    with pytest.raises(nek.NekError):
        ctx.set_geometry(2)
    with pytest.raises(nek.NekError):
        ctx.set_geometry(-1)
    ctx.set_prec("bf16g")
    ctx.set_geometry("stored")
    u32 = u.float()
    s16 = host(ctx.ax_local(u32))
    ctx.set_geometry("trilinear")
    assert np.array_equal(host(ctx.ax_local(u32)), s16)
    ctx.close()


@pytest.mark.parametrize("N,nel,perturb", [(9, (6, 6, 6), 0.0), (7, (5, 3, 4), 0.1), (4, (3, 5, 2), 0.1)])
def test_cg_fp64_trilinear(N, nel, perturb):
    ctx, P = make(N, nel, perturb=perturb)
    f = synth.uniform_load(P.nl, 2)
    _case(f"cg fp64 trilinear N={N} nel={nel}")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000)
    xo, ito, _ = P.cg(f, tol=1e-8, maxit=3000)
    xh = host(x)
    rho = P.true_residual(xh, f)
    dx = np.linalg.norm(xh - xo) / np.linalg.norm(xo)
    print(f"  iters gpu {st['iters']} oracle {ito}  rho* {rho:.2e}  |dx|/|x| {dx:.2e}")
    assert st["status"] == 0 and abs(st["iters"] - ito) <= 1
    assert rho <= 1e-8 and dx <= 1e-9
    ctx.close()


@pytest.mark.parametrize("N,nel", [(9, (5, 4, 4)), (12, (2, 3, 2))])
def test_cg_mixed_trilinear(N, nel):
    """FP32 operator with in-kernel factors inside FP64 refinement (the FP64
    residual updates use the FP64 in-kernel factors): true residual 1e-8."""
    ctx, P = make(N, nel, prec="fp32")
    f = synth.uniform_load(P.nl, 4)
    _case(f"cg mixed fp32 trilinear N={N}")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=5000)
    xh = host(x)
    rho = P.true_residual(xh, f)
    xo, ito, _ = P.cg(f, tol=1e-8, maxit=5000)
    dx = np.linalg.norm(xh - xo) / np.linalg.norm(xo)
    print(f"  inner {st['iters']} outer {st['outer_iters']} (oracle {ito})  rho* {rho:.2e}  |dx|/|x| {dx:.2e}")
    assert st["status"] == 0 and rho <= 1e-8 and dx <= 1e-7
    ctx.close()


@pytest.mark.parametrize("pc", ["jacobi", "fdm"])
def test_pcg_trilinear(pc):
    """Preconditioned FP64 and mixed solves with in-kernel factors: FP64 within
    1 iteration of the oracle's PCG, both to a true residual of 1e-8."""
    from oracle import fdm as ofdm
    N, nel = 7, (4, 3, 3)
    ctx, P = make(N, nel)
    vtx = synth.box_vertices(nel, perturb=0.1, seed=7)
    f = synth.uniform_load(P.nl, 6)
    ctx.set_precond(pc)
    _case(f"pcg {pc} fp64 trilinear")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000)
    if pc == "jacobi":
        xo, ito, _ = P.pcg(f, P.diag(), tol=1e-8, maxit=3000)
    else:
        xo, ito, _ = ofdm.pcg(P, f, ofdm.Fdm(P, vtx).apply, tol=1e-8, maxit=3000)
    rho = P.true_residual(host(x), f)
    print(f"  fp64 iters gpu {st['iters']} oracle {ito}  rho* {rho:.2e}")
    assert st["status"] == 0 and abs(st["iters"] - ito) <= 1 and rho <= 1e-8
    ctx.set_prec("fp32")
    _case(f"pcg {pc} mixed trilinear")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=5000)
    rho = P.true_residual(host(x), f)
    print(f"  mixed inner {st['iters']} outer {st['outer_iters']}  rho* {rho:.2e}")
    assert st["status"] == 0 and rho <= 1e-8
    ctx.close()


def test_batch_refuses_trilinear():
    b = nek.Batch([{"nel": (2, 2, 2), "N": 5}, {"nel": (3, 2, 2), "N": 7}], prec="fp64")
    b.ctx[1].set_geometry("trilinear")
    fs = [torch.rand(n, dtype=torch.float64, device="cuda") for n in b.nl]
    _case("batch with a trilinear member")
    with pytest.raises(nek.NekError):
        b.solve(fs, tol=1e-8, maxit=100, graph=False)
    b.ctx[1].set_geometry("stored")
    xs, st, rc = b.solve(fs, tol=1e-8, maxit=1000, graph=False)
    assert rc == 0 and all(s["status"] == 0 for s in st)
    b.close()
