"""GPU parity of the element-interior fast-diagonalization preconditioner.

Against the oracle (oracle/fdm.py):
  * z = M^-1 r (nek_precond_apply): FP64 within 1e-12 of max|z| (the 1-D
    modes come from different eigensolvers and agree to rounding), FP32
    within 1e-5;
  * FP64 CG with it, 100 fixed iterations: same iteration count, x within
    1e-12 relative, or 10x the oracle's own movement when its diagonal moves
    by one ulp where the loop amplifies rounding;
  * converged solves in every precision: the oracle's true FP64 residual of
    the GPU's x <= tol, FP64 iteration count within 1 of the oracle's, far
    fewer iterations than CG.
"""
import numpy as np
import pytest

import oracle
from oracle import fdm
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


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [(5, (3, 2, 2), 0.0, (1.5, 0.5, 1.0)), (7, (2, 3, 2), 0.1, None), (9, (2, 2, 2), 0.1, None),
         (1, (3, 2, 2), 0.0, None), (2, (2, 2, 3), 0.1, None), (11, (2, 1, 2), 0.1, None), (15, (1, 2, 1), 0.1, None)]


@pytest.mark.parametrize("N,nel,perturb,hi", CASES)
def test_apply_matches_oracle(N, nel, perturb, hi):
    vtx = synth.box_vertices(nel, hi=hi, perturb=perturb, seed=5)
    _case(f"precond_apply fdm N={N} nel={nel}")
    ctx = nek.Context(nel, N, vtx=vtx, precond="fdm")
    P = oracle.Problem(N, nel, vtx)
    F = fdm.Fdm(P, vtx)
    r = (synth.uniform_load(P.nl, 40 + N) - 0.5) * P.mask
    ref = F.apply(r)
    z64 = ctx.precond_apply(torch.from_numpy(r).cuda()).cpu().numpy()
    z32 = ctx.precond_apply(torch.from_numpy(r.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    ref32 = F.apply(r.astype(np.float32).astype(np.float64))
    e64, e32 = rel(z64, ref), rel(z32, ref32)
    print(f"  fp64 err {e64:.2e}  fp32 err {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5
    ctx.close()


@pytest.mark.parametrize("N,nel,perturb,hi", CASES[:4])
def test_fixed_iterations_fp64(N, nel, perturb, hi):
    vtx = synth.box_vertices(nel, hi=hi, perturb=perturb, seed=5)
    _case(f"fdm PCG fp64 100 its N={N} nel={nel}")
    ctx = nek.Context(nel, N, vtx=vtx, precond="fdm")
    P = oracle.Problem(N, nel, vtx)
    F = fdm.Fdm(P, vtx)
    f = synth.uniform_load(P.nl, 41)
    x, st, h = ctx.cg_solve(torch.from_numpy(f).cuda(), tol=0.0, maxit=100, history=True)
    xo, ito, ho = fdm.pcg(P, f, F.apply, tol=0.0, maxit=100)
    # the oracle's own movement when its diagonal changes by one ulp
    eps = np.random.default_rng(0).integers(-1, 2, size=P.ng)
    F.m = F.m * (1 + eps[P.gid] * 2.0 ** -52)
    xs, _, hs = fdm.pcg(P, f, F.apply, tol=0.0, maxit=100)
    sx, sh = rel(xs, xo), float(np.max(np.abs(hs - ho)))
    xg = x.cpu().numpy()
    n = min(len(h), len(ho))
    excess = float(np.max(np.abs(h[:n] - ho[:n]) - np.maximum(1e-10 * ho[:n] + 1e-14, 10 * sh)))
    err = rel(xg, xo)
    print(f"  its gpu {st['iters']} oracle {ito}: x rel err {err:.2e} (sensitivity {sx:.1e}), "
          f"history excess {excess:.2e}")
    if ho[-1] > 1e-13:
        assert st["iters"] == ito
    else:
        assert abs(st["iters"] - ito) <= 2
    assert err <= max(1e-12, 10 * sx) and excess <= 0.0
    ctx.close()


@pytest.mark.parametrize("N,nel,perturb", [(7, (4, 4, 4), 0.0), (5, (3, 3, 2), 0.1), (9, (3, 2, 2), 0.1)])
def test_converged_all_precisions(N, nel, perturb):
    vtx = synth.box_vertices(nel, perturb=perturb, seed=7)
    P = oracle.Problem(N, nel, vtx)
    F = fdm.Fdm(P, vtx)
    f = synth.uniform_load(P.nl, 32)
    fd = torch.from_numpy(f).cuda()
    tol = 1e-8
    _, it_cg, _ = P.cg(f, tol=tol, maxit=5000)
    _, it_f, _ = fdm.pcg(P, f, F.apply, tol=tol, maxit=5000)
    assert it_f < 0.8 * it_cg
    for prec in ("fp64", "fp32", "bf16g"):
        _case(f"converged fdm PCG N={N} nel={nel} prec={prec}")
        ctx = nek.Context(nel, N, vtx=vtx, prec=prec, precond="fdm")
        x, st, _ = ctx.cg_solve(fd, tol=tol, maxit=5000, raise_on_noconv=True)
        res = P.true_residual(x.cpu().numpy(), f)
        print(f"  {prec}: {st['iters']} its ({st['outer_iters']} outer; oracle {it_f}, CG {it_cg}), "
              f"true residual {res:.3e}")
        assert res <= tol
        if prec == "fp64":
            assert abs(st["iters"] - it_f) <= 1
        ctx.close()


def test_switching_to_fdm_and_back():
    N, nel = 5, (3, 2, 2)
    vtx = synth.box_vertices(nel, perturb=0.1, seed=10)
    f = torch.from_numpy(synth.uniform_load(3 * 2 * 2 * 216, 34)).cuda()
    for prec in ("fp64", "fp32"):
        # one fixed kernel configuration for both contexts (no autotuning), so
        # their results can be compared bit for bit
        ctx = nek.Context(nel, N, vtx=vtx, prec=prec, elts_per_wg=-1)
        a, sa, _ = ctx.cg_solve(f, tol=1e-8, maxit=3000)
        a = a.clone()
        ctx.set_precond("fdm")
        b, sb, _ = ctx.cg_solve(f, tol=1e-8, maxit=3000)
        b = b.clone()
        ctx.set_precond("none")
        c, sc, _ = ctx.cg_solve(f, tol=1e-8, maxit=3000)
        fresh = nek.Context(nel, N, vtx=vtx, prec=prec, precond="fdm", elts_per_wg=-1)
        d, sd, _ = fresh.cg_solve(f, tol=1e-8, maxit=3000)
        print(f"  {prec}: none {sa['iters']} its, fdm {sb['iters']}, none again {sc['iters']}")
        assert torch.equal(a, c) and torch.equal(b, d) and sb["iters"] < sa["iters"]
        ctx.close()
        fresh.close()
