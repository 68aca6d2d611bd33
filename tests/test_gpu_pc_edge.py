"""Edge cases of the preconditioned solves (diagonal and fast
diagonalization), in FP64 and mixed precision: exact initial guess, zero
load, iteration cap, non-finite load, run-to-run determinism, the
reliable-update refinement, and the high orders (whose operator kernel keeps
D in LDS and whose block-solve kernel runs 14^3-node interiors).  Converged
results are judged by the oracle's true FP64 residual."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("pc", ["jacobi", "fdm"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_preconditioned_edge_cases(pc, prec):
    N, nel = 5, (3, 3, 3)
    vtx = synth.box_vertices(nel, perturb=0.1, seed=7)
    P = oracle.Problem(N, nel, vtx)
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec, precond=pc)
    f = synth.uniform_load(P.nl, 9)
    xo, _, _ = P.cg(f, tol=1e-12, maxit=3000)
    _case(f"{pc} {prec} converged")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000)
    assert st["status"] == 0 and P.true_residual(x.cpu().numpy(), f) <= 1e-8
    _case(f"{pc} {prec} determinism")
    x2, st2, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000)
    assert torch.equal(x, x2) and st2["iters"] == st["iters"]
    _case(f"{pc} {prec} maxit 3 after a converged run")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-12, maxit=3)
    assert st["iters"] == 3 and st["status"] == nek.NEK_NOCONV
    _case(f"{pc} {prec} exact x0")
    x, st, _ = ctx.cg_solve(dev(f), x0=dev(xo), tol=1e-8, maxit=50)
    assert st["iters"] == 0 and st["status"] == 0
    _case(f"{pc} {prec} zero load")
    x, st, _ = ctx.cg_solve(dev(np.zeros(P.nl)), tol=1e-8, maxit=10)
    assert st["iters"] == 0 and not x.cpu().numpy().any()
    _case(f"{pc} {prec} non-finite load")
    fn = f.copy()
    fn[int(np.flatnonzero(P.mask)[100])] = np.nan   # an unmasked node (the mask would zero a Dirichlet one)
    with pytest.raises(nek.NekError) as ei:
        ctx.cg_solve(dev(fn), tol=1e-8, maxit=10)
    assert ei.value.status == nek.NEK_E_NONFINITE
    _case(f"{pc} {prec} converged again after the errors")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000)
    assert st["status"] == 0 and P.true_residual(x.cpu().numpy(), f) <= 1e-8
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16g"])
def test_fdm_reliable_update(prec):
    N, nel = 7, (3, 3, 3)
    vtx = synth.box_vertices(nel, perturb=0.1, seed=9)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 33)
    _case(f"fdm reliable update {prec}")
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec, precond="fdm", refine_mode=2)
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=5000, raise_on_noconv=True)
    res = P.true_residual(x.cpu().numpy(), f)
    print(f"  {st['iters']} its, {st['outer_iters']} outer, {st['fp64_iters']} FP64, true residual {res:.3e}")
    assert res <= 1e-8
    ctx.close()


@pytest.mark.parametrize("N,nel", [(12, (2, 1, 2)), (15, (1, 2, 1)), (13, (1, 1, 2))])
@pytest.mark.parametrize("pc", ["jacobi", "fdm"])
def test_high_orders(N, nel, pc):
    vtx = synth.box_vertices(nel, perturb=0.1, seed=11)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 35)
    for prec in ("fp64", "fp32"):
        _case(f"{pc} N={N} {prec}")
        ctx = nek.Context(nel, N, vtx=vtx, prec=prec, precond=pc)
        x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=5000, raise_on_noconv=True)
        res = P.true_residual(x.cpu().numpy(), f)
        print(f"  {st['iters']} its, true residual {res:.3e}")
        assert res <= 1e-8
        ctx.close()


@pytest.mark.parametrize("pc", ["jacobi", "fdm"])
def test_tuning_with_preconditioner(pc):
    """The autotuner starts its timing runs as a solve does (z = M^-1 r), so
    the preconditioned kernels never read a z vector nothing has written:
    every configuration gives a finite time of a whole iteration (none of
    the runs ends at once on a non-finite value), and the tuned context
    solves to the tolerance."""
    N, nel = 9, (4, 4, 4)
    vtx = synth.box_vertices(nel, perturb=0.1, seed=13)
    P = oracle.Problem(N, nel, vtx)
    f = dev(synth.uniform_load(P.nl, 36))
    ctx = nek.Context(nel, N, vtx=vtx, prec="fp32", precond=pc)
    _case(f"tune with {pc}")
    best, us = ctx.tune("fp32", iters=8)
    print(f"  us per iteration {[round(u, 1) for u in us]}, best {best}")
    assert all(np.isfinite(u) and u > 0 for u in us)
    # each configuration runs a whole iteration: none of them ends at once
    assert min(us) > 0.3 * max(us)
    x, st, _ = ctx.cg_solve(f, tol=1e-8, maxit=5000, raise_on_noconv=True)
    assert P.true_residual(x.cpu().numpy(), f.cpu().numpy()) <= 1e-8
    ctx.close()
