"""The oracle's 23-bit emulation against the GPU's own FP32 inner CG.

The emulation harness (oracle/nek_vprec.c) predicts how far a CG loop whose
operator, dssum and vector updates round to 23 mantissa bits, with FP64
dot products and scalars, can push the true FP64 residual: its recursive
residual reaches the tolerance while the true one stalls orders of
magnitude above it.  The GPU's mixed solver runs exactly that loop inside
its refinement; with a single refinement step and the inner tolerance set
to the outer one, its returned true residual must show the same stall, at
the level the emulation predicts (within a factor of 5: the GPU fuses
multiply-adds and sums copies in FP64 before rounding, so the two agree
in magnitude, not bit for bit).  The emulation rounds every vector update,
the iterate's included, so the GPU runs with its FP32-stored correction
(corr_fp32), the layout the emulation models.  Each check also runs with
the persistent grid capped at 3 workgroups, so that every workgroup walks
several element groups, the path the kernels take at full size.  With
refinement allowed the same solve must reach the tolerance.
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


@pytest.mark.parametrize("cap", [0, 3])
def test_fp32_inner_cg_stall_matches_emulation(cap):
    nel, N, tol = (4, 4, 4), 7, 1e-8
    vtx = synth.box_vertices(nel)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, synth.SEED_C1)
    print(f"[case] 4^3 N=7 f seed {synth.SEED_C1}: emulated 23-bit CG loop, FP64 dots", flush=True)
    xe, ite, he = oracle.vprec_cg(N, nel, vtx, f, t=(52, 23, 23, 52), mode="rne", tol=tol, maxit=3000)
    emu = P.true_residual(xe, f)
    print(f"emulation: {ite} its, recursive {he[-1]:.3e}, true {emu:.3e}", flush=True)
    assert he[-1] <= tol and emu > 100 * tol

    fd = torch.from_numpy(f).cuda()
    one = nek.Context(nel, N, vtx=vtx, prec="fp32", inner_tol=tol, max_outer=1, corr_fp32=1)
    one.set_max_workgroups(cap)
    x, st, _ = one.cg_solve(fd, tol=tol, maxit=3000)
    torch.cuda.synchronize()
    gpu = P.true_residual(x.cpu().numpy(), f)
    print(f"GPU one refinement step: {st['iters']} inner its, returned {st['true_rel_res']:.3e}, oracle {gpu:.3e}",
          flush=True)
    assert st["outer_iters"] == 1
    assert gpu == pytest.approx(st["true_rel_res"], rel=1e-6)
    assert emu / 5 <= gpu <= emu * 5
    assert abs(st["iters"] - ite) <= 0.1 * ite

    full = nek.Context(nel, N, vtx=vtx, prec="fp32")
    full.set_max_workgroups(cap)
    x, st, _ = full.cg_solve(fd, tol=tol, maxit=3000, raise_on_noconv=True)
    res = P.true_residual(x.cpu().numpy(), f)
    print(f"GPU refinement: {st['outer_iters']} steps, {st['iters']} its, oracle true residual {res:.3e}", flush=True)
    assert res <= tol
    one.close()
    full.close()


@pytest.mark.parametrize("cap", [0, 3])
def test_fp32_inner_pcg_stall_matches_emulation(cap):
    """The same with the diagonal (Jacobi) preconditioner: the 23-bit
    preconditioned loop stalls too, the GPU's FP32 inner PCG at the level the
    emulation predicts (factor 5), and refinement removes the stall."""
    nel, N, tol = (4, 4, 4), 7, 1e-8
    vtx = synth.box_vertices(nel)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, synth.SEED_C1)
    m = P.diag()
    print(f"[case] 4^3 N=7 f seed {synth.SEED_C1}: emulated 23-bit PCG loop, FP64 dots", flush=True)
    xe, ite, he = oracle.vprec_cg(N, nel, vtx, f, t=(52, 23, 23, 52), mode="rne", tol=tol, maxit=3000, m=m)
    emu = P.true_residual(xe, f)
    print(f"emulation: {ite} its, recursive {he[-1]:.3e}, true {emu:.3e}", flush=True)
    assert he[-1] <= tol and emu > 100 * tol

    fd = torch.from_numpy(f).cuda()
    one = nek.Context(nel, N, vtx=vtx, prec="fp32", inner_tol=tol, max_outer=1, precond="jacobi", corr_fp32=1)
    one.set_max_workgroups(cap)
    x, st, _ = one.cg_solve(fd, tol=tol, maxit=3000)
    gpu = P.true_residual(x.cpu().numpy(), f)
    print(f"GPU one refinement step: {st['iters']} inner its, returned {st['true_rel_res']:.3e}, oracle {gpu:.3e}",
          flush=True)
    assert st["outer_iters"] == 1
    assert emu / 5 <= gpu <= emu * 5
    assert abs(st["iters"] - ite) <= 0.1 * ite

    full = nek.Context(nel, N, vtx=vtx, prec="fp32", precond="jacobi")
    full.set_max_workgroups(cap)
    x, st, _ = full.cg_solve(fd, tol=tol, maxit=3000, raise_on_noconv=True)
    res = P.true_residual(x.cpu().numpy(), f)
    print(f"GPU refinement: {st['outer_iters']} steps, {st['iters']} its, oracle true residual {res:.3e}", flush=True)
    assert res <= tol
    one.close()
    full.close()
