"""Semantics of the C-ABI options and statistics, through the C ABI.

  * nek_opts.elts_per_wg: 0 autotunes at the first solve of a precision,
    > 0 picks the configuration with that many elements per workgroup (an
    order without one is refused at set-up), -1 keeps the order's default;
    nek_set_variant overrides it.
  * nek_stats: true_rel_res is the FP64 true residual of the returned x
    (checked against the oracle's), last_rec_res the loop's last recursive
    residual.
  * Refinement stagnation: a refinement step that fails to halve the true
    residual ends the mixed solve with NEK_E_STAGNATION, or with the FP64
    fallback from the current x when it is enabled.  The case is forced
    with one inner iteration per step: on this problem one CG step from
    x = 0 raises the residual norm (the oracle's first step gives 1.91x),
    which CG may do, since it minimises the energy norm of the error.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_elts_per_wg_option():
    nel, N = (4, 3, 3), 9
    f = dev(synth.uniform_load(36 * 1000, 3))
    _case("elts_per_wg = 2 at N=9")
    ctx = nek.Context(nel, N, elts_per_wg=2)
    for prec in ("fp64", "fp32", "bf16g"):
        assert ctx.get_variant(prec) == 2   # EPW options at N=9: 3 (variants 0, 1), 2 (2, 3), 1 (4, 5)
    ctx.cg_solve(f, tol=1e-8, maxit=2000, raise_on_noconv=True)
    assert ctx.get_variant("fp64") == 2   # fixed: no autotuning at the solve
    ctx.close()
    _case("elts_per_wg = 1 at N=9")
    ctx = nek.Context(nel, N, elts_per_wg=1)
    assert ctx.get_variant("fp64") == 4
    ctx.close()
    _case("elts_per_wg = 5 at N=9: no such configuration")
    with pytest.raises(nek.NekError) as ei:
        nek.Context(nel, N, elts_per_wg=5)
    assert ei.value.status == nek.NEK_E_ARG
    with pytest.raises(nek.NekError) as ei:
        nek.Context(nel, N, elts_per_wg=-2)
    assert ei.value.status == nek.NEK_E_ARG
    _case("elts_per_wg = -1: default configuration, untuned")
    ctx = nek.Context(nel, N, elts_per_wg=-1)
    ctx.cg_solve(f, tol=1e-8, maxit=2000, raise_on_noconv=True)
    assert ctx.get_variant("fp64") == 0
    ctx.close()
    _case("elts_per_wg = 0: autotuned at the first solve; set_variant overrides")
    ctx = nek.Context(nel, N, elts_per_wg=0)
    x, st, _ = ctx.cg_solve(f, tol=1e-8, maxit=2000, raise_on_noconv=True)
    v = ctx.get_variant("fp64")
    assert 0 <= v < ctx.num_variants()
    ctx.set_variant("fp64", 5)
    ctx.cg_solve(f, tol=1e-8, maxit=2000, raise_on_noconv=True)
    assert ctx.get_variant("fp64") == 5
    ctx.close()
    _case("batch with elts_per_wg = 1: every order has EPW 1 at N = 7 and 9")
    b = nek.Batch([{"nel": (2, 2, 3), "N": 7}, {"nel": (3, 2, 2), "N": 9}], elts_per_wg=1)
    assert b.get_variant("fp64", 0) == 4 and b.get_variant("fp64", 1) == 4
    b.close()
    with pytest.raises(nek.NekError):
        nek.Batch([{"nel": (2, 2, 2), "N": 9}, {"nel": (2, 2, 2), "N": 4}], elts_per_wg=2)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16g"])
def test_stats_residuals_against_oracle(prec):
    nel, N = (3, 3, 2), 7
    vtx = synth.box_vertices(nel, perturb=0.1, seed=5)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 6)
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec)
    _case(f"stats {prec}")
    x, st, hist = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000, history=True, raise_on_noconv=True)
    rho = P.true_residual(host(x), f)
    print(f"  true {st['true_rel_res']:.3e} oracle {rho:.3e} last recursive {st['last_rec_res']:.3e}")
    assert rho <= 1e-8 and st["true_rel_res"] <= 1e-8
    assert st["true_rel_res"] == pytest.approx(rho, rel=1e-3)
    assert st["last_rec_res"] == pytest.approx(hist[-1], rel=1e-12)
    if prec == "fp64":
        assert st["last_rec_res"] <= 1e-8
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16g"])
def test_refinement_stagnation_and_fp64_fallback(prec):
    nel, N, tol = (4, 4, 4), 7, 1e-8
    vtx = synth.box_vertices(nel)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, synth.SEED_C1)
    _, _, h = P.cg(f, tol=0.0, maxit=1)
    print(f"  oracle: one CG step takes the residual from {h[0]:.3f} to {h[1]:.3f}")
    assert h[1] > 0.5 * h[0]   # the premise of the forced stagnation
    fd = dev(f)
    _case(f"{prec}: one inner iteration per step, no fallback")
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec, inner_maxit=1, fp64_fallback=0)
    with pytest.raises(nek.NekError) as ei:
        ctx.cg_solve(fd, tol=tol, maxit=3000)
    assert ei.value.status == nek.NEK_E_STAGNATION
    ctx.close()
    _case(f"{prec}: one inner iteration per step, FP64 fallback")
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec, inner_maxit=1, fp64_fallback=1)
    x, st, _ = ctx.cg_solve(fd, tol=tol, maxit=3000, raise_on_noconv=True)
    rho = P.true_residual(host(x), f)
    print(f"  iters {st['iters']} outer {st['outer_iters']} fp64 {st['fp64_iters']} rho* {rho:.2e}")
    assert st["status"] == nek.NEK_OK and st["fp64_iters"] > 0
    assert st["iters"] == 1 + st["fp64_iters"] and st["outer_iters"] == 2
    assert rho <= tol
    ctx.close()
