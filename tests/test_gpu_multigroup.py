"""Parity of the persistent CG kernels on the path they take at full size.

The CG operator and gather/update kernels run a capped grid of persistent
workgroups, each walking a contiguous share of the element groups: for every
group after its first a workgroup requests that group's first factor slices
(or trilinear coefficients) and reuses the LDS of the group before.  On the
small meshes of the other parity tests each workgroup takes one group, and
at full size (more than 2048 groups, 1024 for FP64 with in-kernel factors)
every workgroup takes several.  Here nek_set_max_workgroups caps the grid at
a few workgroups so that each walks at least two groups (a ragged share:
the group count is not a multiple of the cap), and the result is judged by
the FP64 oracle, for every kernel configuration of the order:
  * FP64: a fixed number of CG iterations (Table 1), x and the residual
    history element by element <= 1e-12 relative;
  * FP32 operator (one refinement step of exactly that many inner
    iterations): x against the oracle's FP64 iterations, bounded by 10x the deviation
    of the oracle's own 23-bit emulation of that loop (operator, dssum and
    vector updates rounded to binary32's 23 bits, FP64 dots and scalars);
  * BF16-stored factors: the same against the oracle run with its factors
    rounded to bfloat16 (nearest even, from FP64, as the library rounds them).
A mistake in the multi-group walk (a stale factor slice, a group skipped or
walked twice, LDS reused too early) changes x at O(1).

The meshes: the 4^3 N=7 unit-cube box for 100 iterations, and deformed
meshes (interior vertices moved up to 10 %, so the factors differ from
element to element and a stale slice would show).  On the deformed meshes
finite-precision CG stops being reproducible to rounding after some tens of
iterations: the oracle itself, given factors changed by one ulp, moves x by
1e-12 after 60 iterations and 6e-6 after 100 at N=9.  So they run 60 (N=7)
and 40 (N=9) iterations, and each case first checks on the oracle that a
one-ulp change of the factors moves its x by at most 1e-14, the premise of
the 1e-12 bound.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as om
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


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# name: (N, nel, perturb, cap, iterations); the cap is at most a third of
# the smallest group count of any configuration of the order (EPW up to 4
# at N=7, 3 at N=9)
CASES = {"c1": (7, (4, 4, 4), 0.0, 3, 100), "n7def": (7, (4, 4, 4), 0.1, 3, 60),
         "n9def": (9, (4, 3, 3), 0.1, 5, 40)}


@pytest.fixture(scope="module")
def problems():
    out = {}
    for name, (N, nel, pert, cap, its) in CASES.items():
        vtx = synth.box_vertices(nel, perturb=pert, seed=70 + N)
        P = oracle.Problem(N, nel, vtx)
        f = synth.uniform_load(P.nl, synth.SEED_C1)
        xo, ito, ho = P.cg(f, tol=0.0, maxit=its)
        Pu = oracle.Problem(N, nel, vtx)
        Pu.g = Pu.g * (1.0 + 2.0 ** -52)
        xu, _, _ = Pu.cg(f, tol=0.0, maxit=its)
        sens = relmax(xu, xo)
        print(f"  {name}: oracle moved {sens:.1e} by a one-ulp change of g after {its} iterations", flush=True)
        assert sens <= 1e-14
        out[name] = (N, nel, vtx, P, f, xo, ho, cap, its)
    return out


@pytest.mark.parametrize("geom", ["stored", "trilinear"])
@pytest.mark.parametrize("case", list(CASES))
def test_fp64_multigroup_fixed_iterations(problems, case, geom):
    N, nel, vtx, P, f, xo, ho, cap, its = problems[case]
    ctx = nek.Context(nel, N, vtx=vtx, prec="fp64", elts_per_wg=-1)
    ctx.set_geometry(geom)
    fd = dev(f)
    for v in range(ctx.num_variants()):
        for c in (0, cap):
            _case(f"fp64 {case} N={N} nel={nel} geom={geom} variant={v} cap={c} iterations={its}")
            ctx.set_variant("fp64", v)
            ctx.set_max_workgroups(c)
            x, st, hist = ctx.cg_solve(fd, tol=0.0, maxit=its, history=True)
            err = relmax(host(x), xo)
            herr = float(np.abs(hist - ho).max() / ho[0])
            print(f"  x err {err:.2e} history err {herr:.2e}", flush=True)
            assert st["iters"] == its and st["status"] == 0
            assert err <= 1e-12 and herr <= 1e-12
            # the FP64 solve reports the true residual of its x (formed once at exit)
            rho = P.true_residual(host(x), f)
            assert st["true_rel_res"] == pytest.approx(rho, rel=1e-9)
            assert st["last_rec_res"] == pytest.approx(hist[-1], rel=1e-12)
    ctx.close()


@pytest.fixture(scope="module")
def emulated(problems):
    """Deviation of the oracle's 23-bit emulated loop from FP64 after the case's iterations."""
    out = {}
    for name, (N, nel, vtx, P, f, xo, ho, cap, its) in problems.items():
        xe, ite, _ = oracle.vprec_cg(N, nel, vtx, f, t=(52, 23, 23, 52), mode="rne", tol=0.0, maxit=its)
        assert ite == its
        out[name] = relmax(xe, xo)
        print(f"  {name}: 23-bit emulation deviates {out[name]:.2e} from FP64 after {its} iterations", flush=True)
    return out


@pytest.mark.parametrize("corr", [0, 1])
@pytest.mark.parametrize("prec,geom", [("fp32", "stored"), ("fp32", "trilinear"), ("bf16g", "stored")])
@pytest.mark.parametrize("case", list(CASES))
def test_reduced_precision_multigroup_inner_iterations(problems, emulated, case, prec, geom, corr):
    N, nel, vtx, P, f, xo, ho, cap, its = problems[case]
    if prec == "bf16g":
        Pb = oracle.Problem(N, nel, vtx)
        Pb.g = om.bf16(Pb.g)
        ref, _, _ = Pb.cg(f, tol=0.0, maxit=its)
    else:
        ref = xo
    bound = 10 * emulated[case]
    # one refinement step of exactly `its` inner iterations from x = 0
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec, inner_tol=1e-300, inner_maxit=its, max_outer=1,
                      elts_per_wg=-1, corr_fp32=corr)
    ctx.set_geometry(geom)
    fd = dev(f)
    for v in range(ctx.num_variants()):
        for c in (0, cap):
            _case(f"{prec} {case} N={N} geom={geom} corr_fp32={corr} variant={v} cap={c} iterations={its}")
            ctx.set_variant(prec, v)
            ctx.set_max_workgroups(c)
            x, st, hist = ctx.cg_solve(fd, tol=1e-300, maxit=its, history=True)
            err = relmax(host(x), ref)
            print(f"  x err {err:.2e} (bound {bound:.2e}), true residual {st['true_rel_res']:.3e}", flush=True)
            assert st["iters"] == its and st["outer_iters"] == 1 and st["status"] == nek.NEK_NOCONV
            assert err <= bound
            # the inner loop's recursive residuals track the FP64 history
            assert float(np.abs(hist - ho).max() / ho[0]) <= 1e-2
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16g"])
def test_mixed_multigroup_converges(problems, prec):
    """Converged mixed solves at a cap, every configuration: oracle rho* <= tol."""
    N, nel, vtx, P, f, xo, ho, cap, its = problems["n9def"]
    ctx = nek.Context(nel, 9, vtx=vtx, prec=prec, elts_per_wg=-1)
    fd = dev(f)
    for v in range(ctx.num_variants()):
        _case(f"mixed {prec} N=9 variant={v} cap={cap}")
        ctx.set_variant(prec, v)
        ctx.set_max_workgroups(cap)
        x, st, _ = ctx.cg_solve(fd, tol=1e-8, maxit=5000, raise_on_noconv=True)
        rho = P.true_residual(host(x), f)
        print(f"  iters {st['iters']} outer {st['outer_iters']} rho* {rho:.2e} reported {st['true_rel_res']:.2e}")
        assert rho <= 1e-8
        # r = b - A x cancels to ~1e-9 of |b|: the two FP64 evaluations agree to ~1e-5 of it
        assert st["true_rel_res"] == pytest.approx(rho, rel=1e-3)
    ctx.close()


def test_max_workgroups_arguments():
    ctx = nek.Context((2, 2, 2), 5)
    for bad in (-1, 2049):
        with pytest.raises(nek.NekError) as ei:
            ctx.set_max_workgroups(bad)
        assert ei.value.status == nek.NEK_E_ARG
    ctx.set_max_workgroups(2048)
    ctx.set_max_workgroups(0)
    ctx.close()
    b = nek.Batch([{"nel": (2, 2, 2), "N": 5}])
    with pytest.raises(nek.NekError) as ei:
        b.ctx[0].set_max_workgroups(4)
    assert ei.value.status == nek.NEK_E_ARG
    b.close()
