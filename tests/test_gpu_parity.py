"""GPU parity of libnek against the FP64 CPU oracle, through the C ABI.

Tolerances: integer maps and FP64 dssum bit-exact; GLL/D 1e-14 absolute
(D relative to max|D|); g and B 1e-13 of their scale; FP64 operator 1e-12
(max-norm, relative); glsc3 1e-12 relative; 100 fixed FP64 CG iterations
1e-12 relative on x.  Converged solves are judged by the oracle's true FP64
residual on the GPU's x (<= tol) and an iteration count within 1 of the
oracle's.  FP32 / BF16-g operators are compared with the FP64 oracle within
the rounding their storage implies.  Every check prints the error it saw.
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
    nek.load()   # raises when libnek.so is missing: no fallback


def make(N, nel, perturb=0.0, seed=7, hi=None, prec="fp64", want_X=False, **kw):
    vtx = synth.box_vertices(nel, hi=hi, perturb=perturb, seed=seed)
    _case(f"setup N={N} nel={nel} perturb={perturb} prec={prec}")
    ctx = nek.Context(nel, N, vtx=vtx, prec=prec, **kw)
    P = oracle.Problem(N, nel, vtx, want_X=want_X)
    return ctx, P


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


MESHES = [(1, (2, 2, 2)), (2, (3, 1, 2)), (3, (2, 3, 2)), (4, (3, 5, 2)), (5, (2, 2, 3)), (7, (4, 4, 4)),
          (9, (2, 2, 2)), (9, (3, 2, 1)), (11, (2, 1, 2)), (12, (1, 2, 2)), (15, (1, 2, 1))]


@pytest.mark.parametrize("N,nel", MESHES)
def test_setup_matches_oracle(N, nel):
    ctx, P = make(N, nel, perturb=0.1)
    xi, w = oracle.gll(N)
    assert np.abs(ctx.get(nek.NEK_GET_GLL) - xi).max() <= 1e-14
    assert np.abs(ctx.get(nek.NEK_GET_W) - w).max() <= 1e-14
    assert np.abs(ctx.get(nek.NEK_GET_D) - P.D).max() <= 1e-13 * np.abs(P.D).max()
    g = ctx.get(nek.NEK_GET_G)
    scale = np.abs(P.g[:, :3]).max()
    err_g = np.abs(g - P.g).max() / scale
    err_B = relmax(ctx.get(nek.NEK_GET_B), P.B.ravel())
    print(f"  g err {err_g:.2e}  B err {err_B:.2e}")
    assert err_g <= 1e-13 and err_B <= 1e-13
    assert np.array_equal(ctx.get(nek.NEK_GET_GID), P.gid)
    assert np.array_equal(ctx.get(nek.NEK_GET_MULT), P.mult)
    assert np.array_equal(ctx.get(nek.NEK_GET_MASK), P.mask)
    perm, ptr, flag = P.segments()
    assert np.array_equal(ctx.get(nek.NEK_GET_PERM), perm)
    assert np.array_equal(ctx.get(nek.NEK_GET_SEGPTR), ptr)
    assert np.array_equal(ctx.get(nek.NEK_GET_SEGFLAG), flag)
    ctx.close()


@pytest.mark.parametrize("N,nel", MESHES)
def test_ax_fp64(N, nel):
    ctx, P = make(N, nel, perturb=0.1)
    u = synth.uniform_load(P.nl, 100 + N) - 0.5
    _case(f"nek_ax_local fp64 N={N}")
    wl = host(ctx.ax_local(dev(u)))
    e1 = relmax(wl, P.ax_local(u))
    _case(f"nek_ax fp64 N={N}")
    wa = host(ctx.ax(dev(u)))
    e2 = relmax(wa, P.A(u))
    print(f"  ax_local err {e1:.2e}  ax err {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12
    ctx.close()


@pytest.mark.parametrize("N,nel", [(3, (2, 3, 2)), (7, (4, 4, 4)), (9, (3, 2, 2))])
def test_dssum_bit_exact(N, nel):
    ctx, P = make(N, nel)
    w = synth.uniform_load(P.nl, 5) - 0.5
    for masked in (False, True):
        _case(f"nek_dssum fp64 mask={masked}")
        got = host(ctx.dssum(dev(w), mask=masked))
        assert np.array_equal(got, P.dssum(w, masked=masked))
    # FP32: copies summed in FP64 in the same order, rounded once
    w32 = w.astype(np.float32)
    _case("nek_dssum fp32")
    got = host(ctx.dssum(dev(w32, torch.float32), mask=True))
    ref = P.dssum(w32.astype(np.float64), masked=True).astype(np.float32)
    assert np.array_equal(got, ref)
    ctx.close()


def test_glsc3():
    ctx, P = make(5, (3, 2, 4), perturb=0.1)
    a = synth.uniform_load(P.nl, 1) - 0.3
    b = synth.uniform_load(P.nl, 2)
    _case("nek_glsc3")
    got = ctx.glsc3(dev(a), dev(b))
    ref = P.glsc3(a, b)
    print(f"  glsc3 rel err {abs(got - ref) / abs(ref):.2e}")
    assert abs(got - ref) <= 1e-12 * abs(ref)
    got32 = ctx.glsc3(dev(a, torch.float32), dev(b, torch.float32))
    ref32 = P.glsc3(a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
    assert abs(got32 - ref32) <= 1e-12 * abs(ref32)
    ctx.close()


@pytest.mark.parametrize("N,nel", [(7, (4, 4, 4)), (9, (3, 2, 2)), (5, (2, 3, 2)), (11, (2, 3, 2)), (12, (2, 1, 2)),
                                   (15, (1, 2, 1))])
def test_ax_reduced_precision(N, nel):
    ctx, P = make(N, nel, perturb=0.1, prec="fp32")
    u = synth.uniform_load(P.nl, 3) - 0.5
    ref, refA = P.ax_local(u), P.A(u)
    u32 = dev(u, torch.float32)
    _case(f"nek_ax_local fp32 N={N}")
    e32 = relmax(host(ctx.ax_local(u32)).astype(np.float64), ref)
    _case(f"nek_ax fp32 N={N}")
    a32 = relmax(host(ctx.ax(u32)).astype(np.float64), refA)
    ctx.set_prec("bf16g")
    _case(f"nek_ax_local fp32/bf16-g N={N}")
    e16 = relmax(host(ctx.ax_local(u32)).astype(np.float64), ref)
    _case(f"nek_ax fp32/bf16-g N={N}")
    a16 = relmax(host(ctx.ax(u32)).astype(np.float64), refA)
    print(f"  fp32 err {e32:.2e} (assembled {a32:.2e})  bf16-g err {e16:.2e} (assembled {a16:.2e})")
    assert e32 <= 2e-6 and a32 <= 2e-6
    assert e16 <= 1e-2 and a16 <= 1e-2
    ctx.close()


def test_single_element_worked_example():
    """1 element, N=2, unit cube: x_centre = 9/64 for a unit load (hand derivation)."""
    ctx, P = make(2, (1, 1, 1))
    f = np.ones(P.nl)
    _case("cg single element")
    x, st, hist = ctx.cg_solve(dev(f), tol=1e-14, maxit=5, history=True)
    xh = host(x)
    assert st["iters"] == 1 and st["status"] == 0
    assert abs(xh[13] - 9.0 / 64.0) <= 1e-16
    ctx.close()


def test_cg_fp64_fixed_100_iterations():
    """4x4x4 unit-cube elements, N=7, f ~ U[0,1) (seed 1), 100 fixed iterations."""
    ctx, P = make(7, (4, 4, 4))
    f = synth.uniform_load(P.nl, synth.SEED_C1)
    _case("cg fp64 4^3 N=7 100 iterations")
    x, st, hist = ctx.cg_solve(dev(f), tol=0.0, maxit=100, history=True)
    xo, ito, ho = P.cg(f, tol=0.0, maxit=100)
    err = relmax(host(x), xo)
    herr = float(np.abs(hist - ho).max() / ho[0])
    print(f"  x err {err:.2e}  history err {herr:.2e}  res {hist[-1]:.3e}")
    assert st["iters"] == 100 and ito == 100 and st["status"] == 0
    assert err <= 1e-12
    assert herr <= 1e-12
    ctx.close()


@pytest.mark.parametrize("N,nel,perturb", [(9, (6, 6, 6), 0.0), (7, (5, 3, 4), 0.1), (4, (3, 5, 2), 0.1)])
def test_cg_fp64_converged(N, nel, perturb):
    ctx, P = make(N, nel, perturb=perturb)
    f = synth.uniform_load(P.nl, 2)
    _case(f"cg fp64 converge N={N} nel={nel}")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000)
    xo, ito, _ = P.cg(f, tol=1e-8, maxit=3000)
    xh = host(x)
    rho = P.true_residual(xh, f)
    dx = np.linalg.norm(xh - xo) / np.linalg.norm(xo)
    print(f"  iters gpu {st['iters']} oracle {ito}  rho* {rho:.2e}  |dx|/|x| {dx:.2e}")
    assert st["status"] == 0
    assert abs(st["iters"] - ito) <= 1
    assert rho <= 1e-8
    assert dx <= 1e-9
    ctx.close()


def test_cg_initial_guess_and_edge_cases():
    ctx, P = make(5, (3, 3, 3), perturb=0.1)
    f = synth.uniform_load(P.nl, 9)
    xo, ito, _ = P.cg(f, tol=1e-12, maxit=3000)
    _case("cg exact x0")
    x, st, _ = ctx.cg_solve(dev(f), x0=dev(xo), tol=1e-10, maxit=50)
    assert st["iters"] == 0 and st["status"] == 0
    _case("cg perturbed x0")
    x0 = xo + 1e-3 * synth.uniform_load(P.nl, 10)
    x, st, _ = ctx.cg_solve(dev(f), x0=dev(x0), tol=1e-10, maxit=3000)
    assert relmax(host(x), xo) <= 1e-8
    _case("cg x aliases x0")
    xa = dev(x0)
    x, st, _ = ctx.cg_solve(dev(f), x0=xa, x=xa, tol=1e-10, maxit=3000)
    assert relmax(host(xa), xo) <= 1e-8
    _case("cg zero load")
    x, st, _ = ctx.cg_solve(dev(np.zeros(P.nl)), tol=1e-8, maxit=10)
    assert st["iters"] == 0 and not host(x).any()
    _case("cg maxit reached")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-12, maxit=3)
    assert st["iters"] == 3 and st["status"] == nek.NEK_NOCONV
    _case("cg non-finite load")
    fn = f.copy()
    fn[123] = np.nan
    with pytest.raises(nek.NekError) as ei:
        ctx.cg_solve(dev(fn), tol=1e-8, maxit=10)
    assert ei.value.status == nek.NEK_E_NONFINITE
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16g"])
def test_mixed_edge_cases(prec):
    """Refinement edge cases; a run capped at 3 iterations right after a
    converged one checks that the finished run's done flag (which the kernels
    write to pinned host memory) cannot end the next run early."""
    ctx, P = make(5, (3, 3, 3), perturb=0.1, prec=prec)
    f = synth.uniform_load(P.nl, 9)
    xo, _, _ = P.cg(f, tol=1e-12, maxit=3000)
    _case(f"cg mixed {prec} converged")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-8, maxit=3000)
    assert st["status"] == 0 and P.true_residual(host(x), f) <= 1e-8
    _case(f"cg mixed {prec} maxit 3 after a converged run")
    x, st, _ = ctx.cg_solve(dev(f), tol=1e-12, maxit=3)
    assert st["iters"] == 3 and st["status"] == nek.NEK_NOCONV
    _case(f"cg mixed {prec} exact x0")
    x, st, _ = ctx.cg_solve(dev(f), x0=dev(xo), tol=1e-8, maxit=50)
    assert st["iters"] == 0 and st["status"] == 0
    _case(f"cg mixed {prec} zero load")
    x, st, _ = ctx.cg_solve(dev(np.zeros(P.nl)), tol=1e-8, maxit=10)
    assert st["iters"] == 0 and not host(x).any()
    ctx.close()


def test_cg_deterministic():
    ctx, P = make(7, (3, 3, 3), perturb=0.1)
    f = dev(synth.uniform_load(P.nl, 4))
    _case("cg determinism")
    a, sa, ha = ctx.cg_solve(f, tol=1e-8, maxit=2000, history=True)
    a = host(a).copy()
    b, sb, hb = ctx.cg_solve(f, tol=1e-8, maxit=2000, history=True)
    assert sa["iters"] == sb["iters"]
    assert np.array_equal(a, host(b)) and np.array_equal(ha, hb)
    ctx.close()


@pytest.mark.parametrize("prec,mode,N,nel", [("fp32", 0, 9, (5, 4, 4)), ("fp32", 1, 9, (5, 4, 4)),
                                             ("fp32", 2, 9, (5, 4, 4)), ("bf16g", 0, 9, (5, 4, 4)),
                                             ("bf16g", 2, 9, (5, 4, 4)), ("fp32", 0, 11, (3, 3, 2)),
                                             ("bf16g", 0, 11, (3, 3, 2)), ("fp32", 0, 12, (2, 3, 2)),
                                             ("fp32", 0, 15, (2, 2, 2))])
def test_mixed_precision_solve(prec, mode, N, nel):
    """Deformed [0,1]^3 mesh, manufactured forcing: the refined mixed solve
    (mode 1: restarted refinement, 2: reliable update, 0: default for the
    storage) reaches a true FP64 residual of 1e-8 (judged by the oracle)."""
    ctx, P = make(N, nel, perturb=0.1, seed=33, hi=(1.0, 1.0, 1.0), prec=prec, want_X=True, refine_mode=mode)
    noise = synth.normal_noise(P.nl, 1e-3, 34).reshape(P.E, -1)
    f_or = (P.B * (synth.sine_field(P.X) + noise)).ravel()
    Bg = ctx.get(nek.NEK_GET_B).reshape(P.E, -1)
    Xg = ctx.get(nek.NEK_GET_XYZ)
    f_gpu = (Bg * (synth.sine_field(Xg) + noise)).ravel()
    _case(f"cg mixed {prec} mode {mode} N={N}")
    x, st, hist = ctx.cg_solve(dev(f_gpu), tol=1e-8, maxit=5000, history=True)
    xh = host(x)
    rho = P.true_residual(xh, f_or)
    xo, ito, _ = P.cg(f_or, tol=1e-8, maxit=5000)
    dx = np.linalg.norm(xh - xo) / np.linalg.norm(xo)
    print(f"  {prec}: inner iters {st['iters']} outer {st['outer_iters']} fp64 {st['fp64_iters']} "
          f"(oracle fp64 {ito})  rho* {rho:.2e}  |dx|/|x| {dx:.2e}")
    assert st["status"] == 0
    assert rho <= 1e-8
    assert dx <= 1e-7
    ctx.close()


def manufactured_load(ctx, P, noise):
    """f = B (sin pi x sin pi y sin pi z + noise) for each side from its own B and X."""
    f_or = (P.B * (synth.sine_field(P.X) + noise)).ravel()
    Bg = ctx.get(nek.NEK_GET_B).reshape(P.E, -1)
    Xg = ctx.get(nek.NEK_GET_XYZ)
    return f_or, (Bg * (synth.sine_field(Xg) + noise)).ravel()


def test_full_size_16cubed_N9():
    """The benchmarked workload itself: 16^3 unit cubes, N=9, f ~ U[0,1) seed 2,
    tol 1e-8; FP64 and mixed solves judged by the oracle's true residual."""
    nel, N = (16, 16, 16), 9
    vtx = synth.box_vertices(nel)
    _case("setup 16^3 N=9")
    ctx = nek.Context(nel, N, vtx=vtx, prec="fp64")
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, synth.SEED_C2)
    fd = dev(f)
    res = {}
    for prec in ("fp64", "fp32"):
        ctx.set_prec(prec)
        ctx.tune(prec, iters=10)
        _case(f"cg 16^3 N=9 {prec}")
        x, st, _ = ctx.cg_solve(fd, tol=1e-8, maxit=20000)
        xh = host(x)
        res[prec] = (xh, st)
        rho = P.true_residual(xh, f)
        print(f"  {prec}: iters {st['iters']} outer {st['outer_iters']} rho* {rho:.2e}")
        assert st["status"] == 0 and rho <= 1e-8
    dx = np.linalg.norm(res["fp32"][0] - res["fp64"][0]) / np.linalg.norm(res["fp64"][0])
    print(f"  |x_mixed - x_fp64| / |x_fp64| = {dx:.2e}")
    assert dx <= 1e-6
    # factors recomputed in the kernels from the trilinear maps: 1366 element
    # groups over at most 1024 FP64 workgroups, so some walk two
    ctx.set_geometry("trilinear")
    for prec in ("fp64", "fp32"):
        ctx.set_prec(prec)
        ctx.tune(prec, iters=10)
        _case(f"cg 16^3 N=9 {prec} trilinear")
        x, st, _ = ctx.cg_solve(fd, tol=1e-8, maxit=20000)
        xh = host(x)
        rho = P.true_residual(xh, f)
        dx = np.linalg.norm(xh - res[prec][0]) / np.linalg.norm(res[prec][0])
        print(f"  {prec} trilinear: iters {st['iters']} rho* {rho:.2e} |x - x_stored|/|x_stored| {dx:.2e}")
        assert st["status"] == 0 and rho <= 1e-8 and dx <= 1e-6
    ctx.set_geometry("stored")
    # the preconditioners on the benchmarked workload, FP64 and mixed
    for pc in ("jacobi", "fdm", "schwarz"):
        ctx.set_precond(pc)
        for prec in ("fp64", "fp32"):
            ctx.set_prec(prec)
            ctx.tune(prec, iters=10)
            _case(f"cg 16^3 N=9 {prec} {pc}")
            x, st, _ = ctx.cg_solve(fd, tol=1e-8, maxit=20000)
            rho = P.true_residual(host(x), f)
            print(f"  {prec} {pc}: iters {st['iters']} outer {st['outer_iters']} rho* {rho:.2e}")
            assert st["status"] == 0 and rho <= 1e-8 and st["iters"] < res[prec][1]["iters"]
    ctx.close()


def test_full_size_32cubed_N9_bf16g():
    """32^3 elements on [0,1]^3 with interior vertices moved up to 10 %, N=9
    (32.8 M local points), manufactured forcing + N(0, 1e-3) noise, mixed
    solve with BF16-stored g: true FP64 residual <= 1e-8 by the oracle."""
    nel, N = (32, 32, 32), 9
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=synth.SEED_C3_VERTICES)
    _case("setup 32^3 N=9 bf16g")
    ctx = nek.Context(nel, N, vtx=vtx, prec="bf16g")
    P = oracle.Problem(N, nel, vtx, want_X=True)
    noise = synth.normal_noise(P.nl, 1e-3, synth.SEED_C3).reshape(P.E, -1)
    f_or, f_gpu = manufactured_load(ctx, P, noise)
    ctx.tune("bf16g", iters=10)
    _case("cg 32^3 N=9 bf16g")
    x, st, _ = ctx.cg_solve(dev(f_gpu), tol=1e-8, maxit=20000)
    rho = P.true_residual(host(x), f_or)
    print(f"  bf16g: iters {st['iters']} outer {st['outer_iters']} fp64 {st['fp64_iters']} "
          f"t {st['t_solve_s']:.3f}s rho* {rho:.2e}")
    assert st["status"] == 0 and rho <= 1e-8
    # FP64 CG on the same mesh: 16384 element groups over the persistent grid,
    # every workgroup walking several; stored and in-kernel factors
    ctx.set_prec("fp64")
    for geom in ("stored", "trilinear"):
        ctx.set_geometry(geom)
        ctx.tune("fp64", iters=10)
        _case(f"cg 32^3 N=9 fp64 {geom}")
        x64, s64, _ = ctx.cg_solve(dev(f_gpu), tol=1e-8, maxit=20000)
        rho = P.true_residual(host(x64), f_or)
        print(f"  fp64 {geom}: iters {s64['iters']} t {s64['t_solve_s']:.3f}s rho* {rho:.2e} "
              f"reported {s64['true_rel_res']:.2e}")
        assert s64["status"] == 0 and rho <= 1e-8
    ctx.set_geometry("stored")
    ctx.set_prec("bf16g")
    # the same solve with each preconditioner, as the benchmark times it
    for pc in ("jacobi", "fdm", "schwarz"):
        ctx.set_precond(pc)
        ctx.tune("bf16g", iters=10)
        _case(f"cg 32^3 N=9 bf16g {pc}")
        xp, sp, _ = ctx.cg_solve(dev(f_gpu), tol=1e-8, maxit=20000)
        rho = P.true_residual(host(xp), f_or)
        print(f"  bf16g {pc}: iters {sp['iters']} outer {sp['outer_iters']} t {sp['t_solve_s']:.3f}s rho* {rho:.2e}")
        assert sp["status"] == 0 and rho <= 1e-8 and sp["iters"] < st["iters"]
    # Schwarz in the other precisions: FP32-g mixed (vector-ALU window
    # solves by default) and FP64 (matrix-core window solves by default, then
    # the vector-ALU ones)
    for prec, kind in (("fp32", "auto"), ("fp64", "auto"), ("fp64", "valu")):
        ctx.set_prec(prec)
        ctx.set_schwarz_kernel(kind)
        ctx.tune(prec, iters=10)
        _case(f"cg 32^3 N=9 {prec} schwarz kernel={kind}")
        xp, sp, _ = ctx.cg_solve(dev(f_gpu), tol=1e-8, maxit=20000)
        rho = P.true_residual(host(xp), f_or)
        print(f"  {prec} schwarz ({kind}): iters {sp['iters']} outer {sp['outer_iters']} t {sp['t_solve_s']:.3f}s "
              f"rho* {rho:.2e}")
        assert sp["status"] == 0 and rho <= 1e-8 and sp["iters"] < 100
    ctx.close()
