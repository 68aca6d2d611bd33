"""The initial-guess network and its inputs on the GPU, against the FP64 oracle.

Tolerances.  The GPU multiplies bfloat16 operands with FP32 accumulation; the
oracle is run with the same bfloat16 rounding points (oracle.mlp, bf16=True)
and FP64 accumulation, so the two differ by accumulation rounding (~1e-6
relative) and the rare bfloat16 rounding decisions that it moves (each one a
2^-9 relative change of one operand).  Outputs must agree to 1e-4 in norm
(relative), parameter gradients to 2e-3 in norm per tensor, the loss to 1e-5,
and every element of the outputs and gradients within its own bound derived
from those two effects (elementwise_bounds: FP32 accumulation of each sum and
one moved bfloat16 rounding per stored value, propagated to first order);
against the pure FP64 oracle (no bfloat16 anywhere) gradients stay within
5e-2.  Adam (FP32) must agree with the FP64 update of the same gradient to
1e-6 relative.  Features: bfloat16 inputs bit-equal to the oracle's FP64
values rounded once (a tie moved by summation order would be a 2^-8 step in
one entry; none is allowed here), scales to 1e-14; targets to 1e-7.  The
assembled initial guess (projection, energy-norm scaling, fallback) is FP64
on both sides: 1e-10.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as om, x0 as ox0
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
    return t.detach().float().cpu().numpy() if t.dtype == torch.bfloat16 else t.detach().cpu().numpy()


def bf16_rows(a, ld):
    """bfloat16 CUDA matrix [rows, ld] holding a (already bfloat16-representable), zero padded."""
    out = np.zeros((a.shape[0], ld), dtype=np.float32)
    out[:, :a.shape[1]] = a
    return torch.from_numpy(out).cuda().to(torch.bfloat16)


def f32_rows(a, ld):
    out = np.zeros((a.shape[0], ld), dtype=np.float32)
    out[:, :a.shape[1]] = a
    return torch.from_numpy(out).cuda()


def setup_net(sizes, rows, seed):
    r = np.random.default_rng(seed)
    params = synth.mlp_init(sizes, seed)
    for k in (1, 3, 5):
        params[k] = r.normal(0, 0.2, size=params[k].shape).astype(np.float32)
    X = om.bf16(r.normal(size=(rows, sizes[0])))
    T = r.normal(0, 0.5, size=(rows, sizes[-1]))
    return params, X, T


def nrel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


U32 = 2.0 ** -24   # FP32 unit roundoff


def stored_err(v, ev):
    """Bound on |bf16(v') - bf16(v)| for |v' - v| <= ev: zero where no
    bfloat16 rounding boundary (a midpoint between neighbours) lies within
    ev of v, else ev plus one spacing."""
    v = np.asarray(v, dtype=np.float64)
    rv = om.bf16(v)
    _, e = np.frexp(np.where(rv == 0, 1.0, rv))
    spacing = np.ldexp(1.0, e - 8)            # 8 significant bits
    nearest_mid = np.minimum(np.abs(v - (rv + spacing / 2)), np.abs(v - (rv - spacing / 2)))
    flip = (nearest_mid <= ev) | (rv == 0)
    return np.where(flip, ev + spacing, 0.0)


def elementwise_bounds(params, X, T=None):
    """Per-element bounds on |GPU - bf16 oracle| for Y and, with T, for every
    parameter gradient, propagated to first order from the two differences
    the arithmetic allows: FP32 accumulation of a K-term sum (at most
    K u sum |terms|) and, at a bfloat16 storage point, a rounding decision
    moved by that error (stored_err: only where a rounding boundary lies
    within the propagated error).  Activation derivatives enter through
    |silu'| <= 1.1 and |silu''| <= 0.5."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    r = om.bf16
    A0 = r(X)
    W1r, W2r, W3r = r(W1), r(W2), r(W3)
    Z1 = A0 @ W1r.T + b1
    H1 = r(om.silu(Z1))
    Z2 = H1 @ W2r.T + b2
    H2 = r(om.silu(Z2))
    Y = H2 @ W3r.T + b3
    eZ1 = A0.shape[1] * U32 * (np.abs(A0) @ np.abs(W1r).T + np.abs(b1))
    eH1 = stored_err(om.silu(Z1), 1.1 * eZ1)
    eZ2 = H1.shape[1] * U32 * (np.abs(H1) @ np.abs(W2r).T + np.abs(b2)) + eH1 @ np.abs(W2r).T
    eH2 = stored_err(om.silu(Z2), 1.1 * eZ2)
    eY = H2.shape[1] * U32 * (np.abs(H2) @ np.abs(W3r).T + np.abs(b3)) + eH2 @ np.abs(W3r).T
    if T is None:
        return eY
    R, n = X.shape[0], Y.size
    dY = 2.0 * (Y - np.asarray(T, dtype=np.float64)) / n
    e_dY = 2.0 * eY / n
    dYr = r(dY)
    e_dYr = stored_err(dY, e_dY)
    g = []
    e_gW3 = R * U32 * (np.abs(dYr).T @ np.abs(H2)) + e_dYr.T @ np.abs(H2) + np.abs(dYr).T @ eH2
    e_gb3 = R * U32 * np.abs(dY).sum(axis=0) + e_dY.sum(axis=0)
    P2 = dYr @ W3r
    dZ2 = P2 * om.dsilu(Z2)
    e_dZ2 = (W3r.shape[0] * U32 * (np.abs(dYr) @ np.abs(W3r)) + e_dYr @ np.abs(W3r)) * 1.1 + 0.5 * np.abs(P2) * eZ2
    dZ2r = r(dZ2)
    e_dZ2r = stored_err(dZ2, e_dZ2)
    e_gW2 = R * U32 * (np.abs(dZ2r).T @ np.abs(H1)) + e_dZ2r.T @ np.abs(H1) + np.abs(dZ2r).T @ eH1
    e_gb2 = R * U32 * np.abs(dZ2).sum(axis=0) + e_dZ2.sum(axis=0)
    P1 = dZ2r @ W2r
    dZ1 = P1 * om.dsilu(Z1)
    e_dZ1 = (W2r.shape[0] * U32 * (np.abs(dZ2r) @ np.abs(W2r)) + e_dZ2r @ np.abs(W2r)) * 1.1 + 0.5 * np.abs(P1) * eZ1
    dZ1r = r(dZ1)
    e_dZ1r = stored_err(dZ1, e_dZ1)
    e_gW1 = R * U32 * (np.abs(dZ1r).T @ np.abs(A0)) + e_dZ1r.T @ np.abs(A0)
    e_gb1 = R * U32 * np.abs(dZ1).sum(axis=0) + e_dZ1.sum(axis=0)
    return eY, [e_gW1, e_gb1, e_gW2, e_gb2, e_gW3, e_gb3]


def within(a, b, bound, name):
    """Element by element: |a - b| <= bound; reports the largest use of it."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    worst = float((d / np.maximum(bound, 1e-300)).max())
    print(f"  {name}: largest |diff| / bound {worst:.2e}")
    assert np.all(d <= bound), f"{name}: {int((d > bound).sum())} elements beyond their bound"


SHAPES = [((518, 256, 256, 512), 300), ((37, 20, 24, 13), 70), ((8, 64, 64, 8), 64), ((518, 256, 256, 512), 1)]


@pytest.mark.parametrize("sizes,rows", SHAPES)
def test_forward_matches_oracle(sizes, rows):
    if len(sizes) == 4 and sizes[1] != sizes[2]:
        sizes = (sizes[0], sizes[1], sizes[1], sizes[3])
    _case(f"forward sizes={sizes} rows={rows}")
    params, X, _ = setup_net(sizes, rows, 1)
    net = nek.Mlp(sizes[0], sizes[1], sizes[3], params)
    Y = host(net.forward(bf16_rows(X, net.ld_in)))[:, :sizes[3]]
    P64 = [p.astype(np.float64) for p in params]
    Yo, _ = om.forward(P64, X, bf16_points=True)
    Y64, _ = om.forward(P64, X)
    e, e64 = nrel(Y, Yo), nrel(Y, Y64)
    print(f"  |dY|/|Y| vs bf16 oracle {e:.2e}, vs FP64 oracle {e64:.2e}")
    assert e <= 1e-4 and e64 <= 2e-2
    within(Y, Yo, elementwise_bounds(P64, X), "Y")
    net.close()


@pytest.mark.parametrize("sizes,rows", SHAPES[:3] + [((96, 64, 64, 40), 2500)])
def test_loss_and_gradient_match_oracle(sizes, rows):
    """2500 rows: the weight gradients run split along the rows (four pieces, the last one ragged)."""
    if sizes[1] != sizes[2]:
        sizes = (sizes[0], sizes[1], sizes[1], sizes[3])
    _case(f"grad sizes={sizes} rows={rows}")
    params, X, T = setup_net(sizes, rows, 2)
    net = nek.Mlp(sizes[0], sizes[1], sizes[3], params)
    loss, g = net.loss_grad(bf16_rows(X, net.ld_in), f32_rows(T.astype(np.float32), net.ld_out))
    P64 = [p.astype(np.float64) for p in params]
    T32 = T.astype(np.float32).astype(np.float64)
    lo, go = om.loss_and_grads(P64, X, T32, bf16_points=True)
    l64, g64 = om.loss_and_grads(P64, X, T32)
    print(f"  loss {loss:.6e} oracle {lo:.6e}")
    assert abs(loss - lo) <= 1e-5 * lo
    _, eb = elementwise_bounds(P64, X, T32)
    for k, (a, b, c) in enumerate(zip(g, go, g64)):
        e, e64 = nrel(a, b), nrel(a, c)
        print(f"  grad[{k}] shape {b.shape}: vs bf16 oracle {e:.2e}, vs FP64 oracle {e64:.2e}")
        assert e <= 2e-3 and e64 <= 5e-2
        within(a, b, eb[k], f"grad[{k}]")
    net.close()


def test_adam_multi_step_matches_oracle():
    """Three Adam steps on the GPU against the oracle fed the GPU's gradients."""
    sizes = (24, 16, 16, 8)
    params, X, T = setup_net(sizes, 40, 4)
    net = nek.Mlp(24, 16, 8, params)
    Xd, Td = bf16_rows(X, net.ld_in), f32_rows(T.astype(np.float32), net.ld_out)
    P = [p.astype(np.float64) for p in params]
    M = [np.zeros_like(p) for p in P]
    V = [np.zeros_like(p) for p in P]
    for t in (1, 2, 3):
        before = net.get_params()
        _, g = net.loss_grad(Xd, Td)
        net.adam(lr=1e-2)
        after = net.get_params()
        # the oracle step from the GPU's own starting point and gradient
        Pb = [b.astype(np.float64) for b in before]
        P1, M, V = om.adam_step(Pb, [x.astype(np.float64) for x in g], M, V, t, 1e-2)
        for k, (a, b, b0) in enumerate(zip(after, P1, Pb)):
            step_err = np.abs(a - b).max() / max(np.abs(b - b0).max(), 1e-30)
            assert step_err <= 1e-4, (t, k, step_err)
    net.close()


def test_training_fits_a_teacher_network_deterministically():
    sizes = (40, 32, 32, 16)
    r = np.random.default_rng(6)
    teacher = synth.mlp_init(sizes, 60)
    X = om.bf16(r.normal(size=(2048, 40)))
    Tt, _ = om.forward([p.astype(np.float64) for p in teacher], X)
    init = synth.mlp_init(sizes, 61)
    hists, finals = [], []
    for rep in range(2):
        net = nek.Mlp(40, 32, 16, init)
        h = net.train(bf16_rows(X, net.ld_in), f32_rows(Tt.astype(np.float32), net.ld_out), 2048, 256, 400,
                      lr=3e-3, seed=11)
        hists.append(h)
        finals.append(np.concatenate([p.ravel() for p in net.get_params()]))
        net.close()
    print(f"  loss {hists[0][0]:.3e} -> {hists[0][-1]:.3e}")
    assert hists[0][-1] < 0.1 * hists[0][0]
    assert np.array_equal(hists[0], hists[1]) and np.array_equal(finals[0], finals[1])


def _problem(N=7, nel=(3, 2, 2), pert=0.1, seed=21):
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=pert, seed=seed)
    return nek.Context(nel, N, vtx=vtx), oracle.Problem(N, nel, vtx, want_X=True)


def test_grf_matches_generator():
    ctx, P = _problem()
    draw = synth.FourierFieldDraw(31, length=0.2, features=256)
    F = host(nek.grf(ctx, draw, times_B=False))
    Fo = draw(P.X).ravel()
    err = np.abs(F - Fo).max() / np.abs(Fo).max()
    fB = host(nek.grf(ctx, draw, scale=2.0, times_B=True))
    errB = np.abs(fB - 2.0 * Fo * P.B.ravel()).max() / np.abs(2.0 * Fo * P.B.ravel()).max()
    print(f"  grf err {err:.2e}, times 2B err {errB:.2e}")
    assert err <= 1e-12 and errB <= 1e-12
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_features_and_targets_match_oracle(mode):
    ctx, P = _problem()
    draw = synth.FourierFieldDraw(32)
    f_np = (draw(P.X) * P.B.reshape(P.E, -1)).ravel()
    f = torch.from_numpy(f_np).cuda()
    X, s = nek.x0_features(ctx, f, mode=mode)
    Xo, so = ox0.features(P, f_np, mode=mode)
    Xg = host(X)
    n3 = P.n ** 3
    assert np.array_equal(Xg[:, :n3 + 6], om.bf16(Xo))
    assert np.all(Xg[:, n3 + 6:] == 0)
    assert np.abs(host(s) - so).max() <= 1e-14 * so.max()
    x_np, _, _ = P.cg(f_np, tol=1e-10, maxit=3000)
    T = nek.x0_targets(ctx, torch.from_numpy(x_np).cuda(), s, 0.05)
    To = ox0.targets(P, x_np, so, 0.05)
    assert np.abs(host(T)[:, :n3] - To).max() <= 1e-7 * np.abs(To).max()
    ctx.close()


@pytest.mark.parametrize("fit,policy,mode", [(False, 0, 0), (True, 0, 0), (False, 1, 0), (True, 0, 2)])
def test_predict_chain_matches_oracle(fit, policy, mode):
    """nek_x0_predict against oracle.x0.assemble on the GPU network's own outputs."""
    ctx, P = _problem(seed=23)
    n3 = P.n ** 3
    draw = synth.FourierFieldDraw(33)
    f_np = (draw(P.X) * P.B.reshape(P.E, -1)).ravel()
    f = torch.from_numpy(f_np).cuda()
    kappa = 1.0 / (3 * np.pi ** 2)
    net = nek.Mlp(n3 + 6, 64, n3, synth.mlp_init((n3 + 6, 64, 64, n3), 7))
    X, s = nek.x0_features(ctx, f, mode=mode)
    if fit:   # overfit this one problem so that the guess is worth keeping
        x_np, _, _ = P.cg(f_np, tol=1e-10, maxit=3000)
        T = nek.x0_targets(ctx, torch.from_numpy(x_np).cuda(), s, kappa)
        net.train(X, T, P.E, P.E, 300, lr=3e-3, seed=1)
    x0, alpha, rho0, used = nek.x0_predict(ctx, net, f, kappa, policy=policy, mode=mode)
    Y = host(net.forward(X))[:, :n3]
    x0o, ao, ro, uo = ox0.assemble(P, f_np, Y, host(s), kappa, residual_policy=policy == 0)
    print(f"  fit={fit}: alpha {alpha:.6g} (oracle {ao:.6g}) rho0 {rho0:.4g} (oracle {ro:.4g}) used {used}")
    assert used == uo
    if fit or policy == 1:
        assert used
    if used:
        assert abs(alpha - ao) <= 1e-10 * abs(ao) and abs(rho0 - ro) <= 1e-10
        assert np.abs(host(x0) - x0o).max() <= 1e-10 * np.abs(x0o).max()
        # CG from the guess reaches the tolerance
        xs, st, _ = ctx.cg_solve(f, x0=x0, tol=1e-8, maxit=5000)
        assert P.true_residual(host(xs), f_np) <= 1e-8
    else:
        assert np.all(host(x0) == 0)
    net.close()
    ctx.close()


def test_bad_arguments():
    with pytest.raises(nek.NekError):
        nek.Mlp(0, 4, 4)
    ctx, _ = _problem(nel=(1, 1, 1))
    net = nek.Mlp(10, 8, 10)
    f = ctx.new_vector()
    with pytest.raises(nek.NekError):
        nek.x0_predict(ctx, net, f, 1.0)   # network shape does not fit N = 7
    net.close()
    ctx.close()
