"""Pins of the FP64 oracle of the initial-guess network and its feature maps.

What fixes each part (none of it from the oracle itself):
  * bfloat16 rounding: hand-worked values of round-to-nearest-even with 8
    significant bits (ties, carries into the next binade, sign);
  * SiLU and its derivative: closed values and central differences;
  * the gradient: central finite differences of the loss in FP64, every
    parameter tensor, relative agreement 1e-7;
  * Adam: the closed form of the first steps (m_hat = g, v_hat = g^2 for a
    constant gradient, so each step moves by lr * g / (|g| + eps));
  * features: an affine element has shape numbers (1, 1, 1, 0, 0, 0), the
    first three always sum to 3, a constant forcing gives unit inputs;
  * the prediction chain: outputs equal to the targets of the exact discrete
    solution give back that solution with alpha = 1 and rho0 ~ 0; their
    negative gives alpha = -1 and the same x0.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp, x0 as ox0
from paper_2405_11065_amd import synth


def test_bf16_rounding_hand_values():
    u = 2.0 ** -7    # spacing of bfloat16 in [1, 2)
    cases = {1.0: 1.0, 1.0 + u: 1.0 + u, 1.0 + u / 2: 1.0, 1.0 + 3 * u / 2: 1.0 + 2 * u,
             1.0 + u / 2 + 2.0 ** -20: 1.0 + u, 2.0 - u / 2: 2.0, -(1.0 + 3 * u / 2): -(1.0 + 2 * u),
             3.0: 3.0, 0.1: 0.10009765625, 0.0: 0.0, 1e-3: 131 / 128 * 2.0 ** -10}
    for a, want in cases.items():
        assert mlp.bf16(np.array([a]))[0] == want, a


def test_silu_closed_values_and_derivative():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.silu(np.array([1.0]))[0] - 1.0 / (1.0 + np.exp(-1.0))) < 1e-16
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.dsilu(z)).max() < 1e-9
    assert mlp.dsilu(np.array([0.0]))[0] == 0.5


def _tiny(seed=3, sizes=(7, 5, 4, 3), rows=4):
    r = np.random.default_rng(seed)
    params = [p.astype(np.float64) for p in synth.mlp_init(sizes, seed)]
    for k in (1, 3, 5):
        params[k] = r.normal(0, 0.3, size=params[k].shape)
    X = r.normal(size=(rows, sizes[0]))
    T = r.normal(size=(rows, sizes[-1]))
    return params, X, T


@pytest.mark.parametrize("rows", [1, 2, 4])
def test_gradient_matches_central_differences(rows):
    params, X, T = _tiny(rows=rows)
    _, grads = mlp.loss_and_grads(params, X, T)
    h = 1e-6
    for k, p in enumerate(params):
        fd = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            pp = [q.copy() for q in params]
            pp[k][idx] += h
            lp, _ = mlp.loss_and_grads(pp, X, T)
            pp[k][idx] -= 2 * h
            lm, _ = mlp.loss_and_grads(pp, X, T)
            fd[idx] = (lp - lm) / (2 * h)
        err = np.linalg.norm(fd - grads[k]) / max(np.linalg.norm(grads[k]), 1e-300)
        assert err < 1e-7, (k, err)


def test_zero_residual_gives_zero_loss_and_gradient():
    params, X, _ = _tiny()
    Y, _ = mlp.forward(params, X)
    loss, grads = mlp.loss_and_grads(params, X, Y)
    assert loss == 0.0
    assert all(np.all(g == 0) for g in grads)


def test_adam_closed_form_steps():
    g = np.array([0.3, -2.0, 1e-3])
    p0 = np.array([1.0, 2.0, -1.0])
    lr, eps = 1e-2, 1e-8
    P, M, V = mlp.adam_step([p0], [g], [np.zeros(3)], [np.zeros(3)], 1, lr, eps=eps)
    step = lr * g / (np.abs(g) + eps)
    assert np.allclose(P[0], p0 - step, rtol=0, atol=1e-15)
    P2, _, _ = mlp.adam_step(P, [g], M, V, 2, lr, eps=eps)
    assert np.allclose(P2[0], p0 - 2 * step, rtol=0, atol=1e-15)


def test_bf16_points_stay_within_bf16_error():
    params, X, T = _tiny(sizes=(16, 32, 32, 8), rows=6)
    Y64, _ = mlp.forward(params, X)
    Y16, _ = mlp.forward(params, X, bf16_points=True)
    assert np.abs(Y16 - Y64).max() <= 0.05 * np.abs(Y64).max()
    l64, g64 = mlp.loss_and_grads(params, X, T)
    l16, g16 = mlp.loss_and_grads(params, X, T, bf16_points=True)
    assert abs(l16 - l64) <= 0.05 * l64
    for a, b in zip(g16, g64):
        assert np.linalg.norm(a - b) <= 0.1 * np.linalg.norm(b)


def test_features_of_affine_and_deformed_elements():
    P = oracle.Problem(3, (2, 2, 1), synth.box_vertices((2, 2, 1)))
    n3 = P.n ** 3
    f = 2.5 * np.asarray(P.B, dtype=np.float64).ravel()   # F = 2.5 everywhere
    Xin, s = ox0.features(P, f)
    assert Xin.shape == (P.E, n3 + 6)
    assert np.allclose(s, 2.5, rtol=1e-15) and np.allclose(Xin[:, :n3], 1.0, rtol=1e-15)
    assert np.allclose(Xin[:, n3:], [1, 1, 1, 0, 0, 0], atol=1e-14)
    Pd = oracle.Problem(3, (2, 2, 2), synth.box_vertices((2, 2, 2), perturb=0.1, seed=5))
    Xd, _ = ox0.features(Pd, synth.uniform_load(Pd.nl, 1))
    q = Xd[:, Pd.n ** 3:]
    assert np.allclose(q[:, 0] + q[:, 1] + q[:, 2], 3.0, atol=1e-13)
    assert np.abs(q[:, 3:]).max() > 1e-4   # deformation shows in the off-diagonal numbers


def test_prediction_chain_recovers_exact_solution():
    Pd = oracle.Problem(4, (2, 2, 2), synth.box_vertices((2, 2, 2), perturb=0.1, seed=8))
    f = synth.uniform_load(Pd.nl, 2)
    x, it, _ = Pd.cg(f, tol=1e-13, maxit=2000)
    _, s = ox0.features(Pd, f)
    kappa = 0.05
    T = ox0.targets(Pd, x, s, kappa)
    x0, alpha, rho0, used = ox0.assemble(Pd, f, T, s, kappa)
    assert used and abs(alpha - 1.0) < 1e-10 and rho0 < 1e-10
    assert np.abs(x0 - x).max() <= 1e-10 * np.abs(x).max()
    x0n, alpha_n, _, used_n = ox0.assemble(Pd, f, -T, s, kappa)
    assert used_n and abs(alpha_n + 1.0) < 1e-10
    assert np.abs(x0n - x).max() <= 1e-10 * np.abs(x).max()
    z, _, rho_z, used_z = ox0.assemble(Pd, f, np.zeros_like(T), s, kappa)
    assert not used_z and np.all(z == 0)
