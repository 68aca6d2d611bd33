"""Pins of the oracle's element-interior fast-diagonalization preconditioner.

  * the 1-D modes: S^T W_I S = I and K_I S = W_I S Lambda;
  * the interior block solve equals the inverse of the interior block of the
    assembled operator, built by brute force from unit vectors through the C
    oracle, on axis-aligned elements of unequal sides (where the separable
    form is exact);
  * the rest of M^-1 is the inverse diagonal (1 / or_diag) on shared nodes;
  * M^-1 is symmetric in the c-weighted inner product and positive;
  * the Python PCG loop with M^-1 = identity gives or_cg's iterates bit for
    bit, and with the Jacobi M^-1 gives or_pcg's;
  * with the preconditioner the solve matches the dense solve and needs far
    fewer iterations than CG.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from oracle import fdm  # noqa: E402
from paper_2405_11065_amd import synth  # noqa: E402


@pytest.mark.parametrize("N", [2, 3, 5, 7, 9, 11])
def test_interior_modes(N):
    xi, w = oracle.gll(N)
    D = oracle.deriv(N)
    S, lam = fdm.interior_eig(N, D, w)
    WI = np.diag(w[1:N])
    KI = (D.T @ np.diag(w) @ D)[1:N, 1:N]
    assert np.allclose(S.T @ WI @ S, np.eye(N - 1), atol=1e-12)
    assert np.allclose(KI @ S, WI @ S @ np.diag(lam), atol=1e-10 * np.abs(KI).max())
    assert np.all(lam > 0)


@pytest.mark.parametrize("N,nel,hi", [(4, (2, 2, 2), (1.0, 0.6, 1.4)), (5, (3, 1, 2), (1.5, 0.5, 1.0)),
                                      (3, (1, 1, 1), (2.0, 1.0, 0.5))])
def test_interior_solve_is_inverse_of_interior_block(N, nel, hi):
    vtx = synth.box_vertices(nel, hi=hi)
    P = oracle.Problem(N, nel, vtx)
    F = fdm.Fdm(P, vtx)
    n = N + 1
    rng = np.random.default_rng(3)
    for e in range(P.E):
        # interior local indices of element e; those nodes belong to e alone
        idx = np.array([e * n ** 3 + i + n * (j + n * k) for k in range(1, N) for j in range(1, N)
                        for i in range(1, N)])
        Aii = np.empty((idx.size, idx.size))
        for col, l in enumerate(idx):
            u = np.zeros(P.nl)
            u[l] = 1.0
            Aii[:, col] = P.A(u)[idx]
        r = np.zeros(P.nl)
        r[idx] = rng.standard_normal(idx.size)
        z = F.apply(r)
        ref = np.linalg.solve(Aii, r[idx])
        assert np.abs(z[idx] - ref).max() <= 1e-11 * np.abs(ref).max()
    # shared and Dirichlet nodes: inverse diagonal (0 on Dirichlet nodes)
    r = rng.standard_normal(P.nl) * P.mask
    surf = np.ones(P.nl, bool)
    q = np.arange(P.nl) % n ** 3
    i, j, k = q % n, (q // n) % n, q // n ** 2
    surf &= (i == 0) | (i == N) | (j == 0) | (j == N) | (k == 0) | (k == N)
    z = F.apply(r)
    m = P.diag()
    assert np.array_equal(z[surf & (P.mask > 0)], r[surf & (P.mask > 0)] / m[surf & (P.mask > 0)])
    assert np.all(z[P.mask == 0] == 0.0)


def test_preconditioner_symmetric_positive():
    nel, N = (2, 3, 2), 4
    vtx = synth.box_vertices(nel, perturb=0.1, seed=8)
    P = oracle.Problem(N, nel, vtx)
    F = fdm.Fdm(P, vtx)
    rng = np.random.default_rng(4)
    # continuous masked vectors (equal on copies)
    u = P.dssum(P.c * rng.standard_normal(P.nl), masked=True)
    v = P.dssum(P.c * rng.standard_normal(P.nl), masked=True)
    a, b = P.glsc3(u, F.apply(v)), P.glsc3(v, F.apply(u))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert P.glsc3(u, F.apply(u)) > 0


def test_python_loop_is_the_c_loop_bit_for_bit():
    nel, N = (3, 2, 2), 5
    vtx = synth.box_vertices(nel, perturb=0.1, seed=9)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 10)
    x0, it0, h0 = P.cg(f, tol=0.0, maxit=30)
    x1, it1, h1 = fdm.pcg(P, f, lambda r: r, tol=0.0, maxit=30)
    assert it1 == it0 and np.array_equal(x1, x0) and np.array_equal(h1, h0)
    m = P.diag()
    x0, it0, h0 = P.pcg(f, m, tol=0.0, maxit=30)
    x1, it1, h1 = fdm.pcg(P, f, lambda r: r / m, tol=0.0, maxit=30)
    assert it1 == it0 and np.array_equal(x1, x0) and np.array_equal(h1, h0)


def test_fdm_pcg_solves_and_saves_iterations():
    N, nel = 4, (2, 2, 2)
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=12)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 13)
    F = fdm.Fdm(P, vtx)
    x, it, _ = fdm.pcg(P, f, F.apply, tol=1e-13, maxit=2000)
    xr, _, _ = P.cg(f, tol=1e-14, maxit=2000)
    assert np.abs(x - xr).max() <= 1e-11 * np.abs(xr).max()
    nel, N = (4, 4, 4), 7
    vtx = synth.box_vertices(nel)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, synth.SEED_C1)
    F = fdm.Fdm(P, vtx)
    _, it_cg, _ = P.cg(f, tol=1e-8, maxit=3000)
    x, it_f, _ = fdm.pcg(P, f, F.apply, tol=1e-8, maxit=3000)
    assert it_f < 0.65 * it_cg and P.true_residual(x, f) <= 1e-8
