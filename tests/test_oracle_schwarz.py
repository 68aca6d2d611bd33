"""Pins of the oracle's two-level overlapping Schwarz preconditioner.

  * the window variants: S^T W S = I and K S = W S Lambda on the kept nodes;
  * each subdomain solve equals the inverse of the assembled operator
    restricted to the subdomain (built by brute force from unit vectors
    through the C oracle), on box meshes of uniform spacing per direction
    (unequal between directions), where the separable form is exact;
  * the coarse operator equals the Galerkin product P^T A P (brute force)
    on rectilinear meshes of unequal slab spacings, and the coarse term is
    P (P^T A P)^-1 P^T r there;
  * a single element: the subdomain is the whole problem, PCG converges in
    one iteration;
  * M^-1 is symmetric in the c-weighted inner product and positive, also on
    deformed meshes;
  * the two-level signature: PCG iteration counts stay nearly flat from 2^3
    to 8^3 elements while one level (no coarse term) and plain CG grow;
  * the preconditioned solve matches the dense solve.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from oracle import fdm, schwarz  # noqa: E402
from paper_2405_11065_amd import synth  # noqa: E402


def rect_vertices(nel, seed):
    """Rectilinear lattice with random spacings per slab (x fastest)."""
    r = np.random.default_rng(seed)
    ax = [np.concatenate([[0.0], np.cumsum(r.uniform(0.5, 1.5, n))]) for n in nel]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def global_unit(P, g):
    """Continuous vector: 1 on every copy of global node g."""
    return (P.gid == g).astype(np.float64)


@pytest.mark.parametrize("N", [2, 3, 5, 9])
def test_window_modes(N):
    xi, w = oracle.gll(N)
    D = oracle.deriv(N)
    Kw, Ww = schwarz.window_operators(N, D, w)
    assert Kw.shape == (N + 3, N + 3) and np.allclose(Kw, Kw.T)
    for (lo, hi), (keep, S, lam) in schwarz.window_variants(N, D, w).items():
        K = Kw[np.ix_(keep, keep)]
        W = np.diag(Ww[keep])
        assert np.allclose(S.T @ W @ S, np.eye(len(keep)), atol=1e-12)
        assert np.allclose(K @ S, W @ S @ np.diag(lam), atol=1e-10 * np.abs(K).max())
        assert np.all(lam > 0)


@pytest.mark.parametrize("N,nel,hi", [(2, (3, 3, 2), (3.0, 1.5, 1.0)), (3, (3, 2, 2), (2.0, 1.2, 0.9)),
                                      (4, (2, 3, 1), (1.0, 1.0, 0.5))])
def test_subdomain_solve_is_inverse_of_restricted_operator(N, nel, hi):
    vtx = synth.box_vertices(nel, hi=hi)
    P = oracle.Problem(N, nel, vtx)
    M = schwarz.Schwarz(P, vtx)
    Gx, Gy, Gz = M.G
    rng = np.random.default_rng(5)
    for e in range(P.E):
        (ix, _, _), (iy, _, _), (iz, _, _) = M.window(e)
        nodes = [gx + Gx * (gy + Gy * gz) for gz in iz for gy in iy for gx in ix]   # [z][y][x] order
        A = np.empty((len(nodes), len(nodes)))
        for col, g in enumerate(nodes):
            Ag = P.A(global_unit(P, g))
            for row, h in enumerate(nodes):
                A[row, col] = Ag[np.argmax(P.gid == h)]
        rg = np.zeros((Gz, Gy, Gx))
        vals = rng.standard_normal(len(nodes))
        rg.reshape(-1)[nodes] = vals
        got = M.local_solve(e, rg).reshape(-1)
        ref = np.linalg.solve(A, vals)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("N,nel", [(2, (3, 3, 2)), (3, (4, 2, 3)), (5, (3, 3, 3))])
def test_coarse_operator_is_galerkin_product(N, nel):
    vtx = rect_vertices(nel, 9)
    P = oracle.Problem(N, nel, vtx)
    M = schwarz.Schwarz(P, vtx)
    Px, Py, Pz = M.Pd
    nc = [m.shape[1] for m in M.Pd]
    # columns of P in the local layout, one per interior vertex ([vz][vy][vx] order)
    cols = []
    for c in range(nc[2]):
        for b in range(nc[1]):
            for a in range(nc[0]):
                g = np.einsum("i,j,k->kji", Px[:, a], Py[:, b], Pz[:, c])
                cols.append(M.to_local(g))
    Pl = np.stack(cols, axis=1)
    # P^T A P over unique nodes: the c-weighted sum over local copies
    APl = np.stack([P.A(Pl[:, q]) for q in range(Pl.shape[1])], axis=1)
    Ac = (Pl * P.c[:, None]).T @ APl
    assert np.allclose(Ac, Ac.T, atol=1e-12 * np.abs(Ac).max())
    # the separable operator from the 1-D pieces, [vz][vy][vx] with vx fastest
    Hg = schwarz.mean_lengths(nel, vtx).reshape(nel[2], nel[1], nel[0], 3)
    mats = []
    for d in range(3):
        h = Hg[..., d].mean(axis=tuple(a for a in range(3) if a != 2 - d))
        mats.append(schwarz.q1_line(h, N))
    (Kx, Mx), (Ky, My), (Kz, Mz) = mats
    At = np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx))
    assert np.abs(At - Ac).max() <= 1e-12 * np.abs(Ac).max()
    # the coarse term applies P (P^T A P)^-1 P^T
    r = P.dssum(synth.uniform_load(P.nl, 4) - 0.5, masked=True)
    got = M.to_local(M.coarse_correction(M.to_global(r)))
    ref = Pl @ np.linalg.solve(Ac, (Pl * P.c[:, None]).T @ r)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_single_element_is_exact():
    N, nel = 5, (1, 1, 1)
    vtx = synth.box_vertices(nel, hi=(1.0, 0.7, 1.3))
    P = oracle.Problem(N, nel, vtx)
    M = schwarz.Schwarz(P, vtx)
    f = synth.uniform_load(P.nl, 3)
    x, it, _ = fdm.pcg(P, f, M.apply, tol=1e-12, maxit=20)
    assert it == 1
    assert P.true_residual(x, f) <= 1e-13


@pytest.mark.parametrize("pert", [0.0, 0.1])
def test_symmetric_positive(pert):
    N, nel = 4, (3, 2, 3)
    vtx = synth.box_vertices(nel, perturb=pert, seed=8)
    P = oracle.Problem(N, nel, vtx)
    M = schwarz.Schwarz(P, vtx)
    # continuous vectors, zero on the Dirichlet boundary
    u = P.dssum(P.c * (synth.uniform_load(P.nl, 1) - 0.5), masked=True)
    v = P.dssum(P.c * (synth.uniform_load(P.nl, 2) - 0.5), masked=True)
    a, b = P.glsc3(u, M.apply(v)), P.glsc3(v, M.apply(u))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    assert P.glsc3(u, M.apply(u)) > 0 and P.glsc3(v, M.apply(v)) > 0
    z = M.apply(v)   # continuous output: equal copies of every global node
    zg = np.zeros(P.ng)
    zg[P.gid] = z
    assert np.array_equal(zg[P.gid], z)


def test_two_level_iterations_nearly_flat():
    N = 4
    out = {}
    for ne in (2, 4, 8):
        nel = (ne, ne, ne)
        vtx = synth.box_vertices(nel)
        P = oracle.Problem(N, nel, vtx)
        M = schwarz.Schwarz(P, vtx)
        f = synth.uniform_load(P.nl, 1)
        _, i2, _ = fdm.pcg(P, f, M.apply, tol=1e-8, maxit=500)
        _, i1, _ = fdm.pcg(P, f, lambda r: M.apply(r, coarse=False), tol=1e-8, maxit=500)
        _, ic, _ = P.cg(f, tol=1e-8, maxit=2000)
        out[ne] = (i2, i1, ic)
    print(out)
    # 2^3 has no element without a boundary face; from 4^3 on the count is flat
    assert out[8][0] <= 1.3 * out[4][0] and out[4][0] <= 1.8 * out[2][0]
    assert out[8][1] >= 1.4 * out[4][1]        # one level grows with the mesh
    assert out[8][2] >= 1.7 * out[4][2]        # CG even more
    assert out[8][0] * 4 <= out[8][2]


def test_preconditioned_solve_matches_dense():
    N, nel = 3, (2, 2, 2)
    vtx = synth.box_vertices(nel, perturb=0.1, seed=6)
    P = oracle.Problem(N, nel, vtx)
    M = schwarz.Schwarz(P, vtx)
    f = synth.uniform_load(P.nl, 7)
    x, it, _ = fdm.pcg(P, f, M.apply, tol=1e-13, maxit=200)
    # dense solve over the interior global nodes
    G = [v * N + 1 for v in nel]
    gi = np.arange(P.ng)
    gx, gy, gz = gi % G[0], (gi // G[0]) % G[1], gi // (G[0] * G[1])
    inner = gi[(gx > 0) & (gx < G[0] - 1) & (gy > 0) & (gy < G[1] - 1) & (gz > 0) & (gz < G[2] - 1)]
    A = np.empty((inner.size, inner.size))
    first = {g: int(np.argmax(P.gid == g)) for g in inner}
    for col, g in enumerate(inner):
        Ag = P.A(global_unit(P, g))
        A[:, col] = Ag[[first[h] for h in inner]]
    b = P.rhs(f)
    xd = np.linalg.solve(A, b[[first[h] for h in inner]])
    xo = x[[first[h] for h in inner]]
    assert np.abs(xo - xd).max() <= 1e-11 * np.abs(xd).max()
