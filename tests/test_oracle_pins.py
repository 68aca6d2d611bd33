"""Pins for the FP64 CPU oracle: checks against closed forms, invariants and an
independent dense assembly, never against the oracle's own formulas.

Each test names what fixes the expected value.  The paper (Chen et al., Nekbone
case study) states the CG loop (Table 1) and the operator's call structure
(Fig. 2) but not the discretisation, so the spectral-element facts below come
from the mathematics of GLL quadrature and trilinear hexahedra.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import numpy.polynomial.legendre as npleg
import numpy.polynomial.polynomial as nppoly
import pytest

import oracle
from paper_2405_11065_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _val(s):
    s = s.strip()
    neg = s.startswith("-")
    s = s.lstrip("-")
    if s.startswith("sqrt("):
        v = math.sqrt(float(Fraction(s[5:-1])))
    elif "/sqrt(" in s:
        a, b = s.split("/sqrt(")
        v = float(Fraction(a)) / math.sqrt(float(Fraction(b[:-1])))
    else:
        v = float(Fraction(s))
    return -v if neg else v


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


# ----------------------------------------------------------------- GLL and D

@pytest.mark.parametrize("N", [2, 3, 4])
def test_gll_closed_forms(golden, N):
    xi, w = oracle.gll(N)
    ref = golden["gll"][str(N)]
    np.testing.assert_allclose(xi, [_val(v) for v in ref["nodes"]], rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, [_val(v) for v in ref["weights"]], rtol=0, atol=4e-16)


@pytest.mark.parametrize("N", list(range(1, 17)))
def test_gll_roots_and_quadrature(N):
    xi, w = oracle.gll(N)
    # interior nodes = roots of P'_N, found here by NumPy's companion-matrix route
    if N > 1:
        roots = np.sort(npleg.Legendre.basis(N).deriv().roots().real)
        np.testing.assert_allclose(xi[1:-1], roots, rtol=0, atol=1e-13)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    assert np.all(np.diff(xi) > 0)
    # GLL with N+1 points integrates x^k exactly for k <= 2N-1
    for k in range(2 * N):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14, (N, k)
    # and is not exact at degree 2N (so the rule really is Lobatto, not Gauss)
    assert abs(np.dot(w, xi ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-10


def test_deriv_closed_form_N2(golden):
    D = oracle.deriv(2)
    ref = np.array([[_val(v) for v in row] for row in golden["deriv_N2"]["D"]])
    np.testing.assert_allclose(D, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9, 11, 12])
def test_deriv_differentiates_polynomials(N):
    xi, _ = oracle.gll(N)
    D = oracle.deriv(N)
    for k in range(N + 1):
        exact = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        np.testing.assert_allclose(D @ xi ** k, exact, rtol=0, atol=1e-11)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-12)
    # centro-antisymmetry of the GLL derivative: D[N-i, N-j] = -D[i, j]
    np.testing.assert_allclose(D[::-1, ::-1], -D, atol=1e-12)


def _lagrange_deriv_numpy(xi):
    """Independent D: differentiate each Lagrange polynomial built from its roots."""
    n = len(xi)
    Dt = np.empty((n, n))
    for j in range(n):
        others = np.delete(xi, j)
        c = nppoly.polyfromroots(others) / np.prod(xi[j] - others)
        Dt[:, j] = nppoly.polyval(xi, nppoly.polyder(c))
    return Dt


@pytest.mark.parametrize("N", [3, 6, 9])
def test_deriv_matches_lagrange_polynomials(N):
    xi, _ = oracle.gll(N)
    np.testing.assert_allclose(oracle.deriv(N), _lagrange_deriv_numpy(xi), rtol=0, atol=1e-10)


# ------------------------------------------------------------------ numbering

@pytest.mark.parametrize("N,nel", [(1, (2, 2, 2)), (3, (3, 2, 4)), (7, (4, 4, 4))])
def test_numbering_counts(N, nel):
    gid, mult, mask = oracle.numbering(N, nel)
    G = [v * N + 1 for v in nel]
    ng = G[0] * G[1] * G[2]
    assert gid.min() == 0 and gid.max() == ng - 1
    assert len(np.unique(gid)) == ng
    # sum of the multiplicity weights c = 1/mult counts every global node once
    c = 1.0 / mult
    assert abs(c.sum() - ng) < 1e-9 * ng
    # copies per global node equal mult
    counts = np.bincount(gid, minlength=ng)
    assert np.array_equal(counts[gid], mult)
    # masked global nodes: the box surface, prod(G) - prod(G-2)
    masked_unique = len(np.unique(gid[mask == 0]))
    assert masked_unique == ng - (G[0] - 2) * (G[1] - 2) * (G[2] - 2)
    # mult classes: element-interior 1, face 2, edge 4, vertex 8 (for interior lattice nodes)
    n = N + 1
    q = np.arange(len(gid)) % n ** 3
    i, j, k = q % n, (q // n) % n, q // (n * n)
    on = (i == 0) | (i == N), (j == 0) | (j == N), (k == 0) | (k == N)
    nsurf = on[0].astype(int) + on[1] + on[2]
    interior = mask == 1
    assert np.all(mult[interior] == 2 ** nsurf[interior])


@pytest.mark.parametrize("N,nel", [(2, (2, 3, 2)), (4, (3, 3, 3))])
def test_numbering_matches_coordinates(N, nel):
    """Nodes share a global id iff they sit at the same physical point."""
    vtx = synth.box_vertices(nel, perturb=0.1, seed=11)
    _, _, X = oracle.geometry(N, nel, vtx, want_X=True)
    pts = np.round(X.transpose(0, 2, 1).reshape(-1, 3) * 1e8).astype(np.int64)
    _, coord_id = np.unique(pts, axis=0, return_inverse=True)
    gid, _, mask = oracle.numbering(N, nel)
    # same partition: gid -> coord id is a bijection
    pairs = np.unique(np.stack([gid, coord_id.ravel()], 1), axis=0)
    assert len(pairs) == len(np.unique(gid)) == len(np.unique(coord_id))
    # the mask marks exactly the points on the box faces
    lo, hi = vtx.min(0), vtx.max(0)
    P = X.transpose(0, 2, 1).reshape(-1, 3)
    onb = np.any(np.isclose(P, lo, atol=1e-12) | np.isclose(P, hi, atol=1e-12), axis=1)
    assert np.array_equal(onb, mask == 0)


@pytest.mark.parametrize("N,nel", [(1, (2, 2, 2)), (3, (3, 2, 2)), (5, (2, 2, 3))])
def test_segments_sorted_and_complete(N, nel):
    gid, mult, mask = oracle.numbering(N, nel)
    perm, seg_ptr, flag = oracle.segments(N, nel, gid, mask)
    n = N + 1
    q = np.arange(len(gid)) % n ** 3
    i, j, k = q % n, (q // n) % n, q // (n * n)
    surf = np.flatnonzero((i == 0) | (i == N) | (j == 0) | (j == N) | (k == 0) | (k == N))
    order = surf[np.lexsort((surf, gid[surf]))]
    assert np.array_equal(perm, order.astype(np.int32))
    starts = np.flatnonzero(np.r_[True, np.diff(gid[perm]) != 0])
    assert np.array_equal(seg_ptr, np.r_[starts, len(perm)].astype(np.int32))
    assert np.array_equal(flag, (mask[perm[starts]] == 0).astype(np.int8))
    # segment length = multiplicity unless the node is only on the outer boundary
    lens = np.diff(seg_ptr)
    assert np.array_equal(lens, mult[perm[starts]])


# ------------------------------------------------------------------- geometry

@pytest.mark.parametrize("N,nel,hi", [(3, (2, 2, 2), None), (5, (4, 4, 4), (1.0, 1.0, 1.0)), (7, (1, 2, 1), None)])
def test_geometry_affine_closed_form(N, nel, hi):
    vtx = synth.box_vertices(nel, hi=hi)
    g, B, _ = oracle.geometry(N, nel, vtx)
    h = 1.0 if hi is None else 1.0 / nel[0]
    _, w = oracle.gll(N)
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    for q in range(3):
        np.testing.assert_allclose(g[:, q], np.broadcast_to((h / 2) * W, g[:, q].shape), rtol=1e-14)
    np.testing.assert_allclose(g[:, 3:], 0.0, atol=1e-15)
    np.testing.assert_allclose(B, np.broadcast_to((h / 2) ** 3 * W, B.shape), rtol=1e-14)


def test_geometry_deformed_volume():
    nel = (3, 3, 3)
    vtx = synth.box_vertices(nel, hi=(1.0, 2.0, 0.5), perturb=0.1, seed=5)
    for N in (2, 5):
        _, B, X = oracle.geometry(N, nel, vtx, want_X=True)
        assert abs(B.sum() - 1.0) < 1e-13
        # corner GLL nodes coincide with the element vertices
        n = N + 1
        corners = [0, N, N * n, N + N * n, N * n * n, N + N * n * n, N * n + N * n * n, n ** 3 - 1]
        Xc = X[:, :, corners].transpose(0, 2, 1).reshape(-1, 3)
        d = np.min(np.linalg.norm(Xc[:, None, :] - vtx[None, :, :], axis=2), axis=1)
        assert d.max() < 1e-15


def test_geometry_rejects_inverted_element():
    nel = (2, 2, 2)
    vtx = synth.box_vertices(nel)
    centre = 1 + 3 * (1 + 3 * 1)
    vtx[centre] = [2.6, 2.6, 2.6]       # pushes the centre vertex through a corner element
    with pytest.raises(ValueError):
        oracle.geometry(3, nel, vtx)


# ------------------------------------------------------------------- operator

def _problem(N, nel, perturb=0.1, seed=7, hi=None, want_X=False):
    return oracle.Problem(N, nel, synth.box_vertices(nel, hi=hi, perturb=perturb, seed=seed), want_X=want_X)


@pytest.mark.parametrize("N", [2, 5, 9])
def test_ax_annihilates_constants(N):
    P = _problem(N, (3, 2, 2))
    w = P.ax_local(np.ones(P.nl))
    scale = np.abs(P.g).max() * (N + 1) ** 2
    assert np.abs(w).max() < 1e-14 * scale


def test_ax_symmetric():
    P = _problem(5, (2, 3, 2))
    r = synth.rng(3)
    u, v = r.random(P.nl), r.random(P.nl)
    # element level: u_L^T A_L v_L = v_L^T A_L u_L for any local vectors
    a, b = np.dot(u, P.ax_local(v)), np.dot(v, P.ax_local(u))
    assert abs(a - b) < 1e-12 * abs(a)
    # assembled and masked, on continuous vectors (weighted inner product)
    uc, vc = P.dssum(P.c * u), P.dssum(P.c * v)
    a, b = P.glsc3(uc, P.A(vc)), P.glsc3(vc, P.A(uc))
    assert abs(a - b) < 1e-12 * abs(a)
    assert P.glsc3(uc, P.A(uc)) > 0


@pytest.mark.parametrize("N", [2, 4, 7])
def test_volume_identity(N):
    """For u = x_d (a coordinate), a(u,v) = int grad x_d . grad x_e = |Omega| delta_de,
    exact for trilinear elements under GLL quadrature with N >= 2."""
    hi = (1.0, 2.0, 0.5)
    P = _problem(N, (3, 2, 3), hi=hi, want_X=True)
    vol = hi[0] * hi[1] * hi[2]
    Xl = [P.X[:, d].ravel() for d in range(3)]
    AX = [P.ax_local(x) for x in Xl]
    for d in range(3):
        for e in range(3):
            val = np.dot(Xl[d], AX[e])
            assert abs(val - (vol if d == e else 0.0)) < 1e-12, (d, e, val)


def test_worked_example_single_element(golden):
    ref = golden["single_element_N2"]
    P = _problem(2, (1, 1, 1), perturb=0)
    centre = 1 + 3 * (1 + 3 * 1)
    u = np.zeros(P.nl)
    u[centre] = 1.0
    assert abs(P.A(u)[centre] - _val(ref["A_centre"])) < 1e-14
    x, it, _ = P.cg(np.ones(P.nl), tol=1e-14, maxit=5)
    assert abs(x[centre] - _val(ref["x_centre_unit_load"])) < 1e-16
    assert it == 1


def test_worked_example_two_cubed(golden):
    P = _problem(1, (2, 2, 2), perturb=0, hi=(1.0, 1.0, 1.0))
    u = (P.gid == 13).astype(np.float64)
    Au = P.A(u)
    assert np.allclose(Au[P.gid == 13], _val(golden["two_cubed_N1"]["A_centre"]), rtol=0, atol=1e-14)
    assert np.all(Au[P.mask == 0] == 0)


# ------------------------------------------------------------ gather-scatter

def test_dssum_sums_copies_in_order():
    P = _problem(3, (2, 2, 2))
    r = synth.rng(9)
    w = r.random(P.nl)
    s = P.dssum(w, masked=False)
    # brute force: group copies by global id, ascending local index, plain Python sum
    for g_ in r.choice(P.ng, size=200, replace=False):
        idx = np.flatnonzero(P.gid == g_)
        acc = 0.0
        for l in idx:
            acc += float(w[l])
        assert np.all(s[idx] == acc)
    m = P.dssum(w, masked=True)
    assert np.all(m[P.mask == 0] == 0) and np.array_equal(m[P.mask == 1], s[P.mask == 1])


def test_glsc3_vs_exact_sum():
    r = synth.rng(4)
    n = 200_000
    a = r.normal(size=n) * 10.0 ** r.integers(-8, 8, size=n)
    b = r.normal(size=n)
    c = 1.0 / r.choice([1.0, 2.0, 4.0, 8.0], size=n)
    terms = a * c * b
    exact = math.fsum(terms.tolist())
    got = oracle.glsc3(a, c, b)
    assert abs(got - exact) <= 2 * np.spacing(abs(exact))
    plain = oracle.glsc3_plain(a, c, b)
    assert abs(plain - exact) <= 1e-10 * np.abs(terms).sum()


# -------------------------------------------------------------------- solves

def _dense_reference(N, nel, vtx, f):
    """Solution of the dense global system of _dense_system, mapped to local nodes."""
    K, b, cid, free = _dense_system(N, nel, vtx, f)
    xg = np.zeros(len(b))
    xg[free] = np.linalg.solve(K[np.ix_(free, free)], b[free])
    return xg[cid], int(free.sum())


def _dense_system(N, nel, vtx, f):
    """Dense global stiffness from an independent route: Lagrange derivatives by
    NumPy polynomials, J = D X (not the analytic trilinear derivative), J^{-1}
    and det by numpy.linalg, global identification by physical coordinates.
    Returns (K, b, local -> global map, free (non-Dirichlet) global nodes)."""
    xi, w = oracle.gll(N)
    Dt = _lagrange_deriv_numpy(xi)
    n = N + 1
    I = np.eye(n)
    Dr, Ds, Dtt = np.kron(I, np.kron(I, Dt)), np.kron(I, np.kron(Dt, I)), np.kron(Dt, np.kron(I, I))
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    _, _, X = oracle.geometry(N, nel, vtx, want_X=True)
    pts = np.round(X.transpose(0, 2, 1).reshape(-1, 3) * 1e9).astype(np.int64)
    uniq, cid = np.unique(pts, axis=0, return_inverse=True)
    cid = cid.ravel()
    ng = len(uniq)
    K = np.zeros((ng, ng))
    E = X.shape[0]
    for e in range(E):
        Xe = X[e]
        J = np.stack([np.stack([Dm @ Xe[d] for Dm in (Dr, Ds, Dtt)], -1) for d in range(3)], 1)  # [q, d, a]
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)                                   # [q, a, d] = dr_a/dx_d
        Gr = np.stack([Dr, Ds, Dtt], -1)                          # [q, basis, a]
        Gx = np.einsum("qad,qba->qbd", Jinv, Gr)                  # physical gradients
        Ke = np.einsum("q,qad,qbd->ab", W * det, Gx, Gx)
        ids = cid[e * n ** 3:(e + 1) * n ** 3]
        K[np.ix_(ids, ids)] += Ke
    b = np.bincount(cid, weights=f, minlength=ng)
    lo, hi = vtx.min(0), vtx.max(0)
    P = uniq / 1e9
    free = ~np.any(np.isclose(P, lo, atol=1e-8) | np.isclose(P, hi, atol=1e-8), axis=1)
    return K, b, cid, free


def test_cg_matches_dense_solve():
    N, nel = 4, (2, 2, 2)
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=12)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 13)
    xd, nfree = _dense_reference(N, nel, vtx, f)
    x, it, hist = P.cg(f, tol=1e-14, maxit=2000)
    assert np.abs(x - xd).max() <= 1e-12 * np.abs(xd).max()
    assert it <= nfree
    assert P.true_residual(x, f) < 1e-13
    # the exact solution as initial guess survives the projection M o dssum(c o x0)
    _, _, h0 = P.cg(f, x0=xd, tol=1e-14, maxit=2000)
    assert h0[0] < 1e-11
    # a projected initial guess gives the same solution
    x2, _, _ = P.cg(f, x0=xd + 1e-3 * synth.rng(1).random(P.nl), tol=1e-14, maxit=2000)
    assert np.abs(x2 - xd).max() <= 1e-12 * np.abs(xd).max()


def test_cg_fixed_iterations_and_history():
    P = _problem(3, (2, 2, 2), perturb=0)
    f = synth.uniform_load(P.nl, 1)
    x, it, hist = P.cg(f, tol=0.0, maxit=17)
    assert it == 17 and len(hist) == 18 and hist[0] == 1.0
    assert hist[-1] < hist[0]
    # an exact initial guess ends the solve before the first iteration
    xe, _, _ = P.cg(f, tol=1e-14, maxit=500)
    x2, it2, h2 = P.cg(f, x0=xe, tol=1e-10, maxit=5)
    assert it2 == 0 and np.allclose(x2, xe, rtol=4e-16, atol=0)   # projection may move 1 ulp
    x3, it3, _ = P.cg(np.zeros(P.nl), tol=1e-10, maxit=5)
    assert it3 == 0 and not x3.any()


def test_cg_power_of_two_scaling():
    """For affine meshes A(h) = (h/2) A(2); with h/2 a power of two every
    product is scaled exactly, so histories and iteration counts agree bit for bit."""
    f = synth.uniform_load(4 ** 3 * 6 ** 3, 2)
    Pa = _problem(5, (4, 4, 4), perturb=0)
    Pb = _problem(5, (4, 4, 4), perturb=0, hi=(1.0, 1.0, 1.0))
    xa, ia, ha = Pa.cg(f, tol=1e-8, maxit=500)
    xb, ib, hb = Pb.cg(f, tol=1e-8, maxit=500)
    assert ia == ib and np.array_equal(ha, hb)
    assert np.array_equal(xa, xb * 0.25)


def test_manufactured_solution_converges_spectrally():
    """-lap u = 3 pi^2 u for u = sin(pi x) sin(pi y) sin(pi z) on [0,1]^3, on a
    deformed 2^3 mesh: the nodal error must fall geometrically with N."""
    nel = (2, 2, 2)
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=21)
    errs = []
    for N in (3, 5, 7, 9):
        P = oracle.Problem(N, nel, vtx, want_X=True)
        u = synth.sine_field(P.X).ravel()
        f = P.B.ravel() * (3 * np.pi ** 2) * u
        x, it, _ = P.cg(f, tol=1e-14, maxit=5000)
        errs.append(np.abs(x - u)[P.mask == 1].max())
    for a, b in zip(errs, errs[1:]):
        assert b < a / 50, errs
    assert errs[-1] < 1e-9, errs


# ------------------------------------------------- diagonal preconditioner

@pytest.mark.parametrize("N,nel,perturb", [(4, (2, 2, 2), 0.1), (3, (3, 2, 1), 0.1), (5, (1, 2, 2), 0.0)])
def test_diag_is_diagonal_of_dense_stiffness(N, nel, perturb):
    """or_diag against the diagonal of the independently assembled dense K."""
    vtx = synth.box_vertices(nel, hi=tuple(0.5 * v for v in nel), perturb=perturb, seed=21)
    P = oracle.Problem(N, nel, vtx)
    m = P.diag()
    K, _, cid, free = _dense_system(N, nel, vtx, np.zeros(P.nl))
    Kd = np.diag(K)[cid]
    on = free[cid]
    assert np.abs(m[on] - Kd[on]).max() <= 1e-12 * np.abs(Kd[on]).max()
    assert np.all(m[~on] == 1.0) and np.all(m[on] > 0)
    # equal on every copy of a node
    for gval in np.unique(P.gid)[:200]:
        assert np.unique(m[P.gid == gval]).size == 1


def test_pcg_unit_preconditioner_is_cg_bit_for_bit():
    nel, N = (3, 2, 2), 5
    vtx = synth.box_vertices(nel, perturb=0.1, seed=22)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 23)
    x0, it0, h0 = P.cg(f, tol=0.0, maxit=50)
    x1, it1, h1 = P.pcg(f, np.ones(P.nl), tol=0.0, maxit=50)
    assert it1 == it0 and np.array_equal(x1, x0) and np.array_equal(h1, h0)


def test_pcg_power_of_two_scalar_preconditioner_is_cg_bit_for_bit():
    """m = 4: z = r/4, rtz = rtr/4, p and w scale by 1/4, pap by 1/16 and alpha
    by 4, all exactly in binary arithmetic, so x and the residuals equal CG's.
    A loop that mixes up r and z, or alpha's numerator, fails this."""
    nel, N = (2, 2, 2), 4
    vtx = synth.box_vertices(nel, perturb=0.1, seed=24)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 25)
    x0, it0, h0 = P.cg(f, tol=0.0, maxit=40)
    x1, it1, h1 = P.pcg(f, np.full(P.nl, 4.0), tol=0.0, maxit=40)
    assert it1 == it0 and np.array_equal(x1, x0) and np.array_equal(h1, h0)


def test_pcg_matches_dense_solve_and_saves_iterations():
    N, nel = 4, (2, 2, 2)
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=12)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 13)
    xd, nfree = _dense_reference(N, nel, vtx, f)
    x, it, hist = P.pcg(f, P.diag(), tol=1e-14, maxit=2000)
    assert np.abs(x - xd).max() <= 1e-12 * np.abs(xd).max()
    assert it <= nfree and P.true_residual(x, f) < 1e-13
    # Jacobi scaling helps on the spectral-element operator (GLL weights vary
    # strongly across an element)
    nel, N = (4, 4, 4), 7
    vtx = synth.box_vertices(nel)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, synth.SEED_C1)
    _, it_cg, _ = P.cg(f, tol=1e-8, maxit=2000)
    xp, it_pcg, _ = P.pcg(f, P.diag(), tol=1e-8, maxit=2000)
    assert it_pcg < 0.92 * it_cg
    assert P.true_residual(xp, f) <= 1e-8


def test_openmp_build_is_bit_identical():
    """The all-core build of the oracle (OpenMP over elements and element-wise
    updates, serial fixed-order reductions and gather-scatter) returns the
    serial build's iterates and history bit for bit."""
    nel, N = (3, 4, 2), 6
    vtx = synth.box_vertices(nel, perturb=0.1, seed=13)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 14)
    oracle.omp_threads(3)
    a = P.cg(f, tol=0.0, maxit=40)
    b = P.cg(f, tol=0.0, maxit=40, omp=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
