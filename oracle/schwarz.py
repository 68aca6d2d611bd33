"""Oracle of the two-level overlapping Schwarz preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): FP64 NumPy, sharing no
code with the GPU path.

The paper names the call graph of Nekbone's preconditioner only (Fig. 3:
solveM -> h1mg_schwarz -> h1mg_extrude, h1mg_fdm -> h1mg_do_fast ->
h1mg_tnsr3d_el); the algorithm below is the reading this project takes of
it, a two-level additive Schwarz method:

    M^-1 r = sum_e R_e^T A~_e^-1 R_e r  +  P A~_c^-1 P^T r .

Nodes are addressed on the global lattice (gi, gj, gk), gi = ex N + i.

Fine level (overlapping Schwarz, "extrude" + fast diagonalization).  The
subdomain of element e is the element's nodes extended by one node into
each face neighbour: along x the window gi = ex N - 1 .. ex N + N + 1
(N + 3 nodes), clipped to the unknowns 1 .. Gx - 2 (Dirichlet nodes and
nodes beyond the box are left out); likewise along y and z.  R_e picks the
window's values.  A~_e is the separable operator of a uniform mesh of
elements with e's mean edge lengths (hx, hy, hz) restricted to the window:
    A~_e = 1/2 [cx Kw (x) Ww (x) Ww + cy Ww (x) Kw (x) Ww + cz Ww (x) Ww (x) Kw],
cx = hy hz / hx, cy = hx hz / hy, cz = hx hy / hz, where Kw, Ww are the
1-D GLL stiffness D^T W D and mass W of three reference elements assembled
and restricted to the window (own element plus the neighbours' nodes next
to the shared faces).  It is inverted by fast diagonalization: Kw S = Ww S L,
S^T Ww S = I, per direction and window variant (interior, clipped on the
left, on the right, on both sides).  On a uniform box mesh A~_e equals the
restriction R_e A R_e^T of the assembled operator exactly.

Coarse level.  P interpolates the vertex lattice to the GLL nodes with the
trilinear (Q1) functions of the reference coordinates: P = Px (x) Py (x) Pz,
(Px)[gi, v] = l_v(xi_i) for the element ex containing gi, l_0 = (1 - xi)/2,
l_1 = (1 + xi)/2; only interior vertices are coarse unknowns.  A~_c is the
separable Q1 operator of the rectilinear lattice whose spacing along each
direction is the mean length of the elements of that slab, with the 1-D
mass integrated by the GLL rule of order N (exact, i.e. consistent, for
N >= 2):  A~_c = K1x (x) M1y (x) M1z + M1x (x) K1y (x) M1z + M1x (x) M1y (x) K1z,
inverted by fast diagonalization.  For any rectilinear mesh A~_c equals the
Galerkin operator P^T A P.

Both terms are symmetric positive (semi)definite, the sum definite, so
M^-1 serves as solveM in Table 1's loop (oracle.fdm.pcg).
"""
from __future__ import annotations

import numpy as np


def _gll(N):
    import oracle
    return oracle.gll(N)


def window_operators(N: int, D, w):
    """1-D stiffness and (diagonal) mass of three assembled reference elements
    restricted to the N + 3 window nodes: the left neighbour's node N - 1,
    the element's nodes 0..N, the right neighbour's node 1."""
    K = D.T @ np.diag(w) @ D
    n3 = 3 * N + 1
    Ka = np.zeros((n3, n3))
    Wa = np.zeros(n3)
    for q in range(3):
        s = q * N
        Ka[s:s + N + 1, s:s + N + 1] += K
        Wa[s:s + N + 1] += w
    idx = np.arange(N - 1, 2 * N + 2)
    return Ka[np.ix_(idx, idx)], Wa[idx]


def gen_eig_diag(K, m):
    """K S = diag(m) S L with S^T diag(m) S = I."""
    s = 1.0 / np.sqrt(m)
    lam, V = np.linalg.eigh(s[:, None] * K * s[None, :])
    return s[:, None] * V, lam


def window_variants(N: int, D, w):
    """(S, lam) on the kept window indices for the variants (left clipped,
    right clipped) in {0, 1}^2, keyed by (lo, hi)."""
    Kw, Ww = window_operators(N, D, w)
    out = {}
    for lo in (0, 1):
        for hi in (0, 1):
            keep = np.arange(2 if lo else 0, N + 1 if hi else N + 3)
            S, lam = gen_eig_diag(Kw[np.ix_(keep, keep)], Ww[keep])
            out[(lo, hi)] = (keep, S, lam)
    return out


def mean_lengths(nel, vtx):
    """Per element the mean length of its four edges along x, y, z: [E, 3]."""
    nx, ny, nz = (int(v) for v in nel)
    V = np.asarray(vtx, dtype=np.float64).reshape(nz + 1, ny + 1, nx + 1, 3)
    hx = np.linalg.norm(V[:, :, 1:] - V[:, :, :-1], axis=-1)
    hy = np.linalg.norm(V[:, 1:, :] - V[:, :-1, :], axis=-1)
    hz = np.linalg.norm(V[1:, :, :] - V[:-1, :, :], axis=-1)
    Hx = 0.25 * (hx[:-1, :-1] + hx[:-1, 1:] + hx[1:, :-1] + hx[1:, 1:])
    Hy = 0.25 * (hy[:-1, :, :-1] + hy[:-1, :, 1:] + hy[1:, :, :-1] + hy[1:, :, 1:])
    Hz = 0.25 * (hz[:, :-1, :-1] + hz[:, :-1, 1:] + hz[:, 1:, :-1] + hz[:, 1:, 1:])
    return np.stack([Hx, Hy, Hz], axis=-1).reshape(-1, 3)   # e = ex + nx (ey + ny ez)


def q1_line(h, N: int):
    """1-D Q1 stiffness and mass (mass by the GLL rule of order N) assembled on
    a line of len(h) elements of lengths h, restricted to the interior
    vertices."""
    xi, w = _gll(N)
    l0, l1 = (1.0 - xi) / 2.0, (1.0 + xi) / 2.0
    me = np.array([[np.sum(w * l0 * l0), np.sum(w * l0 * l1)], [np.sum(w * l1 * l0), np.sum(w * l1 * l1)]])
    ke = np.array([[1.0, -1.0], [-1.0, 1.0]])
    n = len(h)
    K = np.zeros((n + 1, n + 1))
    M = np.zeros((n + 1, n + 1))
    for e in range(n):
        K[e:e + 2, e:e + 2] += ke / h[e]
        M[e:e + 2, e:e + 2] += me * (h[e] / 2.0)
    return K[1:n, 1:n], M[1:n, 1:n]


def gen_eig(K, M):
    """K S = M S L with S^T M S = I (M symmetric positive definite)."""
    L = np.linalg.cholesky(M)
    Li = np.linalg.inv(L)
    lam, V = np.linalg.eigh(Li @ K @ Li.T)
    return Li.T @ V, lam


def q1_interp(N: int, n: int):
    """(n N + 1) x (n + 1) matrix of the Q1 interpolation along one direction."""
    xi, _ = _gll(N)
    Pm = np.zeros((n * N + 1, n + 1))
    for e in range(n):
        for i in range(N + 1):
            Pm[e * N + i, e] = (1.0 - xi[i]) / 2.0
            Pm[e * N + i, e + 1] = (1.0 + xi[i]) / 2.0
    return Pm


class Schwarz:
    """z = M^-1 r for one problem (oracle.Problem P with vertex lattice vtx)."""

    def __init__(self, P, vtx):
        if P.N < 2:
            raise ValueError("the overlapping Schwarz preconditioner needs N >= 2")
        self.P = P
        N = P.N
        self.nel = P.nel
        self.G = tuple(v * N + 1 for v in P.nel)
        _, w = _gll(N)
        self.var = window_variants(N, P.D, w)
        H = mean_lengths(P.nel, vtx)
        self.c = np.stack([H[:, 1] * H[:, 2] / H[:, 0], H[:, 0] * H[:, 2] / H[:, 1],
                           H[:, 0] * H[:, 1] / H[:, 2]], axis=-1)
        nx, ny, nz = P.nel
        Hg = H.reshape(nz, ny, nx, 3)
        self.coarse = []
        self.Pd = []
        for d, n in enumerate(P.nel):
            h = Hg[..., d].mean(axis=tuple(a for a in range(3) if a != 2 - d))   # slab means along d
            K1, M1 = q1_line(h, N)
            S, lam = gen_eig(K1, M1) if n > 1 else (np.zeros((0, 0)), np.zeros(0))
            self.coarse.append((S, lam))
            self.Pd.append(q1_interp(N, n)[:, 1:n])   # interior vertex columns

    # -- global lattice <-> local layout
    def to_global(self, r):
        P = self.P
        g = np.zeros(P.ng)
        g[P.gid] = r                     # every copy holds the same value
        Gx, Gy, Gz = self.G
        return g.reshape(Gz, Gy, Gx)     # [gk][gj][gi]

    def to_local(self, g):
        return g.reshape(-1)[self.P.gid]

    def window(self, e):
        """Global lattice indices (x, y, z) of element e's subdomain and the
        window variants' (S, lam) along each direction."""
        N = self.P.N
        nx, ny, nz = self.nel
        ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
        parts = []
        for ed, nd in ((ex, nx), (ey, ny), (ez, nz)):
            keep, S, lam = self.var[(int(ed == 0), int(ed == nd - 1))]
            parts.append((ed * N - 1 + keep, S, lam))
        return parts

    def local_solve(self, e, rg):
        """A~_e^-1 R_e r for element e, on its window [z][y][x]."""
        (ix, Sx, lx), (iy, Sy, ly), (iz, Sz, lz) = self.window(e)
        Rl = rg[np.ix_(iz, iy, ix)]                       # [c][b][a]
        T = np.einsum("am,cba->cbm", Sx, Rl)               # S^T along x
        T = np.einsum("bm,cbn->cmn", Sy, T)                # along y
        T = np.einsum("cm,cnp->mnp", Sz, T)                # along z
        cx, cy, cz = self.c[e]
        T = 2.0 * T / (cx * lx[None, None, :] + cy * ly[None, :, None] + cz * lz[:, None, None])
        T = np.einsum("cm,mnp->cnp", Sz, T)                # S along z
        T = np.einsum("bm,cmn->cbn", Sy, T)                # along y
        return np.einsum("am,cbm->cba", Sx, T)             # along x

    def schwarz(self, rg):
        """sum_e R_e^T A~_e^-1 R_e r on the global lattice."""
        z = np.zeros_like(rg)
        for e in range(self.P.E):
            (ix, _, _), (iy, _, _), (iz, _, _) = self.window(e)
            z[np.ix_(iz, iy, ix)] += self.local_solve(e, rg)
        return z

    def coarse_correction(self, rg):
        """P A~_c^-1 P^T r on the global lattice."""
        Px, Py, Pz = self.Pd
        if min(m.shape[1] for m in self.Pd) == 0:
            return np.zeros_like(rg)
        rc = np.einsum("ia,jb,kc,kji->cba", Px, Py, Pz, rg)           # P^T r, [vz][vy][vx]
        (Sx, lx), (Sy, ly), (Sz, lz) = self.coarse
        T = np.einsum("am,cba->cbm", Sx, rc)
        T = np.einsum("bm,cbn->cmn", Sy, T)
        T = np.einsum("cm,cnp->mnp", Sz, T)
        T = T / (lx[None, None, :] + ly[None, :, None] + lz[:, None, None])
        T = np.einsum("cm,mnp->cnp", Sz, T)
        T = np.einsum("bm,cmn->cbn", Sy, T)
        ec = np.einsum("am,cbm->cba", Sx, T)
        return np.einsum("ia,jb,kc,cba->kji", Px, Py, Pz, ec)

    def apply(self, r, coarse: bool = True):
        rg = self.to_global(np.asarray(r, dtype=np.float64))
        z = self.schwarz(rg)
        if coarse:
            z = z + self.coarse_correction(rg)
        return self.to_local(z)
