"""Oracle of the element-interior fast-diagonalization preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): FP64 NumPy, sharing no
code with the GPU path.

The preconditioner is a hybrid block-Jacobi form of the solveM step of the
paper's Table 1, the non-overlapping stage of the Schwarz smoother that
Nekbone's multigrid builds with the fast diagonalization method (Sect. 4.1,
Fig. 3): on the (N-1)^3 interior nodes of every element the element's own
stiffness block is inverted, the other nodes (faces, edges, vertices, shared
between elements) are scaled by the inverse diagonal of the assembled
operator.

Interior block of an element with side lengths (hx, hy, hz).  For an
axis-aligned box the element stiffness is separable,
    A_e = 1/2 [ (hy hz / hx) Wz (x) Wy (x) K + (hx hz / hy) Wz (x) K (x) Wx
              + (hx hy / hz) K (x) Wy (x) Wx ],
K = D^T W D the 1-D GLL stiffness and W = diag(w) the 1-D GLL mass.  On the
interior indices let K_I S = W_I S Lambda with S^T W_I S = I (a generalized
symmetric eigenproblem; W_I is diagonal, so it is the ordinary one of
W_I^-1/2 K_I W_I^-1/2).  Then
    A_II^-1 = 2 (S (x) S (x) S) diag(1 / (cx l_i + cy l_j + cz l_k)) (S (x) S (x) S)^T,
with cx = hy hz / hx, cy = hx hz / hy, cz = hx hy / hz.  For deformed
elements h_d is the mean length of the element's four edges along d (the
block is then an approximation of the element's; the preconditioner stays
symmetric positive definite).
"""
from __future__ import annotations

import numpy as np


def interior_eig(N: int, D, w):
    """S ((N-1) x (N-1), columns = modes) and lambda of K_I S = W_I S Lambda, S^T W_I S = I."""
    K = D.T @ np.diag(w) @ D
    KI = K[1:N, 1:N]
    wi = w[1:N]
    s = 1.0 / np.sqrt(wi)
    C = s[:, None] * KI * s[None, :]
    lam, V = np.linalg.eigh(C)
    S = s[:, None] * V
    return S, lam


def element_scales(nel, vtx):
    """Per element (cx, cy, cz) = (hy hz / hx, hx hz / hy, hx hy / hz), h_d the
    mean of the element's four edge lengths along direction d."""
    nx, ny, nz = (int(v) for v in nel)
    V = np.asarray(vtx, dtype=np.float64).reshape(nz + 1, ny + 1, nx + 1, 3)
    hx = np.linalg.norm(V[:, :, 1:] - V[:, :, :-1], axis=-1)          # [nz+1, ny+1, nx]
    hy = np.linalg.norm(V[:, 1:, :] - V[:, :-1, :], axis=-1)          # [nz+1, ny, nx+1]
    hz = np.linalg.norm(V[1:, :, :] - V[:-1, :, :], axis=-1)          # [nz, ny+1, nx+1]
    Hx = 0.25 * (hx[:-1, :-1] + hx[:-1, 1:] + hx[1:, :-1] + hx[1:, 1:])  # [nz, ny, nx]
    Hy = 0.25 * (hy[:-1, :, :-1] + hy[:-1, :, 1:] + hy[1:, :, :-1] + hy[1:, :, 1:])
    Hz = 0.25 * (hz[:, :-1, :-1] + hz[:, :-1, 1:] + hz[:, 1:, :-1] + hz[:, 1:, 1:])
    c = np.stack([Hy * Hz / Hx, Hx * Hz / Hy, Hx * Hy / Hz], axis=-1)
    return c.reshape(-1, 3)   # element order e = ex + nx (ey + ny ez)


class Fdm:
    """z = M^-1 r for one problem (oracle.Problem P)."""

    def __init__(self, P, vtx):
        self.P = P
        xi, w = _gll(P.N)
        self.S, self.lam = interior_eig(P.N, P.D, w)
        self.c = element_scales(P.nel, vtx)
        self.m = P.diag()   # 1 on Dirichlet nodes, where r is 0

    def apply(self, r):
        P = self.P
        N, n, E = P.N, P.n, P.E
        S, lam = self.S, self.lam
        z = np.asarray(r, dtype=np.float64) / self.m
        R = np.asarray(r, dtype=np.float64).reshape(E, n, n, n)[:, 1:N, 1:N, 1:N]   # [e][k][j][i]
        T = np.einsum("ia,ekji->ekja", S, R)        # S^T along i
        T = np.einsum("jb,ekja->ekba", S, T)        # along j
        T = np.einsum("kc,ekba->ecba", S, T)        # along k
        L = (self.c[:, 0, None, None, None] * lam[None, None, None, :]
             + self.c[:, 1, None, None, None] * lam[None, None, :, None]
             + self.c[:, 2, None, None, None] * lam[None, :, None, None])
        T = 2.0 * T / L
        T = np.einsum("kc,ecba->ekba", S, T)        # S along k
        T = np.einsum("jb,ekba->ekja", S, T)        # along j
        T = np.einsum("ia,ekja->ekji", S, T)        # along i
        Z = z.reshape(E, n, n, n).copy()
        Z[:, 1:N, 1:N, 1:N] = T
        return Z.reshape(-1)


def _gll(N):
    import oracle
    return oracle.gll(N)


def pcg(P, f, minv_apply, x0=None, tol: float = 1e-8, maxit: int = 1000):
    """Table-1 CG with solveM z = minv_apply(r), in the order of or_pcg (the
    operator, dssum, mask and glsc3 are the oracle's).  Returns (x, its, history)."""
    nl = P.nl
    b = P.rhs(f)
    if x0 is not None:
        x = P.dssum(P.c * np.asarray(x0, dtype=np.float64), masked=True)
    else:
        x = np.zeros(nl)
    w = P.A(x)
    r = b - w
    bb = P.glsc3(b, b)
    rn0 = P.glsc3(r, r)
    hist = [np.sqrt(rn0) / np.sqrt(bb) if bb > 0 else 0.0]
    it = 0
    if bb > 0 and not (rn0 == 0.0 or (tol > 0 and np.sqrt(rn0) / np.sqrt(bb) <= tol)):
        rtz1 = 1.0
        p = np.zeros(nl)
        for it in range(1, maxit + 1):
            z = minv_apply(r)
            rtz2 = rtz1
            rtz1 = P.glsc3(r, z)
            if rtz1 == 0.0:
                it -= 1
                break
            beta = 0.0 if it == 1 else rtz1 / rtz2
            p = beta * p + z
            w = P.A(p)
            pap = P.glsc3(w, p)
            if not np.isfinite(pap) or not (pap > 0):
                raise FloatingPointError("PCG breakdown")
            alpha = rtz1 / pap
            x = x + alpha * p
            r = r + (-alpha) * w
            res = np.sqrt(P.glsc3(r, r)) / np.sqrt(bb)
            hist.append(res)
            if tol > 0 and res <= tol:
                break
    return x, it, np.array(hist)
