"""FP64 reference of the learned initial guess around the network.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).

Per element e of a problem (``oracle.Problem``), with F = f / B pointwise (the
forcing values behind the local load vector f = B o F):

  * scale  s_e = sqrt(mean over the element's points of F^2);
  * inputs  [F_e / s_e (the element's (N+1)^3 values, local order),
             q_1..q_6], q_k = (sum_e G_k / sum_e B) / ((q_rr + q_ss + q_tt) / 3)
            with G in the order rr, ss, tt, rs, rt, st: the element's volume
            average of J^-1 J^-T, normalised by its mean diagonal, so the six
            numbers describe the element's shape and not its size;
            an element with s_e = 0 gets zero forcing inputs;
  * targets T_e = x_e / (s_e kappa) for a solution x (0 where s_e = 0);
  * prediction x0_e = y_e s_e kappa for a network output y_e.

The local prediction is then made continuous and scaled:
  x0 <- M o dssum(c o x0)               (the projection nek_cg_solve applies)
  alpha = glsc3(x0, b) / glsc3(x0, A x0) (the A-norm best multiple of x0)
  x0 <- alpha x0,  rho0 = |b - A x0|_c / |b|_c
and the guess is dropped for zero (plain CG from zero) when x0 vanishes after
the projection (glsc3(x0, A x0) <= 0) or alpha is not finite, and, under the
residual policy, when rho0 >= 1.
"""
from __future__ import annotations

import numpy as np


def features(P, f, mode: int = 0):
    """(inputs [E, n3 + 6], scales [E]) of the load vector f on problem P.

    mode 0: element scale s_e = RMS of F over the element, shape numbers q;
    mode 1: global scale S = RMS of F over all local points, shape numbers q;
    mode 2: global scale S, centroid (sum B x / sum B) and q_rs, q_rt, q_st
            (P must be built with want_X)."""
    n3 = P.n ** 3
    B = np.asarray(P.B, dtype=np.float64).reshape(P.E, n3)
    F = np.asarray(f, dtype=np.float64).reshape(P.E, n3) / B
    if mode == 0:
        s = np.sqrt(np.mean(F * F, axis=1))
    else:
        s = np.full(P.E, np.sqrt(np.mean(F * F)))
    Fh = np.zeros_like(F)
    nz = s > 0
    Fh[nz] = F[nz] / s[nz, None]
    g = np.asarray(P.g, dtype=np.float64).reshape(P.E, 6, n3)
    q = g.sum(axis=2) / B.sum(axis=1)[:, None]
    q = q / ((q[:, 0] + q[:, 1] + q[:, 2]) / 3.0)[:, None]
    if mode == 2:
        X = np.asarray(P.X, dtype=np.float64).reshape(P.E, 3, n3)
        cen = (X * B[:, None, :]).sum(axis=2) / B.sum(axis=1)[:, None]
        q = np.concatenate([cen, q[:, 3:]], axis=1)
    return np.concatenate([Fh, q], axis=1), s


def targets(P, x, s, kappa):
    n3 = P.n ** 3
    xe = np.asarray(x, dtype=np.float64).reshape(P.E, n3)
    T = np.zeros_like(xe)
    nz = s > 0
    T[nz] = xe[nz] / (s[nz, None] * kappa)
    return T


def assemble(P, f, Y, s, kappa, residual_policy: bool = True):
    """(x0, alpha, rho0, used) from network outputs Y [E, n3]."""
    x0 = (np.asarray(Y, dtype=np.float64) * (s[:, None] * kappa)).ravel()
    x0 = P.dssum(P.c * x0, masked=True)
    b = P.rhs(f)
    Ax = P.A(x0)
    den = P.glsc3(x0, Ax)
    alpha = P.glsc3(x0, b) / den if den > 0 else np.nan
    if not np.isfinite(alpha):
        return np.zeros(P.nl), alpha, 1.0, False
    x0 = alpha * x0
    r = b - P.A(x0)
    rho0 = np.sqrt(P.glsc3(r, r)) / np.sqrt(P.glsc3(b, b))
    if residual_policy and not rho0 < 1.0:
        return np.zeros(P.nl), alpha, rho0, False
    return x0, alpha, rho0, True
