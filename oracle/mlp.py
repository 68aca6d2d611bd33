"""FP64 reference of the per-element initial-guess network.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``): only tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.
It shares no code with the GPU path.

The network is a plain multilayer perceptron with two hidden layers and the
SiLU activation, silu(z) = z * sigmoid(z):

    Z1 = X W1^T + b1,  H1 = silu(Z1)
    Z2 = H1 W2^T + b2, H2 = silu(Z2)
    Y  = H2 W3^T + b3

trained on the mean squared error L = sum((Y - T)^2) / (rows * outputs) with
Adam (Kingma and Ba, 2015: bias-corrected first and second moments).  The paper
does not contain this network; it is an addition of this project (an initial
guess for the paper's CG solve), so nothing here cites the paper.

Everything is FP64.  With ``bf16=True`` the GEMM operands are rounded to
bfloat16 (round to nearest even) at the points where the GPU stores them in
bfloat16: the input rows, the weight copies, H1 and H2, dY, dZ2 and dZ1.
Products are still accumulated in FP64 and every other quantity (Z, Y, the
bias gradients, Adam) stays FP64, so the GPU, which accumulates in FP32,
differs from this only by accumulation rounding and the rare bfloat16 rounding
decisions that rounding moves.

Parameters are the list [W1, b1, W2, b2, W3, b3] with W_l of shape
(fan_out, fan_in).
"""
from __future__ import annotations

import numpy as np


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of
    a binary32; rounding is applied once, from the float64 value, by scaling
    the value's binade to an integer grid of 2^8 steps per binade.
    """
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = a != 0
    m, e = np.frexp(a[nz])           # a = m * 2^e, 0.5 <= |m| < 1
    q = np.rint(m * 256.0)           # 8 significant bits (1 implicit + 7), rint = ties to even
    out[nz] = np.ldexp(q / 256.0, e)
    return out


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, bf16_points: bool = False):
    """Returns (Y, cache) for the rows of X."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    r = bf16 if bf16_points else (lambda a: np.asarray(a, dtype=np.float64))
    A0 = r(X)
    Z1 = A0 @ r(W1).T + b1
    H1 = r(silu(Z1))
    Z2 = H1 @ r(W2).T + b2
    H2 = r(silu(Z2))
    Y = H2 @ r(W3).T + b3
    return Y, (A0, Z1, H1, Z2, H2)


def loss_and_grads(params, X, T, bf16_points: bool = False):
    """Mean squared error of the network on (X, T) and its gradient w.r.t. every parameter."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    r = bf16 if bf16_points else (lambda a: np.asarray(a, dtype=np.float64))
    Y, (A0, Z1, H1, Z2, H2) = forward(params, X, bf16_points)
    T = np.asarray(T, dtype=np.float64)
    n = Y.size
    D = Y - T
    loss = float(np.sum(D * D) / n)
    dY = 2.0 * D / n
    dYr = r(dY)
    gW3 = dYr.T @ H2
    gb3 = dY.sum(axis=0)
    dZ2 = (dYr @ r(W3)) * dsilu(Z2)
    dZ2r = r(dZ2)
    gW2 = dZ2r.T @ H1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2r @ r(W2)) * dsilu(Z1)
    dZ1r = r(dZ1)
    gW1 = dZ1r.T @ A0
    gb1 = dZ1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step t >= 1); returns new (params, m, v)."""
    P, M, V = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1.0 - beta1) * g
        vi = beta2 * vi + (1.0 - beta2) * g * g
        mh = mi / (1.0 - beta1 ** t)
        vh = vi / (1.0 - beta2 ** t)
        P.append(p - lr * mh / (np.sqrt(vh) + eps))
        M.append(mi)
        V.append(vi)
    return P, M, V
