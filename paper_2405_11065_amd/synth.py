"""Seeded synthetic inputs shared by the GPU path, the tests and the oracle.

Holds none of the solver's arithmetic: it only draws random numbers and lays
out mesh vertices, so both sides receive identical bits.  Every generator
uses NumPy's PCG64 with an explicit seed.

Workloads (the paper's Nekbone inputs are not public, so every workload here
is synthetic):
  * box meshes of unit-cube or [0,1]^3 hexahedra, optionally with interior
    vertices moved by up to +-10 % of the element size;
  * load vectors f ~ U[0,1) per local node;
  * manufactured forcing sin(pi x) sin(pi y) sin(pi z) plus N(0, sigma) noise;
  * Gaussian random fields (squared-exponential kernel) by random Fourier
    features, for training the initial-guess network;
  * batches of independent cube problems, n_e^3 elements with n_e uniform on
    an integer range and the order uniform over a set.
"""
from __future__ import annotations

import numpy as np

# Seeds of the named workloads.
SEED_C1 = 1
SEED_C2 = 2
SEED_C3 = 3
SEED_C3_VERTICES = 3003
SEED_C4 = 4
SEED_C5 = 5


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def box_vertices(nel, lo=(0.0, 0.0, 0.0), hi=None, perturb: float = 0.0, seed: int | None = None):
    """Vertex lattice of a box of nel[0] x nel[1] x nel[2] hexahedra.

    Returns float64 [(nel0+1)(nel1+1)(nel2+1), 3], x-index fastest.  ``hi``
    defaults to lo + nel (unit-cube elements).  With ``perturb`` > 0 every
    interior vertex coordinate moves by U(-perturb*h_d, +perturb*h_d), drawn
    from PCG64(seed) in lattice order (x, y, z per vertex); boundary vertices
    stay put so the box faces remain planar.
    """
    nel = tuple(int(v) for v in nel)
    lo = np.asarray(lo, dtype=np.float64)
    hi = lo + np.asarray(nel, dtype=np.float64) if hi is None else np.asarray(hi, dtype=np.float64)
    axes = [lo[d] + (hi[d] - lo[d]) * (np.arange(nel[d] + 1, dtype=np.float64) / nel[d]) for d in range(3)]
    for d in range(3):
        axes[d][-1] = hi[d]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    v = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).copy()
    if perturb > 0:
        h = (hi - lo) / np.asarray(nel, dtype=np.float64)
        delta = rng(seed).uniform(-1.0, 1.0, size=v.shape) * (perturb * h)[None, :]
        iz, iy, ix = np.meshgrid(np.arange(nel[2] + 1), np.arange(nel[1] + 1), np.arange(nel[0] + 1), indexing="ij")
        interior = ((ix > 0) & (ix < nel[0]) & (iy > 0) & (iy < nel[1]) & (iz > 0) & (iz < nel[2])).ravel()
        v[interior] += delta[interior]
    return v


def uniform_load(n_local: int, seed: int) -> np.ndarray:
    """f ~ U[0,1) per local node, FP64, local order."""
    return rng(seed).random(int(n_local))


def normal_noise(n_local: int, sigma: float, seed: int) -> np.ndarray:
    return rng(seed).normal(0.0, sigma, size=int(n_local))


def sine_field(X: np.ndarray) -> np.ndarray:
    """sin(pi x) sin(pi y) sin(pi z) at coordinates X[..., 3, :] (x, y, z planes)."""
    return np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])


class FourierFieldDraw:
    """One Gaussian random field with squared-exponential covariance.

    exp(-|x-y|^2 / (2 l^2)) is approximated by M random Fourier features:
    F(x) = sqrt(2/M) sum_m a_m cos(omega_m . x + phi_m), omega ~ N(0, I/l^2),
    phi ~ U[0, 2 pi), a ~ N(0, 1).
    """

    def __init__(self, seed: int, length: float = 0.2, features: int = 256):
        r = rng(seed)
        self.omega = r.normal(0.0, 1.0 / length, size=(features, 3))
        self.phi = r.uniform(0.0, 2 * np.pi, size=features)
        self.a = r.normal(0.0, 1.0, size=features)
        self.scale = np.sqrt(2.0 / features)

    def __call__(self, X: np.ndarray) -> np.ndarray:
        """Evaluate at coordinates X[E, 3, n3] -> [E, n3]."""
        E, _, n3 = X.shape
        pts = X.transpose(0, 2, 1).reshape(-1, 3)
        out = np.empty(pts.shape[0])
        step = 1 << 18
        for s in range(0, pts.shape[0], step):
            ph = pts[s:s + step] @ self.omega.T + self.phi[None, :]
            out[s:s + step] = self.scale * (np.cos(ph) @ self.a)
        return out.reshape(E, n3)


def batch_draw(seed: int, nprob: int, ne_range=(2, 24), orders=(5, 7, 9, 11)):
    """Sizes of a batch: problem i is an n_e^3 cube of unit elements of order N.

    n_e ~ uniform integer on [ne_range[0], ne_range[1]], N ~ uniform over
    ``orders``, both drawn from PCG64(seed) per problem (n_e first).
    """
    r = rng(seed)
    out = []
    for _ in range(int(nprob)):
        ne = int(r.integers(ne_range[0], ne_range[1] + 1))
        N = int(orders[int(r.integers(0, len(orders)))])
        out.append({"nel": (ne, ne, ne), "N": N})
    return out


def batch_load_seed(seed: int, i: int) -> int:
    """Seed of problem i's load vector in a batch drawn with ``seed``."""
    return int(seed) * 100003 + int(i)


def mlp_init(sizes, seed: int):
    """Initial parameters [W1, b1, W2, b2, ...] (float32) of a perceptron with
    layer widths ``sizes``: W_l (fan_out, fan_in) ~ U(-a, a) with
    a = sqrt(6 / (fan_in + fan_out)), biases 0; drawn from PCG64(seed) layer
    by layer."""
    r = rng(seed)
    out = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        a = np.sqrt(6.0 / (fi + fo))
        out.append(r.uniform(-a, a, size=(fo, fi)).astype(np.float32))
        out.append(np.zeros(fo, dtype=np.float32))
    return out
