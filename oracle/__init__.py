"""Serial FP64 CPU oracle for the spectral-element Poisson CG solve (Nekbone).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
never loads it, and it shares no code with the GPU path.

The arithmetic lives in ``nek_oracle.c`` (plain serial loops, FP64, built with
``-ffp-contract=off``); this module only marshals NumPy arrays through ctypes
and builds that file with gcc when its shared object is missing.

What each function follows (paper: Chen et al., "Enabling mixed-precision with
the help of tools: A Nekbone case study"):
  * ``cg``        -- the CG loop of Table 1 (solveM = copy, no preconditioner),
  * ``pcg``, ``diag`` -- the same loop with solveM the diagonal (Jacobi)
    preconditioner z = r / m, m the diagonal of the assembled operator,
  * ``ax_local``  -- ax_e of Fig. 2 (local_grad3 -> g1..g6 -> local_grad3_t),
  * ``glsc3``     -- the weighted dot product glsc3(a, c, b) of Table 1,
  * ``dssum``     -- the gather-scatter sum of copies of each shared node,
  * ``gll``, ``deriv``, ``geometry``, ``numbering`` -- the FP64 initialisation
    (kept in double precision in the paper's mixed build, Sect. 6).
The discretisation itself (GLL spectral elements, trilinear hexahedra,
homogeneous Dirichlet box) is not written in the paper; it is pinned by the
closed forms and invariants in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nek_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "nek_vprec.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i8 = ctypes.POINTER(ctypes.c_int8)
_int3 = ctypes.c_int * 3


def build(force: bool = False) -> str:
    """Compile nek_oracle.c into liboracle.so (plain gcc, no FMA contraction)
    and, from the same sources, liboracle_omp.so: -O3 with OpenMP for the
    all-core timing of the CPU baseline (bit-identical results; x86-64-v3,
    so the object built here also runs on the GPU machine's host)."""
    stale = lambda lib: force or not os.path.exists(lib) or os.path.getmtime(lib) < max(map(os.path.getmtime, _SRCS))
    for lib, flags in ((_LIB, ["-O2"]), (_LIB_OMP, ["-O3", "-march=x86-64-v3", "-fopenmp"])):
        if stale(lib):
            tmp = lib + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", *flags, "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                                   "-shared", "-o", tmp] + _SRCS + ["-lm"])
            os.replace(tmp, lib)
    return _LIB


def _get(omp: bool = False):
    global _lib, _lib_omp
    if omp:
        if _lib_omp is None:
            build()
            _lib_omp = _bind(ctypes.CDLL(_LIB_OMP))
        return _lib_omp
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    """Argument types of the oracle's entry points."""
    lib.or_gll.argtypes = [ctypes.c_int, _d, _d]
    lib.or_deriv.argtypes = [ctypes.c_int, _d, _d]
    lib.or_numbering.argtypes = [ctypes.c_int, _int3, _i64, _i32, _i8]
    lib.or_segments.argtypes = [ctypes.c_int, _int3, _i64, _i8, _i32, _i32, _i8, _i64, _i64]
    lib.or_geometry.argtypes = [ctypes.c_int, _int3, _d, _d, _d, _d]
    lib.or_ax_local.argtypes = [ctypes.c_int, ctypes.c_int64, _d, _d, _d, _d]
    lib.or_dssum.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64, _d, _d]
    lib.or_mask.argtypes = [ctypes.c_int64, _i8, _d]
    lib.or_glsc3.argtypes = [ctypes.c_int64, _d, _d, _d]
    lib.or_glsc3.restype = ctypes.c_double
    lib.or_glsc3_plain.argtypes = [ctypes.c_int64, _d, _d, _d]
    lib.or_glsc3_plain.restype = ctypes.c_double
    lib.or_apply_A.argtypes = [ctypes.c_int, _int3, _d, _d, _i64, _i8, _d, _d]
    lib.or_cg.argtypes = [ctypes.c_int, _int3, _d, _d, _i64, _i32, _i8, _d, _d,
                          ctypes.c_double, ctypes.c_int, _d, _d]
    lib.or_diag.argtypes = [ctypes.c_int, _int3, _d, _d, _i64, _i8, _d]
    lib.or_pcg.argtypes = [ctypes.c_int, _int3, _d, _d, _i64, _i32, _i8, _d, _d, _d,
                           ctypes.c_double, ctypes.c_int, _d, _d]
    lib.vp_round.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.vp_round.restype = ctypes.c_double
    lib.vp_perturb.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.vp_perturb.restype = ctypes.c_double
    lib.vp_cg.argtypes = [ctypes.c_int, _int3, _d, _d, _i32, ctypes.c_int, ctypes.c_uint64,
                          ctypes.c_double, ctypes.c_int, _d, _d, _d, _d]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_threads.argtypes = [ctypes.c_int]
    return lib


def omp_threads(n: int | None = None) -> int:
    """Threads of the OpenMP build (setting them when n is given)."""
    lib = _get(omp=True)
    if n is not None:
        lib.or_set_threads(int(n))
    return lib.or_num_threads()


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else ctypes.cast(None, t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gll(N: int):
    """GLL nodes and weights of order N (N+1 points), ascending."""
    xi = np.empty(N + 1)
    w = np.empty(N + 1)
    if _get().or_gll(N, _p(xi, _d), _p(w, _d)):
        raise ValueError("N must be >= 1")
    return xi, w


def deriv(N: int):
    """(N+1)x(N+1) GLL differentiation matrix, D[i, j] = l_j'(x_i)."""
    xi, _ = gll(N)
    D = np.empty((N + 1, N + 1))
    _get().or_deriv(N, _p(xi, _d), _p(D, _d))
    return D


def numbering(N: int, nel):
    """Per local node: global id (int64), multiplicity (int32), Dirichlet mask (int8)."""
    nel = tuple(int(v) for v in nel)
    nl = nel[0] * nel[1] * nel[2] * (N + 1) ** 3
    gid = np.empty(nl, np.int64)
    mult = np.empty(nl, np.int32)
    mask = np.empty(nl, np.int8)
    if _get().or_numbering(N, _int3(*nel), _p(gid, _i64), _p(mult, _i32), _p(mask, _i8)):
        raise MemoryError
    return gid, mult, mask


def segments(N: int, nel, gid, mask):
    """Sorted-segment gather-scatter maps: perm (int32), seg_ptr (int32), seg_flag (int8)."""
    nel = tuple(int(v) for v in nel)
    nl = gid.shape[0]
    perm = np.empty(nl, np.int32)
    seg_ptr = np.empty(nl + 1, np.int32)
    flag = np.empty(nl, np.int8)
    npm = ctypes.c_int64()
    nsg = ctypes.c_int64()
    if _get().or_segments(N, _int3(*nel), _p(gid, _i64), _p(mask, _i8), _p(perm, _i32),
                          _p(seg_ptr, _i32), _p(flag, _i8), ctypes.byref(npm), ctypes.byref(nsg)):
        raise MemoryError
    return perm[:npm.value].copy(), seg_ptr[:nsg.value + 1].copy(), flag[:nsg.value].copy()


def geometry(N: int, nel, vtx, want_X: bool = False):
    """Geometric factors g [E,6,n^3], mass B [E,n^3] and (optional) node coordinates X [E,3,n^3]."""
    nel = tuple(int(v) for v in nel)
    E = nel[0] * nel[1] * nel[2]
    n3 = (N + 1) ** 3
    vtx = _f64(vtx)
    assert vtx.shape == ((nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1), 3)
    g = np.empty((E, 6, n3))
    B = np.empty((E, n3))
    X = np.empty((E, 3, n3)) if want_X else None
    rc = _get().or_geometry(N, _int3(*nel), _p(vtx, _d), _p(g, _d), _p(B, _d), _p(X, _d))
    if rc == -4:
        raise ValueError("inverted element: det J <= 0")
    if rc:
        raise ValueError("bad order N")
    return g, B, X


def ax_local(N: int, D, g, u):
    """Unassembled element stiffness action A_L u (ax_e for every element)."""
    n3 = (N + 1) ** 3
    u = _f64(u)
    E = u.shape[0] // n3
    w = np.empty_like(u)
    _get().or_ax_local(N, E, _p(_f64(D), _d), _p(_f64(g), _d), _p(u, _d), _p(w, _d))
    return w


def dssum(gid, ng: int, w):
    """Sum the copies of each global node (ascending local index) and scatter back."""
    w = _f64(w).copy()
    acc = np.empty(ng)
    _get().or_dssum(w.shape[0], ng, _p(gid, _i64), _p(w, _d), _p(acc, _d))
    return w


def mask_apply(mask, w):
    w = _f64(w).copy()
    _get().or_mask(w.shape[0], _p(np.ascontiguousarray(mask, np.int8), _i8), _p(w, _d))
    return w


def glsc3(a, c, b):
    """Neumaier-compensated serial sum of a*c*b."""
    a, c, b = _f64(a), _f64(c), _f64(b)
    return _get().or_glsc3(a.shape[0], _p(a, _d), _p(c, _d), _p(b, _d))


def glsc3_plain(a, c, b):
    a, c, b = _f64(a), _f64(c), _f64(b)
    return _get().or_glsc3_plain(a.shape[0], _p(a, _d), _p(c, _d), _p(b, _d))


@dataclass
class Problem:
    """One box-mesh Poisson problem with everything the oracle needs, all FP64.

    ``vtx`` is the element-vertex lattice (see paper_2405_11065_amd.synth).
    """
    N: int
    nel: tuple
    vtx: np.ndarray
    want_X: bool = False
    D: np.ndarray = field(init=False)
    g: np.ndarray = field(init=False)
    B: np.ndarray = field(init=False)
    X: np.ndarray = field(init=False)

    def __post_init__(self):
        self.nel = tuple(int(v) for v in self.nel)
        self.E = self.nel[0] * self.nel[1] * self.nel[2]
        self.n = self.N + 1
        self.nl = self.E * self.n ** 3
        self.ng = int(np.prod([v * self.N + 1 for v in self.nel]))
        self.D = deriv(self.N)
        self.g, self.B, self.X = geometry(self.N, self.nel, self.vtx, self.want_X)
        self.gid, self.mult, self.mask = numbering(self.N, self.nel)
        self.c = 1.0 / self.mult.astype(np.float64)

    def ax_local(self, u):
        return ax_local(self.N, self.D, self.g, u)

    def dssum(self, w, masked: bool = True):
        w = dssum(self.gid, self.ng, w)
        return mask_apply(self.mask, w) if masked else w

    def A(self, u):
        """Assembled masked operator: M o dssum(A_L u)."""
        w = np.empty(self.nl)
        _get().or_apply_A(self.N, _int3(*self.nel), _p(self.D, _d), _p(self.g, _d),
                          _p(self.gid, _i64), _p(self.mask, _i8), _p(_f64(u), _d), _p(w, _d))
        return w

    def rhs(self, f):
        """b = M o dssum(f) for a local load vector f."""
        return self.dssum(f, masked=True)

    def glsc3(self, a, b):
        return glsc3(a, self.c, b)

    def segments(self):
        return segments(self.N, self.nel, self.gid, self.mask)

    def cg(self, f, x0=None, tol: float = 1e-8, maxit: int = 1000, omp: bool = False):
        """Table-1 CG (omp: the OpenMP build, bit-identical).  Returns (x,
        iterations, residual history)."""
        x = np.empty(self.nl)
        hist = np.zeros(maxit + 1)
        it = _get(omp).or_cg(self.N, _int3(*self.nel), _p(self.D, _d), _p(self.g, _d),
                          _p(self.gid, _i64), _p(self.mult, _i32), _p(self.mask, _i8),
                          _p(_f64(f), _d), _p(None if x0 is None else _f64(x0), _d),
                          float(tol), int(maxit), _p(x, _d), _p(hist, _d))
        if it == -5:
            raise FloatingPointError("CG breakdown: pAp <= 0")
        if it == -6:
            raise FloatingPointError("CG: non-finite value")
        if it < 0:
            raise MemoryError
        return x, it, hist[:it + 1]

    def diag(self):
        """Diagonal of the assembled masked operator (1 on Dirichlet nodes), per local node."""
        m = np.empty(self.nl)
        if _get().or_diag(self.N, _int3(*self.nel), _p(self.D, _d), _p(self.g, _d), _p(self.gid, _i64),
                          _p(self.mask, _i8), _p(m, _d)):
            raise MemoryError
        return m

    def pcg(self, f, m, x0=None, tol: float = 1e-8, maxit: int = 1000):
        """Table-1 CG with the diagonal preconditioner solveM: z = r / m.
        Returns (x, iterations, residual history)."""
        x = np.empty(self.nl)
        hist = np.zeros(maxit + 1)
        it = _get().or_pcg(self.N, _int3(*self.nel), _p(self.D, _d), _p(self.g, _d),
                           _p(self.gid, _i64), _p(self.mult, _i32), _p(self.mask, _i8), _p(_f64(m), _d),
                           _p(_f64(f), _d), _p(None if x0 is None else _f64(x0), _d),
                           float(tol), int(maxit), _p(x, _d), _p(hist, _d))
        if it == -5:
            raise FloatingPointError("PCG breakdown: pAp <= 0")
        if it == -6:
            raise FloatingPointError("PCG: non-finite value")
        if it < 0:
            raise MemoryError
        return x, it, hist[:it + 1]

    def true_residual(self, x, f):
        """rho* = sqrt(glsc3(r,c,r)) / sqrt(glsc3(b,c,b)), r = b - A x, all FP64."""
        b = self.rhs(f)
        r = b - self.A(x)
        return np.sqrt(self.glsc3(r, r)) / np.sqrt(self.glsc3(b, b))


# ---------------------------------------------------------------- precision emulation
# Region indices and hook modes of nek_vprec.c.
VP_INIT, VP_OP, VP_VEC, VP_DOT = 0, 1, 2, 3
VP_MODES = {"ieee": 0, "rne": 1, "rr": 2, "mca": 3}


def vp_round(x: float, t: int) -> float:
    """x rounded to t explicit mantissa bits (nearest, ties to even)."""
    return _get().vp_round(float(x), int(t))


def vp_perturb(x: float, t: int) -> float:
    """One Monte Carlo perturbation x + 2^(e_x - t) xi (stream continues from the last vp_cg seed)."""
    return _get().vp_perturb(float(x), int(t))


def vprec_cg(N: int, nel, vtx, f, t=(52, 52, 52, 52), mode: str = "ieee", seed: int = 0,
             tol: float = 0.0, maxit: int = 100, want_g: bool = False, m=None):
    """The oracle's init and Table-1 CG with every FP operation passed through
    the precision hook of nek_vprec.c: t = mantissa bits of the regions
    (init, operator + dssum, vector updates, dot products and scalars); mode
    one of 'ieee', 'rne' (round to t bits), 'rr' (random rounding of
    results), 'mca' (perturbed operands and results).  With m (a diagonal
    per local node) the loop is the preconditioned one of Problem.pcg.
    Returns (x, iterations, recursive residual history[, g])."""
    nel = tuple(int(v) for v in nel)
    E = nel[0] * nel[1] * nel[2]
    nl = E * (N + 1) ** 3
    x = np.empty(nl)
    hist = np.zeros(maxit + 1)
    g = np.empty((E, 6, (N + 1) ** 3)) if want_g else None
    tt = np.ascontiguousarray(t, dtype=np.int32)
    assert tt.shape == (4,)
    it = _get().vp_cg(N, _int3(*nel), _p(_f64(vtx), _d), _p(_f64(f), _d), _p(tt, _i32), VP_MODES[mode],
                      int(seed) & (2 ** 64 - 1), float(tol), int(maxit), _p(x, _d), _p(hist, _d), _p(g, _d),
                      _p(None if m is None else _f64(m), _d))
    if it == -4:
        raise ValueError("inverted element: det J <= 0")
    if it == -1:
        raise MemoryError
    if it < 0:
        # breakdown or non-finite value under the emulated precision: a result, not an error
        return x, it, hist, g
    return (x, it, hist[:it + 1], g) if want_g else (x, it, hist[:it + 1])
