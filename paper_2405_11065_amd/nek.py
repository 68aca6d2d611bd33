"""Thin ctypes binding of libnek (include/nek.h).

Argument marshalling only: every step of the solve runs in libnek's HIP
kernels.  torch supplies device memory and the HIP stream; no torch math is
done here on solver data.  Loading fails loudly if libnek.so is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnek.so")

NEK_OK, NEK_NOCONV = 0, 1
NEK_E_ARG, NEK_E_HIP, NEK_E_OOM, NEK_E_JACOBIAN = -1, -2, -3, -4
NEK_E_BREAKDOWN, NEK_E_NONFINITE, NEK_E_STAGNATION, NEK_E_SCRATCH = -5, -6, -7, -8
NEK_NOALLOC_SCRATCH_BYTES = 32 << 20
NEK_PREC_FP64, NEK_PREC_FP32, NEK_PREC_BF16G = 0, 1, 2
NEK_F64, NEK_F32 = 0, 1
(NEK_GET_GLL, NEK_GET_W, NEK_GET_D, NEK_GET_G, NEK_GET_B, NEK_GET_GID, NEK_GET_MULT, NEK_GET_MASK,
 NEK_GET_PERM, NEK_GET_SEGPTR, NEK_GET_SEGFLAG, NEK_GET_XYZ, NEK_GET_DIAG) = range(13)
NEK_PC_NONE, NEK_PC_JACOBI, NEK_PC_FDM, NEK_PC_SCHWARZ = 0, 1, 2, 3
PC_NAMES = {"none": NEK_PC_NONE, "jacobi": NEK_PC_JACOBI, "fdm": NEK_PC_FDM, "schwarz": NEK_PC_SCHWARZ}
(NEK_SIZE_NLOCAL, NEK_SIZE_NGLOBAL, NEK_SIZE_E, NEK_SIZE_NPERM, NEK_SIZE_NSEG, NEK_SIZE_N) = range(6)

PREC_NAMES = {"fp64": NEK_PREC_FP64, "fp32": NEK_PREC_FP32, "bf16g": NEK_PREC_BF16G}
NEK_GSRC_STORED, NEK_GSRC_TRILINEAR = 0, 1
GEOM_NAMES = {"stored": NEK_GSRC_STORED, "trilinear": NEK_GSRC_TRILINEAR}

# every entry point declared in include/nek.h
EXPORTS = ("nek_setup", "nek_free", "nek_size", "nek_get", "nek_set_prec", "nek_set_precond", "nek_set_geometry",
           "nek_set_max_workgroups", "nek_set_operator_kernel", "nek_set_schwarz_kernel",
           "nek_set_update_kernel", "nek_precond_apply", "nek_ax_local", "nek_ax", "nek_ax_noalloc",
           "nek_dssum", "nek_glsc3", "nek_cg_solve", "nek_prof_enable", "nek_prof_read", "nek_num_variants",
           "nek_tune", "nek_set_variant", "nek_get_variant", "nek_setup_batch", "nek_batch_free",
           "nek_batch_size", "nek_batch_ctx", "nek_batch_mesh_of", "nek_batch_orders", "nek_batch_tune", "nek_batch_set_variant",
           "nek_batch_get_variant", "nek_cg_solve_batch", "nek_batch_counters", "nek_strerror",
           "nek_mlp_create", "nek_mlp_free", "nek_mlp_num_params", "nek_mlp_get_params", "nek_mlp_set_params",
           "nek_mlp_forward", "nek_mlp_loss_grad", "nek_mlp_adam", "nek_mlp_train", "nek_x0_features",
           "nek_x0_targets", "nek_x0_predict", "nek_grf")

NEK_MAX_VARIANTS = 6
SCHWARZ_KERNELS = {"auto": 0, "mfma": 1, "valu": 2}
UPDATE_KERNELS = {"auto": 0, "gather": 1, "exchange": 2}
OPERATOR_KERNELS = {"valu": 0, "mfma": 1}
NEK_BATCH_NO_GRAPH = 1


class nek_mesh(ctypes.Structure):
    _fields_ = [("nel", ctypes.c_int * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("vtx", ctypes.POINTER(ctypes.c_double))]


class nek_opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("inner_tol", ctypes.c_double), ("inner_maxit", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("fp64_fallback", ctypes.c_int), ("elts_per_wg", ctypes.c_int),
                ("refine_mode", ctypes.c_int), ("precond", ctypes.c_int), ("corr_fp32", ctypes.c_int)]


class nek_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("fp64_iters", ctypes.c_int),
                ("status", ctypes.c_int), ("true_rel_res", ctypes.c_double), ("last_rec_res", ctypes.c_double),
                ("t_solve_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NekError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status} ({strerror(status)})")


_lib = None


def load(path: str = LIB_PATH):
    """Load libnek.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnek.so not found at {path}: build it with `python -m paper_2405_11065_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    lib.nek_setup.argtypes = [ctypes.POINTER(nek_mesh), ctypes.c_int, ctypes.POINTER(nek_opts), vp,
                              ctypes.POINTER(vp)]
    lib.nek_free.argtypes = [vp]
    lib.nek_free.restype = None
    lib.nek_size.argtypes = [vp, ctypes.c_int, i64p]
    lib.nek_get.argtypes = [vp, ctypes.c_int, vp]
    lib.nek_set_prec.argtypes = [vp, ctypes.c_int]
    lib.nek_set_precond.argtypes = [vp, ctypes.c_int]
    lib.nek_set_geometry.argtypes = [vp, ctypes.c_int]
    lib.nek_set_max_workgroups.argtypes = [vp, ctypes.c_int]
    lib.nek_set_schwarz_kernel.argtypes = [vp, ctypes.c_int]
    lib.nek_set_update_kernel.argtypes = [vp, ctypes.c_int]
    lib.nek_set_operator_kernel.argtypes = [vp, ctypes.c_int]
    lib.nek_precond_apply.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.nek_ax_local.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.nek_ax.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.nek_ax_noalloc.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.nek_dssum.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int]
    lib.nek_glsc3.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.nek_cg_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int, vp, ctypes.POINTER(nek_stats), vp]
    lib.nek_prof_enable.argtypes = [vp, ctypes.c_int]
    lib.nek_prof_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), i64p, ctypes.c_int]
    lib.nek_num_variants.argtypes = [vp]
    lib.nek_tune.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_int)]
    lib.nek_set_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.nek_get_variant.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.nek_setup_batch.argtypes = [ctypes.c_int, ctypes.POINTER(nek_mesh), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(nek_opts), vp, ctypes.POINTER(vp)]
    lib.nek_batch_free.argtypes = [vp]
    lib.nek_batch_free.restype = None
    lib.nek_batch_size.argtypes = [vp]
    lib.nek_batch_ctx.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp)]
    lib.nek_batch_mesh_of.argtypes = [vp, ctypes.c_int]
    lib.nek_batch_orders.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.nek_batch_tune.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.nek_batch_set_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.nek_batch_get_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.nek_cg_solve_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(vp), ctypes.POINTER(nek_stats), ctypes.c_int]
    lib.nek_batch_counters.argtypes = [vp, i64p, i64p]
    dp, fp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)
    lib.nek_mlp_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, vp, ctypes.POINTER(vp)]
    lib.nek_mlp_free.argtypes = [vp]
    lib.nek_mlp_free.restype = None
    lib.nek_mlp_num_params.argtypes = [vp]
    lib.nek_mlp_num_params.restype = ctypes.c_int64
    lib.nek_mlp_get_params.argtypes = [vp, fp]
    lib.nek_mlp_set_params.argtypes = [vp, fp]
    lib.nek_mlp_forward.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int64, vp, ctypes.c_int]
    lib.nek_mlp_loss_grad.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int64, dp, fp]
    lib.nek_mlp_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
    lib.nek_mlp_train.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_float, ctypes.c_uint64, fp]
    lib.nek_x0_features.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, vp]
    lib.nek_x0_targets.argtypes = [vp, vp, vp, ctypes.c_double, vp, ctypes.c_int]
    lib.nek_x0_predict.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, vp, dp, dp,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.nek_grf.argtypes = [vp, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int, vp]
    lib.nek_strerror.argtypes = [ctypes.c_int]
    lib.nek_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load().nek_strerror(int(status)).decode()
    except RuntimeError:
        return "libnek not loaded"


def _check(rc, what, ok=(NEK_OK,)):
    if rc not in ok:
        raise NekError(rc, what)
    return rc


def _torch():
    import torch
    return torch


def _mesh(nel, vtx=None, lo=(0.0, 0.0, 0.0), hi=None):
    """(nek_mesh, nel tuple, vertex array kept alive by the caller)."""
    nel = tuple(int(v) for v in nel)
    lo = tuple(float(v) for v in lo)
    hi = tuple(lo[d] + nel[d] for d in range(3)) if hi is None else tuple(float(v) for v in hi)
    m = nek_mesh()
    m.nel[:] = nel
    m.lo[:] = lo
    m.hi[:] = hi
    keep = None
    if vtx is not None:
        keep = np.ascontiguousarray(vtx, dtype=np.float64)
        nv = (nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1)
        if keep.shape != (nv, 3):
            raise ValueError(f"vtx must have shape ({nv}, 3)")
        m.vtx = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return m, nel, keep


def _opts(prec="fp64", inner_tol=0.0, inner_maxit=0, max_outer=0, fp64_fallback=1, refine_mode=0, precond="none",
          elts_per_wg=0, corr_fp32=0):
    o = nek_opts()
    o.prec = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    o.inner_tol = float(inner_tol)
    o.inner_maxit = int(inner_maxit)
    o.max_outer = int(max_outer)
    o.fp64_fallback = int(fp64_fallback)
    o.refine_mode = int(refine_mode)
    o.precond = PC_NAMES[precond] if isinstance(precond, str) else int(precond)
    o.elts_per_wg = int(elts_per_wg)
    o.corr_fp32 = int(corr_fp32)
    return o


class Context:
    """One box mesh of order N on the current GPU (nek_setup / nek_free)."""

    def __init__(self, nel, N, vtx=None, lo=(0.0, 0.0, 0.0), hi=None, prec="fp64", inner_tol=0.0,
                 inner_maxit=0, max_outer=0, fp64_fallback=1, refine_mode=0, precond="none", stream=None,
                 elts_per_wg=0, corr_fp32=0):
        torch = _torch()
        self._lib = load()
        self.N = int(N)
        m, self.nel, self._vtx = _mesh(nel, vtx, lo, hi)
        o = _opts(prec, inner_tol, inner_maxit, max_outer, fp64_fallback, refine_mode, precond, elts_per_wg,
                  corr_fp32)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        _check(self._lib.nek_setup(ctypes.byref(m), self.N, ctypes.byref(o), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h)), "nek_setup")
        self._owned = True
        self._init_handle(h)

    @classmethod
    def _borrow(cls, handle, N, nel, owner):
        """A view of a context owned by a batch (never freed here)."""
        self = cls.__new__(cls)
        self._lib = load()
        self.N = int(N)
        self.nel = tuple(nel)
        self._vtx = None
        self.stream = None
        self._owned = False
        self._owner = owner
        self._init_handle(handle)
        return self

    def _init_handle(self, h):
        torch = _torch()
        self._h = h
        self.nl = self.size(NEK_SIZE_NLOCAL)
        self.E = self.size(NEK_SIZE_E)
        self.ng = self.size(NEK_SIZE_NGLOBAL)
        self.device = torch.device("cuda", torch.cuda.current_device())

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            if self._owned:
                self._lib.nek_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries
    def size(self, what: int) -> int:
        out = ctypes.c_int64()
        _check(self._lib.nek_size(self._h, int(what), ctypes.byref(out)), "nek_size")
        return out.value

    def get(self, what: int) -> np.ndarray:
        n = self.N + 1
        shapes = {NEK_GET_GLL: (n, np.float64), NEK_GET_W: (n, np.float64), NEK_GET_D: ((n, n), np.float64),
                  NEK_GET_G: ((self.E, 6, n ** 3), np.float64), NEK_GET_B: (self.nl, np.float64),
                  NEK_GET_GID: (self.nl, np.int64), NEK_GET_MULT: (self.nl, np.int32),
                  NEK_GET_MASK: (self.nl, np.int8), NEK_GET_PERM: (self.size(NEK_SIZE_NPERM), np.int32),
                  NEK_GET_SEGPTR: (self.size(NEK_SIZE_NSEG) + 1, np.int32),
                  NEK_GET_SEGFLAG: (self.size(NEK_SIZE_NSEG), np.int8),
                  NEK_GET_XYZ: ((self.E, 3, n ** 3), np.float64), NEK_GET_DIAG: (self.nl, np.float64)}
        shape, dt = shapes[what]
        out = np.empty(shape, dtype=dt)
        _check(self._lib.nek_get(self._h, int(what), out.ctypes.data_as(ctypes.c_void_p)), "nek_get")
        return out

    def set_prec(self, prec):
        _check(self._lib.nek_set_prec(self._h, PREC_NAMES[prec] if isinstance(prec, str) else int(prec)),
               "nek_set_prec")

    def set_precond(self, precond):
        """'none' (Table 1 with solveM a copy), 'jacobi' (z = r / diagonal) or 'fdm'
        (element-interior fast-diagonalization block solve, diagonal elsewhere)."""
        _check(self._lib.nek_set_precond(self._h, PC_NAMES[precond] if isinstance(precond, str) else int(precond)),
               "nek_set_precond")

    def set_geometry(self, geom):
        """'stored' (read g1..g6 per point) or 'trilinear' (FP64 and FP32 operators
        recompute them in the kernel from each element's trilinear map)."""
        _check(self._lib.nek_set_geometry(self._h, GEOM_NAMES[geom] if isinstance(geom, str) else int(geom)),
               "nek_set_geometry")

    def set_max_workgroups(self, n: int):
        """Cap the persistent / reduction grid at n workgroups (0 = default)."""
        _check(self._lib.nek_set_max_workgroups(self._h, int(n)), "nek_set_max_workgroups")

    def set_operator_kernel(self, kind: str):
        """D contractions of the plain operator pass (ax_local, ax): "valu" (default) or "mfma"."""
        _check(self._lib.nek_set_operator_kernel(self._h, OPERATOR_KERNELS[kind]), "nek_set_operator_kernel")

    def set_schwarz_kernel(self, kind: str):
        """Kernel of the Schwarz window solves: "auto" (default: matrix cores for FP64
        vectors, vector ALUs for FP32), "mfma" or "valu"."""
        _check(self._lib.nek_set_schwarz_kernel(self._h, SCHWARZ_KERNELS[kind]), "nek_set_schwarz_kernel")

    def set_update_kernel(self, kind: str):
        """How the CG update kernel and nek_ax's assembly collect the copies of face
        nodes: "auto" (default), "gather" (all from memory) or "exchange" (x-face copies
        of elements one workgroup walks swapped through LDS).  Bit-identical results."""
        _check(self._lib.nek_set_update_kernel(self._h, UPDATE_KERNELS[kind]), "nek_set_update_kernel")

    def precond_apply(self, r, z=None):
        """z = M^-1 r with the context's preconditioner."""
        dt = self._vec(r, "r")
        z = torch_empty_like(r) if z is None else z
        if self._vec(z, "z") != dt or z.data_ptr() == r.data_ptr():
            raise ValueError("z must match r's dtype and not alias it")
        _check(self._lib.nek_precond_apply(self._h, r.data_ptr(), z.data_ptr(), dt), "nek_precond_apply")
        return z

    # -- argument checks (host side, before any kernel sees the pointers)
    def _vec(self, t, what):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{what}: expected a CUDA tensor")
        if t.dtype not in (torch.float64, torch.float32):
            raise TypeError(f"{what}: dtype must be float64 or float32")
        if t.numel() != self.nl or not t.is_contiguous():
            raise ValueError(f"{what}: expected a contiguous vector of {self.nl} entries")
        return NEK_F64 if t.dtype == torch.float64 else NEK_F32

    def new_vector(self, dtype=None):
        torch = _torch()
        return torch.empty(self.nl, dtype=dtype or torch.float64, device=self.device)

    # -- operator
    def ax_local(self, u, w=None):
        dt = self._vec(u, "u")
        w = torch_empty_like(u) if w is None else w
        if self._vec(w, "w") != dt or w.data_ptr() == u.data_ptr():
            raise ValueError("w must match u's dtype and not alias it")
        _check(self._lib.nek_ax_local(self._h, u.data_ptr(), w.data_ptr(), dt), "nek_ax_local")
        return w

    def ax(self, u, w=None):
        dt = self._vec(u, "u")
        w = torch_empty_like(u) if w is None else w
        if self._vec(w, "w") != dt or w.data_ptr() == u.data_ptr():
            raise ValueError("w must match u's dtype and not alias it")
        _check(self._lib.nek_ax(self._h, u.data_ptr(), w.data_ptr(), dt), "nek_ax")
        return w

    def ax_noalloc(self, u, w):
        """nek_ax through the library's static scratch: no device allocation (w must be given)."""
        dt = self._vec(u, "u")
        if self._vec(w, "w") != dt or w.data_ptr() == u.data_ptr():
            raise ValueError("w must match u's dtype and not alias it")
        _check(self._lib.nek_ax_noalloc(self._h, u.data_ptr(), w.data_ptr(), dt), "nek_ax_noalloc")
        return w

    def dssum(self, w, mask=True):
        dt = self._vec(w, "w")
        _check(self._lib.nek_dssum(self._h, w.data_ptr(), dt, int(bool(mask))), "nek_dssum")
        return w

    def glsc3(self, a, b):
        dt = self._vec(a, "a")
        if self._vec(b, "b") != dt:
            raise ValueError("a and b must share a dtype")
        out = ctypes.c_double()
        _check(self._lib.nek_glsc3(self._h, a.data_ptr(), b.data_ptr(), dt, ctypes.byref(out)), "nek_glsc3")
        return out.value

    def prof_enable(self, every: int):
        _check(self._lib.nek_prof_enable(self._h, int(every)), "nek_prof_enable")

    def prof_read(self, kernel: int, reset: bool = True):
        """(total ms, sampled launches) of kernel 0 (operator) or 1 (gather/update)."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(self._lib.nek_prof_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n), int(reset)),
               "nek_prof_read")
        return ms.value, n.value

    def num_variants(self) -> int:
        n = self._lib.nek_num_variants(self._h)
        _check(min(n, 0), "nek_num_variants")
        return n

    def tune(self, prec, iters: int = 20):
        """Time every CG kernel configuration; select the fastest.  Returns (best, us_per_iter list)."""
        pv = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
        n = self.num_variants()
        us = (ctypes.c_double * n)()
        best = ctypes.c_int()
        _check(self._lib.nek_tune(self._h, pv, int(iters), us, ctypes.byref(best)), "nek_tune")
        return best.value, list(us)

    def set_variant(self, prec, variant: int):
        pv = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
        _check(self._lib.nek_set_variant(self._h, pv, int(variant)), "nek_set_variant")

    def get_variant(self, prec) -> int:
        pv = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
        v = ctypes.c_int()
        _check(self._lib.nek_get_variant(self._h, pv, ctypes.byref(v)), "nek_get_variant")
        return v.value

    def cg_solve(self, f, x0=None, tol=1e-8, maxit=1000, x=None, history=False, raise_on_noconv=False):
        """Solve A x = M dssum(f).  Returns (x, stats dict, history or None)."""
        torch = _torch()
        for t, nm in ((f, "f"), (x0, "x0"), (x, "x")):
            if t is not None and (self._vec(t, nm) != NEK_F64):
                raise TypeError(f"{nm}: nek_cg_solve takes float64 vectors")
        if x is None:
            x = self.new_vector(torch.float64)
        hist = np.zeros(int(maxit) + 1) if history else None
        st = nek_stats()
        rc = self._lib.nek_cg_solve(self._h, f.data_ptr(), x0.data_ptr() if x0 is not None else None, float(tol),
                                    int(maxit), x.data_ptr(), ctypes.byref(st),
                                    hist.ctypes.data_as(ctypes.c_void_p) if history else None)
        _check(rc, "nek_cg_solve", ok=(NEK_OK,) if raise_on_noconv else (NEK_OK, NEK_NOCONV))
        d = st.as_dict()
        if history:
            hist = hist[:min(int(maxit), max(0, d["iters"])) + 1]
        return x, d, hist


class Batch:
    """Many box problems solved together (nek_setup_batch, nek_cg_solve_batch, nek_batch_*).

    problems: sequence of dicts with keys nel, N and optionally vtx, lo, hi.
    The options (prec, inner_tol, ...) are common to all problems.
    """

    def __init__(self, problems, prec="fp64", inner_tol=0.0, inner_maxit=0, max_outer=0, fp64_fallback=1,
                 refine_mode=0, stream=None, elts_per_wg=0, corr_fp32=0):
        torch = _torch()
        self._lib = load()
        n = len(problems)
        meshes = (nek_mesh * n)()
        Ns = (ctypes.c_int * n)()
        self._keep = []
        self.specs = []
        for i, p in enumerate(problems):
            m, nel, keep = _mesh(p["nel"], p.get("vtx"), p.get("lo", (0.0, 0.0, 0.0)), p.get("hi"))
            meshes[i] = m
            Ns[i] = int(p["N"])
            self._keep.append(keep)
            self.specs.append((nel, int(p["N"])))
        o = _opts(prec, inner_tol, inner_maxit, max_outer, fp64_fallback, refine_mode, elts_per_wg=elts_per_wg,
                  corr_fp32=corr_fp32)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        _check(self._lib.nek_setup_batch(n, meshes, Ns, ctypes.byref(o), ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(h)), "nek_setup_batch")
        self._h = h
        self._keep = None
        self.n = n
        self.ctx = []
        for i in range(n):
            ch = ctypes.c_void_p()
            _check(self._lib.nek_batch_ctx(self._h, i, ctypes.byref(ch)), "nek_batch_ctx")
            self.ctx.append(Context._borrow(ch, self.specs[i][1], self.specs[i][0], self))
        self.nl = [c.nl for c in self.ctx]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            for c in self.ctx:
                c.close()
            self._lib.nek_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def mesh_of(self, i):
        """Index of the problem whose set-up data problem i shares (i if its own)."""
        k = self._lib.nek_batch_mesh_of(self._h, int(i))
        _check(min(k, 0), "nek_batch_mesh_of")
        return k

    def orders(self):
        out = (ctypes.c_int * 16)()
        k = self._lib.nek_batch_orders(self._h, out)
        _check(min(k, 0), "nek_batch_orders")
        return list(out[:k])

    def tune(self, prec, iters: int = 20):
        """Per order: fastest configuration (dict N -> (best, us_per_iter list))."""
        pv = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
        orders = self.orders()
        us = (ctypes.c_double * (NEK_MAX_VARIANTS * len(orders)))()
        _check(self._lib.nek_batch_tune(self._h, pv, int(iters), us), "nek_batch_tune")
        res = {}
        for g, N in enumerate(orders):
            i = next(k for k in range(self.n) if self.specs[k][1] == N)
            row = [t for t in us[g * NEK_MAX_VARIANTS:(g + 1) * NEK_MAX_VARIANTS]]
            res[N] = (self.get_variant(prec, i), row[:self.ctx[i].num_variants()])
        return res

    def set_variant(self, prec, N: int, variant: int):
        pv = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
        _check(self._lib.nek_batch_set_variant(self._h, pv, int(N), int(variant)), "nek_batch_set_variant")

    def get_variant(self, prec, i: int) -> int:
        pv = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
        v = ctypes.c_int()
        _check(self._lib.nek_batch_get_variant(self._h, pv, int(i), ctypes.byref(v)), "nek_batch_get_variant")
        return v.value

    def counters(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.nek_batch_counters(self._h, ctypes.byref(a), ctypes.byref(b)), "nek_batch_counters")
        return a.value, b.value

    def solve(self, fs, x0s=None, tol=1e-8, maxit=1000, xs=None, graph=True, raise_on_noconv=False):
        """Solve every problem; returns (xs, list of stats dicts, overall status)."""
        torch = _torch()
        if len(fs) != self.n or (x0s is not None and len(x0s) != self.n):
            raise ValueError(f"expected {self.n} vectors")
        if xs is None:
            xs = [torch.empty(self.nl[i], dtype=torch.float64, device=self.ctx[i].device) for i in range(self.n)]
        for i in range(self.n):
            for t, nm in ((fs[i], "f"), (xs[i], "x")) + (((x0s[i], "x0"),) if x0s is not None else ()):
                if t is not None and self.ctx[i]._vec(t, f"{nm}[{i}]") != NEK_F64:
                    raise TypeError(f"{nm}[{i}]: nek_cg_solve_batch takes float64 vectors")
        P = ctypes.c_void_p * self.n
        fa = P(*[t.data_ptr() for t in fs])
        xa = P(*[t.data_ptr() for t in xs])
        x0a = P(*[(t.data_ptr() if t is not None else None) for t in x0s]) if x0s is not None else None
        st = (nek_stats * self.n)()
        rc = self._lib.nek_cg_solve_batch(self._h, fa, x0a, float(tol), int(maxit), xa, st,
                                          0 if graph else NEK_BATCH_NO_GRAPH)
        _check(rc, "nek_cg_solve_batch", ok=(NEK_OK,) if raise_on_noconv else (NEK_OK, NEK_NOCONV))
        return xs, [s.as_dict() for s in st], rc


def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dev2d(t, dtype, cols, what):
    """Check a contiguous CUDA matrix with at least ``cols`` columns; returns its pitch."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or t.dim() != 2 or not t.is_contiguous():
        raise TypeError(f"{what}: expected a contiguous 2-D CUDA tensor of {dtype}")
    if t.shape[1] < cols:
        raise ValueError(f"{what}: needs at least {cols} columns")
    return int(t.shape[1])


class Mlp:
    """Initial-guess network n_in -> n_hidden -> n_hidden -> n_out (include/nek_mlp.h)."""

    def __init__(self, n_in, n_hidden, n_out, params=None, stream=None):
        torch = _torch()
        self._lib = load()
        self.n_in, self.n_hidden, self.n_out = int(n_in), int(n_hidden), int(n_out)
        self.ld_in = (self.n_in + 7) // 8 * 8
        self.ld_out = (self.n_out + 7) // 8 * 8
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        flat = None if params is None else self.flatten(params)
        _check(self._lib.nek_mlp_create(self.n_in, self.n_hidden, self.n_out, None if flat is None else _f32p(flat),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "nek_mlp_create")
        self._h = h
        self.num_params = int(self._lib.nek_mlp_num_params(self._h))

    def shapes(self):
        i, h, o = self.n_in, self.n_hidden, self.n_out
        return [(h, i), (h,), (h, h), (h,), (o, h), (o,)]

    def flatten(self, params):
        out = []
        for p, shp in zip(params, self.shapes()):
            a = np.asarray(p, dtype=np.float32)
            if a.shape != shp:
                raise ValueError(f"parameter shape {a.shape} != {shp}")
            out.append(a.ravel())
        return np.ascontiguousarray(np.concatenate(out))

    def unflatten(self, flat):
        out, k = [], 0
        for shp in self.shapes():
            n = int(np.prod(shp))
            out.append(flat[k:k + n].reshape(shp))
            k += n
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.nek_mlp_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        flat = np.empty(self.num_params, dtype=np.float32)
        _check(self._lib.nek_mlp_get_params(self._h, _f32p(flat)), "nek_mlp_get_params")
        return self.unflatten(flat)

    def set_params(self, params):
        flat = self.flatten(params)
        _check(self._lib.nek_mlp_set_params(self._h, _f32p(flat)), "nek_mlp_set_params")

    def forward(self, X, rows=None, Y=None):
        torch = _torch()
        ldx = _dev2d(X, torch.bfloat16, self.n_in, "X")
        rows = X.shape[0] if rows is None else int(rows)
        if Y is None:
            Y = torch.empty((rows, self.ld_out), dtype=torch.float32, device=X.device)
        ldy = _dev2d(Y, torch.float32, self.n_out, "Y")
        if ldx % 8 or X.shape[0] < rows or Y.shape[0] < rows:
            raise ValueError("X pitch must be a multiple of 8 and X, Y must hold rows rows")
        _check(self._lib.nek_mlp_forward(self._h, X.data_ptr(), ldx, rows, Y.data_ptr(), ldy), "nek_mlp_forward")
        return Y

    def loss_grad(self, X, T, rows=None):
        """(loss, gradient list in parameter order)."""
        torch = _torch()
        ldx = _dev2d(X, torch.bfloat16, self.n_in, "X")
        ldt = _dev2d(T, torch.float32, self.n_out, "T")
        rows = X.shape[0] if rows is None else int(rows)
        if ldx % 8 or X.shape[0] < rows or T.shape[0] < rows:
            raise ValueError("X pitch must be a multiple of 8 and X, T must hold rows rows")
        loss = ctypes.c_double()
        g = np.empty(self.num_params, dtype=np.float32)
        _check(self._lib.nek_mlp_loss_grad(self._h, X.data_ptr(), ldx, T.data_ptr(), ldt, rows, ctypes.byref(loss),
                                           _f32p(g)), "nek_mlp_loss_grad")
        return loss.value, self.unflatten(g)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(self._lib.nek_mlp_adam(self._h, lr, beta1, beta2, eps), "nek_mlp_adam")

    def train(self, X, T, nsamples, batch, steps, lr=1e-3, seed=0, history=True):
        torch = _torch()
        ldx = _dev2d(X, torch.bfloat16, self.n_in, "X")
        ldt = _dev2d(T, torch.float32, self.n_out, "T")
        if ldx % 8 or X.shape[0] < nsamples or T.shape[0] < nsamples:
            raise ValueError("X pitch must be a multiple of 8 and X, T must hold nsamples rows")
        hist = np.empty(int(steps), dtype=np.float32) if history else None
        _check(self._lib.nek_mlp_train(self._h, X.data_ptr(), ldx, T.data_ptr(), ldt, int(nsamples), int(batch),
                                       int(steps), float(lr), int(seed), None if hist is None else _f32p(hist)),
               "nek_mlp_train")
        return hist


def x0_features(ctx, f, X=None, s=None, mode=0):
    """(X bfloat16 [E, ld], s float64 [E]) of the load vector f."""
    torch = _torch()
    n3 = (ctx.N + 1) ** 3
    if X is None:
        X = torch.empty((ctx.E, (n3 + 6 + 7) // 8 * 8), dtype=torch.bfloat16, device=f.device)
    if s is None:
        s = torch.empty(ctx.E, dtype=torch.float64, device=f.device)
    ldx = _dev2d(X, torch.bfloat16, n3 + 6, "X")
    if ctx._vec(f, "f") != NEK_F64 or X.shape[0] < ctx.E or s.numel() < ctx.E or s.dtype != torch.float64:
        raise ValueError("f must be float64 and X, s must hold E rows")
    _check(ctx._lib.nek_x0_features(ctx._h, f.data_ptr(), int(mode), X.data_ptr(), ldx, s.data_ptr()),
           "nek_x0_features")
    return X, s


def x0_targets(ctx, x, s, kappa, T=None):
    torch = _torch()
    n3 = (ctx.N + 1) ** 3
    if T is None:
        T = torch.empty((ctx.E, (n3 + 7) // 8 * 8), dtype=torch.float32, device=x.device)
    ldt = _dev2d(T, torch.float32, n3, "T")
    if ctx._vec(x, "x") != NEK_F64 or T.shape[0] < ctx.E:
        raise ValueError("x must be float64 and T must hold E rows")
    _check(ctx._lib.nek_x0_targets(ctx._h, x.data_ptr(), s.data_ptr(), float(kappa), T.data_ptr(), ldt),
           "nek_x0_targets")
    return T


NEK_X0_RESIDUAL, NEK_X0_ENERGY = 0, 1


def x0_predict(ctx, mlp, f, kappa, x0=None, policy=NEK_X0_RESIDUAL, mode=0):
    """(x0, alpha, rho0, used) -- see nek_x0_predict."""
    if ctx._vec(f, "f") != NEK_F64:
        raise TypeError("f must be float64")
    if x0 is None:
        x0 = ctx.new_vector()
    elif ctx._vec(x0, "x0") != NEK_F64:
        raise TypeError("x0 must be float64")
    a, r, u = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    _check(ctx._lib.nek_x0_predict(ctx._h, mlp._h, f.data_ptr(), int(mode), float(kappa), int(policy), x0.data_ptr(),
                                   ctypes.byref(a),
                                   ctypes.byref(r), ctypes.byref(u)), "nek_x0_predict")
    return x0, a.value, r.value, bool(u.value)


def grf(ctx, draw, scale=1.0, times_B=True, out=None):
    """Forcing sample of a random-Fourier-feature draw (omega, phi, a, scale attributes) on ctx's nodes."""
    if out is None:
        out = ctx.new_vector()
    om = np.ascontiguousarray(draw.omega, dtype=np.float64)
    ph = np.ascontiguousarray(draw.phi, dtype=np.float64)
    am = np.ascontiguousarray(draw.a, dtype=np.float64)
    if om.shape != (ph.size, 3) or am.size != ph.size:
        raise ValueError("omega must be [nfeat, 3] with phi and a of nfeat entries")
    d = ctypes.POINTER(ctypes.c_double)
    _check(ctx._lib.nek_grf(ctx._h, ph.size, om.ctypes.data_as(d), ph.ctypes.data_as(d), am.ctypes.data_as(d),
                            float(scale) * float(draw.scale), int(bool(times_B)), out.data_ptr()), "nek_grf")
    return out


def torch_empty_like(t):
    return _torch().empty_like(t)
