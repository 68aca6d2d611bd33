"""CPU checks of libnek: every declared symbol is exported, and the host-side
set-up (GLL rule, D, geometry, numbering, segment maps) matches the FP64
oracle -- bit for bit on every integer map.  No GPU is touched."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2405_11065_amd import nek, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("nek.h", "nek_host.h", "nek_mlp.h")]


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"\b(nek_\w+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nek.LIB_PATH):
        pytest.fail("libnek.so is not built (python -m paper_2405_11065_amd.build)")
    return ctypes.CDLL(nek.LIB_PATH)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(nek.EXPORTS) <= set(names)


def test_strerror_covers_statuses(lib):
    lib.nek_strerror.restype = ctypes.c_char_p
    msgs = {s: lib.nek_strerror(s).decode() for s in range(-8, 2)}
    assert len(set(msgs.values())) == 10
    assert lib.nek_strerror(42).decode() == "unknown status"


def _i3(nel):
    return (ctypes.c_int * 3)(*nel)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def host_maps(lib, N, nel):
    nl = int(np.prod(nel)) * (N + 1) ** 3
    gid = np.empty(nl, np.int64)
    mult = np.empty(nl, np.int32)
    mask = np.empty(nl, np.int8)
    assert lib.nek_host_numbering(N, _i3(nel), _ptr(gid), _ptr(mult), _ptr(mask)) == 0
    npm, nsg = ctypes.c_int64(), ctypes.c_int64()
    assert lib.nek_host_segment_sizes(N, _i3(nel), ctypes.byref(npm), ctypes.byref(nsg)) == 0
    perm = np.empty(npm.value, np.int32)
    ptr = np.empty(nsg.value + 1, np.int32)
    flag = np.empty(nsg.value, np.int8)
    assert lib.nek_host_segments(N, _i3(nel), _ptr(perm), _ptr(ptr), _ptr(flag)) == 0
    return gid, mult, mask, perm, ptr, flag


@pytest.mark.parametrize("N,nel", [(1, (1, 1, 1)), (2, (3, 1, 2)), (3, (2, 2, 2)), (5, (3, 4, 2)),
                                   (7, (4, 4, 4)), (9, (2, 3, 2)), (15, (1, 2, 1))])
def test_host_maps_bit_exact(lib, N, nel):
    gid, mult, mask, perm, ptr, flag = host_maps(lib, N, nel)
    ogid, omult, omask = oracle.numbering(N, nel)
    operm, optr, oflag = oracle.segments(N, nel, ogid, omask)
    assert np.array_equal(gid, ogid)
    assert np.array_equal(mult, omult)
    assert np.array_equal(mask, omask)
    assert np.array_equal(perm, operm)
    assert np.array_equal(ptr, optr)
    assert np.array_equal(flag, oflag)


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_host_gll_and_deriv(lib, N):
    xi, w = np.empty(N + 1), np.empty(N + 1)
    D = np.empty((N + 1) ** 2)
    assert lib.nek_host_gll(N, _ptr(xi), _ptr(w)) == 0
    assert lib.nek_host_deriv(N, _ptr(D)) == 0
    oxi, ow = oracle.gll(N)
    np.testing.assert_allclose(xi, oxi, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, ow, rtol=0, atol=1e-14)
    oD = oracle.deriv(N)
    assert np.abs(D.reshape(N + 1, N + 1) - oD).max() <= 1e-13 * np.abs(oD).max()


@pytest.mark.parametrize("N,nel,perturb", [(3, (2, 2, 2), 0.0), (7, (3, 2, 2), 0.1), (9, (2, 2, 3), 0.1)])
def test_host_geometry(lib, N, nel, perturb):
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=perturb, seed=17)
    E, n3 = int(np.prod(nel)), (N + 1) ** 3
    g, B, X = np.empty((E, 6, n3)), np.empty((E, n3)), np.empty((E, 3, n3))
    assert lib.nek_host_geometry(N, _i3(nel), _ptr(vtx), _ptr(g), _ptr(B), _ptr(X)) == 0
    og, oB, oX = oracle.geometry(N, nel, vtx, want_X=True)
    # G's natural scale is its diagonal; off-diagonal entries that vanish on
    # affine elements are compared against it
    scale = np.abs(og[:, :3]).max()
    for q in range(6):
        assert np.abs(g[:, q] - og[:, q]).max() <= 1e-13 * scale, q
    assert np.abs(B - oB).max() <= 1e-13 * np.abs(oB).max()
    assert np.abs(X - oX).max() <= 1e-15


def test_host_geometry_rejects_inverted(lib):
    nel = (2, 2, 2)
    vtx = synth.box_vertices(nel)
    vtx[13] = [2.6, 2.6, 2.6]
    n3 = 4 ** 3
    g, B = np.empty((8, 6, n3)), np.empty((8, n3))
    assert lib.nek_host_geometry(3, _i3(nel), _ptr(vtx), _ptr(g), _ptr(B), None) == nek.NEK_E_JACOBIAN


def test_host_rejects_bad_arguments(lib):
    xi = np.empty(20)
    assert lib.nek_host_gll(0, _ptr(xi), _ptr(xi)) == nek.NEK_E_ARG
    assert lib.nek_host_gll(16, _ptr(xi), _ptr(xi)) == nek.NEK_E_ARG
    assert lib.nek_host_numbering(3, _i3((0, 1, 1)), None, None, None) == nek.NEK_E_ARG


@pytest.mark.parametrize("N", [2, 3, 5, 7, 9, 11, 15])
def test_host_fdm_matches_oracle(lib, N):
    """Interior modes by the library's Jacobi rotations against the oracle's
    NumPy eigensolver: eigenvalues, and S Lambda^-1 S^T = K_I^-1 (independent
    of the order and signs of the modes); element factors from the lattice."""
    from oracle import fdm
    nel = (3, 2, 2)
    vtx = synth.box_vertices(nel, perturb=0.1, seed=4)
    m = N - 1
    S, lam, cf = np.empty(m * m), np.empty(m), np.empty(3 * 12)
    assert lib.nek_host_fdm(N, _i3(nel), _ptr(vtx), _ptr(S), _ptr(lam), _ptr(cf)) == 0
    xi, w = oracle.gll(N)
    So, lo = fdm.interior_eig(N, oracle.deriv(N), w)
    np.testing.assert_allclose(np.sort(lam), np.sort(lo), rtol=1e-12)
    S = S.reshape(m, m)
    np.testing.assert_allclose(S @ np.diag(1 / lam) @ S.T, So @ np.diag(1 / lo) @ So.T, rtol=0,
                               atol=1e-12 * np.abs(So @ np.diag(1 / lo) @ So.T).max())
    np.testing.assert_allclose(cf.reshape(-1, 3), fdm.element_scales(nel, vtx), rtol=1e-14)


@pytest.mark.parametrize("N,nel,perturb", [(1, (2, 2, 1), 0.1), (5, (3, 2, 2), 0.1), (9, (2, 3, 2), 0.2),
                                           (15, (1, 2, 1), 0.1), (4, (2, 2, 2), 0.0)])
def test_host_trilinear_matches_oracle(lib, N, nel, perturb):
    """The element maps behind the in-kernel geometric factors: they reproduce
    the 8 vertices at the reference corners, and the factors the kernels form
    from them -- rows K = det(J) J^-1 from cross products of the map's
    derivatives, f = w_i w_j w_k / det(J), G = f K K^T -- equal the oracle's g
    (J by GLL differentiation of the mapped nodes) to rounding."""
    vtx = synth.box_vertices(nel, perturb=perturb, seed=11)
    E = nel[0] * nel[1] * nel[2]
    coef = np.empty(E * 24)
    assert lib.nek_host_trilinear(N, _i3(nel), _ptr(vtx), _ptr(coef)) == 0
    A = coef.reshape(E, 3, 8)
    V = vtx.reshape(nel[2] + 1, nel[1] + 1, nel[0] + 1, 3)
    scale = np.abs(vtx).max()
    for e in range(E):
        ex, ey, ez = e % nel[0], (e // nel[0]) % nel[1], e // (nel[0] * nel[1])
        for v in range(8):
            r, s, t = (1.0 if v & 1 else -1.0), (1.0 if v & 2 else -1.0), (1.0 if v & 4 else -1.0)
            mono = np.array([1, r, s, t, r * s, r * t, s * t, r * s * t])
            want = V[ez + (v >> 2), ey + ((v >> 1) & 1), ex + (v & 1)]
            assert np.abs(A[e] @ mono - want).max() <= 1e-15 * scale
    xi, w = oracle.gll(N)
    P = oracle.Problem(N, nel, vtx)
    n = N + 1
    t, s, r = np.meshgrid(xi, xi, xi, indexing="ij")          # [k][j][i]
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    G = np.empty((E, 6, n, n, n))
    for e in range(E):
        a = A[e]                                                 # [d][m]
        xr = a[:, 1, None, None, None] + a[:, 4, None, None, None] * s + a[:, 5, None, None, None] * t \
            + a[:, 7, None, None, None] * s * t
        xs = a[:, 2, None, None, None] + a[:, 4, None, None, None] * r + a[:, 6, None, None, None] * t \
            + a[:, 7, None, None, None] * r * t
        xt = a[:, 3, None, None, None] + a[:, 5, None, None, None] * r + a[:, 6, None, None, None] * s \
            + a[:, 7, None, None, None] * r * s
        cr, cs, ct = np.cross(xs, xt, axis=0), np.cross(xt, xr, axis=0), np.cross(xr, xs, axis=0)
        det = np.sum(xr * cr, axis=0)
        assert (det > 0).all()
        f = W / det
        for q, (p1, p2) in enumerate(((cr, cr), (cs, cs), (ct, ct), (cr, cs), (cr, ct), (cs, ct))):
            G[e, q] = f * np.sum(p1 * p2, axis=0)
    g = P.g.reshape(E, 6, n, n, n)
    err = np.abs(G - g).max() / np.abs(g[:, :3]).max()
    print(f"  factors from the maps vs oracle g: {err:.2e}")
    assert err <= 1e-13


def test_host_trilinear_inverted_element(lib):
    nel = (2, 1, 1)
    vtx = synth.box_vertices(nel)
    V = vtx.reshape(2, 2, 3, 3)
    V[:, :, 1, 0] = 2.5          # the middle vertex plane past the right face: element 1 inverted
    coef = np.empty(2 * 24)
    assert lib.nek_host_trilinear(3, _i3(nel), _ptr(V.ravel()), _ptr(coef)) == nek.NEK_E_JACOBIAN
    assert lib.nek_host_trilinear(0, _i3(nel), _ptr(vtx), _ptr(coef)) == nek.NEK_E_ARG


@pytest.mark.parametrize("N,nel,perturb", [(2, (3, 2, 4), 0.1), (5, (4, 3, 2), 0.1), (9, (3, 3, 3), 0.0),
                                           (15, (2, 1, 3), 0.1)])
def test_host_schwarz_matches_oracle(lib, N, nel, perturb):
    """Window and coarse modes by the library's Cholesky and Jacobi rotations
    against the oracle's NumPy ones: for every window variant and coarse
    direction, S Lambda^-1 S^T (the inverse of the 1-D operator, independent
    of the order and signs of the modes) and S^T W S = I."""
    from oracle import schwarz
    vtx = synth.box_vertices(nel, perturb=perturb, seed=12)
    NW = N + 3
    Sw, lw = np.empty(4 * NW * NW), np.empty(4 * NW)
    nc = sum((n - 1) ** 2 for n in nel)
    Sc, lc = np.empty(max(nc, 1)), np.empty(max(sum(n - 1 for n in nel), 1))
    assert lib.nek_host_schwarz(N, _i3(nel), _ptr(vtx), _ptr(Sw), _ptr(lw), _ptr(Sc), _ptr(lc)) == 0
    xi, w = oracle.gll(N)
    D = oracle.deriv(N)
    Kw, Ww = schwarz.window_operators(N, D, w)
    for (lo, hi), (keep, So, lo_) in schwarz.window_variants(N, D, w).items():
        v = lo + 2 * hi
        S = Sw[v * NW * NW:(v + 1) * NW * NW].reshape(NW, NW)
        lam = lw[v * NW:(v + 1) * NW]
        m = len(keep)
        drop = np.setdiff1d(np.arange(NW), keep)
        assert not S[drop].any() and not S[:, m:].any() and np.all(lam[m:] == 1.0)
        Sk = S[keep][:, :m]
        np.testing.assert_allclose(np.sort(lam[:m]), np.sort(lo_), rtol=1e-11)
        ref = So @ np.diag(1 / lo_) @ So.T
        np.testing.assert_allclose(Sk @ np.diag(1 / lam[:m]) @ Sk.T, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
        np.testing.assert_allclose(Sk.T @ np.diag(Ww[keep]) @ Sk, np.eye(m), atol=1e-11)
    P = oracle.Problem(N, nel, vtx)
    M = schwarz.Schwarz(P, vtx)
    so = lo2 = 0
    for d, n in enumerate(nel):
        m = n - 1
        if m == 0:
            continue
        S = Sc[so:so + m * m].reshape(m, m)
        lam = lc[lo2:lo2 + m]
        So, lo_ = M.coarse[d]
        np.testing.assert_allclose(np.sort(lam), np.sort(lo_), rtol=1e-11)
        ref = So @ np.diag(1 / lo_) @ So.T
        np.testing.assert_allclose(S @ np.diag(1 / lam) @ S.T, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
        so += m * m
        lo2 += m
