// Device kernels of libnek (gfx950).  Internal header, included once by
// nek_lib.hip.
//
// Hot path of one CG iteration (the loop of the paper's Table 1, no
// preconditioner): two launches per iteration.
//   k_ax<CG>(it)    alpha and rtr of iteration it-1 from the previous
//                   kernels' partials; x += alpha_{it-1} p_{it-1} (add2s2
//                   for x, deferred one iteration because this kernel reads
//                   p anyway); beta; p = beta p + r (add2s1);
//                   w_L = A_L p (ax_e: local_grad3, g1..g6, local_grad3_t);
//                   per-workgroup partials of p.w_L.
//   k_cg_update(it) alpha = rtz / pap; for every local point S = sum of the
//                   copies of w_L at its global node (dssum), mask,
//                   r -= alpha S (add2s2 for r); partials of glsc3(r, c, r).
// Because p is continuous and zero on the Dirichlet boundary,
// glsc3(M dssum(A_L p), c, p) = sum_l p_l (A_L p)_l in exact arithmetic, so
// pap needs no gather and alpha is known right after the operator.  The
// operator kernel launched once more after the last iteration applies the
// pending x update and publishes the final state.
//
// Reductions without atomics or fences: a kernel writes one FP64 partial
// per workgroup with a plain store; every workgroup of a LATER kernel sums
// all of them in the same fixed order (so all obtain the identical value),
// the kernel boundary making the stores visible.  Device-scope fences would
// write back and invalidate a whole XCD's L2 per workgroup on gfx950.  The
// CG state and the partials are double-buffered by iteration parity; only
// workgroup 0 writes the state slot of the current iteration.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace nek {

constexpr int UPD_BS = 256;      // block size of the pointwise kernels
constexpr int MAXB = 2048;       // cap on workgroups of any reducing kernel (partials per region)

// Elements per workgroup of the operator kernel for each NP = N+1, chosen so
// EPW*NP^2 fills whole 64-lane waves where possible and the FP64 LDS
// footprint 3*EPW*NP^3*8 stays within 160 KB.
constexpr int epw_for(int NP)
{
    return NP == 2 ? 16 : NP == 3 ? 7 : NP == 4 ? 8 : NP == 5 ? 5 : NP == 6 ? 7 : NP == 7 ? 9
         : NP == 8 ? 4 : NP == 9 ? 4 : NP == 10 ? 3 : NP == 11 ? 2 : NP == 12 ? 2 : 1;
}

// CG state entering iteration it, in slot it & 1.
struct IterState {
    double rtz;      // glsc3(r, c, z) of the current residual, z = M^-1 r (z = r without preconditioner)
    double rtr;      // glsc3(r, c, r): the stopping test and the residual history
    double beta;
    int iter;        // iterations completed
    int done;
    int status;      // 0, -5 (breakdown) or -6 (non-finite)
    int conv;        // stopped by the tolerance (or r == 0)
};

struct Scal {
    IterState st[2];
    IterState fin;        // state of the iteration that ended the run
    double hist_den;      // history entry = sqrt(rtz / hist_den)
    double stop_den;      // stop when sqrt(rtz) / sqrt(stop_den) <= stop_tol
    double stop_tol;      // <= 0: run to maxit
    double red[4];        // results of standalone reductions
    int maxit;
    int hist_off;         // history index of iteration 0 of this run
    int k2flag[2];        // status of k_cg_update(it) in slot it & 1
    int done_host;        // set once a run is done
    int resume;           // 1: the run continues the previous search direction
    int *host_done;       // device alias of a pinned host flag mirroring done_host (or null)
};

// A flag in pinned host memory, written by a system-scope store so that the
// host sees it once the writing kernel has completed.
__device__ __forceinline__ void set_host_flag(int *f, int v)
{
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

struct Box { int nx, ny, nz; };

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so neighbouring elements share an L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned X = 8, x = b % X, slot = b / X, q = nb / X, r = nb % X;
    return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// Deterministic block sum (fixed order); the result is valid in thread 0.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *sbuf)
{
    if constexpr (BS % 64 == 0) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        constexpr int NW = BS / 64;
        if ((threadIdx.x & 63) == 0) sbuf[threadIdx.x >> 6] = v;
        __syncthreads();
        double s = 0.0;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < NW; ++q) s += sbuf[q];
        }
        __syncthreads();
        return s;
    } else {
        // partial last wave: lanes past BS do not exist, so reduce in LDS
        sbuf[threadIdx.x] = v;
        __syncthreads();
        constexpr int P2 = BS <= 1 ? 1 : 1 << (32 - __builtin_clz(BS - 1));
#pragma unroll
        for (int s = P2 / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s && threadIdx.x + s < BS) sbuf[threadIdx.x] += sbuf[threadIdx.x + s];
            __syncthreads();
        }
        double r = sbuf[0];
        __syncthreads();
        return r;
    }
}

// 1 / m for a multiplicity m in {1, 2, 4, 8}: exact, so (v * inv_mult(m))
// equals v / m bit for bit without a division.
__device__ __forceinline__ double inv_mult(int m)
{
    return m == 1 ? 1.0 : m == 2 ? 0.5 : m == 4 ? 0.25 : 0.125;
}

// Fixed-order sums of NA arrays of per-workgroup partials, returned to every
// thread of the block.  The first NT threads (whole waves: lanes past the
// last full wave do not exist for shuffles) each add the pairs
// (P[2q], P[2q + 1]) for q = t, t + NT, t + 2 NT, ..., low entry first, with
// a batch of U pairs per array loaded (16 bytes each) before the first add
// (U bounds the registers the loads in flight take);
// then a butterfly within each wave and the waves in order, broadcast
// through LDS.  The order of one array's sum does not depend on NA or U, so
// every kernel of block size BS that sums the same partials, alone or
// together with another array, gets the bit-identical value.  Each P[a] is
// 16-byte aligned and readable up to the next even count (P[n] when n is
// odd, a value that is not added): the partial slots hold MAXB entries.
template <int BS, int NA, bool WIDE = false>
__device__ __forceinline__ void sum_all_n(const double *const *P, const int *n, double *sbuf, double *out)
{
    constexpr int NW = BS >= 64 ? BS / 64 : 1;
    constexpr int NT = BS >= 64 ? NW * 64 : BS;
    // pairs in flight per thread: 8 per array below 256 threads, except three
    // arrays without WIDE (4 each), which would cost 4-byte operator kernels
    // a wave per SIMD; FP64 ones have the registers (WIDE) and then sum 2048
    // partials in one batch of loads instead of two
    constexpr int U = NT >= 256 || (NA >= 3 && !WIDE) ? 4 : 8;
    double v[NA];
    int nmax = 0;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        v[a] = 0.0;
        nmax = max(nmax, n[a]);
    }
    if (threadIdx.x < NT)
        for (int q0 = threadIdx.x; 2 * q0 < nmax; q0 += U * NT) {
            double2 t[NA][U];
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = q0 + u * NT;
                    t[a][u] = 2 * q < n[a] ? reinterpret_cast<const double2 *>(P[a])[q] : double2{0.0, 0.0};
                }
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    v[a] += t[a][u].x;
                    v[a] += 2 * (q0 + u * NT) + 1 < n[a] ? t[a][u].y : 0.0;
                }
        }
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        if constexpr (BS >= 64) {
            double w = v[a];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
            if (threadIdx.x < NT && (threadIdx.x & 63) == 0) sbuf[threadIdx.x >> 6] = w;
            __syncthreads();
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) s += sbuf[q];
            __syncthreads();
            out[a] = s;
        } else {
            out[a] = block_sum<BS>(v[a], sbuf);   // LDS tree, result in every thread
        }
    }
}

template <int BS>
__device__ __forceinline__ double sum_all(const double *__restrict__ P, int n, double *sbuf)
{
    const double *ps[1] = {P};
    const int ns[1] = {n};
    double out[1];
    sum_all_n<BS, 1>(ps, ns, sbuf, out);
    return out[0];
}

// Start of iteration it: fold the partials of iteration it-1 into the state
// (identically in every workgroup) and decide whether to stop.  Returns the
// state and the pending x update alpha_{it-1} (when iteration it-1
// completed).  Workgroup 0, thread 0 publishes the state.
struct Begin {
    IterState cur;
    double alpha_prev;
    bool xupd;
};

// With PC (diagonal preconditioner), P2 holds the partials of glsc3(r, c, z)
// and P4 those of glsc3(r, c, r); without it P2 holds glsc3(r, c, r) and P4
// is unused.
template <int BS, bool PC = false, bool WIDE = false>
__device__ __forceinline__ Begin cg_begin(Scal *__restrict__ sc, const double *__restrict__ P1prev, int nb1,
                                          const double *__restrict__ P2prev, int nb2, int it,
                                          double *__restrict__ hist, double *sbuf, bool writer,
                                          const double *__restrict__ P4prev = nullptr)
{
    const IterState prev = sc->st[(it - 1) & 1];
    Begin B{prev, 0.0, false};
    IterState &cur = B.cur;
    if (!prev.done) {
        if (it == 1) {
            if (!sc->resume) cur.beta = 0.0;   // a resumed run keeps beta set at its start
            cur.iter = 0;
        } else {
            const int f = sc->k2flag[(it - 1) & 1];
            if (f) {
                cur.status = f;
                cur.done = 1;
            } else {
                // the sums with their loads in flight together
                constexpr int NS = PC ? 3 : 2;
                const double *ps[3] = {P1prev, P2prev, P4prev};
                const int ns[3] = {nb1, nb2, nb2};
                double sums[3];
                sum_all_n<BS, NS, WIDE>(ps, ns, sbuf, sums);
                B.alpha_prev = prev.rtz / sums[0];
                B.xupd = true;
                const double rtz = sums[1];
                const double rtr = PC ? sums[2] : rtz;
                cur.iter = it - 1;
                cur.rtz = rtz;
                cur.rtr = rtr;
                cur.beta = rtz / prev.rtz;
                if (writer && hist) hist[sc->hist_off + it - 1] = sqrt(rtr / sc->hist_den);
                if (!__builtin_isfinite(rtr) || !__builtin_isfinite(rtz)) {
                    cur.status = -6;
                    cur.done = 1;
                } else if (rtr == 0.0 || (sc->stop_tol > 0 && sqrt(rtr) / sqrt(sc->stop_den) <= sc->stop_tol)) {
                    cur.conv = 1;
                    cur.done = 1;
                }
            }
        }
        if (!cur.done && cur.iter >= sc->maxit) cur.done = 1;
    }
    if (writer) {
        sc->st[it & 1] = cur;
        if (cur.done) {
            sc->done_host = 1;
            if (sc->host_done) set_host_flag(sc->host_done, 1);
            sc->fin = cur;
        }
    }
    return B;
}

// ------------------------------------------------------ geometric factors

// The six factors of one point are stored together ([E][NP^3][6], order
// G_rr, G_ss, G_tt, G_rs, G_rt, G_st) and fetched with wide loads.
template <typename GT> struct GLoad;
template <> struct GLoad<double> {
    struct Raw { double2 a, b, c; };
    __device__ static Raw load(const double *p)
    {
        const double2 *q = reinterpret_cast<const double2 *>(p);
        return Raw{q[0], q[1], q[2]};
    }
    template <typename T> __device__ static void unpack(const Raw &r, T o[6])
    {
        o[0] = r.a.x; o[1] = r.a.y; o[2] = r.b.x; o[3] = r.b.y; o[4] = r.c.x; o[5] = r.c.y;
    }
};
template <> struct GLoad<float> {
    struct Raw { float2 a, b, c; };
    __device__ static Raw load(const float *p)
    {
        const float2 *q = reinterpret_cast<const float2 *>(p);
        return Raw{q[0], q[1], q[2]};
    }
    template <typename T> __device__ static void unpack(const Raw &r, T o[6])
    {
        o[0] = r.a.x; o[1] = r.a.y; o[2] = r.b.x; o[3] = r.b.y; o[4] = r.c.x; o[5] = r.c.y;
    }
};
template <> struct GLoad<uint16_t> {   // BF16 bit patterns, two per 32-bit word
    struct Raw { uint32_t a, b, c; };
    __device__ static Raw load(const uint16_t *p)
    {
        const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
        return Raw{q[0], q[1], q[2]};
    }
    template <typename T> __device__ static void unpack(const Raw &r, T o[6])
    {
        o[0] = __uint_as_float(r.a << 16); o[1] = __uint_as_float(r.a & 0xffff0000u);
        o[2] = __uint_as_float(r.b << 16); o[3] = __uint_as_float(r.b & 0xffff0000u);
        o[4] = __uint_as_float(r.c << 16); o[5] = __uint_as_float(r.c & 0xffff0000u);
    }
};

// Geometric factors recomputed in the kernel from each element's trilinear
// map instead of read from memory.  Every element is the trilinear image of
// its 8 vertices, x(r,s,t) = a0 + a1 r + a2 s + a3 t + a4 rs + a5 rt + a6 st
// + a7 rst per coordinate, so with J = [x_r x_s x_t]
//   x_r = (a1 + a4 s) + (a5 + a7 s) t,  x_s = (a2 + a4 r) + (a6 + a7 r) t,
//   x_t = a3 + a5 r + a6 s + a7 r s,
// and with c_r = x_s x x_t, c_s = x_t x x_r, c_t = x_r x x_s (the rows of
// det(J) J^-1) and det(J) = x_r . c_r the factors are
//   G_ab = w_i w_j w_k (c_a . c_b) / det(J),
// the same quantities the stored arrays hold (applied without forming them).  Buffer layout, in the
// vector type: a header of TRI_HDR entries (GLL nodes xi[NP], then weights
// w[NP]), then per element 3 records of 8 (a1..a7 and a zero, one record per
// coordinate).  The tag type selects this path wherever a factor-storage
// type is expected; it is never dereferenced as such.
template <typename T> struct TriG { T v; };
template <typename GT> struct TriOf { static constexpr bool value = false; using type = void; };
template <typename T> struct TriOf<TriG<T>> { static constexpr bool value = true; using type = T; };
constexpr int TRI_HDR = 32;   // 2 * MAX_NP
constexpr int TRI_REC = 24;   // entries per element

template <typename T> struct GLoad<TriG<T>> {
    struct Raw {};
    __device__ static Raw load(const TriG<T> *) { return Raw{}; }
    template <typename U> __device__ static void unpack(const Raw &, U o[6])
    {
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = 0;
    }
};

// The 24 coefficients of one element, loaded with 16-byte loads.
template <typename T> struct TriRaw { T a[TRI_REC]; };
template <typename T> __device__ __forceinline__ TriRaw<T> tri_load(const T *__restrict__ rec)
{
    TriRaw<T> o;
    if constexpr (sizeof(T) == 4) {
        const float4 *q = reinterpret_cast<const float4 *>(rec);
#pragma unroll
        for (int m = 0; m < TRI_REC / 4; ++m) {
            const float4 v = q[m];
            o.a[4 * m + 0] = v.x; o.a[4 * m + 1] = v.y; o.a[4 * m + 2] = v.z; o.a[4 * m + 3] = v.w;
        }
    } else {
        const double2 *q = reinterpret_cast<const double2 *>(rec);
#pragma unroll
        for (int m = 0; m < TRI_REC / 2; ++m) {
            const double2 v = q[m];
            o.a[2 * m + 0] = v.x; o.a[2 * m + 1] = v.y;
        }
    }
    return o;
}

// Column (r, s) = (xi_i, xi_j) of one element: the parts of x_r and x_s
// that do not depend on t, and x_t.
template <typename T> struct TriCol { T pr[3], qr[3], ps[3], qs[3], xt[3]; };
template <typename T> __device__ __forceinline__ TriCol<T> tri_col(const TriRaw<T> &R, T r, T s)
{
    TriCol<T> c;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T *a = R.a + 8 * d;   // a1..a7 at a[0..6]
        c.pr[d] = a[0] + a[3] * s;
        c.qr[d] = a[4] + a[6] * s;
        c.ps[d] = a[1] + a[3] * r;
        c.qs[d] = a[5] + a[6] * r;
        c.xt[d] = a[2] + a[4] * r + (a[5] + a[6] * r) * s;
    }
    return c;
}

// 1 / d: the hardware reciprocal, refined by two Newton steps in FP64.
__device__ __forceinline__ float tri_rcp(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double tri_rcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// At t = xi_k: the rows c_r, c_s, c_t of det(J) J^-1 (K[a][d] = c_a[d]) and
// f = w_i w_j w_k / det(J).  Applied to the reference gradient
// (u_r, u_s, u_t) the factors give G (u_r, u_s, u_t) = f K (K^T (u_r, u_s, u_t)),
// 21 operations instead of forming the six factors (24) and applying them (9).
template <typename T> __device__ __forceinline__ void tri_rows(const TriCol<T> &c, T t, T wijk, T K[3][3], T &f)
{
    T xr[3], xs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        xr[d] = c.pr[d] + c.qr[d] * t;
        xs[d] = c.ps[d] + c.qs[d] * t;
    }
    const T *xt = c.xt;
    K[0][0] = xs[1] * xt[2] - xs[2] * xt[1];
    K[0][1] = xs[2] * xt[0] - xs[0] * xt[2];
    K[0][2] = xs[0] * xt[1] - xs[1] * xt[0];
    K[1][0] = xt[1] * xr[2] - xt[2] * xr[1];
    K[1][1] = xt[2] * xr[0] - xt[0] * xr[2];
    K[1][2] = xt[0] * xr[1] - xt[1] * xr[0];
    K[2][0] = xr[1] * xs[2] - xr[2] * xs[1];
    K[2][1] = xr[2] * xs[0] - xr[0] * xs[2];
    K[2][2] = xr[0] * xs[1] - xr[1] * xs[0];
    const T det = xr[0] * K[0][0] + xr[1] * K[0][1] + xr[2] * K[0][2];
    f = wijk * tri_rcp(det);
}

// (w_r, w_s, w_t) = f K K^T (u_r, u_s, u_t).
template <typename T>
__device__ __forceinline__ void tri_apply(const T K[3][3], T f, T ur, T us, T ut, T &wr, T &ws, T &wt)
{
    T v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = f * (K[0][d] * ur + K[1][d] * us + K[2][d] * ut);
    wr = K[0][0] * v[0] + K[0][1] * v[1] + K[0][2] * v[2];
    ws = K[1][0] * v[0] + K[1][1] * v[1] + K[1][2] * v[2];
    wt = K[2][0] * v[0] + K[2][1] * v[1] + K[2][2] * v[2];
}

// ---------------------------------------------------------------- operator

// One workgroup = EPW elements x (NP x NP) threads; thread (i, j) walks the
// k-column of its element.  u is staged in LDS for the r and s derivatives;
// the t derivative uses the thread's own column in registers.  wr, ws go
// through LDS for the transposed derivatives, wt stays in registers.  The
// uniform entries D[k][l] of the t contractions come through the scalar
// cache.  The six factors of slice k + PD are in flight while slice k is
// computed.  CG mode fuses p = beta p + r before, and sum p.(A_L p) after.
// A row of RP (a multiple of 4) 4-byte values from 16-byte aligned LDS.
template <int RP, typename T> __device__ __forceinline__ void load_row(const T *__restrict__ src, T out[RP])
{
    static_assert(sizeof(T) == 4 && RP % 4 == 0, "rows of 4-byte values, pitch a multiple of 4");
#pragma unroll
    for (int q = 0; q < RP / 4; ++q) {
        const float4 v = reinterpret_cast<const float4 *>(src)[q];
        out[4 * q + 0] = __builtin_bit_cast(T, v.x);
        out[4 * q + 1] = __builtin_bit_cast(T, v.y);
        out[4 * q + 2] = __builtin_bit_cast(T, v.z);
        out[4 * q + 3] = __builtin_bit_cast(T, v.w);
    }
}

// LDS layout of the operator kernel.  4-byte types keep every slice as rows
// of a pitch rounded up to 4 entries, with a transposed copy of u and ws
// stored transposed, so that every derivative sum reads one contiguous,
// 16-byte aligned row (128-bit LDS reads); FP64, bound by HBM rather than
// LDS, keeps three plain NP^3 arrays.
template <int NP, typename T> struct AxLds {
    static constexpr bool ROWS = sizeof(T) == 4;
    static constexpr int RP = ROWS ? (NP + 3) / 4 * 4 : NP;   // row pitch
    static constexpr int SL = NP * RP;                         // one k slice
    static constexpr int EL = NP * SL;                         // one element
    static constexpr int NARR = ROWS ? 4 : 3;
};
template <int NP, int EPW, typename T> constexpr size_t ax_lds_bytes()
{
    return (size_t)AxLds<NP, T>::NARR * EPW * AxLds<NP, T>::EL * sizeof(T);
}

// Body of the operator kernel for one problem: workgroup blk of the
// problem's nblk workgroups.
template <int NP, int EPW, int PD, typename T, typename GT, bool CG, typename XT, bool PC = false>
__device__ __forceinline__ void ax_body(const T *__restrict__ src, T *__restrict__ p, T *__restrict__ w,
                                        const GT *__restrict__ g, const T *__restrict__ D, XT *__restrict__ x,
                                        Scal *__restrict__ sc, double *__restrict__ P1cur,
                                        const double *__restrict__ P1prev, const double *__restrict__ P2prev,
                                        int nb2, int it, double *__restrict__ hist, int E, int ngroups,
                                        unsigned blk, unsigned nblk, const double *__restrict__ P4prev = nullptr)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, BS = EPW * NP2;
    using GL = GLoad<GT>;
    using L = AxLds<NP, T>;
    constexpr bool ROWS = L::ROWS;
    constexpr int RP = L::RP, SL = L::SL, EL = L::EL;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *su = reinterpret_cast<T *>(smem_raw);
    T *sr = su + EPW * EL;
    T *ss = sr + EPW * EL;
    T *sut = ROWS ? ss + EPW * EL : su;   // transposed u (rows only)
    __shared__ double sbuf[BS];
    __shared__ T sD[NP * NP];

    const int tid = threadIdx.x;
    const int el = tid / NP2, ij = tid - el * NP2;
    const unsigned lb = xcd_block(blk, nblk);
    const int g0 = (int)(((long)lb * ngroups) / nblk);
    const int g1 = (int)(((long)(lb + 1) * ngroups) / nblk);
    const int i = ij % NP, j = ij / NP;
    T *sue = su + el * EL, *sre = sr + el * EL, *sse = ss + el * EL, *sute = sut + el * EL;

    // FP32: the thread's rows/columns of D live in registers.  FP64 reads
    // them from LDS instead (no register spills; FP64 has bandwidth slack).
    constexpr bool DREG = sizeof(T) == 4;
    T Dri[DREG ? NP : 1], Dsj[DREG ? NP : 1], DTi[DREG ? NP : 1], DTj[DREG ? NP : 1];
    // The first PD slices of g of a group; those of the first group are
    // requested before the CG prologue, so their latency overlaps its
    // reduction.  Threads past the last element work on a copy of element
    // E-1 and store nothing (local indices fit in 32 bits, checked at set-up).
    typename GL::Raw gb[PD];
    // in-kernel factors: the element's coefficients are requested where the
    // stored path requests its first slices
    constexpr bool TRI = TriOf<GT>::value;
    using TV = std::conditional_t<TRI, T, float>;
    const TV *tg = reinterpret_cast<const TV *>(g);
    TriRaw<TV> traw;
    TV txi = 0, txj = 0, twij = 0;
    if constexpr (TRI) {
        static_assert(std::is_same_v<typename TriOf<GT>::type, T>, "factors in the vectors' type");
        txi = tg[i];
        txj = tg[j];
        twij = tg[NP + i] * tg[NP + j];
    }
    auto g_first = [&](int grp) {
        const int e = grp * EPW + el;
        const int ec = e < E ? e : E - 1;
        if constexpr (TRI) {
            traw = tri_load<TV>(tg + TRI_HDR + (size_t)ec * TRI_REC);
        } else {
            const GT *ge = g + (size_t)(ec * NP3 + ij) * 6;
#pragma unroll
            for (int s = 0; s < PD; ++s)
                if (s < NP) gb[s] = GL::load(ge + (size_t)s * NP2 * 6);
        }
    };
    if (g0 < g1) g_first(g0);
    T beta = 0;
    bool first = false, xupd = false;
    double alpha_prev = 0.0;
    if constexpr (CG) {
        const Begin B =
            cg_begin<BS, PC, sizeof(T) == 8>(sc, P1prev, (int)nblk, P2prev, nb2, it, hist, sbuf, blk == 0 && tid == 0,
                                             P4prev);
        xupd = B.xupd;
        alpha_prev = B.alpha_prev;
        if (B.cur.done) {
            // last call of a run: only the pending x += alpha p
            if (xupd)
                for (int grp = g0; grp < g1; ++grp) {
                    const int e = grp * EPW + el;
                    if (e >= E) continue;
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const int idx = e * NP3 + k * NP2 + ij;
                        x[idx] = (XT)((double)x[idx] + alpha_prev * (double)p[idx]);
                    }
                }
            return;
        }
        beta = (T)B.cur.beta;
        first = it == 1 && !sc->resume;
    }
    // From NP = 12 on, keeping all four sets of D entries for the whole
    // kernel would cost a wave per SIMD: each phase then reloads its two
    // sets from a copy of D and of D^T in LDS, so only two are live at once.
    constexpr bool DPH = DREG && NP >= 12;
    __shared__ __align__(16) T sDD[DPH ? 2 * NP * NP : 1];
    auto d_rows = [&](const T *base, T a[], T b[]) {
        if constexpr (NP % 4 == 0 && sizeof(T) == 4) {
            load_row<NP>(base + i * NP, a);
            load_row<NP>(base + j * NP, b);
        } else {
#pragma unroll
            for (int l = 0; l < NP; ++l) {
                a[l] = base[i * NP + l];
                b[l] = base[j * NP + l];
            }
        }
    };
    if constexpr (DPH) {
        for (int q = tid; q < NP * NP; q += BS) {
            sDD[q] = D[q];
            sDD[NP * NP + q] = D[(q % NP) * NP + q / NP];
        }
    } else if constexpr (DREG) {
#pragma unroll
        for (int l = 0; l < NP; ++l) {
            Dri[l] = D[i * NP + l];
            Dsj[l] = D[j * NP + l];
            DTi[l] = D[l * NP + i];
            DTj[l] = D[l * NP + j];
        }
    } else {
        for (int q = tid; q < NP * NP; q += BS) sD[q] = D[q];
    }
#define NEK_DR(l) (DREG ? Dri[DREG ? (l) : 0] : sD[i * NP + (l)])
#define NEK_DS(l) (DREG ? Dsj[DREG ? (l) : 0] : sD[j * NP + (l)])
#define NEK_DTI(l) (DREG ? DTi[DREG ? (l) : 0] : sD[(l) * NP + i])
#define NEK_DTJ(l) (DREG ? DTj[DREG ? (l) : 0] : sD[(l) * NP + j])
    double pap = 0.0;

    for (int grp = g0; grp < g1; ++grp) {
        const int e = grp * EPW + el;
        const bool valid = e < E;
        const int base = (valid ? e : E - 1) * NP3 + ij;
        const GT *ge = TRI ? g : g + (size_t)base * 6;
        if (grp > g0) g_first(grp);
        T u[NP];
        __syncthreads();   // LDS of the previous group is free
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int idx = base + k * NP2;
            T v;
            if constexpr (CG) {
                const T rv = src[idx];
                const T po = p[idx];
                if (xupd && valid) x[idx] = (XT)((double)x[idx] + alpha_prev * (double)po);
                v = first ? rv : beta * po + rv;
                if (valid) p[idx] = v;
            } else {
                v = src[idx];
            }
            u[k] = v;
            sue[k * SL + j * RP + i] = v;
            if constexpr (ROWS) sute[k * SL + i * RP + j] = v;
        }
        __syncthreads();
        if constexpr (DPH) d_rows(sDD, Dri, Dsj);   // rows i and j of D
        TriCol<TV> tcol;
        if constexpr (TRI) tcol = tri_col<TV>(traw, txi, txj);
        T wt[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            __builtin_amdgcn_sched_barrier(0);
            T gk[6];
            TV tK[3][3], tf = 0;
            if constexpr (TRI) tri_rows<TV>(tcol, tg[k], twij * tg[NP + k], tK, tf);
            else GL::unpack(gb[k % PD], gk);
            T ur = 0, us = 0, ut = 0;
            if constexpr (ROWS) {
                T rr[RP], rs[RP];
                load_row<RP>(sue + k * SL + j * RP, rr);
                load_row<RP>(sute + k * SL + i * RP, rs);
#pragma unroll
                for (int l = 0; l < NP; ++l) {
                    ur += NEK_DR(l) * rr[l];
                    us += NEK_DS(l) * rs[l];
                    ut += D[k * NP + l] * u[l];
                }
            } else {
#pragma unroll
                for (int l = 0; l < NP; ++l) {
                    ur += NEK_DR(l) * sue[k * NP2 + j * NP + l];
                    us += NEK_DS(l) * sue[k * NP2 + l * NP + i];
                    ut += D[k * NP + l] * u[l];
                }
            }
            // wr by rows of constant j; ws by rows of constant i (transposed)
            T gr, gs, gt;
            if constexpr (TRI) {
                tri_apply<TV>(tK, tf, ur, us, ut, gr, gs, gt);
            } else {
                gr = gk[0] * ur + gk[3] * us + gk[4] * ut;
                gs = gk[3] * ur + gk[1] * us + gk[5] * ut;
                gt = gk[4] * ur + gk[5] * us + gk[2] * ut;
            }
            sre[k * SL + j * RP + i] = gr;
            sse[k * SL + (ROWS ? i * RP + j : j * NP + i)] = gs;
            wt[k] = gt;
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (!TRI)
                if (k + PD < NP) gb[k % PD] = GL::load(ge + (size_t)(k + PD) * NP2 * 6);
        }
        __syncthreads();
        if constexpr (DPH) d_rows(sDD + NP * NP, DTi, DTj);   // columns i and j of D
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            // plain form: one slice at a time.  Left free, the scheduler
            // hoists the LDS rows of every slice ahead of the arithmetic
            // (148-155 VGPRs at NP = 10, 220 for FP64); the CG form keeps its
            // own order (pinning it slows the FP64 kernel by 2-5 %)
            if constexpr (!CG) __builtin_amdgcn_sched_barrier(0);
            T acc = 0;
            if constexpr (ROWS) {
                T rr[RP], rs[RP];
                load_row<RP>(sre + k * SL + j * RP, rr);
                load_row<RP>(sse + k * SL + i * RP, rs);
#pragma unroll
                for (int l = 0; l < NP; ++l) acc += NEK_DTI(l) * rr[l];
#pragma unroll
                for (int l = 0; l < NP; ++l) acc += NEK_DTJ(l) * rs[l];
            } else {
#pragma unroll
                for (int l = 0; l < NP; ++l) acc += NEK_DTI(l) * sre[k * NP2 + j * NP + l];
#pragma unroll
                for (int l = 0; l < NP; ++l) acc += NEK_DTJ(l) * sse[k * NP2 + l * NP + i];
            }
#pragma unroll
            for (int l = 0; l < NP; ++l) acc += D[l * NP + k] * wt[l];
            if (valid) w[base + k * NP2] = acc;
            if (CG && valid) pap += (double)u[k] * (double)acc;
        }
    }
#undef NEK_DR
#undef NEK_DS
#undef NEK_DTI
#undef NEK_DTJ
    if constexpr (CG) {
        const double s = block_sum<BS>(pap, sbuf);
        if (tid == 0) P1cur[blk] = s;
    }
}

template <int NP, int EPW, int PD, typename T, typename GT, bool CG, typename XT, bool PC = false>
__global__ __launch_bounds__(EPW *NP *NP) void k_ax(const T *__restrict__ src, T *__restrict__ p,
                                                    T *__restrict__ w, const GT *__restrict__ g,
                                                    const T *__restrict__ D, XT *__restrict__ x,
                                                    Scal *__restrict__ sc, double *__restrict__ P1cur,
                                                    const double *__restrict__ P1prev,
                                                    const double *__restrict__ P2prev, int nb2, int it,
                                                    double *__restrict__ hist, int E, int ngroups,
                                                    const double *__restrict__ P4prev)
{
    ax_body<NP, EPW, PD, T, GT, CG, XT, PC>(src, p, w, g, D, x, sc, P1cur, P1prev, P2prev, nb2, it, hist, E,
                                            ngroups, blockIdx.x, gridDim.x, P4prev);
}

// ----------------------------------------------------------- gather-scatter

// Position of a local point and the copies of its global node.
template <int NP> struct PointInfo {
    long e;
    int i, j, k, ex, ey, ez;
    bool masked;
    int mult;
};

template <int NP>
__device__ __forceinline__ PointInfo<NP> locate(unsigned t, Box b)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    PointInfo<NP> P;
    const unsigned e = t / NP3, q = t - e * NP3;
    P.e = e;
    P.i = q % NP;
    P.j = (q / NP) % NP;
    P.k = q / NP2;
    P.ex = e % b.nx;
    const unsigned eyz = e / b.nx;
    P.ey = eyz % b.ny;
    P.ez = eyz / b.ny;
    const bool bx = (P.i == 0 && P.ex == 0) || (P.i == N && P.ex == b.nx - 1);
    const bool by = (P.j == 0 && P.ey == 0) || (P.j == N && P.ey == b.ny - 1);
    const bool bz = (P.k == 0 && P.ez == 0) || (P.k == N && P.ez == b.nz - 1);
    P.masked = bx || by || bz;
    const int mx = ((P.i == 0 && P.ex > 0) || (P.i == N && P.ex < b.nx - 1)) ? 2 : 1;
    const int my = ((P.j == 0 && P.ey > 0) || (P.j == N && P.ey < b.ny - 1)) ? 2 : 1;
    const int mz = ((P.k == 0 && P.ez > 0) || (P.k == N && P.ez < b.nz - 1)) ? 2 : 1;
    P.mult = mx * my * mz;
    return P;
}

// Sum over the copies of the point's global node, in ascending local index
// (copies lie in distinct elements; ascending (dz, dy, dx) is ascending e),
// starting from 0.0 like a serial sum.  With WEIGHT each copy is scaled by
// c = 1/mult first.  The (up to two) copies per direction are fixed-size
// register pairs, so no private memory is used.
template <int NP, typename T, bool WEIGHT>
__device__ __forceinline__ double gather_copies(const T *__restrict__ w, const PointInfo<NP> &P, Box b)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    // per direction: number of copies n?, element offsets d?0 < d?1, local coordinates c?0, c?1
    int nx = 1, dx0 = 0, dx1 = 0, cx0 = P.i, cx1 = 0;
    if (P.i == 0 && P.ex > 0) { nx = 2; dx0 = -1; cx0 = N; dx1 = 0; cx1 = 0; }
    else if (P.i == N && P.ex < b.nx - 1) { nx = 2; dx0 = 0; cx0 = N; dx1 = 1; cx1 = 0; }
    int ny = 1, dy0 = 0, dy1 = 0, cy0 = P.j, cy1 = 0;
    if (P.j == 0 && P.ey > 0) { ny = 2; dy0 = -1; cy0 = N; dy1 = 0; cy1 = 0; }
    else if (P.j == N && P.ey < b.ny - 1) { ny = 2; dy0 = 0; cy0 = N; dy1 = 1; cy1 = 0; }
    int nz = 1, dz0 = 0, dz1 = 0, cz0 = P.k, cz1 = 0;
    if (P.k == 0 && P.ez > 0) { nz = 2; dz0 = -1; cz0 = N; dz1 = 0; cz1 = 0; }
    else if (P.k == N && P.ez < b.nz - 1) { nz = 2; dz0 = 0; cz0 = N; dz1 = 1; cz1 = 0; }
    const double c = WEIGHT ? inv_mult(nx * ny * nz) : 1.0;
    const long sy = b.nx, sz = (long)b.nx * b.ny;
    double s = 0.0;
#pragma unroll
    for (int az = 0; az < 2; ++az) {
        if (az >= nz) break;
        const long oz = (az ? dz1 : dz0) * sz;
        const int kz = az ? cz1 : cz0;
#pragma unroll
        for (int ay = 0; ay < 2; ++ay) {
            if (ay >= ny) break;
            const long oy = (ay ? dy1 : dy0) * sy;
            const int jy = ay ? cy1 : cy0;
#pragma unroll
            for (int ax = 0; ax < 2; ++ax) {
                if (ax >= nx) break;
                const long ee = P.e + (ax ? dx1 : dx0) + oy + oz;
                const int ix = ax ? cx1 : cx0;
                const double v = (double)w[ee * NP3 + ix + NP * jy + NP2 * kz];
                s += WEIGHT ? c * v : v;
            }
        }
    }
    return s;
}

// Second kernel of CG iteration it: alpha = rtz / pap, then for every
// unmasked point S = sum of the copies of w_L at its global node (in a fixed
// pairwise order that every copy reproduces bit for bit), r -= alpha S, and
// partials of glsc3(r, c, r).
// Same workgroup shape as the operator (EPW elements x NP^2 threads walking
// k-columns).  All loads of a column are issued before any is used: the own
// column of r and w, the columns of w in the x, y and xy neighbours (for
// threads on those faces), and the neighbouring slices in z.
// The copies that a column (e, i, j) shares with neighbouring elements, for
// the fixed-order sums of the gather-scatter: the own column, the columns of
// the x, y and xy neighbours in the same k-range (offsets offX, offY, offXY
// from the element start; loaded only where the neighbour exists), and the
// end nodes of those four columns in the elements below (slice N of e - oz,
// meeting k = 0) and above (slice 0 of e + oz, meeting k = N).  For FP32
// the eight end-node loads are issued without a branch from addresses that
// are always valid (the element's own column when a neighbour is absent) and
// absent copies are then replaced by 0: as single conditional loads they
// would each end in a wait for every load in flight.
template <int NP, typename T>
__device__ __forceinline__ void load_copies(const T *__restrict__ we, int oz, bool hx, bool hy, bool hzm, bool hzp,
                                            int ij, int offX, int offY, int offXY, T wo[NP], T wx[NP], T wy[NP],
                                            T wxy[NP], T zm[4], T zp[4])
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    const bool hxy = hx && hy;
    const int cX = hx ? offX : ij, cY = hy ? offY : ij, cXY = hxy ? offXY : ij;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        wo[k] = we[k * NP2 + ij];
        wx[k] = wy[k] = wxy[k] = (T)0;
    }
    if (hx) {
#pragma unroll
        for (int k = 0; k < NP; ++k) wx[k] = we[k * NP2 + offX];
    }
    if (hy) {
#pragma unroll
        for (int k = 0; k < NP; ++k) wy[k] = we[k * NP2 + offY];
    }
    if (hxy) {
#pragma unroll
        for (int k = 0; k < NP; ++k) wxy[k] = we[k * NP2 + offXY];
    }
    if constexpr (sizeof(T) == 8) {
        // FP64: conditional loads (eight more values in flight would cost a
        // wave of occupancy per SIMD)
#pragma unroll
        for (int q = 0; q < 4; ++q) zm[q] = zp[q] = (T)0;
        if (hzm) {
            const T *wz = we - oz * NP3 + N * NP2;
            zm[0] = wz[ij];
            if (hx) zm[1] = wz[offX];
            if (hy) zm[2] = wz[offY];
            if (hxy) zm[3] = wz[offXY];
        }
        if (hzp) {
            const T *wz = we + oz * NP3;
            zp[0] = wz[ij];
            if (hx) zp[1] = wz[offX];
            if (hy) zp[2] = wz[offY];
            if (hxy) zp[3] = wz[offXY];
        }
    } else {
        const T *wm = hzm ? we - oz * NP3 + N * NP2 : we;
        const T *wp = hzp ? we + oz * NP3 : we;
        const T m0 = wm[ij], m1 = wm[cX], m2 = wm[cY], m3 = wm[cXY];
        const T p0 = wp[ij], p1 = wp[cX], p2 = wp[cY], p3 = wp[cXY];
        zm[0] = hzm ? m0 : (T)0;
        zm[1] = (hzm && hx) ? m1 : (T)0;
        zm[2] = (hzm && hy) ? m2 : (T)0;
        zm[3] = (hzm && hxy) ? m3 : (T)0;
        zp[0] = hzp ? p0 : (T)0;
        zp[1] = (hzp && hx) ? p1 : (T)0;
        zp[2] = (hzp && hy) ? p2 : (T)0;
        zp[3] = (hzp && hxy) ? p3 : (T)0;
    }
}

// One column (e, i, j) of the update kernel: its residual and every copy of
// its nodes, loaded together.
// With PC the column also holds the preconditioner diagonal m of its nodes.
template <int NP, typename T, bool PC = false> struct UpdCol {
    int e, ez;
    bool valid, hx, hy, hzm, hzp;
    T rv[NP], wo[NP], wx[NP], wy[NP], wxy[NP], zm[4], zp[4];
    T dv[PC ? NP : 1];
};

template <int NP, int EPW, typename T, bool PC>
__device__ __forceinline__ void upd_load(UpdCol<NP, T, PC> &c, const T *__restrict__ r, const T *__restrict__ w,
                                         const T *__restrict__ dg, int grp, int el, int i, int j, int ij, Box box,
                                         int E)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    c.e = grp * EPW + el;
    c.valid = false;
    if (c.e >= E) return;
    const int ex = c.e % box.nx;
    const int eyz = c.e / box.nx;
    const int ey = eyz % box.ny;
    c.ez = eyz / box.ny;
    if ((i == 0 && ex == 0) || (i == N && ex == box.nx - 1) || (j == 0 && ey == 0) || (j == N && ey == box.ny - 1))
        return;   // the whole column lies on the Dirichlet boundary
    c.valid = true;
    c.hx = (i == 0 && ex > 0) || (i == N && ex < box.nx - 1);
    c.hy = (j == 0 && ey > 0) || (j == N && ey < box.ny - 1);
    const bool xneg = i == 0, yneg = j == 0;   // neighbour sits below (dx or dy = -1)
    const int ox = xneg ? -1 : 1, oy = yneg ? -box.nx : box.nx;
    const int colX = (xneg ? N : 0) + NP * j, colY = i + NP * (yneg ? N : 0);
    const int colXY = (xneg ? N : 0) + NP * (yneg ? N : 0);
    c.hzm = c.ez > 0;
    c.hzp = c.ez < box.nz - 1;
    const int oz = box.nx * box.ny;   // local indices fit in 32 bits (checked at set-up)
#pragma unroll
    for (int k = 0; k < NP; ++k) c.rv[k] = r[c.e * NP3 + k * NP2 + ij];
    if constexpr (PC) {
#pragma unroll
        for (int k = 0; k < NP; ++k) c.dv[k] = dg[c.e * NP3 + k * NP2 + ij];
    }
    load_copies<NP>(w + c.e * NP3, oz, c.hx, c.hy, c.hzm, c.hzp, ij, ox * NP3 + colX, oy * NP3 + colY,
                    (ox + oy) * NP3 + colXY, c.wo, c.wx, c.wy, c.wxy, c.zm, c.zp);
}

// Gathered sum S of every node of the column (fixed pairwise order, see
// upd_body), r -= alpha S, and the column's part of sum c r^2.
// With PC the vector is z = r / m instead of r: z -= alpha S / m, and the
// parts of sum c r z (into part) and sum c r^2 (into part2), r = m z.
template <int NP, typename T, bool PC>
__device__ __forceinline__ void upd_apply(const UpdCol<NP, T, PC> &c, T *__restrict__ r, double alpha, int ij,
                                          Box box, double &part, double &part2)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    auto plane = [](double o, double X, double Y, double XY) -> double { return (o + X) + (Y + XY); };
    const int mxy = (c.hx ? 2 : 1) * (c.hy ? 2 : 1);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        if ((k == 0 && c.ez == 0) || (k == N && c.ez == box.nz - 1)) continue;   // Dirichlet slice
        double S = plane((double)c.wo[k], (double)c.wx[k], (double)c.wy[k], (double)c.wxy[k]);
        int m = mxy;
        if (k == 0 && c.hzm) {
            S = plane((double)c.zm[0], (double)c.zm[1], (double)c.zm[2], (double)c.zm[3]) + S;
            m *= 2;
        }
        if (k == N && c.hzp) {
            S = S + plane((double)c.zp[0], (double)c.zp[1], (double)c.zp[2], (double)c.zp[3]);
            m *= 2;
        }
        if constexpr (PC) {
            const double d = (double)c.dv[k];
            // FP32 vectors: the quotient in FP32 (the FP64 division sequence
            // would cost a wave of occupancy); identical on every copy
            double q;
            if constexpr (sizeof(T) == 4) q = (double)((float)S / c.dv[k]);
            else q = S / d;
            const T zn = (T)((double)c.rv[k] - alpha * q);
            r[c.e * NP3 + k * NP2 + ij] = zn;
            const double rn = d * (double)zn;
            part += (rn * (double)zn) * inv_mult(m);
            part2 += (rn * rn) * inv_mult(m);
        } else {
            const T rn = (T)((double)c.rv[k] - alpha * S);
            r[c.e * NP3 + k * NP2 + ij] = rn;
            part += ((double)rn * (double)rn) * inv_mult(m);
        }
    }
}

// Gather-scatter + mask of w = A_L p fused with r -= alpha M dssum(w) and the
// partials of rtr = glsc3(r, c, r).  Copies in one plane of constant k (own,
// x and y neighbours, the diagonal one; zero when absent, and adding +0.0 is
// exact) are summed as (own + X) + (Y + XY), pairing copies of the same y row
// first; the planes below and above are then added in turn.  IEEE addition
// is commutative, so every copy of a node computes the bit-identical value
// and r stays exactly continuous.
// With PC (diagonal preconditioner dg, 1 on Dirichlet nodes) r holds z =
// r / m and the kernel writes the partials of glsc3(r, c, z) to P2cur and
// of glsc3(r, c, r) to P4cur.  The unpreconditioned kernels run this form
// only when asked to (nek_set_update_kernel); by default they run
// upd_body_x (below), which takes the x-face copies shared inside a
// workgroup from LDS and adds the same values in the same order.
template <int NP, int EPW, typename T, bool PC = false>
__device__ __forceinline__ void upd_body(T *__restrict__ r, const T *__restrict__ w, Scal *__restrict__ sc,
                                         const double *__restrict__ P1cur, int nb1, double *__restrict__ P2cur,
                                         int it, Box box, int E, int ngroups, unsigned blk, unsigned nblk,
                                         const T *__restrict__ dg = nullptr, double *__restrict__ P4cur = nullptr)
{
    constexpr int NP2 = NP * NP, BS = EPW * NP2;
    __shared__ double sbuf[BS];
    const IterState cur = sc->st[it & 1];
    if (cur.done) return;
    const int tid = threadIdx.x;
    const int el = tid / NP2, ij = tid - el * NP2;
    const int i = ij % NP, j = ij / NP;
    const unsigned lb = xcd_block(blk, nblk);
    const int g0 = (int)(((long)lb * ngroups) / nblk);
    const int g1 = (int)(((long)(lb + 1) * ngroups) / nblk);
    // FP32 columns are loaded before the reduction; FP64 ones, and those of
    // the preconditioned kernel, after it (held across the reduction they
    // would cost a wave of occupancy per SIMD)
    constexpr bool early = sizeof(T) == 4 && !PC;
    UpdCol<NP, T, PC> c;
    c.valid = false;
    if (early && g0 < g1) upd_load<NP, EPW, T, PC>(c, r, w, dg, g0, el, i, j, ij, box, E);
    const double pap = sum_all<BS>(P1cur, nb1, sbuf);
    const bool writer = blk == 0 && tid == 0;
    if (!__builtin_isfinite(pap) || !(pap > 0)) {
        if (writer) sc->k2flag[it & 1] = __builtin_isfinite(pap) ? -5 : -6;
        return;
    }
    const double alpha = cur.rtz / pap;
    double part = 0.0, part2 = 0.0;
    if constexpr (early) {
        for (int grp = g0; grp < g1; ++grp) {
            if (grp > g0) upd_load<NP, EPW, T, PC>(c, r, w, dg, grp, el, i, j, ij, box, E);
            if (c.valid) upd_apply<NP, T, PC>(c, r, alpha, ij, box, part, part2);
        }
    } else {
        constexpr int NP3 = NP2 * NP, N = NP - 1;
        const int oz = box.nx * box.ny;
        for (int grp = g0; grp < g1; ++grp) {
            const int e = grp * EPW + el;
            if (e >= E) continue;
            const int ex = e % box.nx;
            const int eyz = e / box.nx;
            const int ey = eyz % box.ny, ez = eyz / box.ny;
            if ((i == 0 && ex == 0) || (i == N && ex == box.nx - 1) || (j == 0 && ey == 0) ||
                (j == N && ey == box.ny - 1))
                continue;   // the whole column lies on the Dirichlet boundary
            const bool hx = (i == 0 && ex > 0) || (i == N && ex < box.nx - 1);
            const bool hy = (j == 0 && ey > 0) || (j == N && ey < box.ny - 1);
            const bool xneg = i == 0, yneg = j == 0;
            const int ox = xneg ? -1 : 1, oy = yneg ? -box.nx : box.nx;
            const int colX = (xneg ? N : 0) + NP * j, colY = i + NP * (yneg ? N : 0);
            const int colXY = (xneg ? N : 0) + NP * (yneg ? N : 0);
            UpdCol<NP, T, PC> cg;
            cg.e = e;
            cg.ez = ez;
            cg.hx = hx;
            cg.hy = hy;
            cg.hzm = ez > 0;
            cg.hzp = ez < box.nz - 1;
#pragma unroll
            for (int k = 0; k < NP; ++k) cg.rv[k] = r[e * NP3 + k * NP2 + ij];
            if constexpr (PC) {
#pragma unroll
                for (int k = 0; k < NP; ++k) cg.dv[k] = dg[e * NP3 + k * NP2 + ij];
            }
            load_copies<NP>(w + e * NP3, oz, hx, hy, cg.hzm, cg.hzp, ij, ox * NP3 + colX, oy * NP3 + colY,
                            (ox + oy) * NP3 + colXY, cg.wo, cg.wx, cg.wy, cg.wxy, cg.zm, cg.zp);
            upd_apply<NP, T, PC>(cg, r, alpha, ij, box, part, part2);
        }
    }
    const double s = block_sum<BS>(part, sbuf);
    if (tid == 0) P2cur[blk] = s;
    if constexpr (PC) {
        const double s2 = block_sum<BS>(part2, sbuf);
        if (tid == 0) P4cur[blk] = s2;
    }
    if (writer) sc->k2flag[it & 1] = 0;
}

// Where a column of the update kernel finds the copies at its x face.  The
// face columns of two x-adjacent elements (i = N of the left one, i = 0 of
// the right one, same j) need each other's copies: the partner's own column
// is this column's x copy, the partner's y-neighbour column its xy copy and
// the partner's z end nodes (own and y neighbour) its x and xy end nodes.
//   xin:  the partner is in the same element group; the two swap through LDS.
//   cin:  the partner is the last element of the group this workgroup
//         walked just before (left face of the group's first element).
//   cout: this column is that partner for the next group of the walk.
// Otherwise (first group of a walk, right face of the last element) the x
// copies are gathered from memory as in upd_load.
struct XRole { bool xin, cin, cout, in_mesh; };

// The copies of one column (of w; the update kernel reads its column of r
// after the exchange, which keeps fewer registers live across the barrier:
// 162 instead of 176 VGPRs for FP64 at NP = 10, three waves per SIMD).
template <int NP, int EPW, typename T>
__device__ __forceinline__ XRole upd_load_x(UpdCol<NP, T, false> &c, const T *__restrict__ w, int grp, int g0,
                                            int g1, int el, int i, int j, int ij, Box box, int E)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    XRole xr{false, false, false, false};
    c.e = grp * EPW + el;
    c.valid = false;
    if (c.e >= E) return xr;
    xr.in_mesh = true;
    const int ex = c.e % box.nx;
    const int eyz = c.e / box.nx;
    const int ey = eyz % box.ny;
    c.ez = eyz / box.ny;
    if ((i == 0 && ex == 0) || (i == N && ex == box.nx - 1) || (j == 0 && ey == 0) || (j == N && ey == box.ny - 1))
        return xr;   // the whole column lies on the Dirichlet boundary
    c.valid = true;
    c.hx = (i == 0 && ex > 0) || (i == N && ex < box.nx - 1);
    c.hy = (j == 0 && ey > 0) || (j == N && ey < box.ny - 1);
    const bool xneg = i == 0, yneg = j == 0;
    // x-adjacent elements of one group, or of consecutive groups of one walk,
    // are consecutive local elements; the partner exists (hx) in the same row
    xr.xin = c.hx && (xneg ? el > 0 : el < EPW - 1);
    xr.cin = c.hx && xneg && el == 0 && grp > g0;
    xr.cout = c.hx && !xneg && el == EPW - 1 && grp + 1 < g1;
    const int ox = xneg ? -1 : 1, oy = yneg ? -box.nx : box.nx;
    const int colX = (xneg ? N : 0) + NP * j, colY = i + NP * (yneg ? N : 0);
    const int colXY = (xneg ? N : 0) + NP * (yneg ? N : 0);
    c.hzm = c.ez > 0;
    c.hzp = c.ez < box.nz - 1;
    const int oz = box.nx * box.ny;   // local indices fit in 32 bits (checked at set-up)
    load_copies<NP>(w + c.e * NP3, oz, c.hx && !xr.xin && !xr.cin, c.hy, c.hzm, c.hzp, ij, ox * NP3 + colX,
                    oy * NP3 + colY, (ox + oy) * NP3 + colXY, c.wo, c.wx, c.wy, c.wxy, c.zm, c.zp);
    return xr;
}

// A face column's values for its x partner (2 NP + 4 entries at sl), and the
// partner's values taken as this column's x and xy copies.
template <int NP, typename T>
__device__ __forceinline__ void xf_publish(T *sl, const UpdCol<NP, T, false> &c)
{
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        sl[k] = c.wo[k];
        sl[NP + k] = c.wy[k];
    }
    sl[2 * NP] = c.zm[0];
    sl[2 * NP + 1] = c.zm[2];
    sl[2 * NP + 2] = c.zp[0];
    sl[2 * NP + 3] = c.zp[2];
}

template <int NP, typename T>
__device__ __forceinline__ void xf_take(const T *sl, UpdCol<NP, T, false> &c)
{
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        c.wx[k] = sl[k];
        c.wxy[k] = sl[NP + k];
    }
    c.zm[1] = sl[2 * NP];
    c.zm[3] = sl[2 * NP + 1];
    c.zp[1] = sl[2 * NP + 2];
    c.zp[3] = sl[2 * NP + 3];
}

// The unpreconditioned update (upd_body without PC) with x-face copies
// exchanged in LDS between the columns that XRole pairs.  Every copy enters
// the same fixed-order sums with the same value as when gathered from
// memory, so the result is bit-identical to the gathering form.  A walk
// takes consecutive element groups; the exchange buffer is double-buffered
// and the carry between groups triple-buffered by group, so one barrier per
// group orders every write before its reads and after the previous reads of
// the same slot.
template <int NP, int EPW, typename T>
__device__ __forceinline__ void upd_body_x(T *__restrict__ r, const T *__restrict__ w, Scal *__restrict__ sc,
                                           const double *__restrict__ P1cur, int nb1, double *__restrict__ P2cur,
                                           int it, Box box, int E, int ngroups, unsigned blk, unsigned nblk)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, BS = EPW * NP2;
    constexpr int FV = 2 * NP + 4, FS = FV + 1;   // published values of a face column; odd slot stride
    __shared__ double sbuf[BS];
    __shared__ T xf[2][EPW][2][NP][FS];   // [group parity][element][face i = 0 / i = N][j][value]
    __shared__ T cf[3][NP][FS];           // [group mod 3][j][value]
    const IterState cur = sc->st[it & 1];
    if (cur.done) return;
    const int tid = threadIdx.x;
    const int el = tid / NP2, ij = tid - el * NP2;
    const int i = ij % NP, j = ij / NP;
    const int side = i == 0 ? 0 : 1;
    const unsigned lb = xcd_block(blk, nblk);
    const int g0 = (int)(((long)lb * ngroups) / nblk);
    const int g1 = (int)(((long)(lb + 1) * ngroups) / nblk);
    // FP32 copies of the first group are loaded before the reduction, FP64
    // ones after it (held across the reduction they would cost a wave of
    // occupancy per SIMD)
    constexpr bool early = sizeof(T) == 4;
    UpdCol<NP, T, false> c;
    XRole xr{false, false, false, false};
    c.valid = false;
    if (early && g0 < g1) xr = upd_load_x<NP, EPW, T>(c, w, g0, g0, g1, el, i, j, ij, box, E);
    const double pap = sum_all<BS>(P1cur, nb1, sbuf);
    const bool writer = blk == 0 && tid == 0;
    if (!__builtin_isfinite(pap) || !(pap > 0)) {
        if (writer) sc->k2flag[it & 1] = __builtin_isfinite(pap) ? -5 : -6;
        return;
    }
    const double alpha = cur.rtz / pap;
    double part = 0.0, part2 = 0.0;
    int buf = 0, c3 = 0, p3 = 2;   // exchange slot; carry slot written now and by the previous group
    for (int grp = g0; grp < g1; ++grp) {
        if (!early || grp > g0) xr = upd_load_x<NP, EPW, T>(c, w, grp, g0, g1, el, i, j, ij, box, E);
        if (c.valid && (xr.xin || xr.cout)) xf_publish<NP, T>(xr.xin ? xf[buf][el][side][j] : cf[c3][j], c);
        __syncthreads();
        if (c.valid) {
#pragma unroll
            for (int k = 0; k < NP; ++k) c.rv[k] = r[c.e * NP3 + k * NP2 + ij];
            if (xr.xin || xr.cin) xf_take<NP, T>(xr.xin ? xf[buf][el + (i == 0 ? -1 : 1)][side ^ 1][j] : cf[p3][j], c);
            upd_apply<NP, T, false>(c, r, alpha, ij, box, part, part2);
        }
        buf ^= 1;
        p3 = c3;
        c3 = c3 == 2 ? 0 : c3 + 1;
    }
    const double s = block_sum<BS>(part, sbuf);
    if (tid == 0) P2cur[blk] = s;
    if (writer) sc->k2flag[it & 1] = 0;
}

// When the exchange forms run (0: always, INT_MAX: never): the update
// kernel by default at every size (fewest element groups per workgroup), the
// assembly pass of nek_ax when its workgroups walk at least this many
// elements each.  The assembly's exchange form also changes its grid (one
// group per workgroup when gathering, a capped grid of walking workgroups
// when exchanging) and is the faster one only beyond the caches (32^3 N=9:
// 3-6 % faster; 16^3: within -2 / +3.5 %).
constexpr int UPD_X_MIN_GROUPS = 0;
constexpr int ASM_X_MIN_ELEMENTS = 6;

// Elements per workgroup of the assembly pass, per order and independent of
// the operator's configuration (the pass reduces nothing, so any grouping
// gives the same output): the count, within 512 threads and 48 KB of FP64
// exchange buffers, whose EPW * NP^2 threads fill 64-lane waves best.  At
// NP = 10 that is 5 (500 threads in 8 waves): the 32^3 N=9 exchange form
// takes 72-74 us (FP32) and 139-145 us (FP64) against 78 and 173 us with
// two elements per workgroup.
constexpr int asm_epw(int NP)
{
    return NP == 2 ? 80 : NP == 3 ? 42 : NP == 4 ? 28 : NP == 5 ? 15 : NP == 6 ? 14 : NP == 7 ? 9 : NP == 8 ? 8
         : NP == 9 ? 6 : NP == 10 ? 5 : NP == 11 ? 4 : NP <= 13 ? 3 : NP <= 15 ? 2 : 1;
}

// The unpreconditioned update of one workgroup: the exchange form when the
// walk has at least xmin groups per workgroup, the gathering form
// otherwise.  The exchange form pays one barrier per element group for the
// copies it does not gather; with its column of r read after the barrier it
// is the faster one on MI355X both beyond the caches (32^3 N=9: FP32 123 ->
// 97 us, FP64 222 -> 200 us per launch) and for cache-resident problems
// (16^3 N=9 solves 0.3-2.5 % faster in every configuration), so the update
// kernel takes it by default.  Both forms add the same values in the same
// order with the same workgroups, so they give bit-identical results and
// partials.
template <int NP, int EPW, typename T>
__device__ __forceinline__ void upd_body_nopc(T *__restrict__ r, const T *__restrict__ w, Scal *__restrict__ sc,
                                              const double *__restrict__ P1cur, int nb1, double *__restrict__ P2cur,
                                              int it, Box box, int E, int ngroups, unsigned blk, unsigned nblk,
                                              int xmin)
{
    if ((long)ngroups >= (long)xmin * nblk) {
        upd_body_x<NP, EPW, T>(r, w, sc, P1cur, nb1, P2cur, it, box, E, ngroups, blk, nblk);
        return;
    }
    upd_body<NP, EPW, T>(r, w, sc, P1cur, nb1, P2cur, it, box, E, ngroups, blk, nblk);
}

// wout = M o dssum(win) out of place, for whole columns: the copies of every
// node are gathered exactly as in upd_body (same columns, same fixed pairwise
// order), summed in FP64 and rounded once; Dirichlet nodes get 0.
template <int NP, int EPW, typename T>
__global__ __launch_bounds__(EPW *NP *NP) void k_assemble(const T *__restrict__ win, T *__restrict__ wout, Box box,
                                                          int E, int ngroups)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    const int tid = threadIdx.x;
    const int el = tid / NP2, ij = tid - el * NP2;
    const int i = ij % NP, j = ij / NP;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int g0 = (int)(((long)lb * ngroups) / gridDim.x);
    const int g1 = (int)(((long)(lb + 1) * ngroups) / gridDim.x);
    const int oz = box.nx * box.ny;
    for (int grp = g0; grp < g1; ++grp) {
        const int e = grp * EPW + el;
        if (e >= E) continue;
        const int ex = e % box.nx;
        const int eyz = e / box.nx;
        const int ey = eyz % box.ny, ez = eyz / box.ny;
        T *oe = wout + e * NP3;
        if ((i == 0 && ex == 0) || (i == N && ex == box.nx - 1) || (j == 0 && ey == 0) ||
            (j == N && ey == box.ny - 1)) {
#pragma unroll
            for (int k = 0; k < NP; ++k) oe[k * NP2 + ij] = (T)0;
            continue;
        }
        const bool hx = (i == 0 && ex > 0) || (i == N && ex < box.nx - 1);
        const bool hy = (j == 0 && ey > 0) || (j == N && ey < box.ny - 1);
        const bool xneg = i == 0, yneg = j == 0;
        const int ox = xneg ? -1 : 1, oy = yneg ? -box.nx : box.nx;
        const int colX = (xneg ? N : 0) + NP * j, colY = i + NP * (yneg ? N : 0);
        const int colXY = (xneg ? N : 0) + NP * (yneg ? N : 0);
        const bool hzm = ez > 0, hzp = ez < box.nz - 1;
        const T *we = win + e * NP3;
        T wo[NP], wx[NP], wy[NP], wxy[NP], zm[4], zp[4];
        load_copies<NP>(we, oz, hx, hy, hzm, hzp, ij, ox * NP3 + colX, oy * NP3 + colY, (ox + oy) * NP3 + colXY, wo, wx,
                        wy, wxy, zm, zp);
        auto plane = [](double o, double X, double Y, double XY) -> double { return (o + X) + (Y + XY); };
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            double S = plane((double)wo[k], (double)wx[k], (double)wy[k], (double)wxy[k]);
            if (k == 0 && hzm) S = plane((double)zm[0], (double)zm[1], (double)zm[2], (double)zm[3]) + S;
            if (k == N && hzp) S = S + plane((double)zp[0], (double)zp[1], (double)zp[2], (double)zp[3]);
            const bool dir = (k == 0 && ez == 0) || (k == N && ez == box.nz - 1);
            oe[k * NP2 + ij] = dir ? (T)0 : (T)S;
        }
    }
}

// k_assemble with the x-face copies of elements walked by one workgroup
// swapped through LDS (see upd_body_x): a capped grid of workgroups, each
// walking consecutive element groups.  The same values enter the same sums,
// so the output is bit-identical to k_assemble's.
template <int NP, int EPW, typename T>
__global__ __launch_bounds__(EPW *NP *NP) void k_assemble_x(const T *__restrict__ win, T *__restrict__ wout, Box box,
                                                            int E, int ngroups)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    constexpr int FS = 2 * NP + 5;
    __shared__ T xf[2][EPW][2][NP][FS];
    __shared__ T cf[3][NP][FS];
    const int tid = threadIdx.x;
    const int el = tid / NP2, ij = tid - el * NP2;
    const int i = ij % NP, j = ij / NP;
    const int side = i == 0 ? 0 : 1;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int g0 = (int)(((long)lb * ngroups) / gridDim.x);
    const int g1 = (int)(((long)(lb + 1) * ngroups) / gridDim.x);
    int buf = 0, c3 = 0, p3 = 2;
    for (int grp = g0; grp < g1; ++grp) {
        UpdCol<NP, T, false> c;
        const XRole xr = upd_load_x<NP, EPW, T>(c, win, grp, g0, g1, el, i, j, ij, box, E);
        if (c.valid && (xr.xin || xr.cout)) xf_publish<NP, T>(xr.xin ? xf[buf][el][side][j] : cf[c3][j], c);
        __syncthreads();
        if (xr.in_mesh) {
            T *oe = wout + c.e * NP3;
            if (!c.valid) {   // a column on the x or y Dirichlet faces
#pragma unroll
                for (int k = 0; k < NP; ++k) oe[k * NP2 + ij] = (T)0;
            } else {
                if (xr.xin || xr.cin)
                    xf_take<NP, T>(xr.xin ? xf[buf][el + (i == 0 ? -1 : 1)][side ^ 1][j] : cf[p3][j], c);
                auto plane = [](double o, double X, double Y, double XY) -> double { return (o + X) + (Y + XY); };
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    double S = plane((double)c.wo[k], (double)c.wx[k], (double)c.wy[k], (double)c.wxy[k]);
                    if (k == 0 && c.hzm) S = plane((double)c.zm[0], (double)c.zm[1], (double)c.zm[2], (double)c.zm[3]) + S;
                    if (k == N && c.hzp) S = S + plane((double)c.zp[0], (double)c.zp[1], (double)c.zp[2], (double)c.zp[3]);
                    const bool dir = (k == 0 && c.ez == 0) || (k == N && c.ez == box.nz - 1);
                    oe[k * NP2 + ij] = dir ? (T)0 : (T)S;
                }
            }
        }
        buf ^= 1;
        p3 = c3;
        c3 = c3 == 2 ? 0 : c3 + 1;
    }
}

// Occupancy target of the preconditioned update kernel (waves per SIMD).
// Its FP32 columns plus the diagonal take 134 VGPRs at NP = 10, one wave
// per SIMD fewer than the unpreconditioned kernel; the target brings it
// back at the cost of 4 spilled registers (25.1 instead of 26.7 us at 16^3
// N=9), and stays at what fits without heavy spilling for higher orders.
// FP64 (173 VGPRs at NP = 10) is left free: forcing 3 waves spilled 6
// registers and ran slower (47.1 against 43.2 us).
template <int NP, typename T> constexpr int pc_update_waves()
{
    return sizeof(T) == 4 ? (NP <= 10 ? 4 : NP <= 12 ? 3 : 2) : 1;
}

template <int NP, int EPW, typename T>
__global__ __launch_bounds__(EPW *NP *NP) __attribute__((amdgpu_waves_per_eu(pc_update_waves<NP, T>())))
void k_cg_update_pc(T *__restrict__ r, const T *__restrict__ w, Scal *__restrict__ sc, const double *__restrict__ P1cur,
                    int nb1, double *__restrict__ P2cur, int it, Box box, int E, int ngroups, const T *__restrict__ dg,
                    double *__restrict__ P4cur)
{
    upd_body<NP, EPW, T, true>(r, w, sc, P1cur, nb1, P2cur, it, box, E, ngroups, blockIdx.x, gridDim.x, dg, P4cur);
}

template <int NP, int EPW, typename T>
__global__ __launch_bounds__(EPW *NP *NP) void k_cg_update(T *__restrict__ r, const T *__restrict__ w,
                                                           Scal *__restrict__ sc, const double *__restrict__ P1cur,
                                                           int nb1, double *__restrict__ P2cur, int it, Box box,
                                                           int E, int ngroups, int xmin)
{
    upd_body_nopc<NP, EPW, T>(r, w, sc, P1cur, nb1, P2cur, it, box, E, ngroups, blockIdx.x, gridDim.x, xmin);
}

// ------------------------------------------------------------- batched CG

// One problem of a batch: its vectors (element type fixed by the launch), its
// factors, CG state and partials, and the size nblk of its share of the
// batched grid.  The launch's owner map gives each workgroup its problem and
// its block index within that share; block j sits at a grid index congruent
// to j mod 8, so it runs on the same XCD as block j of a solo launch, and
// the blocks j of problems that share one mesh sit next to each other, so
// their reads of the same factors meet in that XCD's L2.
struct BatchProb {
    void *r, *p, *w;       // residual, search direction, A_L p (T)
    const void *g;         // geometric factors (GT)
    void *x;               // FP64 iterate (FP64 solve) or inner correction (FP64, or FP32)
    Scal *sc;
    double *partials;      // pAp by parity, then rtr by parity (MAXB each)
    double *hist;
    Box box;
    int E, ngroups, nblk, active;
};

// Iteration number of a batched launch: the chunk base kept on the device
// (advanced by k_batch_advance at the start of every chunk) plus the launch's
// position in the chunk, so one recorded chunk serves every chunk of a run.
__device__ __forceinline__ int batch_it(const int *__restrict__ base, int it_local) { return *base + it_local; }

// The operator kernel of every problem of one order in one launch: workgroup
// b runs the solo body as block owner[b].y of problem owner[b].x (none if
// owner[b].x < 0).
template <int NP, int EPW, int PD, typename T, typename GT, typename XT>
__global__ __launch_bounds__(EPW *NP *NP) void k_ax_batch(const BatchProb *__restrict__ tab,
                                                          const int2 *__restrict__ owner, const T *__restrict__ D,
                                                          int it_local, const int *__restrict__ base)
{
    const int2 o = owner[blockIdx.x];
    if (o.x < 0) return;
    const BatchProb P = tab[o.x];
    if (!P.active) return;
    const int it = batch_it(base, it_local);
    ax_body<NP, EPW, PD, T, GT, true, XT>(
        (const T *)P.r, (T *)P.p, (T *)P.w, (const GT *)P.g, D, (XT *)P.x, P.sc, P.partials + (it & 1) * MAXB,
        P.partials + ((it - 1) & 1) * MAXB, P.partials + (2 + ((it - 1) & 1)) * MAXB, P.nblk, it, P.hist, P.E,
        P.ngroups, (unsigned)o.y, P.nblk);
}

template <int NP, int EPW, typename T>
__global__ __launch_bounds__(EPW *NP *NP) void k_cg_update_batch(const BatchProb *__restrict__ tab,
                                                                 const int2 *__restrict__ owner, int it_local,
                                                                 const int *__restrict__ base)
{
    const int2 o = owner[blockIdx.x];
    if (o.x < 0) return;
    const BatchProb P = tab[o.x];
    if (!P.active) return;
    const int it = batch_it(base, it_local);
    upd_body_nopc<NP, EPW, T>((T *)P.r, (const T *)P.w, P.sc, P.partials + (it & 1) * MAXB, P.nblk,
                              P.partials + (2 + (it & 1)) * MAXB, it, P.box, P.E, P.ngroups, (unsigned)o.y, P.nblk,
                              UPD_X_MIN_GROUPS);
}

// out = M o sum over copies of (c o) in: the right-hand side b = M dssum(f)
// and the initial-guess projection x = M dssum(c x0).
template <int NP, typename T, bool WEIGHT>
__global__ __launch_bounds__(UPD_BS) void k_gather(const T *__restrict__ in, T *__restrict__ out, Box box, unsigned nl)
{
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> P = locate<NP>(t, box);
        out[t] = P.masked ? (T)0 : (T)gather_copies<NP, T, WEIGHT>(in, P, box);
    }
}

// r = b - M dssum(w) (FP64); partials of glsc3(r, c, r).
template <int NP>
__global__ __launch_bounds__(UPD_BS) void k_resid(const double *__restrict__ b, const double *__restrict__ w,
                                                  double *__restrict__ r, double *__restrict__ P, Box box,
                                                  unsigned nl)
{
    __shared__ double sbuf[UPD_BS];
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> Pt = locate<NP>(t, box);
        double v = 0.0;
        if (!Pt.masked) v = b[t] - gather_copies<NP, double, false>(w, Pt, box);
        r[t] = v;
        part += (v * v) * inv_mult(Pt.mult);
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (threadIdx.x == 0) P[blockIdx.x] = s;
}

// Partials of sum_l a_l c_l b_l with c = 1/mult (glsc3).
template <int NP, typename TA, typename TB>
__global__ __launch_bounds__(UPD_BS) void k_glsc3(const TA *__restrict__ a, const TB *__restrict__ bv,
                                                  double *__restrict__ P, Box box, unsigned nl)
{
    __shared__ double sbuf[UPD_BS];
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> Pt = locate<NP>(t, box);
        part += ((double)a[t] * (double)bv[t]) * inv_mult(Pt.mult);
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (threadIdx.x == 0) P[blockIdx.x] = s;
}

// r32 = (float) r64, d = 0, and partials of glsc3(r32, c, r32): start of an
// inner (FP32-operator) solve of the refinement loop; the correction d is
// FP64 or FP32.
template <int NP, typename DT>
__global__ __launch_bounds__(UPD_BS) void k_inner_start(const double *__restrict__ r64, float *__restrict__ r32,
                                                        DT *__restrict__ d, double *__restrict__ P, Box box,
                                                        unsigned nl)
{
    __shared__ double sbuf[UPD_BS];
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> Pt = locate<NP>(t, box);
        const float v = (float)r64[t];
        r32[t] = v;
        d[t] = (DT)0;
        part += ((double)v * (double)v) * inv_mult(Pt.mult);
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (threadIdx.x == 0) P[blockIdx.x] = s;
}

// Element-interior fast-diagonalization preconditioner (solveM): z = M^-1 r
// with, on the (N-1)^3 interior nodes of every element, the inverse of the
// element's separable interior stiffness block,
//   2 (S (x) S (x) S) diag(1 / (cx l_i + cy l_j + cz l_k)) (S (x) S (x) S)^T,
// (S, l: the 1-D interior modes, S^T W_I S = I; cx, cy, cz: the element's
// factors), and z = r / m on the other nodes (m the assembled diagonal, 1 on
// Dirichlet nodes).  A workgroup of NP^2 threads walks a contiguous range of
// elements; thread (i, j) holds the k-column (i, j).  S^T is applied along k
// in registers, then along j and i through LDS; the way back runs along i
// and j through LDS and along k in registers.  Writes z and, per workgroup,
// the partial of glsc3(r, c, z) to P[blockIdx.x].  With sc set the kernel is
// a CG step of iteration it and does nothing once the run has ended.
template <int NP, typename T>
__global__ __launch_bounds__(NP *NP) void k_pc_fdm(const T *__restrict__ r, T *__restrict__ z,
                                                   const T *__restrict__ m, const T *__restrict__ S,
                                                   const T *__restrict__ lam, const T *__restrict__ cf,
                                                   double *__restrict__ P, Box box, int E,
                                                   const Scal *__restrict__ sc, int it)
{
    constexpr int N = NP - 1, NI = NP - 2, NP2 = NP * NP, NP3 = NP2 * NP, BS = NP2;
    constexpr int NIa = NI > 0 ? NI : 1, NI2 = NIa * NIa, NI3 = NI2 * NIa;
    __shared__ T sS[NI2];   // S[node * NI + mode]
    __shared__ T sl[NIa];
    __shared__ T bufA[NI3], bufB[NI3];
    __shared__ double sbuf[BS];
    if (sc && sc->st[it & 1].done) return;
    const int tid = threadIdx.x;
    for (int q = tid; q < NI * NI; q += BS) sS[q] = S[q];
    for (int q = tid; q < NI; q += BS) sl[q] = lam[q];
    const int i = tid % NP, j = tid / NP;
    const bool inner = NI > 0 && i >= 1 && i <= N - 1 && j >= 1 && j <= N - 1;
    const int ii = i - 1, jj = j - 1;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int e0 = (int)(((long)lb * E) / gridDim.x), e1 = (int)(((long)(lb + 1) * E) / gridDim.x);
    double part = 0.0;
    __syncthreads();
    for (int e = e0; e < e1; ++e) {
        const int ex = e % box.nx, eyz = e / box.nx;
        const int ey = eyz % box.ny, ez = eyz / box.ny;
        const T *re = r + (long)e * NP3;
        const T *me = m + (long)e * NP3;
        T rv[NP], zv[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) rv[k] = re[k * NP2 + tid];
        if (inner) {
            zv[0] = rv[0] / me[tid];
            zv[N] = rv[N] / me[N * NP2 + tid];
        } else {
#pragma unroll
            for (int k = 0; k < NP; ++k) zv[k] = rv[k] / me[k * NP2 + tid];
        }
        T t[NIa];
        if (inner) {   // S^T along k (registers)
#pragma unroll
            for (int a = 0; a < NI; ++a) {
                T acc = 0;
#pragma unroll
                for (int kk = 0; kk < NI; ++kk) acc += sS[kk * NI + a] * rv[kk + 1];
                bufA[a * NI2 + jj * NI + ii] = acc;
            }
        }
        __syncthreads();
        if (inner) {   // S^T along j: thread (ii, b = jj)
#pragma unroll
            for (int a = 0; a < NI; ++a) {
                T acc = 0;
#pragma unroll
                for (int jp = 0; jp < NI; ++jp) acc += sS[jp * NI + jj] * bufA[a * NI2 + jp * NI + ii];
                t[a] = acc;
            }
#pragma unroll
            for (int a = 0; a < NI; ++a) bufB[a * NI2 + jj * NI + ii] = t[a];
        }
        __syncthreads();
        if (inner) {   // S^T along i: thread (c = ii, b = jj); scale the modes
            const T cx = cf[3 * e], cy = cf[3 * e + 1], cz = cf[3 * e + 2];
            const T lxy = cx * sl[ii] + cy * sl[jj];
#pragma unroll
            for (int a = 0; a < NI; ++a) {
                T acc = 0;
#pragma unroll
                for (int ip = 0; ip < NI; ++ip) acc += sS[ip * NI + ii] * bufB[a * NI2 + jj * NI + ip];
                t[a] = (T)2 * acc / (lxy + cz * sl[a]);
            }
#pragma unroll
            for (int a = 0; a < NI; ++a) bufA[a * NI2 + jj * NI + ii] = t[a];
        }
        __syncthreads();
        if (inner) {   // S along i: thread (i = ii, b = jj)
#pragma unroll
            for (int a = 0; a < NI; ++a) {
                T acc = 0;
#pragma unroll
                for (int c = 0; c < NI; ++c) acc += sS[ii * NI + c] * bufA[a * NI2 + jj * NI + c];
                t[a] = acc;
            }
#pragma unroll
            for (int a = 0; a < NI; ++a) bufB[a * NI2 + jj * NI + ii] = t[a];
        }
        __syncthreads();
        if (inner) {   // S along j, then along k (registers)
#pragma unroll
            for (int a = 0; a < NI; ++a) {
                T acc = 0;
#pragma unroll
                for (int b = 0; b < NI; ++b) acc += sS[jj * NI + b] * bufB[a * NI2 + b * NI + ii];
                t[a] = acc;
            }
#pragma unroll
            for (int kk = 0; kk < NI; ++kk) {
                T acc = 0;
#pragma unroll
                for (int a = 0; a < NI; ++a) acc += sS[kk * NI + a] * t[a];
                zv[kk + 1] = acc;
            }
        }
        // next element: its first LDS writes (bufA) follow every thread's last
        // reads of bufA above; its bufB writes follow its first barrier
        T *ze = z + (long)e * NP3;
        const int mx = ((i == 0 && ex > 0) || (i == N && ex < box.nx - 1)) ? 2 : 1;
        const int my = ((j == 0 && ey > 0) || (j == N && ey < box.ny - 1)) ? 2 : 1;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            ze[k * NP2 + tid] = zv[k];
            const int mz = ((k == 0 && ez > 0) || (k == N && ez < box.nz - 1)) ? 2 : 1;
            part += ((double)rv[k] * (double)zv[k]) * inv_mult(mx * my * mz);
        }
    }
    const double sum = block_sum<BS>(part, sbuf);
    if (tid == 0) P[blockIdx.x] = sum;
}

// ------------------------------------- two-level overlapping Schwarz (solveM)
//
// M^-1 r = sum_e R_e^T A~_e^-1 R_e r + P A~_c^-1 P^T r  (see nek.h,
// NEK_PC_SCHWARZ).  The window of element e along x is the global lattice
// line gi = ex N - 1 .. ex N + N + 1 (NW = N + 3 nodes, window index
// a = gi - ex N + 1); nodes on or past the Dirichlet boundary carry no
// unknown (zero rows of the padded modes S, zero values).

// A row of RP (a multiple of 16 / sizeof(T)) entries from 16-byte aligned LDS.
template <int RP, typename T> __device__ __forceinline__ void lds_row(const T *__restrict__ src, T out[RP])
{
    constexpr int V = 16 / sizeof(T);
    static_assert(RP % V == 0, "row pitch a multiple of the 16-byte vector");
#pragma unroll
    for (int q = 0; q < RP / V; ++q) {
        const uint4 v = reinterpret_cast<const uint4 *>(src)[q];
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int t = 0; t < V; ++t) {
            if constexpr (sizeof(T) == 4) out[V * q + t] = __builtin_bit_cast(T, w[t]);
            else out[V * q + t] = __builtin_bit_cast(T, (unsigned long long)w[2 * t] | ((unsigned long long)w[2 * t + 1] << 32));
        }
    }
}

// Window node a of element coordinate ed (of nd) along one direction: the
// element and local index holding a copy of it, or false when the node is
// not an unknown (a Dirichlet node or past the boundary).
template <int NP>
__device__ __forceinline__ bool win_node(int a, int ed, int nd, int &eo, int &io)
{
    constexpr int N = NP - 1;
    const int g = ed * N - 1 + a, G = nd * N + 1;
    if (g <= 0 || g >= G - 1) return false;
    eo = a == 0 ? ed - 1 : a == N + 2 ? ed + 1 : ed;
    io = a == 0 ? N - 1 : a == N + 2 ? 1 : a - 1;
    return true;
}

// The NW mode rows of one direction (pitch SP) read in order with two in
// flight: row a + 1 is requested before row a is used, so an LDS read's
// latency overlaps the previous row's products (one row at a time exposed it
// NW times per pass; all rows at once took 210 VGPRs instead of 76).
template <int NW, int SP, typename T, typename F>
__device__ __forceinline__ void rows_pipelined(const T *__restrict__ base, F body)
{
    T cur[SP], nxt[SP];
    lds_row<SP>(base, cur);
#pragma unroll
    for (int a = 0; a < NW; ++a) {
        __builtin_amdgcn_sched_barrier(0);
        if (a + 1 < NW) lds_row<SP>(base + (a + 1) * SP, nxt);
        body(a, cur);
#pragma unroll
        for (int q = 0; q < SP; ++q) cur[q] = nxt[q];
    }
}

// Local solves: a workgroup of NW^2 threads walks a contiguous range of
// elements (persistent grid).  The window of r
// is staged in LDS (rows of pitch NW + 1); six passes apply S^T along x, y, z,
// the scaling 2 / (cx l_a + cy l_b + cz l_c), and S back along z, y, x, each
// pass one line per thread held in registers (the z passes share a thread's
// column).  Writes the window solution u[e][c][b][a] and the element's eight
// coarse moments mom[e][v] = sum over its nodes of c_l l_v(x) r_l, v = vx +
// 2 vy + 4 vz (c_l = 1 / multiplicity, separable; l_0 = (1-x)/2, l_1 =
// (1+x)/2).  With sc set, a CG step of iteration it (nothing after the run
// has ended).
template <int NP, typename T>
__global__ __launch_bounds__((NP + 2) * (NP + 2)) void k_asm_local(
    const T *__restrict__ r, T *__restrict__ u, double *__restrict__ mom, const T *__restrict__ Sw,
    const T *__restrict__ lamw, const T *__restrict__ cf, const double *__restrict__ ell, Box box, int E,
    const Scal *__restrict__ sc, int it)
{
    constexpr int N = NP - 1, NW = NP + 2, PW = NW + 1, NW2 = NW * NW, NP2 = NP * NP, NP3 = NP2 * NP;
    constexpr int VS = 16 / sizeof(T), SP = (NW + VS - 1) / VS * VS;   // mode rows padded to 16 bytes
    __shared__ T buf[NW * NW * PW];
    __shared__ __align__(16) T sS[3][NW][SP];
    __shared__ T sl[3][NW];
    __shared__ double mx[2][NP2];
    __shared__ double my[4][NP];
    if (sc && sc->st[it & 1].done) return;
    const int tid = threadIdx.x;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int eb = (int)(((long)lb * E) / gridDim.x), ee = (int)(((long)(lb + 1) * E) / gridDim.x);
    for (int q = eb; q < ee; ++q) {   // column-major: z fastest (the previous window overlaps this one)
    __syncthreads();   // the previous element's LDS reads are done
    const int ez = q % box.nz, col = q / box.nz, ex = col % box.nx, ey = col / box.nx;
    const int e = ex + box.nx * (ey + box.ny * ez);
    // the modes of each direction's clipping variant, as 16-byte aligned rows
    // in LDS (a thread's pass reads one row per output or input entry)
    const int vx = (ex == 0 ? 1 : 0) + (ex == box.nx - 1 ? 2 : 0);
    const int vy = (ey == 0 ? 1 : 0) + (ey == box.ny - 1 ? 2 : 0);
    const int vz = (ez == 0 ? 1 : 0) + (ez == box.nz - 1 ? 2 : 0);
    {
        const int a = tid % NW, m = tid / NW;   // NW^2 threads: one entry per direction each
        sS[0][a][m] = Sw[vx * NW2 + a * NW + m];
        sS[1][a][m] = Sw[vy * NW2 + a * NW + m];
        sS[2][a][m] = Sw[vz * NW2 + a * NW + m];
        if (m < SP - NW) {   // padding of the rows
            sS[0][a][NW + m] = sS[1][a][NW + m] = sS[2][a][NW + m] = (T)0;
        }
    }
    if (tid < NW) {
        sl[0][tid] = lamw[vx * NW + tid];
        sl[1][tid] = lamw[vy * NW + tid];
        sl[2][tid] = lamw[vz * NW + tid];
    }
    // the window of r: thread (a, b) loads its column along z, every load
    // issued without a branch (a node that is not an unknown reads a valid
    // address, the element's own node 0, and its value is replaced by 0)
    {
        const int a = tid % NW, b = tid / NW;
        int e0 = ex, i0 = 0, e1 = ey, i1 = 0;
        const bool hx = win_node<NP>(a, ex, box.nx, e0, i0), hy = win_node<NP>(b, ey, box.ny, e1, i1);
        if (!hx) { e0 = ex; i0 = 0; }
        if (!hy) { e1 = ey; i1 = 0; }
        const long col = (long)(e0 + box.nx * e1) * NP3 + i0 + NP * i1;
        const long zst = (long)box.nx * box.ny * NP3;
        T v[NW];
        bool ok[NW];
#pragma unroll
        for (int c = 0; c < NW; ++c) {
            int e2 = ez, i2 = 0;
            ok[c] = hx && hy && win_node<NP>(c, ez, box.nz, e2, i2);
            if (!ok[c]) { e2 = ez; i2 = 0; }
            v[c] = r[col + zst * e2 + NP2 * i2];
        }
#pragma unroll
        for (int c = 0; c < NW; ++c) buf[a + PW * (b + NW * c)] = ok[c] ? v[c] : (T)0;
    }
    __syncthreads();
    // coarse moments: along x per (j, k) line of the element's own nodes, then y, then z
    auto cw = [&](int i, int edd, int ndd, int side) -> double {
        const double l = ell[side * NP + i];
        const bool shared = (i == 0 && edd > 0) || (i == N && edd < ndd - 1);
        return shared ? 0.5 * l : l;
    };
    if (tid < NP2) {
        const int j = tid % NP, k = tid / NP;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const double v = (double)buf[(i + 1) + PW * ((j + 1) + NW * (k + 1))];
            s0 += cw(i, ex, box.nx, 0) * v;
            s1 += cw(i, ex, box.nx, 1) * v;
        }
        mx[0][k * NP + j] = s0;
        mx[1][k * NP + j] = s1;
    }
    __syncthreads();
    if (tid < 2 * NP) {
        const int xa = tid & 1, k = tid >> 1;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            s0 += cw(j, ey, box.ny, 0) * mx[xa][k * NP + j];
            s1 += cw(j, ey, box.ny, 1) * mx[xa][k * NP + j];
        }
        my[xa][k] = s0;
        my[2 + xa][k] = s1;
    }
    __syncthreads();
    if (tid < 8) {
        const int xa = tid & 1, yb = (tid >> 1) & 1, zc = tid >> 2;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) s += cw(k, ez, box.nz, zc) * my[2 * yb + xa][k];
        mom[(long)e * 8 + tid] = s;
    }
    // fast diagonalization; thread t takes line (t % NW, t / NW) of each pass
    const int p0 = tid % NW, p1 = tid / NW;
    T in[NW], out[NW];
    // S^T along x: line (b, c) = (p0, p1)
#pragma unroll
    for (int a = 0; a < NW; ++a) in[a] = buf[a + PW * (p0 + NW * p1)];
#pragma unroll
    for (int m = 0; m < NW; ++m) out[m] = 0;
    rows_pipelined<NW, SP, T>(&sS[0][0][0], [&](int a, const T *row) {
#pragma unroll
        for (int m = 0; m < NW; ++m) out[m] += row[m] * in[a];
    });
#pragma unroll
    for (int m = 0; m < NW; ++m) buf[m + PW * (p0 + NW * p1)] = out[m];
    __syncthreads();
    // S^T along y: line (a, c) = (p0, p1)
#pragma unroll
    for (int b = 0; b < NW; ++b) in[b] = buf[p0 + PW * (b + NW * p1)];
#pragma unroll
    for (int m = 0; m < NW; ++m) out[m] = 0;
    rows_pipelined<NW, SP, T>(&sS[1][0][0], [&](int b, const T *row) {
#pragma unroll
        for (int m = 0; m < NW; ++m) out[m] += row[m] * in[b];
    });
#pragma unroll
    for (int m = 0; m < NW; ++m) buf[p0 + PW * (m + NW * p1)] = out[m];
    __syncthreads();
    // along z: line (a, b) = (p0, p1) = modes (ma, mb); S^T, scale, S
    {
        const T cx = cf[3 * e], cy = cf[3 * e + 1], cz = cf[3 * e + 2];
        const T lxy = cx * sl[0][p0] + cy * sl[1][p1];
#pragma unroll
        for (int c = 0; c < NW; ++c) in[c] = buf[p0 + PW * (p1 + NW * c)];
#pragma unroll
        for (int m = 0; m < NW; ++m) out[m] = 0;
        rows_pipelined<NW, SP, T>(&sS[2][0][0], [&](int c, const T *row) {
#pragma unroll
            for (int m = 0; m < NW; ++m) out[m] += row[m] * in[c];
        });
#pragma unroll
        for (int m = 0; m < NW; ++m) out[m] = (T)2 * out[m] / (lxy + cz * sl[2][m]);
        rows_pipelined<NW, SP, T>(&sS[2][0][0], [&](int c, const T *row) {
            T acc = 0;
#pragma unroll
            for (int m = 0; m < NW; ++m) acc += row[m] * out[m];
            in[c] = acc;
        });
#pragma unroll
        for (int c = 0; c < NW; ++c) buf[p0 + PW * (p1 + NW * c)] = in[c];
    }
    __syncthreads();
    // S along y: line (a, c)
#pragma unroll
    for (int m = 0; m < NW; ++m) in[m] = buf[p0 + PW * (m + NW * p1)];
    rows_pipelined<NW, SP, T>(&sS[1][0][0], [&](int b, const T *row) {
        T acc = 0;
#pragma unroll
        for (int m = 0; m < NW; ++m) acc += row[m] * in[m];
        out[b] = acc;
    });
#pragma unroll
    for (int b = 0; b < NW; ++b) buf[p0 + PW * (b + NW * p1)] = out[b];
    __syncthreads();
    // S along x: line (b, c); to memory
#pragma unroll
    for (int m = 0; m < NW; ++m) in[m] = buf[m + PW * (p0 + NW * p1)];
    T *ue = u + (long)e * NW2 * NW + NW * (p0 + NW * p1);
    rows_pipelined<NW, SP, T>(&sS[0][0][0], [&](int a, const T *row) {
        T acc = 0;
#pragma unroll
        for (int m = 0; m < NW; ++m) acc += row[m] * in[m];
        ue[a] = acc;
    });
    }
}

// ---- the same local solves on the matrix cores
//
// Each pass of the fast diagonalization is a product of the NW^2 lines of the
// window (one of the three directions running along the line) with an NW x NW
// matrix of 1-D modes: (NW^2 x NW) x (NW x NW).  v_mfma_*_16x16x4 multiplies a
// 16 x 4 block of lines by a 4 x 16 block of modes into a 16 x 16 block held
// by one wave; lane l supplies line l mod 16 at contracted index l / 16 and
// mode (l mod 16) at the same contracted index, and receives four outputs of
// column l mod 16 (rows 4 (l / 16) + q for FP32, l / 16 + 4 q for FP64: the
// two instructions order their outputs differently).  Lines and modes past NW
// are zero-padded; the modes stay in LDS and each lane reads its few operands
// once per pass, so the per-thread row reads of the VALU form disappear.
template <typename T> struct Mfma16;
template <> struct Mfma16<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V mma(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};
template <> struct Mfma16<double> {
    typedef double V __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V mma(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};

// One pass: out(L, m) = sum_k A(L, k) B(k, m) over the NW^2 lines L and the
// NW outputs m; wave w of NWV takes the line tiles w, w + NWV, ...  a_at(L, k)
// and b_at(k, m) read the operands, put(L, m, v) stores a result.
template <int NW, int NWV, typename T, typename FA, typename FB, typename FO>
__device__ __forceinline__ void mfma_pass(int wave, int lane, FA a_at, FB b_at, FO put)
{
    using M = Mfma16<T>;
    constexpr int NL = NW * NW, MT = (NL + 15) / 16, NT = (NW + 15) / 16, KT = (NW + 3) / 4;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        T bop[KT];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const int k = 4 * kt + lk, m = 16 * nt + lr;
            bop[kt] = (k < NW && m < NW) ? b_at(k, m) : (T)0;
        }
        for (int mt = wave; mt < MT; mt += NWV) {
            typename M::V acc = {0, 0, 0, 0};
            const int L = 16 * mt + lr;
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                const int k = 4 * kt + lk;
                const T a = (L < NL && k < NW) ? a_at(L, k) : (T)0;
                acc = M::mma(a, bop[kt], acc);
            }
            const int m = 16 * nt + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int Lo = 16 * mt + M::row(lane, q);
                if (Lo < NL && m < NW) put(Lo, m, acc[q]);
            }
        }
    }
}

// The local solves of k_asm_local (same window, moments, outputs and order of
// the fast-diagonalization steps) with every pass on the matrix cores: a
// workgroup of 4 waves walks a contiguous range of elements; the passes
// ping-pong between two LDS copies of the window.
template <int NP, typename T>
__global__ __launch_bounds__(256) void k_asm_local_mfma(
    const T *__restrict__ r, T *__restrict__ u, double *__restrict__ mom, const T *__restrict__ Sw,
    const T *__restrict__ lamw, const T *__restrict__ cf, const double *__restrict__ ell, Box box, int E,
    const Scal *__restrict__ sc, int it)
{
    constexpr int N = NP - 1, NW = NP + 2, PW = NW + 1, NW2 = NW * NW, NP2 = NP * NP, NP3 = NP2 * NP;
    constexpr int BS = 256, NWV = BS / 64;
    __shared__ T b0[NW * NW * PW], b1[NW * NW * PW];
    __shared__ T sS[3][NW][NW];
    __shared__ T sl[3][NW];
    __shared__ double mx[2][NP2];
    __shared__ double my[4][NP];
    if (sc && sc->st[it & 1].done) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int eb = (int)(((long)lb * E) / gridDim.x), ee = (int)(((long)(lb + 1) * E) / gridDim.x);
    auto ix = [](int a, int b, int c) { return a + PW * (b + NW * c); };
    for (int q = eb; q < ee; ++q) {   // column-major: z fastest (the previous window overlaps this one)
        __syncthreads();   // the previous element's LDS reads are done
        const int ez = q % box.nz, col = q / box.nz, ex = col % box.nx, ey = col / box.nx;
        const int e = ex + box.nx * (ey + box.ny * ez);
        const int vx = (ex == 0 ? 1 : 0) + (ex == box.nx - 1 ? 2 : 0);
        const int vy = (ey == 0 ? 1 : 0) + (ey == box.ny - 1 ? 2 : 0);
        const int vz = (ez == 0 ? 1 : 0) + (ez == box.nz - 1 ? 2 : 0);
        for (int q = tid; q < NW2; q += BS) {
            const int a = q / NW, m = q % NW;
            sS[0][a][m] = Sw[vx * NW2 + q];
            sS[1][a][m] = Sw[vy * NW2 + q];
            sS[2][a][m] = Sw[vz * NW2 + q];
        }
        if (tid < NW) {
            sl[0][tid] = lamw[vx * NW + tid];
            sl[1][tid] = lamw[vy * NW + tid];
            sl[2][tid] = lamw[vz * NW + tid];
        }
        // the window of r by columns along z, every load issued without a
        // branch (a node that is not an unknown reads the element's own node
        // 0 and its value is replaced by 0)
        for (int col = tid; col < NW2; col += BS) {
            const int a = col % NW, b = col / NW;
            int e0 = ex, i0 = 0, e1 = ey, i1 = 0;
            const bool hx = win_node<NP>(a, ex, box.nx, e0, i0), hy = win_node<NP>(b, ey, box.ny, e1, i1);
            if (!hx) { e0 = ex; i0 = 0; }
            if (!hy) { e1 = ey; i1 = 0; }
            const long cb = (long)(e0 + box.nx * e1) * NP3 + i0 + NP * i1;
            const long zst = (long)box.nx * box.ny * NP3;
            T v[NW];
            bool ok[NW];
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                int e2 = ez, i2 = 0;
                ok[c] = hx && hy && win_node<NP>(c, ez, box.nz, e2, i2);
                if (!ok[c]) { e2 = ez; i2 = 0; }
                v[c] = r[cb + zst * e2 + NP2 * i2];
            }
#pragma unroll
            for (int c = 0; c < NW; ++c) b0[ix(a, b, c)] = ok[c] ? v[c] : (T)0;
        }
        __syncthreads();
        // coarse moments, as in k_asm_local
        auto cw = [&](int i, int edd, int ndd, int side) -> double {
            const double l = ell[side * NP + i];
            const bool shared = (i == 0 && edd > 0) || (i == N && edd < ndd - 1);
            return shared ? 0.5 * l : l;
        };
        if (tid < NP2) {
            const int j = tid % NP, k = tid / NP;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const double v = (double)b0[ix(i + 1, j + 1, k + 1)];
                s0 += cw(i, ex, box.nx, 0) * v;
                s1 += cw(i, ex, box.nx, 1) * v;
            }
            mx[0][k * NP + j] = s0;
            mx[1][k * NP + j] = s1;
        }
        __syncthreads();
        if (tid < 2 * NP) {
            const int xa = tid & 1, k = tid >> 1;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                s0 += cw(j, ey, box.ny, 0) * mx[xa][k * NP + j];
                s1 += cw(j, ey, box.ny, 1) * mx[xa][k * NP + j];
            }
            my[xa][k] = s0;
            my[2 + xa][k] = s1;
        }
        __syncthreads();
        if (tid < 8) {
            const int xa = tid & 1, yb = (tid >> 1) & 1, zc = tid >> 2;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < NP; ++k) s += cw(k, ez, box.nz, zc) * my[2 * yb + xa][k];
            mom[(long)e * 8 + tid] = s;
        }
        // S^T along x: lines (b, c)
        mfma_pass<NW, NWV, T>(
            wave, lane, [&](int L, int k) { return b0[ix(k, L % NW, L / NW)]; },
            [&](int k, int m) { return sS[0][k][m]; },
            [&](int L, int m, T v) { b1[ix(m, L % NW, L / NW)] = v; });
        __syncthreads();
        // S^T along y: lines (a, c)
        mfma_pass<NW, NWV, T>(
            wave, lane, [&](int L, int k) { return b1[ix(L % NW, k, L / NW)]; },
            [&](int k, int m) { return sS[1][k][m]; },
            [&](int L, int m, T v) { b0[ix(L % NW, m, L / NW)] = v; });
        __syncthreads();
        // S^T along z: lines (a, b) of modes; scaled by 2 / (cx l_a + cy l_b + cz l_c)
        {
            const T cx = cf[3 * e], cy = cf[3 * e + 1], cz = cf[3 * e + 2];
            mfma_pass<NW, NWV, T>(
                wave, lane, [&](int L, int k) { return b0[ix(L % NW, L / NW, k)]; },
                [&](int k, int m) { return sS[2][k][m]; },
                [&](int L, int m, T v) {
                    const int a = L % NW, b = L / NW;
                    b1[ix(a, b, m)] = (T)2 * v / (cx * sl[0][a] + cy * sl[1][b] + cz * sl[2][m]);
                });
        }
        __syncthreads();
        // S along z
        mfma_pass<NW, NWV, T>(
            wave, lane, [&](int L, int k) { return b1[ix(L % NW, L / NW, k)]; },
            [&](int k, int m) { return sS[2][m][k]; },
            [&](int L, int m, T v) { b0[ix(L % NW, L / NW, m)] = v; });
        __syncthreads();
        // S along y
        mfma_pass<NW, NWV, T>(
            wave, lane, [&](int L, int k) { return b0[ix(L % NW, k, L / NW)]; },
            [&](int k, int m) { return sS[1][m][k]; },
            [&](int L, int m, T v) { b1[ix(L % NW, m, L / NW)] = v; });
        __syncthreads();
        // S along x, to the window solution u[e][c][b][a]
        T *ue = u + (long)e * NW2 * NW;
        mfma_pass<NW, NWV, T>(
            wave, lane, [&](int L, int k) { return b1[ix(k, L % NW, L / NW)]; },
            [&](int k, int m) { return sS[0][m][k]; },
            [&](int L, int m, T v) { ue[m + NW * L] = v; });
    }
}

// The plain local operator w = A_L u (local_grad3, the six factors,
// local_grad3_t; Fig. 2) with its six D contractions on the matrix cores:
// each is the product of the NP^2 lines of the element along one direction
// with D or D^T (mfma_pass with NW = NP); the factors are applied per point
// on the vector ALUs between the two halves.  A workgroup of 4 waves walks a
// contiguous range of elements.  The measured alternative to ax_body's
// vector-ALU contractions (nek_set_operator_kernel); NP <= 12 (four LDS
// copies of the element).
template <int NP, typename T, typename GT>
__global__ __launch_bounds__(256) void k_ax_mfma(const T *__restrict__ u, T *__restrict__ w,
                                                 const GT *__restrict__ g, const T *__restrict__ D, int E)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, PWn = NP + 1, NWV = 4, SZ = NP * NP * PWn;
    using GL = GLoad<GT>;
    __shared__ T su[SZ], sr[SZ], ss[SZ], st[SZ];
    __shared__ T sD[NP * NP];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int q = tid; q < NP * NP; q += 256) sD[q] = D[q];
    auto ix = [](int i, int j, int k) { return i + PWn * (j + NP * k); };
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int eb = (int)(((long)lb * E) / gridDim.x), ee = (int)(((long)(lb + 1) * E) / gridDim.x);
    for (int e = eb; e < ee; ++e) {
        __syncthreads();   // the previous element's LDS reads are done (and sD written)
        for (int p = tid; p < NP3; p += 256) su[ix(p % NP, (p / NP) % NP, p / NP2)] = u[(long)e * NP3 + p];
        __syncthreads();
        // ur = D u along r, us along s, ut along t
        mfma_pass<NP, NWV, T>(
            wave, lane, [&](int L, int l) { return su[ix(l, L % NP, L / NP)]; },
            [&](int l, int m) { return sD[m * NP + l]; }, [&](int L, int m, T v) { sr[ix(m, L % NP, L / NP)] = v; });
        mfma_pass<NP, NWV, T>(
            wave, lane, [&](int L, int l) { return su[ix(L % NP, l, L / NP)]; },
            [&](int l, int m) { return sD[m * NP + l]; }, [&](int L, int m, T v) { ss[ix(L % NP, m, L / NP)] = v; });
        mfma_pass<NP, NWV, T>(
            wave, lane, [&](int L, int l) { return su[ix(L % NP, L / NP, l)]; },
            [&](int l, int m) { return sD[m * NP + l]; }, [&](int L, int m, T v) { st[ix(L % NP, L / NP, m)] = v; });
        __syncthreads();
        for (int p = tid; p < NP3; p += 256) {
            const int a = ix(p % NP, (p / NP) % NP, p / NP2);
            T gk[6];
            GL::unpack(GL::load(g + ((long)e * NP3 + p) * 6), gk);
            const T ur = sr[a], us = ss[a], ut = st[a];
            sr[a] = gk[0] * ur + gk[3] * us + gk[4] * ut;
            ss[a] = gk[3] * ur + gk[1] * us + gk[5] * ut;
            st[a] = gk[4] * ur + gk[5] * us + gk[2] * ut;
        }
        __syncthreads();
        // w = D^T wr + D^T ws + D^T wt, accumulated in su
        mfma_pass<NP, NWV, T>(
            wave, lane, [&](int L, int l) { return sr[ix(l, L % NP, L / NP)]; },
            [&](int l, int m) { return sD[l * NP + m]; }, [&](int L, int m, T v) { su[ix(m, L % NP, L / NP)] = v; });
        __syncthreads();
        mfma_pass<NP, NWV, T>(
            wave, lane, [&](int L, int l) { return ss[ix(L % NP, l, L / NP)]; },
            [&](int l, int m) { return sD[l * NP + m]; }, [&](int L, int m, T v) { su[ix(L % NP, m, L / NP)] += v; });
        __syncthreads();
        mfma_pass<NP, NWV, T>(
            wave, lane, [&](int L, int l) { return st[ix(L % NP, L / NP, l)]; },
            [&](int l, int m) { return sD[l * NP + m]; },
            [&](int L, int m, T v) {
                const int i = L % NP, j = L / NP;
                w[(long)e * NP3 + i + NP * (j + NP * m)] = su[ix(i, j, m)] + v;
            });
    }
}

// Subdomains of one direction holding global lattice node ed N + i: the
// element coordinates (ascending) and the node's window index in each.
template <int NP>
__device__ __forceinline__ int win_cands(int i, int ed, int nd, int eo[3], int ao[3])
{
    constexpr int N = NP - 1;
    int n = 0;
    if (i <= 1 && ed > 0) { eo[n] = ed - 1; ao[n++] = i + N + 1; }
    eo[n] = ed; ao[n++] = i + 1;
    if (i >= N - 1 && ed < nd - 1) { eo[n] = ed + 1; ao[n++] = i - N + 1; }
    return n;
}

// z = sum over the subdomains holding each node of their window solutions
// (ascending element order: every copy of a node forms the identical sum)
// + the trilinear interpolation of the coarse correction ec (vertex lattice,
// 0 on the boundary; weights by reference coordinate, so copies agree bit
// for bit), 0 on Dirichlet nodes; partials of glsc3(r, c, z) to P.  A
// workgroup of NP^2 threads walks a contiguous range of elements in
// column-major order (z fastest), thread (i, j) its k-column: the x and y
// subdomains and the coarse weights along x and y are the column's, only the
// z part changes along it, and the window below, read for the lowest layers,
// is the one the workgroup read for the previous element.  With sc set, a CG
// step of iteration it.
template <int NP, typename T>
__global__ __launch_bounds__(NP *NP) void k_asm_gather(const T *__restrict__ r, T *__restrict__ z,
                                                       const T *__restrict__ u, const double *__restrict__ ec,
                                                       const double *__restrict__ ell, double *__restrict__ P,
                                                       Box box, int E, const Scal *__restrict__ sc, int it)
{
    constexpr int N = NP - 1, NW = NP + 2, NW3 = NW * NW * NW, NP2 = NP * NP, NP3 = NP2 * NP, BS = NP2;
    __shared__ double sbuf[BS];
    if (sc && sc->st[it & 1].done) return;
    const int tid = threadIdx.x, i = tid % NP, j = tid / NP;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int e0 = (int)(((long)lb * E) / gridDim.x), e1 = (int)(((long)(lb + 1) * E) / gridDim.x);
    const long vx = box.nx + 1, vy = box.ny + 1;
    const double lx0 = ell[i], lx1 = ell[NP + i], ly0 = ell[j], ly1 = ell[NP + j];
    double part = 0.0;
    for (int q = e0; q < e1; ++q) {
        const int ez = q % box.nz, col = q / box.nz, ex = col % box.nx, ey = col / box.nx;
        const int e = ex + box.nx * (ey + box.ny * ez);
        const bool dir_xy = (i == 0 && ex == 0) || (i == N && ex == box.nx - 1) || (j == 0 && ey == 0) ||
                            (j == N && ey == box.ny - 1);
        int exo[3] = {ex, ex, ex}, axo[3] = {1, 1, 1}, eyo[3] = {ey, ey, ey}, ayo[3] = {1, 1, 1};
        const int nx = win_cands<NP>(i, ex, box.nx, exo, axo);
        const int ny = win_cands<NP>(j, ey, box.ny, eyo, ayo);
        // coarse correction of the column: along x, then y, per z-layer of vertices
        double tz[2];
#pragma unroll
        for (int dz = 0; dz < 2; ++dz) {
            double ty[2];
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const double *row = ec + ex + vx * ((ey + dy) + vy * (ez + dz));
                ty[dy] = lx0 * row[0] + lx1 * row[1];
            }
            tz[dz] = ly0 * ty[0] + ly1 * ty[1];
        }
        const T *re = r + (long)e * NP3 + tid;
        T *ze = z + (long)e * NP3 + tid;
        // every load of the column first: r, then for each (y, x) subdomain
        // pair its column in the own z-layer and the two end nodes that the
        // layers below and above contribute (pairs and layers that do not
        // exist read the element's own window and are not added)
        constexpr int CX = NP >= 4 ? 2 : 3;   // subdomains per direction holding a node
        const bool zlo = ez > 0, zhi = ez < box.nz - 1;
        const long zs = (long)box.nx * box.ny;
        T rv[NP], own[CX * CX][NP], zl[CX * CX][2], zh[CX * CX][2];
#pragma unroll
        for (int k = 0; k < NP; ++k) rv[k] = re[k * NP2];
#pragma unroll
        for (int qy = 0; qy < CX; ++qy)
#pragma unroll
            for (int qx = 0; qx < CX; ++qx) {
                const bool ok = qy < ny && qx < nx;
                const long eo = ok ? exo[qx] + (long)box.nx * (eyo[qy] + (long)box.ny * ez) : (long)e;
                const T *uo = u + eo * NW3 + (ok ? axo[qx] + NW * ayo[qy] : 1 + NW);
                const T *ul = zlo && ok ? uo - zs * NW3 : uo;
                const T *uh = zhi && ok ? uo + zs * NW3 : uo;
#pragma unroll
                for (int k = 0; k < NP; ++k) own[qy * CX + qx][k] = uo[NW * NW * (k + 1)];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    zl[qy * CX + qx][q] = ul[NW * NW * (q + N + 1)];
                    zh[qy * CX + qx][q] = uh[NW * NW * q];
                }
            }
        const int mx = ((i == 0 && ex > 0) || (i == N && ex < box.nx - 1)) ? 2 : 1;
        const int my = ((j == 0 && ey > 0) || (j == N && ey < box.ny - 1)) ? 2 : 1;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            double zv = 0.0;
            const bool dir = dir_xy || (k == 0 && ez == 0) || (k == N && ez == box.nz - 1);
            if (!dir) {
                // ascending element order: the layer below, the own layer, the layer above
                double sm = 0.0;
                if (k <= 1 && zlo) {
#pragma unroll
                    for (int qy = 0; qy < CX; ++qy)
#pragma unroll
                        for (int qx = 0; qx < CX; ++qx)
                            if (qy < ny && qx < nx) sm += (double)zl[qy * CX + qx][k];
                }
#pragma unroll
                for (int qy = 0; qy < CX; ++qy)
#pragma unroll
                    for (int qx = 0; qx < CX; ++qx)
                        if (qy < ny && qx < nx) sm += (double)own[qy * CX + qx][k];
                if (k >= N - 1 && zhi) {
#pragma unroll
                    for (int qy = 0; qy < CX; ++qy)
#pragma unroll
                        for (int qx = 0; qx < CX; ++qx)
                            if (qy < ny && qx < nx) sm += (double)zh[qy * CX + qx][k - (N - 1)];
                }
                zv = sm + (ell[k] * tz[0] + ell[NP + k] * tz[1]);
            }
            const T zt = (T)zv;
            ze[k * NP2] = zt;
            const int mz = ((k == 0 && ez > 0) || (k == N && ez < box.nz - 1)) ? 2 : 1;
            part += ((double)rv[k] * (double)zt) * inv_mult(mx * my * mz);
        }
    }
    const double sum = block_sum<BS>(part, sbuf);
    if (tid == 0) P[blockIdx.x] = sum;
}

// Start of a preconditioned run: r -> z = r / m in place (m the diagonal,
// 1 on Dirichlet nodes), each quotient formed in FP64 and rounded once, and
// partials of glsc3(r, c, z).
template <int NP, typename T>
__global__ __launch_bounds__(UPD_BS) void k_pc_start(T *__restrict__ r, const T *__restrict__ dg,
                                                     double *__restrict__ P, Box box, unsigned nl)
{
    __shared__ double sbuf[UPD_BS];
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> Pt = locate<NP>(t, box);
        const double rv = (double)r[t];
        const T z = (T)(rv / (double)dg[t]);
        r[t] = z;
        part += (rv * (double)z) * inv_mult(Pt.mult);
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (threadIdx.x == 0) P[blockIdx.x] = s;
}

}  // namespace nek
