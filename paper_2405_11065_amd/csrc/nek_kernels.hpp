// Device kernels of libnek (gfx950).  Internal header, included once by
// nek_lib.hip.
//
// Hot path of one CG iteration (the loop of the paper's Table 1, no
// preconditioner): two launches per iteration.
//   k_ax<CG>(it)    beta from the previous iteration's rtr, p = beta p + r
//                   (add2s1), w_L = A_L p (ax_e: local_grad3, g1..g6,
//                   local_grad3_t), and per-workgroup partials of p.w_L.
//   k_cg_update(it) alpha = rtz / pap, then for every local point:
//                   S = sum of the copies of w_L at its global node (dssum),
//                   mask, x += alpha p, r -= alpha S, and per-workgroup
//                   partials of glsc3(r, c, r).
// Because p is continuous and zero on the Dirichlet boundary,
// glsc3(M dssum(A_L p), c, p) = sum_l p_l (A_L p)_l in exact arithmetic, so
// pap needs no gather and alpha is known right after the operator.
//
// Reductions without atomics or fences: a kernel writes one FP64 partial
// per workgroup with a plain store; every workgroup of the NEXT kernel sums
// all of them in the same fixed order (so all obtain the identical value),
// the kernel boundary making the stores visible.  Device-scope fences would
// write back and invalidate a whole XCD's L2 per workgroup on gfx950.  The
// CG state is double-buffered by iteration parity; only workgroup 0 writes
// the slot of the current iteration.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nek {

constexpr int UPD_BS = 256;      // block size of the pointwise kernels

// CG state entering iteration it, in slot it & 1.
struct IterState {
    double rtz;      // glsc3(r, c, r) of the current residual
    double beta;
    int iter;        // iterations completed
    int done;
    int status;      // 0, -5 (breakdown) or -6 (non-finite)
    int conv;        // stopped by the tolerance (or r == 0)
};

struct Scal {
    IterState st[2];
    IterState fin;        // final state, written by k_cg_finish
    double hist_den;      // history entry = sqrt(rtz / hist_den)
    double stop_den;      // stop when sqrt(rtz) / sqrt(stop_den) <= stop_tol
    double stop_tol;      // <= 0: run to maxit
    double red[4];        // results of standalone reductions
    int maxit;
    int hist_off;         // history index of iteration 0 of this run
    int k2flag[2];        // status of k_cg_update(it) in slot it & 1
    int done_host;        // set once a run is done; polled by the host
};

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

// Sum of P[0..n) in a fixed order, returned to every thread of the block.
template <int BS>
__device__ __forceinline__ double sum_all(const double *__restrict__ P, int n, double *sbuf)
{
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += BS) v += P[q];
    double s = block_sum<BS>(v, sbuf);
    if (threadIdx.x == 0) sbuf[0] = s;
    __syncthreads();
    s = sbuf[0];
    __syncthreads();
    return s;
}

// Start of iteration it: fold the previous update kernel's rtr partials into
// the state (identically in every workgroup) and decide whether to stop.
// Workgroup 0, thread 0 publishes the state (and, when done, the host flag).
template <int BS>
__device__ __forceinline__ IterState cg_begin(Scal *__restrict__ sc, const double *__restrict__ P2, int nb2,
                                              int it, double *__restrict__ hist, double *sbuf, bool writer)
{
    const IterState prev = sc->st[(it - 1) & 1];
    IterState cur = prev;
    if (!prev.done) {
        if (it == 1) {
            cur.beta = 0.0;
            cur.iter = 0;
        } else {
            const int f = sc->k2flag[(it - 1) & 1];
            if (f) {
                cur.status = f;
                cur.done = 1;
            } else {
                const double rtr = sum_all<BS>(P2, nb2, sbuf);
                cur.iter = it - 1;
                cur.rtz = rtr;
                cur.beta = rtr / prev.rtz;
                if (writer && hist) hist[sc->hist_off + it - 1] = sqrt(rtr / sc->hist_den);
                if (!__builtin_isfinite(rtr)) {
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
        if (cur.done) sc->done_host = 1;
    }
    return cur;
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

// ---------------------------------------------------------------- operator

// One workgroup = EPW elements x (NP x NP) threads; thread (i, j) walks the
// k-column of its element.  u is staged in LDS for the r and s derivatives;
// the t derivative uses the thread's own column in registers.  wr, ws go
// through LDS for the transposed derivatives, wt stays in registers.  The
// uniform entries D[k][l] of the t contractions come through the scalar
// cache.  The six factors of slice k + PD are in flight while slice k is
// computed.  CG mode fuses p = beta p + r before, and sum p.(A_L p) after.
template <int NP, int EPW, int PD, typename T, typename GT, bool CG>
__global__ __launch_bounds__(EPW *NP *NP) void k_ax(const T *__restrict__ src, T *__restrict__ p,
                                                    T *__restrict__ w, const GT *__restrict__ g,
                                                    const T *__restrict__ D, Scal *__restrict__ sc,
                                                    double *__restrict__ P1, const double *__restrict__ P2,
                                                    int nb2, int it, double *__restrict__ hist, int E,
                                                    int ngroups)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, BS = EPW * NP2;
    using GL = GLoad<GT>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *su = reinterpret_cast<T *>(smem_raw);
    T *sr = su + EPW * NP3;
    T *ss = sr + EPW * NP3;
    __shared__ double sbuf[BS];
    __shared__ T sD[NP * NP];

    const int tid = threadIdx.x;
    T beta = 0;
    bool first = false;
    if constexpr (CG) {
        const IterState cur = cg_begin<BS>(sc, P2, nb2, it, hist, sbuf, blockIdx.x == 0 && tid == 0);
        if (cur.done) return;
        beta = (T)cur.beta;
        first = it == 1;
    }
    const int el = tid / NP2, ij = tid - el * NP2;
    const int i = ij % NP, j = ij / NP;
    T *sue = su + el * NP3, *sre = sr + el * NP3, *sse = ss + el * NP3;

    // FP32: the thread's rows/columns of D live in registers.  FP64 reads
    // them from LDS instead (no register spills; FP64 has bandwidth slack).
    constexpr bool DREG = sizeof(T) == 4;
    T Dri[DREG ? NP : 1], Dsj[DREG ? NP : 1], DTi[DREG ? NP : 1], DTj[DREG ? NP : 1];
    if constexpr (DREG) {
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
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int g0 = (int)(((long)lb * ngroups) / gridDim.x);
    const int g1 = (int)(((long)(lb + 1) * ngroups) / gridDim.x);
    double pap = 0.0;

    for (int grp = g0; grp < g1; ++grp) {
        const long e = (long)grp * EPW + el;
        const bool valid = e < E;
        // threads past the last element compute on a copy of element E-1 and
        // store nothing
        const long ec = valid ? e : (long)E - 1;
        const long base = ec * NP3 + ij;
        const GT *ge = g + (size_t)base * 6;
        typename GL::Raw gb[PD];
#pragma unroll
        for (int s = 0; s < PD; ++s)
            if (s < NP) gb[s] = GL::load(ge + (size_t)s * NP2 * 6);
        T u[NP];
        __syncthreads();   // LDS of the previous group is free
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const long idx = base + k * NP2;
            T v;
            if constexpr (CG) {
                const T rv = src[idx];
                v = first ? rv : beta * p[idx] + rv;
                if (valid) p[idx] = v;
            } else {
                v = src[idx];
            }
            u[k] = v;
            sue[k * NP2 + ij] = v;
        }
        __syncthreads();
        T wt[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            __builtin_amdgcn_sched_barrier(0);
            T gk[6];
            GL::unpack(gb[k % PD], gk);
            T ur = 0, us = 0, ut = 0;
#pragma unroll
            for (int l = 0; l < NP; ++l) {
                ur += NEK_DR(l) * sue[k * NP2 + j * NP + l];
                us += NEK_DS(l) * sue[k * NP2 + l * NP + i];
                ut += D[k * NP + l] * u[l];
            }
            sre[k * NP2 + ij] = gk[0] * ur + gk[3] * us + gk[4] * ut;
            sse[k * NP2 + ij] = gk[3] * ur + gk[1] * us + gk[5] * ut;
            wt[k] = gk[4] * ur + gk[5] * us + gk[2] * ut;
            __builtin_amdgcn_sched_barrier(0);
            if (k + PD < NP) gb[k % PD] = GL::load(ge + (size_t)(k + PD) * NP2 * 6);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            T acc = 0;
#pragma unroll
            for (int l = 0; l < NP; ++l) acc += NEK_DTI(l) * sre[k * NP2 + j * NP + l];
#pragma unroll
            for (int l = 0; l < NP; ++l) acc += NEK_DTJ(l) * sse[k * NP2 + l * NP + i];
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
        if (tid == 0) P1[blockIdx.x] = s;
    }
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
    const double c = WEIGHT ? 1.0 / (double)(nx * ny * nz) : 1.0;
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

template <typename T, typename XT> struct UpdArgs {
    XT *x;             // solution (FP64 CG) or correction (mixed inner)
    const T *p;
    T *r;
    const T *w;        // A_L p, unassembled
    Scal *sc;
    const double *P1;  // pAp partials of k_ax(it)
    double *P2;        // rtr partials written here
    int nb1;
    int it;
    Box box;
    unsigned nl;
};

template <int NP, typename T, typename XT>
__global__ __launch_bounds__(UPD_BS) void k_cg_update(UpdArgs<T, XT> a)
{
    __shared__ double sbuf[UPD_BS];
    const IterState cur = a.sc->st[a.it & 1];
    if (cur.done) return;
    const double pap = sum_all<UPD_BS>(a.P1, a.nb1, sbuf);
    const bool writer = blockIdx.x == 0 && threadIdx.x == 0;
    if (!__builtin_isfinite(pap) || !(pap > 0)) {
        if (writer) a.sc->k2flag[a.it & 1] = __builtin_isfinite(pap) ? -5 : -6;
        return;
    }
    const double alpha = cur.rtz / pap;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * a.nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * a.nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> P = locate<NP>(t, a.box);
        if (P.masked) continue;   // r, x, p are zero there and stay zero
        const double S = gather_copies<NP, T, false>(a.w, P, a.box);
        a.x[t] = (XT)((double)a.x[t] + alpha * (double)a.p[t]);
        const T rn = (T)((double)a.r[t] - alpha * S);
        a.r[t] = rn;
        part += ((double)rn * (double)rn) / (double)P.mult;
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (threadIdx.x == 0) a.P2[blockIdx.x] = s;
    if (writer) a.sc->k2flag[a.it & 1] = 0;
}

// End of a CG run: fold the last update's partials and publish the final
// state (one workgroup).
__global__ __launch_bounds__(UPD_BS) void k_cg_finish(Scal *__restrict__ sc, const double *__restrict__ P2, int nb2,
                                                      int it, double *__restrict__ hist)
{
    __shared__ double sbuf[UPD_BS];
    const IterState cur = cg_begin<UPD_BS>(sc, P2, nb2, it, hist, sbuf, threadIdx.x == 0);
    if (threadIdx.x == 0) sc->fin = cur;
}

// Start of a CG run: rtz = red[rslot]; stop and history denominators; the
// initial residual test.
__global__ void k_cg_start(Scal *sc, double *hist, int rslot, int hist_off, double stop_tol, int maxit,
                           int stop_on_initial)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double bb = sc->red[0];
    const double rtz = sc->red[rslot];
    IterState s{};
    s.rtz = rtz;
    s.beta = 0.0;
    s.iter = 0;
    sc->hist_den = bb;
    sc->stop_den = stop_on_initial ? rtz : bb;
    sc->stop_tol = stop_tol;
    sc->maxit = maxit;
    sc->hist_off = hist_off;
    sc->k2flag[0] = sc->k2flag[1] = 0;
    if (hist) hist[hist_off] = bb > 0 ? sqrt(rtz / bb) : 0.0;
    if (!__builtin_isfinite(bb) || !__builtin_isfinite(rtz)) {
        s.status = -6;
        s.done = 1;
    } else if (bb == 0.0 || rtz == 0.0 ||
               (!stop_on_initial && stop_tol > 0 && sqrt(rtz) / sqrt(sc->stop_den) <= stop_tol)) {
        s.conv = 1;
        s.done = 1;
    } else if (maxit <= 0) {
        s.done = 1;
    }
    sc->st[0] = s;
    sc->st[1] = s;
    sc->fin = s;
    sc->done_host = s.done;
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

// Standalone reductions write one partial per workgroup; k_red_final sums
// them in a fixed order into red[slot].
__global__ __launch_bounds__(UPD_BS) void k_red_final(const double *__restrict__ P, int n, Scal *sc, int slot)
{
    __shared__ double sbuf[UPD_BS];
    const double s = sum_all<UPD_BS>(P, n, sbuf);
    if (threadIdx.x == 0) sc->red[slot] = s;
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
        part += (v * v) / (double)Pt.mult;
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
        part += ((double)a[t] * (double)bv[t]) / (double)Pt.mult;
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (threadIdx.x == 0) P[blockIdx.x] = s;
}

// r32 = (float) r64, d = 0, and partials of glsc3(r32, c, r32): start of an
// inner (FP32-operator) solve of the refinement loop.
template <int NP>
__global__ __launch_bounds__(UPD_BS) void k_inner_start(const double *__restrict__ r64, float *__restrict__ r32,
                                                        double *__restrict__ d, double *__restrict__ P, Box box,
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
        d[t] = 0.0;
        part += ((double)v * (double)v) / (double)Pt.mult;
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (threadIdx.x == 0) P[blockIdx.x] = s;
}

// Standalone sorted-segment dssum: one thread per segment, copies summed in
// ascending local index (perm order) from 0.0, written back to every copy.
template <typename T>
__global__ __launch_bounds__(UPD_BS) void k_dssum_seg(T *__restrict__ w, const int32_t *__restrict__ perm,
                                                      const int32_t *__restrict__ seg_ptr,
                                                      const int8_t *__restrict__ flag, unsigned nseg, int apply_mask)
{
    const unsigned s = blockIdx.x * UPD_BS + threadIdx.x;
    if (s >= nseg) return;
    const int b = seg_ptr[s], e = seg_ptr[s + 1];
    if (apply_mask && flag[s]) {
        for (int q = b; q < e; ++q) w[perm[q]] = (T)0;
        return;
    }
    double acc = 0.0;
    for (int q = b; q < e; ++q) acc += (double)w[perm[q]];
    const T v = (T)acc;
    for (int q = b; q < e; ++q) w[perm[q]] = v;
}

// Rounding of the FP64 geometric factors to the storage precision.
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double x)
{
    // Round-to-nearest-even directly from binary64 (no double rounding via
    // binary32).  Values below the binary32 normal range flush to signed 0.
    const unsigned long long u = __double_as_longlong(x);
    const unsigned sign = (unsigned)(u >> 63);
    const int ex = (int)((u >> 52) & 0x7ff);
    const unsigned long long man = u & 0xfffffffffffffULL;
    if (ex == 0x7ff) return (uint16_t)((sign << 15) | 0x7f80u | (man ? 0x40u : 0u));
    const int eb = ex - 1023 + 127;
    if (ex == 0 || eb <= 0) return (uint16_t)(sign << 15);
    if (eb >= 0xff) return (uint16_t)((sign << 15) | 0x7f80u);
    unsigned bits = (sign << 15) | ((unsigned)eb << 7) | (unsigned)(man >> 45);
    const unsigned long long rest = man & ((1ULL << 45) - 1);
    const unsigned long long half = 1ULL << 44;
    if (rest > half || (rest == half && (bits & 1u))) bits += 1u;   // carries into the exponent correctly
    return (uint16_t)bits;
}

__global__ void k_g_to_f32(const double *__restrict__ g, float *__restrict__ o, unsigned long n)
{
    for (unsigned long t = blockIdx.x * (unsigned long)blockDim.x + threadIdx.x; t < n; t += (unsigned long)gridDim.x * blockDim.x)
        o[t] = (float)g[t];
}

__global__ void k_g_to_bf16(const double *__restrict__ g, uint16_t *__restrict__ o, unsigned long n)
{
    for (unsigned long t = blockIdx.x * (unsigned long)blockDim.x + threadIdx.x; t < n; t += (unsigned long)gridDim.x * blockDim.x)
        o[t] = f64_to_bf16_rne(g[t]);
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, T v, unsigned long n)
{
    for (unsigned long t = blockIdx.x * (unsigned long)blockDim.x + threadIdx.x; t < n; t += (unsigned long)gridDim.x * blockDim.x)
        p[t] = v;
}

// x += d (FP64).
__global__ void k_axpy1(double *__restrict__ x, const double *__restrict__ d, unsigned long n)
{
    for (unsigned long t = blockIdx.x * (unsigned long)blockDim.x + threadIdx.x; t < n; t += (unsigned long)gridDim.x * blockDim.x)
        x[t] += d[t];
}

}  // namespace nek
