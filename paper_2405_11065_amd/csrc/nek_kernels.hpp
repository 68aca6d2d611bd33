// Device kernels of libnek (gfx950).  Internal header, included once by
// nek_lib.hip.
//
// Hot path of one CG iteration (the loop of the paper's Table 1, no
// preconditioner), two launches:
//   k_cg_ax     p = beta p + r (add2s1), w_L = A_L p (ax_e: local_grad3,
//               g1..g6, local_grad3_t), and p.w_L summed over all local
//               points; its last workgroup forms alpha = rtz / pap.
//   k_cg_update for every local point: S = sum of the copies of w_L at the
//               point's global node (dssum), mask, x += alpha p,
//               r -= alpha S, rtr = glsc3(r, c, r); its last workgroup forms
//               beta, the residual history and the stopping decision.
// Because p is continuous and zero on the Dirichlet boundary,
// glsc3(M dssum(A_L p), c, p) = sum_l p_l (A_L p)_l exactly in real
// arithmetic, so pap needs no gather and alpha is known right after ax.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nek {

constexpr int UPD_BS = 256;     // block size of the pointwise kernels

// Device-resident CG state.  All scalars of the solve live here so an
// iteration never waits for the host.
struct Scal {
    double rtz;        // glsc3(r, c, r) of the current residual
    double rtz_prev;
    double alpha, beta, pap;
    double hist_den;   // history entry = sqrt(rtz / hist_den)
    double stop_den;   // stop when sqrt(rtz) / sqrt(stop_den) <= stop_tol
    double stop_tol;   // <= 0: run to maxit
    double red[4];     // results of standalone reductions
    int iter;          // iterations completed in this CG run
    int maxit;
    int hist_off;      // history index of iteration 0 of this run
    int done;
    int status;        // 0, NEK_E_BREAKDOWN or NEK_E_NONFINITE
    int conv;          // 1 when stopped by the tolerance (or r == 0)
    unsigned ctr[4];   // arrival counters of the last-workgroup reductions
};

struct Box { int nx, ny, nz; };

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so neighbouring elements share an L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned X = 8, x = b % X, slot = b / X, q = nb / X, r = nb % X;
    return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

template <typename GT> __device__ __forceinline__ float g_to_f32(GT v);
template <> __device__ __forceinline__ float g_to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float g_to_f32<uint16_t>(uint16_t v)
{
    return __uint_as_float(((unsigned)v) << 16);
}
template <typename T, typename GT> __device__ __forceinline__ T load_g(const GT *p)
{
    return (T)g_to_f32<GT>(*p);
}
template <> __device__ __forceinline__ double load_g<double, double>(const double *p) { return *p; }

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

// Publish this workgroup's partial and report whether it arrived last.
__device__ __forceinline__ bool arrive_last(unsigned *ctr, double *partials, double v, int *s_flag)
{
    if (threadIdx.x == 0) {
        __hip_atomic_store(&partials[blockIdx.x], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned prev = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = prev == gridDim.x - 1;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Sum of all partials in a fixed order, by the last workgroup (thread 0).
template <int BS>
__device__ __forceinline__ double sum_partials(const double *partials, double *sbuf)
{
    __threadfence();
    double v = 0.0;
    for (unsigned q = threadIdx.x; q < gridDim.x; q += BS)
        v += __hip_atomic_load(&partials[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum<BS>(v, sbuf);
}

// ---------------------------------------------------------------- operator

// One workgroup = EPW elements x (NP x NP) threads; thread (i, j) walks the
// k-column of its element.  u is staged in LDS for the r and s derivatives;
// the t derivative uses the thread's own column in registers.  wr, ws go
// through LDS for the transposed derivatives, wt stays in registers.  The
// uniform entries D[k][l] of the t contractions come through the scalar
// cache.  CG mode fuses p = beta p + r before, and sum p.(A_L p) after.
template <int NP, int EPW, typename T, typename GT, bool CG>
__global__ __launch_bounds__(EPW *NP *NP) void k_ax(const T *__restrict__ src, T *__restrict__ p,
                                                    T *__restrict__ w, const GT *__restrict__ g,
                                                    const T *__restrict__ D, Scal *__restrict__ sc,
                                                    double *__restrict__ partials, int E, int ngroups)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, BS = EPW * NP2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *su = reinterpret_cast<T *>(smem_raw);
    T *sr = su + EPW * NP3;
    T *ss = sr + EPW * NP3;
    __shared__ double sbuf[BS];
    __shared__ int s_flag;

    if (CG && sc->done) return;
    const int tid = threadIdx.x;
    const int el = tid / NP2, ij = tid - el * NP2;
    const int i = ij % NP, j = ij / NP;
    T *sue = su + el * NP3, *sre = sr + el * NP3, *sse = ss + el * NP3;

    // FP32: the thread's rows/columns of D live in registers.  FP64 has the
    // bandwidth slack to read them from LDS instead (no register spills).
    constexpr bool DREG = sizeof(T) == 4;
    __shared__ T sD[NP * NP];
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
    T beta = 0;
    bool first = false;
    if (CG) {
        beta = (T)sc->beta;
        first = sc->iter == 0;
    }
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int g0 = (int)(((long)lb * ngroups) / gridDim.x);
    const int g1 = (int)(((long)(lb + 1) * ngroups) / gridDim.x);
    double pap = 0.0;

    for (int grp = g0; grp < g1; ++grp) {
        const long e = (long)grp * EPW + el;
        const bool valid = e < E;
        // threads past the last element compute on a copy of element E-1 and
        // store nothing
        const long base = (valid ? e : (long)E - 1) * NP3 + ij;
        T u[NP];
        __syncthreads();   // LDS of the previous group is free
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const long idx = base + k * NP2;
            T v;
            if (CG) {
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
        const GT *ge = g + (base - ij) * 6 + ij;
        // software pipeline over k: the six factors of slice k+1 are in
        // flight while slice k is computed (bounded register use)
        T gc[6], gn[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) gc[q] = load_g<T, GT>(ge + q * NP3);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (k + 1 < NP) {
#pragma unroll
                for (int q = 0; q < 6; ++q) gn[q] = load_g<T, GT>(ge + q * NP3 + (k + 1) * NP2);
            }
            __builtin_amdgcn_sched_barrier(0);
            T ur = 0, us = 0, ut = 0;
#pragma unroll
            for (int l = 0; l < NP; ++l) {
                ur += NEK_DR(l) * sue[k * NP2 + j * NP + l];
                us += NEK_DS(l) * sue[k * NP2 + l * NP + i];
                ut += D[k * NP + l] * u[l];
            }
            sre[k * NP2 + ij] = gc[0] * ur + gc[3] * us + gc[4] * ut;
            sse[k * NP2 + ij] = gc[3] * ur + gc[1] * us + gc[5] * ut;
            wt[k] = gc[4] * ur + gc[5] * us + gc[2] * ut;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 6; ++q) gc[q] = gn[q];
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

    if (CG) {
        double s = block_sum<BS>(pap, sbuf);
        if (arrive_last(&sc->ctr[0], partials, s, &s_flag)) {
            double tot = sum_partials<BS>(partials, sbuf);
            if (tid == 0) {
                sc->pap = tot;
                if (!__builtin_isfinite(tot)) {
                    sc->status = -6;
                    sc->done = 1;
                } else if (!(tot > 0)) {
                    sc->status = -5;
                    sc->done = 1;
                } else {
                    sc->alpha = sc->rtz / tot;
                }
                __hip_atomic_store(&sc->ctr[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
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
// c = 1/mult first.
template <int NP, typename T, bool WEIGHT>
__device__ __forceinline__ double gather_copies(const T *__restrict__ w, const PointInfo<NP> &P, Box b)
{
    constexpr int NP2 = NP * NP, NP3 = NP2 * NP, N = NP - 1;
    int dxo[2], ixo[2], nxo = 0, dyo[2], jyo[2], nyo = 0, dzo[2], kzo[2], nzo = 0;
    if (P.i == 0 && P.ex > 0) { dxo[0] = -1; ixo[0] = N; dxo[1] = 0; ixo[1] = 0; nxo = 2; }
    else if (P.i == N && P.ex < b.nx - 1) { dxo[0] = 0; ixo[0] = N; dxo[1] = 1; ixo[1] = 0; nxo = 2; }
    else { dxo[0] = 0; ixo[0] = P.i; nxo = 1; }
    if (P.j == 0 && P.ey > 0) { dyo[0] = -1; jyo[0] = N; dyo[1] = 0; jyo[1] = 0; nyo = 2; }
    else if (P.j == N && P.ey < b.ny - 1) { dyo[0] = 0; jyo[0] = N; dyo[1] = 1; jyo[1] = 0; nyo = 2; }
    else { dyo[0] = 0; jyo[0] = P.j; nyo = 1; }
    if (P.k == 0 && P.ez > 0) { dzo[0] = -1; kzo[0] = N; dzo[1] = 0; kzo[1] = 0; nzo = 2; }
    else if (P.k == N && P.ez < b.nz - 1) { dzo[0] = 0; kzo[0] = N; dzo[1] = 1; kzo[1] = 0; nzo = 2; }
    else { dzo[0] = 0; kzo[0] = P.k; nzo = 1; }
    const double c = WEIGHT ? 1.0 / (double)(nxo * nyo * nzo) : 1.0;
    double s = 0.0;
    for (int cz = 0; cz < nzo; ++cz)
        for (int cy = 0; cy < nyo; ++cy)
            for (int cx = 0; cx < nxo; ++cx) {
                const long ee = P.e + dxo[cx] + (long)b.nx * (dyo[cy] + (long)b.ny * dzo[cz]);
                const double v = (double)w[ee * NP3 + ixo[cx] + NP * jyo[cy] + NP2 * kzo[cz]];
                s += WEIGHT ? c * v : v;
            }
    return s;
}

template <typename T, typename XT> struct UpdArgs {
    XT *x;             // solution (FP64 CG) or correction (mixed inner)
    const T *p;
    T *r;
    const T *w;        // A_L p, unassembled
    Scal *sc;
    double *partials;
    double *hist;
    Box box;
    unsigned nl;
};

template <int NP, typename T, typename XT>
__global__ __launch_bounds__(UPD_BS) void k_cg_update(UpdArgs<T, XT> a)
{
    __shared__ double sbuf[UPD_BS];
    __shared__ int s_flag;
    if (a.sc->done) return;
    const double alpha = a.sc->alpha;
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
    if (arrive_last(&a.sc->ctr[1], a.partials, s, &s_flag)) {
        const double rtr = sum_partials<UPD_BS>(a.partials, sbuf);
        if (threadIdx.x == 0) {
            Scal *sc = a.sc;
            const int it = sc->iter + 1;
            sc->iter = it;
            if (a.hist) a.hist[sc->hist_off + it] = sqrt(rtr / sc->hist_den);
            sc->rtz_prev = sc->rtz;
            sc->rtz = rtr;
            sc->beta = rtr / sc->rtz_prev;
            if (!__builtin_isfinite(rtr)) {
                sc->status = -6;
                sc->done = 1;
            } else if (rtr == 0.0 || (sc->stop_tol > 0 && sqrt(rtr) / sqrt(sc->stop_den) <= sc->stop_tol)) {
                sc->conv = 1;
                sc->done = 1;
            } else if (it >= sc->maxit) {
                sc->done = 1;
            }
            __hip_atomic_store(&sc->ctr[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
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

// r = b - M dssum(w) (FP64) and red[slot] = glsc3(r, c, r).
template <int NP>
__global__ __launch_bounds__(UPD_BS) void k_resid(const double *__restrict__ b, const double *__restrict__ w,
                                                  double *__restrict__ r, Scal *sc, double *partials, int slot,
                                                  Box box, unsigned nl)
{
    __shared__ double sbuf[UPD_BS];
    __shared__ int s_flag;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> P = locate<NP>(t, box);
        double v = 0.0;
        if (!P.masked) v = b[t] - gather_copies<NP, double, false>(w, P, box);
        r[t] = v;
        part += (v * v) / (double)P.mult;
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (arrive_last(&sc->ctr[2], partials, s, &s_flag)) {
        const double tot = sum_partials<UPD_BS>(partials, sbuf);
        if (threadIdx.x == 0) {
            sc->red[slot] = tot;
            __hip_atomic_store(&sc->ctr[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// red[slot] = sum_l a_l c_l b_l with c = 1/mult (glsc3).
template <int NP, typename TA, typename TB>
__global__ __launch_bounds__(UPD_BS) void k_glsc3(const TA *__restrict__ a, const TB *__restrict__ bv, Scal *sc,
                                                  double *partials, int slot, Box box, unsigned nl)
{
    __shared__ double sbuf[UPD_BS];
    __shared__ int s_flag;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> P = locate<NP>(t, box);
        part += ((double)a[t] * (double)bv[t]) / (double)P.mult;
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (arrive_last(&sc->ctr[2], partials, s, &s_flag)) {
        const double tot = sum_partials<UPD_BS>(partials, sbuf);
        if (threadIdx.x == 0) {
            sc->red[slot] = tot;
            __hip_atomic_store(&sc->ctr[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Start of a CG run: rtz = red[rslot]; stop and history denominators; the
// initial residual test.
__global__ void k_cg_start(Scal *sc, double *hist, int rslot, int hist_off, double stop_tol, int maxit,
                           int stop_on_initial)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double bb = sc->red[0];
    const double rtz = sc->red[rslot];
    sc->rtz = rtz;
    sc->rtz_prev = 1.0;
    sc->alpha = sc->beta = sc->pap = 0.0;
    sc->hist_den = bb;
    sc->stop_den = stop_on_initial ? rtz : bb;
    sc->stop_tol = stop_tol;
    sc->iter = 0;
    sc->maxit = maxit;
    sc->hist_off = hist_off;
    sc->status = 0;
    sc->conv = 0;
    sc->done = 0;
    if (hist) hist[hist_off] = bb > 0 ? sqrt(rtz / bb) : 0.0;
    if (!__builtin_isfinite(bb) || !__builtin_isfinite(rtz)) {
        sc->status = -6;
        sc->done = 1;
    } else if (bb == 0.0 || rtz == 0.0 ||
               (stop_tol > 0 && sqrt(rtz) / sqrt(sc->stop_den) <= stop_tol && !stop_on_initial)) {
        sc->conv = 1;
        sc->done = 1;
    } else if (maxit <= 0) {
        sc->done = 1;
    }
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

// r32 = (float) r64, d = 0 and red[slot] = glsc3(r32, c, r32): start of an
// inner (FP32-operator) solve of the refinement loop.
template <int NP>
__global__ __launch_bounds__(UPD_BS) void k_inner_start(const double *__restrict__ r64, float *__restrict__ r32,
                                                        double *__restrict__ d, Scal *sc, double *partials, int slot,
                                                        Box box, unsigned nl)
{
    __shared__ double sbuf[UPD_BS];
    __shared__ int s_flag;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned t0 = (unsigned)(((unsigned long)lb * nl) / gridDim.x);
    const unsigned t1 = (unsigned)(((unsigned long)(lb + 1) * nl) / gridDim.x);
    double part = 0.0;
    for (unsigned t = t0 + threadIdx.x; t < t1; t += UPD_BS) {
        const PointInfo<NP> P = locate<NP>(t, box);
        const float v = (float)r64[t];
        r32[t] = v;
        d[t] = 0.0;
        part += ((double)v * (double)v) / (double)P.mult;
    }
    const double s = block_sum<UPD_BS>(part, sbuf);
    if (arrive_last(&sc->ctr[2], partials, s, &s_flag)) {
        const double tot = sum_partials<UPD_BS>(partials, sbuf);
        if (threadIdx.x == 0) {
            sc->red[slot] = tot;
            __hip_atomic_store(&sc->ctr[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// x += d (FP64).
__global__ void k_axpy1(double *__restrict__ x, const double *__restrict__ d, unsigned long n)
{
    for (unsigned long t = blockIdx.x * (unsigned long)blockDim.x + threadIdx.x; t < n; t += (unsigned long)gridDim.x * blockDim.x)
        x[t] += d[t];
}

}  // namespace nek
