// Order-independent device kernels of libnek (gfx950): CG start, reduction
// finish, sorted-segment dssum, precision conversion of g, fills.  Internal
// header, included only by nek_lib.hip.
#pragma once
#include "nek_bf16.hpp"
#include "nek_kernels.hpp"

namespace nek {

// Start of a CG run: rtz = red[rslot] (glsc3(r, c, z); for an
// unpreconditioned run z = r), rtr = red[rtr_slot] (glsc3(r, c, r)); stop
// and history denominators; the initial residual test on rtr.
// A resumed run (rtz_prev > 0) keeps the search direction: its first
// p = z + beta p with beta = rtz / rtz_prev (reliable update).
__global__ void k_cg_start(Scal *sc, double *hist, int rslot, int rtr_slot, int hist_off, double stop_tol, int maxit,
                           int stop_on_initial, double rtz_prev)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double bb = sc->red[0];
    const double rtz = sc->red[rslot];
    const double rtr = sc->red[rtr_slot];
    IterState s{};
    s.rtz = rtz;
    s.rtr = rtr;
    s.beta = rtz_prev > 0 ? rtz / rtz_prev : 0.0;
    s.iter = 0;
    sc->resume = rtz_prev > 0 ? 1 : 0;
    sc->hist_den = bb;
    sc->stop_den = stop_on_initial ? rtr : bb;
    sc->stop_tol = stop_tol;
    sc->maxit = maxit;
    sc->hist_off = hist_off;
    sc->k2flag[0] = sc->k2flag[1] = 0;
    if (hist) hist[hist_off] = bb > 0 ? sqrt(rtr / bb) : 0.0;
    if (!__builtin_isfinite(bb) || !__builtin_isfinite(rtz) || !__builtin_isfinite(rtr)) {
        s.status = -6;
        s.done = 1;
    } else if (bb == 0.0 || rtr == 0.0 || rtz == 0.0 ||
               (!stop_on_initial && stop_tol > 0 && sqrt(rtr) / sqrt(sc->stop_den) <= stop_tol)) {
        s.conv = 1;
        s.done = 1;
    } else if (maxit <= 0) {
        s.done = 1;
    }
    sc->st[0] = s;
    sc->st[1] = s;
    sc->fin = s;
    sc->done_host = s.done;
    if (sc->host_done) set_host_flag(sc->host_done, s.done);
}

// Standalone reductions write one partial per workgroup; k_red_final sums
// them in a fixed order into red[slot].
__global__ __launch_bounds__(UPD_BS) void k_red_final(const double *__restrict__ P, int n, Scal *sc, int slot)
{
    __shared__ double sbuf[UPD_BS];
    const double s = sum_all<UPD_BS>(P, n, sbuf);
    if (threadIdx.x == 0) sc->red[slot] = s;
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
    // A node of a hexahedral mesh has at most 8 copies: their indices, then
    // their values, are requested together (predicated), so a segment costs
    // two dependent loads instead of two per copy; longer segments of
    // general maps finish in the loop after.  Sum in ascending copy order.
    constexpr int K = 8;
    const int n = e - b;
    int idx[K];
#pragma unroll
    for (int q = 0; q < K; ++q) idx[q] = q < n ? perm[b + q] : 0;
    if (apply_mask && flag[s]) {
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (q < n) w[idx[q]] = (T)0;
        for (int q = b + K; q < e; ++q) w[perm[q]] = (T)0;
        return;
    }
    T v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = q < n ? w[idx[q]] : (T)0;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (q < n) acc += (double)v[q];
    for (int q = b + K; q < e; ++q) acc += (double)w[perm[q]];
    const T r = (T)acc;
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (q < n) w[idx[q]] = r;
    for (int q = b + K; q < e; ++q) w[perm[q]] = r;
}

// Rounding of the FP64 geometric factors to the storage precision.
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

// Batched runs: advance the device chunk base by one chunk.
__global__ void k_batch_advance(int *base, int step)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *base += step;
}

// Batched runs: *out (a pinned host flag) = 1 when every listed problem
// (non-null entry) has finished its run, else 0.
__global__ __launch_bounds__(256) void k_batch_alldone(Scal *const *__restrict__ scs, int nprob, int *out)
{
    int pending = 0;
    for (int i = threadIdx.x; i < nprob; i += 256)
        if (scs[i] && !scs[i]->done_host) pending = 1;
    pending = __syncthreads_or(pending);
    if (threadIdx.x == 0) set_host_flag(out, !pending);
}

// Coarse solve of the two-level Schwarz preconditioner in three launches on
// the interior vertices (mx x my x mz = n_d - 1 per direction, x fastest),
// each workgroup staging its slab or plane in LDS (dynamic: the slab, then
// the modes it applies):
//   k_coarse_xy<true>  one workgroup per z-slab: the coarse right-hand side
//                      P^T r of the slab's vertices from the elements'
//                      moments (the eight elements around a vertex in
//                      ascending order), then S^T along x and along y -> a;
//   k_coarse_z         one workgroup per y-plane: S^T along z, the scaling
//                      1 / (lx + ly + lz), S along z -> b;
//   k_coarse_xy<false> one workgroup per z-slab: S along y and along x, into
//                      the vertex lattice ec (its boundary stays 0).
// Modes S are [vertex][mode] per direction.  With sc set, a CG step of
// iteration it (nothing after the run has ended).
template <bool FWD>
__global__ __launch_bounds__(256) void k_coarse_xy(const double *__restrict__ src, const double *__restrict__ Sx,
                                                   const double *__restrict__ Sy, double *__restrict__ dst, Box box,
                                                   const Scal *__restrict__ sc, int it)
{
    extern __shared__ double cl[];
    if (sc && sc->st[it & 1].done) return;
    const int mx = box.nx - 1, my = box.ny - 1;
    const int vz = blockIdx.x;   // interior z-index, vertex vz + 1
    const int tid = threadIdx.x, bs = blockDim.x, ns = mx * my;
    double *sl = cl, *t = cl + ns, *sx = t + ns, *sy = sx + mx * mx;
    for (int q = tid; q < mx * mx; q += bs) sx[q] = Sx[q];
    for (int q = tid; q < my * my; q += bs) sy[q] = Sy[q];
    if constexpr (FWD) {
        for (int q = tid; q < ns; q += bs) {
            const int ix = q % mx + 1, iy = q / mx + 1, iz = vz + 1;
            double s = 0.0;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const long e = (ix - 1 + dx) + (long)box.nx * ((iy - 1 + dy) + (long)box.ny * (iz - 1 + dz));
                        s += src[e * 8 + (1 - dx) + 2 * (1 - dy) + 4 * (1 - dz)];
                    }
            sl[q] = s;
        }
    } else {
        for (int q = tid; q < ns; q += bs) sl[q] = src[(long)vz * ns + q];
    }
    __syncthreads();
    if constexpr (FWD) {
        for (int q = tid; q < ns; q += bs) {   // along x: t[y][m] = sum_k Sx[k][m] sl[y][k]
            const int m = q % mx, y = q / mx;
            double acc = 0.0;
            for (int k = 0; k < mx; ++k) acc += sx[k * mx + m] * sl[y * mx + k];
            t[q] = acc;
        }
        __syncthreads();
        for (int q = tid; q < ns; q += bs) {   // along y: out[m][x] = sum_k Sy[k][m] t[k][x]
            const int x = q % mx, m = q / mx;
            double acc = 0.0;
            for (int k = 0; k < my; ++k) acc += sy[k * my + m] * t[k * mx + x];
            dst[(long)vz * ns + q] = acc;
        }
    } else {
        for (int q = tid; q < ns; q += bs) {   // along y: t[y][x] = sum_m Sy[y][m] sl[m][x]
            const int x = q % mx, y = q / mx;
            double acc = 0.0;
            for (int m = 0; m < my; ++m) acc += sy[y * my + m] * sl[m * mx + x];
            t[q] = acc;
        }
        __syncthreads();
        const long vx = box.nx + 1, vy = box.ny + 1;
        for (int q = tid; q < ns; q += bs) {   // along x: ec[x][y] = sum_m Sx[x][m] t[y][m]
            const int x = q % mx, y = q / mx;
            double acc = 0.0;
            for (int m = 0; m < mx; ++m) acc += sx[x * mx + m] * t[y * mx + m];
            dst[(x + 1) + vx * ((y + 1) + vy * (vz + 1))] = acc;
        }
    }
}

__global__ __launch_bounds__(256) void k_coarse_z(const double *__restrict__ a, const double *__restrict__ Sz,
                                                  const double *__restrict__ lx, const double *__restrict__ ly,
                                                  const double *__restrict__ lz, double *__restrict__ b, Box box,
                                                  const Scal *__restrict__ sc, int it)
{
    extern __shared__ double cl[];
    if (sc && sc->st[it & 1].done) return;
    const int mx = box.nx - 1, my = box.ny - 1, mz = box.nz - 1;
    const int y = blockIdx.x, tid = threadIdx.x, bs = blockDim.x, np = mx * mz;
    double *pl = cl, *t = cl + np, *sz = t + np;
    for (int q = tid; q < mz * mz; q += bs) sz[q] = Sz[q];
    for (int q = tid; q < np; q += bs) {   // plane [z][x]
        const int x = q % mx, z = q / mx;
        pl[q] = a[(long)z * mx * my + (long)y * mx + x];
    }
    __syncthreads();
    for (int q = tid; q < np; q += bs) {   // t[m][x] = sum_k Sz[k][m] pl[k][x] / (lx + ly + lz)
        const int x = q % mx, m = q / mx;
        double acc = 0.0;
        for (int k = 0; k < mz; ++k) acc += sz[k * mz + m] * pl[k * mx + x];
        t[q] = acc / (lx[x] + ly[y] + lz[m]);
    }
    __syncthreads();
    for (int q = tid; q < np; q += bs) {   // back along z
        const int x = q % mx, z = q / mx;
        double acc = 0.0;
        for (int m = 0; m < mz; ++m) acc += sz[z * mz + m] * t[m * mx + x];
        b[(long)z * mx * my + (long)y * mx + x] = acc;
    }
}

// x += d: FP64 iterate, FP64 or FP32 correction of an inner solve.
template <typename DT>
__global__ void k_axpy1(double *__restrict__ x, const DT *__restrict__ d, unsigned long n)
{
    for (unsigned long t = blockIdx.x * (unsigned long)blockDim.x + threadIdx.x; t < n; t += (unsigned long)gridDim.x * blockDim.x)
        x[t] += (double)d[t];
}

}  // namespace nek
