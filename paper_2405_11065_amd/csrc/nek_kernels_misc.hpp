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

// Coarse solve of the two-level Schwarz preconditioner, one workgroup: the
// coarse right-hand side P^T r of the interior vertices from the elements'
// moments (the up to eight elements around a vertex in ascending order),
// then S^T along x, y, z, the scaling 1 / (lx + ly + lz), and S back along
// z, y, x (per-direction modes S [vertex][mode] of n_d - 1 interior
// vertices), through the two scratch buffers a and b (interior vertices,
// x fastest).  ec receives the result on the whole vertex lattice, 0 on the
// boundary.  With sc set, a CG step of iteration it.
__global__ __launch_bounds__(1024) void k_asm_coarse(const double *__restrict__ mom, const double *__restrict__ Sx,
                                                     const double *__restrict__ Sy, const double *__restrict__ Sz,
                                                     const double *__restrict__ lx, const double *__restrict__ ly,
                                                     const double *__restrict__ lz, double *__restrict__ a,
                                                     double *__restrict__ b, double *__restrict__ ec, Box box,
                                                     const Scal *__restrict__ sc, int it)
{
    if (sc && sc->st[it & 1].done) return;
    const int tid = threadIdx.x, bs = blockDim.x;
    const int mx = box.nx - 1, my = box.ny - 1, mz = box.nz - 1;
    const long vx = box.nx + 1, vy = box.ny + 1, nv = vx * vy * (box.nz + 1);
    const long nc = (long)mx * my * mz;
    for (long q = tid; q < nv; q += bs) ec[q] = 0.0;
    for (long q = tid; q < nc; q += bs) {
        const int ix = (int)(q % mx) + 1, iy = (int)((q / mx) % my) + 1, iz = (int)(q / ((long)mx * my)) + 1;
        double s = 0.0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const long e = (ix - 1 + dx) + (long)box.nx * ((iy - 1 + dy) + (long)box.ny * (iz - 1 + dz));
                    s += mom[e * 8 + (1 - dx) + 2 * (1 - dy) + 4 * (1 - dz)];
                }
        a[q] = s;
    }
    __syncthreads();
    if (nc == 0) return;
    // one line per thread: in (stride st, n entries) -> out, out[m] = sum_k S[k][m] in[k] (fwd) or
    // out[k] = sum_m S[k][m] in[m] (back)
    auto pass = [&](const double *in, double *out, const double *S, int n, long st, long nlines, auto base_of,
                    bool fwd) {
        for (long l = tid; l < nlines; l += bs) {
            const long o = base_of(l);
            for (int m = 0; m < n; ++m) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k) acc += (fwd ? S[k * n + m] : S[m * n + k]) * in[o + k * st];
                out[o + m * st] = acc;
            }
        }
        __syncthreads();
    };
    auto bx = [&](long l) { return l * mx; };                                       // lines along x: (y, z)
    auto by = [&](long l) { return (l % mx) + (long)mx * my * (l / mx); };          // along y: (x, z)
    auto bz = [&](long l) { return l; };                                            // along z: (x, y)
    pass(a, b, Sx, mx, 1, (long)my * mz, bx, true);
    pass(b, a, Sy, my, mx, (long)mx * mz, by, true);
    pass(a, b, Sz, mz, (long)mx * my, (long)mx * my, bz, true);
    for (long q = tid; q < nc; q += bs) {
        const int ix = (int)(q % mx), iy = (int)((q / mx) % my), iz = (int)(q / ((long)mx * my));
        b[q] = b[q] / (lx[ix] + ly[iy] + lz[iz]);
    }
    __syncthreads();
    pass(b, a, Sz, mz, (long)mx * my, (long)mx * my, bz, false);
    pass(a, b, Sy, my, mx, (long)mx * mz, by, false);
    pass(b, a, Sx, mx, 1, (long)my * mz, bx, false);
    for (long q = tid; q < nc; q += bs) {
        const int ix = (int)(q % mx) + 1, iy = (int)((q / mx) % my) + 1, iz = (int)(q / ((long)mx * my)) + 1;
        ec[ix + vx * (iy + vy * iz)] = a[q];
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
