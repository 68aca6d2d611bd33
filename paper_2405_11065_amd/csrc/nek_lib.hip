// libnek: C ABI over the gfx950 kernels of the spectral-element Poisson CG
// solve (see include/nek.h for the contract of every entry point).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "nek.h"
#include "nek_kernels.hpp"
#include "nek_setup.hpp"

using namespace nek;

namespace {

constexpr int MAX_NP = 16;        // N <= 15
constexpr int MAXB = 2048;        // cap on workgroups of any reducing kernel
constexpr int CHUNK_ITERS = 16;   // CG iterations enqueued between flag polls

// Elements per workgroup of the operator kernel for each NP = N+1, chosen so
// EPW*NP^2 fills whole 64-lane waves where possible and the FP64 LDS
// footprint 3*EPW*NP^3*8 stays within 160 KB.
constexpr int epw_for(int NP)
{
    return NP == 2 ? 16 : NP == 3 ? 7 : NP == 4 ? 8 : NP == 5 ? 5 : NP == 6 ? 7 : NP == 7 ? 9
         : NP == 8 ? 4 : NP == 9 ? 4 : NP == 10 ? 3 : NP == 11 ? 2 : NP == 12 ? 2 : 1;
}

// Slices of geometric factors in flight per thread (register budget:
// 12 / 6 / 3 VGPRs per slice for FP64 / FP32 / BF16 storage).
template <typename GT> constexpr int pd_for() { return sizeof(GT) == 8 ? 2 : sizeof(GT) == 4 ? 4 : 6; }

#define NEK_NP_SWITCH(np, ...)                                   \
    switch (np) {                                                \
    case 2: { constexpr int NP = 2; __VA_ARGS__; } break;        \
    case 3: { constexpr int NP = 3; __VA_ARGS__; } break;        \
    case 4: { constexpr int NP = 4; __VA_ARGS__; } break;        \
    case 5: { constexpr int NP = 5; __VA_ARGS__; } break;        \
    case 6: { constexpr int NP = 6; __VA_ARGS__; } break;        \
    case 7: { constexpr int NP = 7; __VA_ARGS__; } break;        \
    case 8: { constexpr int NP = 8; __VA_ARGS__; } break;        \
    case 9: { constexpr int NP = 9; __VA_ARGS__; } break;        \
    case 10: { constexpr int NP = 10; __VA_ARGS__; } break;      \
    case 11: { constexpr int NP = 11; __VA_ARGS__; } break;      \
    case 12: { constexpr int NP = 12; __VA_ARGS__; } break;      \
    case 13: { constexpr int NP = 13; __VA_ARGS__; } break;      \
    case 14: { constexpr int NP = 14; __VA_ARGS__; } break;      \
    case 15: { constexpr int NP = 15; __VA_ARGS__; } break;      \
    case 16: { constexpr int NP = 16; __VA_ARGS__; } break;      \
    default: return NEK_E_ARG;                                   \
    }

#define HIP_TRY(expr)                                            \
    do {                                                         \
        if ((expr) != hipSuccess) return NEK_E_HIP;              \
    } while (0)

int g_num_cu = 0;

int num_cu()
{
    if (!g_num_cu) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            g_num_cu = v;
        else
            g_num_cu = 256;
    }
    return g_num_cu;
}

template <typename T> int dalloc(T *&p, size_t count)
{
    if (p) return NEK_OK;
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return NEK_E_OOM;
    p = static_cast<T *>(q);
    return NEK_OK;
}

template <typename T> void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

struct nek_ctx {
    int N = 0, NP = 0;
    int nel[3] = {0, 0, 0};
    long E = 0, nl = 0, ng = 0, nperm = 0, nseg = 0;
    Box box{};
    hipStream_t stream = nullptr;
    nek_opts opts{};
    int prec = NEK_PREC_FP64;

    std::vector<double> xi, w, D, vtx;

    // device data; g* are stored per point: [E][NP^3][6]
    double *D64 = nullptr;
    float *D32 = nullptr;
    double *g64 = nullptr;
    float *g32 = nullptr;
    uint16_t *g16 = nullptr;
    double *B = nullptr;
    int32_t *perm = nullptr, *segptr = nullptr;
    int8_t *segflag = nullptr;
    Scal *sc = nullptr;
    double *partials = nullptr;   // 3 regions of MAXB: operator, update, other
    double *hist = nullptr;
    long hist_cap = 0;
    // work vectors
    double *b = nullptr, *r64 = nullptr, *p64 = nullptr, *w64 = nullptr, *d64 = nullptr;
    float *r32 = nullptr, *p32 = nullptr, *w32 = nullptr;
    int *hflags = nullptr;   // pinned
    hipEvent_t ev[2] = {nullptr, nullptr};
    // sampled kernel timing (nek_prof_*)
    int prof_every = 0;
    long prof_tick = 0;
    std::vector<hipEvent_t> prof_pool;
    std::vector<int> prof_pending;     // event triples awaiting resolution
    double prof_ms[2] = {0, 0};
    long prof_n[2] = {0, 0};

    double *P1() { return partials; }
    double *P2() { return partials + MAXB; }
    double *P3() { return partials + 2 * MAXB; }
};

namespace {

unsigned red_grid(const nek_ctx *c)
{
    long want = (c->nl + UPD_BS - 1) / UPD_BS;
    long cap = std::min<long>(MAXB / 2, 4L * num_cu());
    return (unsigned)std::max<long>(1, std::min(want, cap));
}

template <int NP> int ax_groups(const nek_ctx *c) { return (int)((c->E + epw_for(NP) - 1) / epw_for(NP)); }

template <int NP> unsigned ax_grid(const nek_ctx *c)
{
    long want = ax_groups<NP>(c);
    long cap = std::min<long>(MAXB, 8L * num_cu());
    return (unsigned)std::max<long>(1, std::min(want, cap));
}

template <int NP, typename T, typename GT, bool CG>
int launch_ax(nek_ctx *c, const T *src, T *p, T *w, const GT *g, const T *D, int it)
{
    constexpr int EPW = epw_for(NP);
    constexpr int PD = pd_for<GT>();
    constexpr int BS = EPW * NP * NP;
    const size_t shm = 3ul * EPW * NP * NP * NP * sizeof(T);
    static bool attr_done = false;
    if (!attr_done) {
        if (shm > 65536)
            HIP_TRY(hipFuncSetAttribute((const void *)k_ax<NP, EPW, PD, T, GT, CG>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        attr_done = true;
    }
    hipLaunchKernelGGL((k_ax<NP, EPW, PD, T, GT, CG>), dim3(ax_grid<NP>(c)), dim3(BS), shm, c->stream, src, p, w, g,
                       D, c->sc, c->P1(), c->P2(), (int)red_grid(c), it, c->hist, (int)c->E, ax_groups<NP>(c));
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int prof_take(nek_ctx *c)
{
    // index of a free event triple, creating one when the pool is exhausted
    const size_t used = c->prof_pending.size();
    if (3 * used + 3 > c->prof_pool.size()) {
        for (int q = 0; q < 3; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            c->prof_pool.push_back(e);
        }
    }
    c->prof_pending.push_back((int)used);
    return (int)used;
}

// Fold the elapsed times of recorded triples into the totals (stream idle).
int prof_resolve(nek_ctx *c)
{
    for (int t : c->prof_pending) {
        float a = 0, b = 0;
        if (hipEventElapsedTime(&a, c->prof_pool[3 * t], c->prof_pool[3 * t + 1]) != hipSuccess ||
            hipEventElapsedTime(&b, c->prof_pool[3 * t + 1], c->prof_pool[3 * t + 2]) != hipSuccess)
            return NEK_E_HIP;
        c->prof_ms[0] += a;
        c->prof_ms[1] += b;
        c->prof_n[0] += 1;
        c->prof_n[1] += 1;
    }
    c->prof_pending.clear();
    return NEK_OK;
}

// CG iteration it (1-based): operator + pAp partials, then gather/update +
// rtr partials.  When sampled timing is on, every prof_every-th iteration is
// bracketed by events.
template <int NP, typename T, typename GT, typename XT>
int launch_cg_iter(nek_ctx *c, int it, XT *x, T *r, T *p, T *w, const GT *g, const T *D)
{
    int slot = -1;
    if (c->prof_every > 0 && (c->prof_tick++ % c->prof_every) == 0) {
        if ((slot = prof_take(c)) < 0) return NEK_E_HIP;
        HIP_TRY(hipEventRecord(c->prof_pool[3 * slot], c->stream));
    }
    int rc = launch_ax<NP, T, GT, true>(c, r, p, w, g, D, it);
    if (rc) return rc;
    if (slot >= 0) HIP_TRY(hipEventRecord(c->prof_pool[3 * slot + 1], c->stream));
    UpdArgs<T, XT> u{x, p, r, w, c->sc, c->P1(), c->P2(), (int)ax_grid<NP>(c), it, c->box, (unsigned)c->nl};
    hipLaunchKernelGGL((k_cg_update<NP, T, XT>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, u);
    HIP_TRY(hipGetLastError());
    if (slot >= 0) HIP_TRY(hipEventRecord(c->prof_pool[3 * slot + 2], c->stream));
    return NEK_OK;
}

int ensure_hist(nek_ctx *c, long need)
{
    if (need <= c->hist_cap) return NEK_OK;
    dfree(c->hist);
    long cap = std::max<long>(need, 4096);
    if (dalloc(c->hist, cap)) return NEK_E_OOM;
    c->hist_cap = cap;
    return NEK_OK;
}

int ensure_g(nek_ctx *c, int prec)
{
    const unsigned long n = (unsigned long)c->E * 6 * c->NP * c->NP * c->NP;
    const int grid = 4 * num_cu();
    if (prec == NEK_PREC_FP32 && !c->g32) {
        if (dalloc(c->g32, n)) return NEK_E_OOM;
        hipLaunchKernelGGL(k_g_to_f32, dim3(grid), dim3(256), 0, c->stream, c->g64, c->g32, n);
        HIP_TRY(hipGetLastError());
    }
    if (prec == NEK_PREC_BF16G && !c->g16) {
        if (dalloc(c->g16, n)) return NEK_E_OOM;
        hipLaunchKernelGGL(k_g_to_bf16, dim3(grid), dim3(256), 0, c->stream, c->g64, c->g16, n);
        HIP_TRY(hipGetLastError());
    }
    return NEK_OK;
}

template <typename T> int fill(nek_ctx *c, T *p, T v, unsigned long n)
{
    hipLaunchKernelGGL((k_fill<T>), dim3(4 * num_cu()), dim3(256), 0, c->stream, p, v, n);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int red_final(nek_ctx *c, int slot)
{
    hipLaunchKernelGGL(k_red_final, dim3(1), dim3(UPD_BS), 0, c->stream, c->P3(), (int)red_grid(c), c->sc, slot);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int glsc3_to_slot(nek_ctx *c, const void *a, const void *b, int dtype, int slot)
{
    NEK_NP_SWITCH(c->NP, {
        if (dtype == NEK_F64)
            hipLaunchKernelGGL((k_glsc3<NP, double, double>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream,
                               (const double *)a, (const double *)b, c->P3(), c->box, (unsigned)c->nl);
        else
            hipLaunchKernelGGL((k_glsc3<NP, float, float>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream,
                               (const float *)a, (const float *)b, c->P3(), c->box, (unsigned)c->nl);
    });
    HIP_TRY(hipGetLastError());
    return red_final(c, slot);
}

template <typename T> int gather_launch(nek_ctx *c, const T *in, T *out, bool weighted)
{
    NEK_NP_SWITCH(c->NP, {
        if (weighted)
            hipLaunchKernelGGL((k_gather<NP, T, true>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, in, out,
                               c->box, (unsigned)c->nl);
        else
            hipLaunchKernelGGL((k_gather<NP, T, false>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, in, out,
                               c->box, (unsigned)c->nl);
    });
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int ax_local_launch(nek_ctx *c, const void *u, void *w, int dtype, int prec)
{
    NEK_NP_SWITCH(c->NP, {
        if (dtype == NEK_F64)
            return launch_ax<NP, double, double, false>(c, (const double *)u, nullptr, (double *)w, c->g64, c->D64, 0);
        if (prec == NEK_PREC_BF16G)
            return launch_ax<NP, float, uint16_t, false>(c, (const float *)u, nullptr, (float *)w, c->g16, c->D32, 0);
        return launch_ax<NP, float, float, false>(c, (const float *)u, nullptr, (float *)w, c->g32, c->D32, 0);
    });
    return NEK_OK;
}

// r = b - M dssum(w) and red[slot] = glsc3(r, c, r)
int resid_launch(nek_ctx *c, const double *b, const double *w, double *r, int slot)
{
    NEK_NP_SWITCH(c->NP, {
        hipLaunchKernelGGL((k_resid<NP>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, b, w, r, c->P3(), c->box,
                           (unsigned)c->nl);
    });
    HIP_TRY(hipGetLastError());
    return red_final(c, slot);
}

int start_launch(nek_ctx *c, int rslot, int hist_off, double stop_tol, int maxit, int stop_on_initial)
{
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(64), 0, c->stream, c->sc, c->hist, rslot, hist_off, stop_tol, maxit,
                       stop_on_initial);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int read_scal(nek_ctx *c, Scal &h)
{
    HIP_TRY(hipMemcpyAsync(&h, c->sc, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return NEK_OK;
}

// Enqueue CG iterations it = 1, 2, ... in chunks until the device reports
// the run done or maxit iterations are enqueued; the flag of chunk k is read
// while chunk k+1 runs.  Then the finishing kernel publishes the final state.
template <typename IterFn> int run_cg(nek_ctx *c, int maxit, IterFn iter)
{
    int launched = 0, pend = -1, slot = 0;
    while (launched < maxit) {
        const int n = std::min(CHUNK_ITERS, maxit - launched);
        for (int q = 0; q < n; ++q) {
            int rc = iter(launched + q + 1);
            if (rc) return rc;
        }
        launched += n;
        HIP_TRY(hipMemcpyAsync(&c->hflags[slot], &c->sc->done_host, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipEventRecord(c->ev[slot], c->stream));
        if (pend >= 0) {
            HIP_TRY(hipEventSynchronize(c->ev[pend]));
            if (c->hflags[pend]) break;
        }
        pend = slot;
        slot ^= 1;
    }
    hipLaunchKernelGGL(k_cg_finish, dim3(1), dim3(UPD_BS), 0, c->stream, c->sc, c->P2(), (int)red_grid(c),
                       launched + 1, c->hist);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    return NEK_OK;
}

int ensure_fp64_work(nek_ctx *c)
{
    if (dalloc(c->b, c->nl) || dalloc(c->r64, c->nl) || dalloc(c->p64, c->nl) || dalloc(c->w64, c->nl))
        return NEK_E_OOM;
    return NEK_OK;
}

// b = M dssum(f); x = M dssum(c x0) or 0; r = b - A x; red[0] = b.b, red[1] = r.r
int cg_prologue(nek_ctx *c, const double *f, const double *x0, double *x, double *r)
{
    int rc = gather_launch<double>(c, f, c->b, false);
    if (rc) return rc;
    if (x0) {
        if ((rc = gather_launch<double>(c, x0, x == x0 ? c->w64 : x, true))) return rc;
        if (x == x0) HIP_TRY(hipMemcpyAsync(x, c->w64, c->nl * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if ((rc = ax_local_launch(c, x, c->w64, NEK_F64, NEK_PREC_FP64))) return rc;
        if ((rc = resid_launch(c, c->b, c->w64, r, 1))) return rc;
    } else {
        if ((rc = fill<double>(c, x, 0.0, c->nl))) return rc;
        HIP_TRY(hipMemcpyAsync(r, c->b, c->nl * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if ((rc = glsc3_to_slot(c, r, r, NEK_F64, 1))) return rc;
    }
    return glsc3_to_slot(c, c->b, c->b, NEK_F64, 0);
}

int cg_fp64_iterations(nek_ctx *c, double *x, int maxit)
{
    return run_cg(c, maxit, [&](int it) -> int {
        NEK_NP_SWITCH(c->NP, {
            return launch_cg_iter<NP, double, double, double>(c, it, x, c->r64, c->p64, c->w64, c->g64, c->D64);
        });
        return NEK_OK;
    });
}

int finish_status(const IterState &s, double tol)
{
    if (s.status) return s.status;
    if (tol > 0 && !s.conv) return NEK_NOCONV;
    return NEK_OK;
}

int solve_fp64(nek_ctx *c, const double *f, const double *x0, double tol, int maxit, double *x, nek_stats *st)
{
    int rc = ensure_fp64_work(c);
    if (rc) return rc;
    if ((rc = cg_prologue(c, f, x0, x, c->r64))) return rc;
    if ((rc = start_launch(c, 1, 0, tol, maxit, 0))) return rc;
    if ((rc = cg_fp64_iterations(c, x, maxit))) return rc;
    Scal h;
    if ((rc = read_scal(c, h))) return rc;
    st->iters = h.fin.iter;
    st->rel_res = h.hist_den > 0 ? std::sqrt(h.fin.rtz / h.hist_den) : 0.0;
    return finish_status(h.fin, tol);
}

// Iterative refinement: FP64 outer residual with FP64 g; inner CG with an
// FP32 operator (FP32 or BF16 g), FP64 reductions/scalars and FP64 correction.
int solve_mixed(nek_ctx *c, const double *f, const double *x0, double tol, int maxit, double *x, nek_stats *st)
{
    int rc;
    if ((rc = ensure_fp64_work(c)) || (rc = ensure_g(c, c->prec))) return rc;
    if (dalloc(c->d64, c->nl) || dalloc(c->r32, c->nl) || dalloc(c->p32, c->nl) || dalloc(c->w32, c->nl))
        return NEK_E_OOM;
    const bool bf16 = c->prec == NEK_PREC_BF16G;
    const double tau = c->opts.inner_tol > 0 ? c->opts.inner_tol : (bf16 ? 1e-2 : 1e-4);
    const int inner_cap = c->opts.inner_maxit > 0 ? c->opts.inner_maxit : 4000;
    const int max_outer = c->opts.max_outer > 0 ? c->opts.max_outer : 30;

    if ((rc = cg_prologue(c, f, x0, x, c->r64))) return rc;
    Scal h;
    if ((rc = read_scal(c, h))) return rc;
    const double bb = h.red[0];
    if (!std::isfinite(bb) || !std::isfinite(h.red[1])) return NEK_E_NONFINITE;
    double rho = bb > 0 ? std::sqrt(h.red[1]) / std::sqrt(bb) : 0.0;
    int total = 0, outer = 0, status = NEK_OK;
    double rho_prev = INFINITY;
    st->rel_res = rho;
    while (true) {
        if (bb == 0.0 || rho <= tol) break;
        if (outer >= max_outer || total >= maxit) { status = NEK_NOCONV; break; }
        if (outer > 0 && rho > 0.5 * rho_prev) {
            if (!c->opts.fp64_fallback) { status = NEK_E_STAGNATION; break; }
            // finish in FP64 from the current x (restart of the Krylov space)
            if ((rc = start_launch(c, 1, total, tol, maxit - total, 0))) return rc;
            if ((rc = cg_fp64_iterations(c, x, maxit - total))) return rc;
            if ((rc = read_scal(c, h))) return rc;
            st->fp64_iters = h.fin.iter;
            total += h.fin.iter;
            if ((rc = ax_local_launch(c, x, c->w64, NEK_F64, NEK_PREC_FP64))) return rc;
            if ((rc = resid_launch(c, c->b, c->w64, c->r64, 1))) return rc;
            if ((rc = read_scal(c, h))) return rc;
            rho = std::sqrt(h.red[1]) / std::sqrt(bb);
            status = h.fin.status ? h.fin.status : (rho <= tol ? NEK_OK : NEK_NOCONV);
            ++outer;
            break;
        }
        // inner solve of A d = r with the FP32 operator
        NEK_NP_SWITCH(c->NP, {
            hipLaunchKernelGGL((k_inner_start<NP>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, c->r64, c->r32,
                               c->d64, c->P3(), c->box, (unsigned)c->nl);
        });
        HIP_TRY(hipGetLastError());
        if ((rc = red_final(c, 1))) return rc;
        const double tau_k = std::min(0.5, std::max(tau, 0.3 * tol / rho));
        const int cap = std::min(inner_cap, maxit - total);
        if ((rc = start_launch(c, 1, total, tau_k, cap, 1))) return rc;
        rc = run_cg(c, cap, [&](int it) -> int {
            NEK_NP_SWITCH(c->NP, {
                if (bf16)
                    return launch_cg_iter<NP, float, uint16_t, double>(c, it, c->d64, c->r32, c->p32, c->w32, c->g16,
                                                                       c->D32);
                return launch_cg_iter<NP, float, float, double>(c, it, c->d64, c->r32, c->p32, c->w32, c->g32,
                                                                c->D32);
            });
            return NEK_OK;
        });
        if (rc) return rc;
        if ((rc = read_scal(c, h))) return rc;
        total += h.fin.iter;
        if (h.fin.status) { status = h.fin.status; break; }
        hipLaunchKernelGGL(k_axpy1, dim3(4 * num_cu()), dim3(256), 0, c->stream, x, c->d64, (unsigned long)c->nl);
        HIP_TRY(hipGetLastError());
        // true FP64 residual of the updated x
        if ((rc = ax_local_launch(c, x, c->w64, NEK_F64, NEK_PREC_FP64))) return rc;
        if ((rc = resid_launch(c, c->b, c->w64, c->r64, 1))) return rc;
        if ((rc = read_scal(c, h))) return rc;
        rho_prev = rho;
        rho = std::sqrt(h.red[1]) / std::sqrt(bb);
        ++outer;
        if (!std::isfinite(rho)) { status = NEK_E_NONFINITE; break; }
    }
    st->iters = total;
    st->outer_iters = outer;
    st->rel_res = rho;
    return status;
}

// [E][6][n3] <-> [E][n3][6]
void planes_to_points(const double *src, double *dst, long E, long n3)
{
    for (long e = 0; e < E; ++e)
        for (long q = 0; q < n3; ++q)
            for (int f = 0; f < 6; ++f) dst[(e * n3 + q) * 6 + f] = src[(e * 6 + f) * n3 + q];
}

void points_to_planes(const double *src, double *dst, long E, long n3)
{
    for (long e = 0; e < E; ++e)
        for (long q = 0; q < n3; ++q)
            for (int f = 0; f < 6; ++f) dst[(e * 6 + f) * n3 + q] = src[(e * n3 + q) * 6 + f];
}

}  // namespace

extern "C" {

const char *nek_strerror(int s)
{
    switch (s) {
    case NEK_OK: return "ok";
    case NEK_NOCONV: return "not converged within maxit";
    case NEK_E_ARG: return "invalid argument";
    case NEK_E_HIP: return "HIP runtime error";
    case NEK_E_OOM: return "out of memory";
    case NEK_E_JACOBIAN: return "inverted element (det J <= 0)";
    case NEK_E_BREAKDOWN: return "CG breakdown (pAp <= 0)";
    case NEK_E_NONFINITE: return "non-finite value in a reduction";
    case NEK_E_STAGNATION: return "mixed-precision refinement stagnated";
    default: return "unknown status";
    }
}

void nek_free(nek_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    dfree(c->D64); dfree(c->D32); dfree(c->g64); dfree(c->g32); dfree(c->g16); dfree(c->B);
    dfree(c->perm); dfree(c->segptr); dfree(c->segflag); dfree(c->sc); dfree(c->partials); dfree(c->hist);
    dfree(c->b); dfree(c->r64); dfree(c->p64); dfree(c->w64); dfree(c->d64);
    dfree(c->r32); dfree(c->p32); dfree(c->w32);
    if (c->hflags) (void)hipHostFree(c->hflags);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->prof_pool) (void)hipEventDestroy(e);
    delete c;
}

int nek_setup(const nek_mesh *mesh, int N, const nek_opts *opts, void *stream, nek_ctx **out)
{
    if (!mesh || !out || N < 1 || N + 1 > MAX_NP) return NEK_E_ARG;
    *out = nullptr;
    for (int d = 0; d < 3; ++d)
        if (mesh->nel[d] < 1) return NEK_E_ARG;
    const long NP = N + 1, n3 = NP * NP * NP;
    const long E = (long)mesh->nel[0] * mesh->nel[1] * mesh->nel[2];
    if (E * n3 >= (1L << 31)) return NEK_E_ARG;
    if (opts && (opts->prec < NEK_PREC_FP64 || opts->prec > NEK_PREC_BF16G || opts->elts_per_wg != 0))
        return NEK_E_ARG;
    nek_ctx *c = new (std::nothrow) nek_ctx;
    if (!c) return NEK_E_OOM;
    c->N = N;
    c->NP = (int)NP;
    for (int d = 0; d < 3; ++d) c->nel[d] = mesh->nel[d];
    c->box = Box{mesh->nel[0], mesh->nel[1], mesh->nel[2]};
    c->E = E;
    c->nl = E * n3;
    c->ng = ((long)mesh->nel[0] * N + 1) * ((long)mesh->nel[1] * N + 1) * ((long)mesh->nel[2] * N + 1);
    c->stream = (hipStream_t)stream;
    if (opts) c->opts = *opts;
    c->prec = c->opts.prec;

    gll_rule(N, c->xi, c->w);
    deriv_matrix(c->xi, c->D);
    if (mesh->vtx)
        c->vtx.assign(mesh->vtx, mesh->vtx + 3 * (size_t)(mesh->nel[0] + 1) * (mesh->nel[1] + 1) * (mesh->nel[2] + 1));
    else
        uniform_vertices(mesh->nel, mesh->lo, mesh->hi, c->vtx);

    int rc = NEK_OK;
    auto fail = [&](int code) { nek_free(c); return code; };
    std::vector<double> hg((size_t)E * 6 * n3), hB((size_t)c->nl);
    if (geometry(N, c->nel, c->vtx, c->xi, c->w, c->D, hg.data(), hB.data(), nullptr)) return fail(NEK_E_JACOBIAN);
    {
        std::vector<double> pts(hg.size());
        planes_to_points(hg.data(), pts.data(), E, n3);
        hg.swap(pts);
    }
    std::vector<int32_t> perm, segptr;
    std::vector<int8_t> segflag;
    segment_maps(N, c->nel, perm, segptr, segflag);
    c->nperm = (long)perm.size();
    c->nseg = (long)segflag.size();
    std::vector<float> D32(c->D.begin(), c->D.end());

    if (dalloc(c->D64, NP * NP) || dalloc(c->D32, NP * NP) || dalloc(c->g64, hg.size()) || dalloc(c->B, hB.size()) ||
        dalloc(c->perm, perm.size()) || dalloc(c->segptr, segptr.size()) || dalloc(c->segflag, segflag.size()) ||
        dalloc(c->sc, 1) || dalloc(c->partials, 3 * MAXB))
        return fail(NEK_E_OOM);
    if (hipHostMalloc((void **)&c->hflags, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) return fail(NEK_E_OOM);
    for (auto &e : c->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(NEK_E_HIP);
    // synchronous uploads: the host staging vectors die at return
    if (hipMemcpy(c->D64, c->D.data(), NP * NP * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->D32, D32.data(), NP * NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->g64, hg.data(), hg.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->B, hB.data(), hB.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->perm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->segptr, segptr.data(), segptr.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->segflag, segflag.data(), segflag.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->sc, 0, sizeof(Scal)) != hipSuccess ||
        hipMemset(c->partials, 0, 3 * MAXB * sizeof(double)) != hipSuccess)
        return fail(NEK_E_HIP);
    if ((rc = ensure_g(c, c->prec))) return fail(rc);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(NEK_E_HIP);
    *out = c;
    return NEK_OK;
}

int nek_size(const nek_ctx *c, int what, int64_t *out)
{
    if (!c || !out) return NEK_E_ARG;
    switch (what) {
    case NEK_SIZE_NLOCAL: *out = c->nl; break;
    case NEK_SIZE_NGLOBAL: *out = c->ng; break;
    case NEK_SIZE_E: *out = c->E; break;
    case NEK_SIZE_NPERM: *out = c->nperm; break;
    case NEK_SIZE_NSEG: *out = c->nseg; break;
    case NEK_SIZE_N: *out = c->N; break;
    default: return NEK_E_ARG;
    }
    return NEK_OK;
}

int nek_get(nek_ctx *c, int what, void *o)
{
    if (!c || !o) return NEK_E_ARG;
    const size_t NP = c->NP, n3 = NP * NP * NP;
    auto d2h = [&](void *dst, const void *src, size_t bytes) -> int {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return NEK_E_HIP;
        return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess ? NEK_OK : NEK_E_HIP;
    };
    switch (what) {
    case NEK_GET_GLL: std::memcpy(o, c->xi.data(), NP * sizeof(double)); return NEK_OK;
    case NEK_GET_W: std::memcpy(o, c->w.data(), NP * sizeof(double)); return NEK_OK;
    case NEK_GET_D: std::memcpy(o, c->D.data(), NP * NP * sizeof(double)); return NEK_OK;
    case NEK_GET_G: {
        std::vector<double> pts((size_t)c->E * 6 * n3);
        int rc = d2h(pts.data(), c->g64, pts.size() * sizeof(double));
        if (rc == NEK_OK) points_to_planes(pts.data(), (double *)o, c->E, (long)n3);
        return rc;
    }
    case NEK_GET_B: return d2h(o, c->B, (size_t)c->nl * sizeof(double));
    case NEK_GET_GID: numbering(c->N, c->nel, (int64_t *)o, nullptr, nullptr); return NEK_OK;
    case NEK_GET_MULT: numbering(c->N, c->nel, nullptr, (int32_t *)o, nullptr); return NEK_OK;
    case NEK_GET_MASK: numbering(c->N, c->nel, nullptr, nullptr, (int8_t *)o); return NEK_OK;
    case NEK_GET_PERM: return d2h(o, c->perm, (size_t)c->nperm * sizeof(int32_t));
    case NEK_GET_SEGPTR: return d2h(o, c->segptr, (size_t)(c->nseg + 1) * sizeof(int32_t));
    case NEK_GET_SEGFLAG: return d2h(o, c->segflag, (size_t)c->nseg);
    case NEK_GET_XYZ: {
        std::vector<double> g((size_t)c->E * 6 * n3), B((size_t)c->nl);
        return geometry(c->N, c->nel, c->vtx, c->xi, c->w, c->D, g.data(), B.data(), (double *)o) ? NEK_E_JACOBIAN
                                                                                                  : NEK_OK;
    }
    default: return NEK_E_ARG;
    }
}

int nek_set_prec(nek_ctx *c, int prec)
{
    if (!c || prec < NEK_PREC_FP64 || prec > NEK_PREC_BF16G) return NEK_E_ARG;
    int rc = ensure_g(c, prec);
    if (rc) return rc;
    c->prec = prec;
    return NEK_OK;
}

int nek_ax_local(nek_ctx *c, const void *u, void *w, int dtype)
{
    if (!c || !u || !w || (dtype != NEK_F64 && dtype != NEK_F32)) return NEK_E_ARG;
    int prec = dtype == NEK_F64 ? NEK_PREC_FP64 : (c->prec == NEK_PREC_BF16G ? NEK_PREC_BF16G : NEK_PREC_FP32);
    int rc = ensure_g(c, prec);
    if (rc) return rc;
    return ax_local_launch(c, u, w, dtype, prec);
}

int nek_dssum(nek_ctx *c, void *w, int dtype, int apply_mask)
{
    if (!c || !w || (dtype != NEK_F64 && dtype != NEK_F32)) return NEK_E_ARG;
    const unsigned grid = (unsigned)((c->nseg + UPD_BS - 1) / UPD_BS);
    if (dtype == NEK_F64)
        hipLaunchKernelGGL(k_dssum_seg<double>, dim3(grid), dim3(UPD_BS), 0, c->stream, (double *)w, c->perm,
                           c->segptr, c->segflag, (unsigned)c->nseg, apply_mask);
    else
        hipLaunchKernelGGL(k_dssum_seg<float>, dim3(grid), dim3(UPD_BS), 0, c->stream, (float *)w, c->perm,
                           c->segptr, c->segflag, (unsigned)c->nseg, apply_mask);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int nek_ax(nek_ctx *c, const void *u, void *w, int dtype)
{
    if (u == w) return NEK_E_ARG;
    int rc = nek_ax_local(c, u, w, dtype);
    if (rc) return rc;
    return nek_dssum(c, w, dtype, 1);
}

int nek_glsc3(nek_ctx *c, const void *a, const void *b, int dtype, double *out)
{
    if (!c || !a || !b || !out || (dtype != NEK_F64 && dtype != NEK_F32)) return NEK_E_ARG;
    int rc = glsc3_to_slot(c, a, b, dtype, 3);
    if (rc) return rc;
    Scal h;
    if ((rc = read_scal(c, h))) return rc;
    *out = h.red[3];
    return NEK_OK;
}

int nek_prof_enable(nek_ctx *c, int every)
{
    if (!c || every < 0) return NEK_E_ARG;
    c->prof_every = every;
    c->prof_tick = 0;
    return NEK_OK;
}

int nek_prof_read(nek_ctx *c, int kernel, double *total_ms, int64_t *count, int reset)
{
    if (!c || kernel < 0 || kernel > 1 || !total_ms || !count) return NEK_E_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess || prof_resolve(c) != NEK_OK) return NEK_E_HIP;
    *total_ms = c->prof_ms[kernel];
    *count = c->prof_n[kernel];
    if (reset) {
        c->prof_ms[kernel] = 0;
        c->prof_n[kernel] = 0;
    }
    return NEK_OK;
}

int nek_cg_solve(nek_ctx *c, const double *f, const double *x0, double tol, int maxit, double *x, nek_stats *stats,
                 double *res_hist)
{
    if (!c || !f || !x || maxit < 0) return NEK_E_ARG;
    nek_stats st{};
    int rc = ensure_hist(c, (long)maxit + 1);
    if (rc) return rc;
    auto t0 = std::chrono::steady_clock::now();
    if (c->prec == NEK_PREC_FP64)
        rc = solve_fp64(c, f, x0, tol, maxit, x, &st);
    else
        rc = solve_mixed(c, f, x0, tol, maxit, x, &st);
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc >= 0) rc = NEK_E_HIP;
    st.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc != NEK_E_HIP && prof_resolve(c) != NEK_OK) rc = NEK_E_HIP;
    st.status = rc;
    if (res_hist && rc != NEK_E_HIP) {
        const long n = std::min<long>(maxit, std::max(0, st.iters)) + 1;
        if (hipMemcpy(res_hist, c->hist, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) rc = NEK_E_HIP;
    }
    if (stats) *stats = st;
    return rc;
}

}  // extern "C"
