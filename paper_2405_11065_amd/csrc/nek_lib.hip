// libnek: C ABI over the gfx950 kernels of the spectral-element Poisson CG
// solve (see include/nek.h for the contract of every entry point).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "nek.h"
#include "nek_internal.hpp"
#include "nek_kernels_misc.hpp"
#include "nek_setup.hpp"

using namespace nek;

// Static device scratch of nek_ax_noalloc (the unassembled A_L u of one call).
// In host code `scratch` names a host-side stand-in, not device memory: host
// code reaches the array only through the per-device address that
// hipGetSymbolAddress returns (noalloc_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[NEK_NOALLOC_SCRATCH_BYTES];

namespace nek {

int g_num_cu = 0;

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// Device address of this device's copy of `scratch`, looked up once per
// device (with the device current) and kept.
int noalloc_scratch_ptr(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return NEK_E_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NEK_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NEK_OK;
}

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

const NpOps *np_ops_2();
const NpOps *np_ops_3();
const NpOps *np_ops_4();
const NpOps *np_ops_5();
const NpOps *np_ops_6();
const NpOps *np_ops_7();
const NpOps *np_ops_8();
const NpOps *np_ops_9();
const NpOps *np_ops_10();
const NpOps *np_ops_11();
const NpOps *np_ops_12();
const NpOps *np_ops_13();
const NpOps *np_ops_14();
const NpOps *np_ops_15();
const NpOps *np_ops_16();

const NpOps *np_ops(int NP)
{
    switch (NP) {
    case 2: return np_ops_2();
    case 3: return np_ops_3();
    case 4: return np_ops_4();
    case 5: return np_ops_5();
    case 6: return np_ops_6();
    case 7: return np_ops_7();
    case 8: return np_ops_8();
    case 9: return np_ops_9();
    case 10: return np_ops_10();
    case 11: return np_ops_11();
    case 12: return np_ops_12();
    case 13: return np_ops_13();
    case 14: return np_ops_14();
    case 15: return np_ops_15();
    case 16: return np_ops_16();
    default: return nullptr;
    }
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

// CG iteration it (1-based): operator (+ the pending x update) and pAp
// partials, then gather/update and rtr partials.  With final set, only the
// operator kernel runs: it applies the last x update and publishes the final
// state.  When sampled timing is on, every prof_every-th iteration is
// bracketed by events.
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
    if (nek_ctx *o = c->mesh_owner) {
        const int rc = ensure_g(o, prec);
        c->g32 = o->g32;
        c->g16 = o->g16;
        return rc;
    }
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

int fill_f64(nek_ctx *c, double *p, double v, unsigned long n) { return fill<double>(c, p, v, n); }

int fill_i32(hipStream_t s, int *p, int v, unsigned long n)
{
    hipLaunchKernelGGL((k_fill<int>), dim3(1), dim3(256), 0, s, p, v, n);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int batch_advance_launch(hipStream_t s, int *base, int step)
{
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, base, step);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int batch_alldone_launch(hipStream_t s, Scal *const *scs, int nprob, int *out)
{
    hipLaunchKernelGGL(k_batch_alldone, dim3(1), dim3(256), 0, s, scs, nprob, out);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int red_final(nek_ctx *c, int slot)
{
    hipLaunchKernelGGL(k_red_final, dim3(1), dim3(UPD_BS), 0, c->stream, c->P3(), (int)red_grid(c), c->sc, slot);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

const NpOps *ops(const nek_ctx *c) { return np_ops(c->NP); }

int glsc3_to_slot(nek_ctx *c, const void *a, const void *b, int dtype, int slot)
{
    const int rc = dtype == NEK_F64 ? ops(c)->glsc3_64(c, (const double *)a, (const double *)b)
                                    : ops(c)->glsc3_32(c, (const float *)a, (const float *)b);
    return rc ? rc : red_final(c, slot);
}

int gather_launch(nek_ctx *c, const double *in, double *out, bool weighted)
{
    return ops(c)->gather64(c, in, out, weighted);
}

int ax_local_launch(nek_ctx *c, const void *u, void *w, int dtype, int prec)
{
    if (dtype == NEK_F64) return ops(c)->ax64(c, (const double *)u, (double *)w);
    if (prec == NEK_PREC_BF16G) return ops(c)->ax16(c, (const float *)u, (float *)w);
    return ops(c)->ax32(c, (const float *)u, (float *)w);
}

// r = b - M dssum(w) and red[slot] = glsc3(r, c, r)
int resid_launch(nek_ctx *c, const double *b, const double *w, double *r, int slot)
{
    const int rc = ops(c)->resid(c, b, w, r);
    return rc ? rc : red_final(c, slot);
}

int ensure_diag(nek_ctx *c)
{
    if (c->dg64 && c->dg32) return NEK_OK;
    const long n3 = (long)c->NP * c->NP * c->NP;
    std::vector<double> hg((size_t)c->E * 6 * n3), hB((size_t)c->nl), m((size_t)c->nl);
    if (geometry(c->N, c->nel, c->vtx, c->xi, c->w, c->D, hg.data(), hB.data(), nullptr)) return NEK_E_JACOBIAN;
    assembled_diagonal(c->N, c->nel, c->D, hg.data(), m.data());
    std::vector<float> m32(m.begin(), m.end());   // round to nearest even
    if (dalloc(c->dg64, c->nl) || dalloc(c->dg32, c->nl)) return NEK_E_OOM;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->dg64, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->dg32, m32.data(), m32.size() * sizeof(float), hipMemcpyHostToDevice));
    return NEK_OK;
}

int ensure_tri(nek_ctx *c)
{
    if (c->tri64 && c->tri32) return NEK_OK;
    std::vector<double> t;
    if (trilinear_coefs(c->N, c->nel, c->vtx, c->xi, c->w, TRI_HDR, t)) return NEK_E_JACOBIAN;
    std::vector<float> t32(t.begin(), t.end());   // round to nearest even
    if (dalloc(c->tri64, t.size()) || dalloc(c->tri32, t.size())) return NEK_E_OOM;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->tri64, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->tri32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
    return NEK_OK;
}

int ensure_fdm(nek_ctx *c)
{
    int rc = ensure_diag(c);
    if (rc) return rc;
    if (c->fdmS64 && c->z64 && c->z32) return NEK_OK;
    std::vector<double> S, L, C((size_t)3 * c->E);
    fdm_modes(c->N, c->w, c->D, S, L);
    fdm_scales(c->nel, c->vtx, C.data());
    std::vector<float> S32(S.begin(), S.end()), L32(L.begin(), L.end()), C32(C.begin(), C.end());
    if (dalloc(c->fdmS64, S.size()) || dalloc(c->fdmL64, L.size()) || dalloc(c->fdmC64, C.size()) ||
        dalloc(c->fdmS32, S.size()) || dalloc(c->fdmL32, L.size()) || dalloc(c->fdmC32, C.size()) ||
        dalloc(c->z64, c->nl) || dalloc(c->z32, c->nl))
        return NEK_E_OOM;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!S.empty()) {
        HIP_TRY(hipMemcpy(c->fdmS64, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->fdmL64, L.data(), L.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->fdmS32, S32.data(), S32.size() * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->fdmL32, L32.data(), L32.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(c->fdmC64, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->fdmC32, C32.data(), C32.size() * sizeof(float), hipMemcpyHostToDevice));
    return NEK_OK;
}

int ensure_schwarz(nek_ctx *c)
{
    // the coarse slabs and planes are staged in LDS: at most 64 interior
    // vertices per direction (meshes of up to 65 elements along each)
    if (c->N < 2 || c->nel[0] > 65 || c->nel[1] > 65 || c->nel[2] > 65) return NEK_E_ARG;
    if (c->asmS64 && c->asmU64 && c->z64 && c->z32) return NEK_OK;
    const int NP = c->NP, NW = NP + 2;
    std::vector<double> S, L, CS, CL, ell((size_t)2 * NP), C((size_t)3 * c->E);
    schwarz_windows(c->N, c->w, c->D, S, L);
    schwarz_coarse(c->N, c->nel, c->vtx, c->xi, c->w, CS, CL, c->asmCoff, c->asmCloff);
    for (int i = 0; i < NP; ++i) {
        ell[i] = (1.0 - c->xi[i]) / 2.0;
        ell[NP + i] = (1.0 + c->xi[i]) / 2.0;
    }
    fdm_scales(c->nel, c->vtx, C.data());
    std::vector<float> S32(S.begin(), S.end()), L32(L.begin(), L.end()), C32(C.begin(), C.end());
    const long nv = (long)(c->nel[0] + 1) * (c->nel[1] + 1) * (c->nel[2] + 1);
    const long ncv = (long)(c->nel[0] - 1) * (c->nel[1] - 1) * (c->nel[2] - 1);
    const size_t nu = (size_t)c->E * NW * NW * NW;
    if (dalloc(c->asmS64, S.size()) || dalloc(c->asmL64, L.size()) || dalloc(c->asmS32, S.size()) ||
        dalloc(c->asmL32, L.size()) || dalloc(c->asmEll, ell.size()) || dalloc(c->asmCS, CS.size()) ||
        dalloc(c->asmCL, CL.size()) || dalloc(c->fdmC64, C.size()) || dalloc(c->fdmC32, C.size()) ||
        dalloc(c->asmU64, nu) || dalloc(c->asmU32, nu) || dalloc(c->asmMom, (size_t)8 * c->E) ||
        dalloc(c->asmEc, nv) || dalloc(c->asmTmp, 2 * ncv) || dalloc(c->z64, c->nl) || dalloc(c->z32, c->nl))
        return NEK_E_OOM;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->asmS64, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->asmL64, L.data(), L.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->asmS32, S32.data(), S32.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->asmL32, L32.data(), L32.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->asmEll, ell.data(), ell.size() * sizeof(double), hipMemcpyHostToDevice));
    if (!CS.empty()) {
        HIP_TRY(hipMemcpy(c->asmCS, CS.data(), CS.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->asmCL, CL.data(), CL.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(c->fdmC64, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->fdmC32, C32.data(), C32.size() * sizeof(float), hipMemcpyHostToDevice));
    // the coarse correction's boundary vertices are never written: zero once
    const int rc = fill_f64(c, c->asmEc, 0.0, (unsigned long)nv);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return NEK_OK;
}

int asm_coarse_launch(nek_ctx *c, const Scal *sc, int it)
{
    const int mx = c->box.nx - 1, my = c->box.ny - 1, mz = c->box.nz - 1;
    if (mx <= 0 || my <= 0 || mz <= 0) return NEK_OK;   // no interior vertex: ec stays 0
    const long ncv = (long)mx * my * mz;
    const double *S = c->asmCS, *L = c->asmCL;
    double *a = c->asmTmp, *b = c->asmTmp + ncv;
    const size_t lxy = (size_t)(2 * mx * my + mx * mx + my * my) * sizeof(double);
    const size_t lz = (size_t)(2 * mx * mz + mz * mz) * sizeof(double);
    static bool attr_done = false;   // up to 128 KB of LDS at 64 interior vertices per direction
    if (!attr_done) {
        const int big = 160 * 1024;
        HIP_TRY(hipFuncSetAttribute((const void *)k_coarse_xy<true>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
        HIP_TRY(hipFuncSetAttribute((const void *)k_coarse_xy<false>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
        HIP_TRY(hipFuncSetAttribute((const void *)k_coarse_z, hipFuncAttributeMaxDynamicSharedMemorySize, big));
        attr_done = true;
    }
    hipLaunchKernelGGL(k_coarse_xy<true>, dim3(mz), dim3(256), lxy, c->stream, c->asmMom, S + c->asmCoff[0],
                       S + c->asmCoff[1], a, c->box, sc, it);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_coarse_z, dim3(my), dim3(256), lz, c->stream, a, S + c->asmCoff[2], L + c->asmCloff[0],
                       L + c->asmCloff[1], L + c->asmCloff[2], b, c->box, sc, it);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_coarse_xy<false>, dim3(mz), dim3(256), lxy, c->stream, b, S + c->asmCoff[0],
                       S + c->asmCoff[1], c->asmEc, c->box, sc, it);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int ensure_precond(nek_ctx *c, int pc)
{
    return pc == NEK_PC_FDM ? ensure_fdm(c) : pc == NEK_PC_SCHWARZ ? ensure_schwarz(c)
         : pc == NEK_PC_JACOBI ? ensure_diag(c) : NEK_OK;
}

int pc_start64(nek_ctx *c, double *r, int *rtz_slot)
{
    *rtz_slot = 1;
    if (!c->precond) return NEK_OK;
    int rc;
    if (c->precond == NEK_PC_FDM || c->precond == NEK_PC_SCHWARZ) {
        if (!c->z64) return NEK_E_ARG;
        rc = c->precond == NEK_PC_FDM ? ops(c)->pc_fdm64(c, r, c->z64, c->P3(), red_grid(c), false, 0)
                                      : ops(c)->pc_asm64(c, r, c->z64, c->P3(), red_grid(c), false, 0);
    } else {
        if (!c->dg64) return NEK_E_ARG;
        rc = ops(c)->pc_start64(c, r, c->dg64);
    }
    if (rc) return rc;
    *rtz_slot = 2;
    return red_final(c, 2);
}

int pc_start32(nek_ctx *c, float *r, int *rtz_slot)
{
    *rtz_slot = 1;
    if (!c->precond) return NEK_OK;
    int rc;
    if (c->precond == NEK_PC_FDM || c->precond == NEK_PC_SCHWARZ) {
        if (!c->z32) return NEK_E_ARG;
        rc = c->precond == NEK_PC_FDM ? ops(c)->pc_fdm32(c, r, c->z32, c->P3(), red_grid(c), false, 0)
                                      : ops(c)->pc_asm32(c, r, c->z32, c->P3(), red_grid(c), false, 0);
    } else {
        if (!c->dg32) return NEK_E_ARG;
        rc = ops(c)->pc_start32(c, r, c->dg32);
    }
    if (rc) return rc;
    *rtz_slot = 2;
    return red_final(c, 2);
}

// one CG iteration of the context at precision prec on its work vectors;
// x is FP64 at FP64, else the correction of an inner solve (FP64 unless
// opts.corr_fp32)
int cg_iter(nek_ctx *c, int prec, int variant, int it, bool final, void *x)
{
    if (prec == NEK_PREC_FP64)
        return ops(c)->cg_iter64(c, variant, it, final, (double *)x, c->r64, c->p64, c->w64, c->g64, c->D64);
    const bool x64 = !c->opts.corr_fp32;
    if (prec == NEK_PREC_BF16G)
        return ops(c)->cg_iter16(c, variant, it, final, x, x64, c->r32, c->p32, c->w32, c->g16, c->D32);
    return ops(c)->cg_iter32(c, variant, it, final, x, x64, c->r32, c->p32, c->w32, c->g32, c->D32);
}

int true_residual(nek_ctx *c, const double *x, double bb, double *rho)
{
    int rc;
    if ((rc = ax_local_launch(c, x, c->w64, NEK_F64, NEK_PREC_FP64)) || (rc = resid_launch(c, c->b, c->w64, c->r64, 1)))
        return rc;
    Scal h;
    if ((rc = read_scal(c, h))) return rc;
    *rho = bb > 0 ? std::sqrt(h.red[1]) / std::sqrt(bb) : 0.0;
    return NEK_OK;
}

int variant_for_epw(int NP, int epw)
{
    const NpOps *o = np_ops(NP);
    if (!o) return -1;
    for (int v = 0; v < o->nvariants; v += 2)   // even variants: the default prefetch depth
        if (o->variant_epw(v) == epw) return v;
    return -1;
}

int autotune_if_needed(nek_ctx *c, int prec)
{
    if (c->tuned[prec] || c->opts.elts_per_wg != 0) return NEK_OK;
    return nek_tune(c, prec, 20, nullptr, nullptr);
}

int start_launch(nek_ctx *c, int rslot, int hist_off, double stop_tol, int maxit, int stop_on_initial,
                 double rtz_prev, int rtr_slot)
{
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(64), 0, c->stream, c->sc, c->hist, rslot,
                       rtr_slot < 0 ? rslot : rtr_slot, hist_off, stop_tol, maxit, stop_on_initial, rtz_prev);
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
// while chunk k+1 runs.  Then one more operator launch applies the pending x
// update and publishes the final state.
template <typename IterFn> int run_cg(nek_ctx *c, int maxit, IterFn iter)
{
    int launched = 0, pend = -1, slot = 0;
    // Schwarz-preconditioned runs take a few iterations per refinement step:
    // shorter chunks enqueue fewer iterations past the end of a run
    const int chunk = c->precond == NEK_PC_SCHWARZ ? 4 : CHUNK_ITERS;
    while (launched < maxit) {
        const int n = std::min(chunk, maxit - launched);
        for (int q = 0; q < n; ++q) {
            int rc = iter(launched + q + 1, false);
            if (rc) return rc;
        }
        launched += n;
        HIP_TRY(hipEventRecord(c->ev[slot], c->stream));
        if (pend >= 0) {
            // the run's kernels write hflags[0] themselves (k_cg_start, then
            // the operator kernel that ends the run): no copy in the stream
            HIP_TRY(hipEventSynchronize(c->ev[pend]));
            if (__atomic_load_n(&c->hflags[0], __ATOMIC_ACQUIRE)) break;
        }
        pend = slot;
        slot ^= 1;
    }
    int rc = iter(launched + 1, true);
    if (rc) return rc;
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
    int rc = gather_launch(c, f, c->b, false);
    if (rc) return rc;
    if (x0) {
        if ((rc = gather_launch(c, x0, x == x0 ? c->w64 : x, true))) return rc;
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
    return run_cg(c, maxit, [&](int it, bool final) -> int {
        return cg_iter(c, NEK_PREC_FP64, c->variant[NEK_PREC_FP64], it, final, x);
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
    int rs = 1;
    if ((rc = pc_start64(c, c->r64, &rs))) return rc;
    if ((rc = start_launch(c, rs, 0, tol, maxit, 0, 0.0, 1))) return rc;
    if ((rc = cg_fp64_iterations(c, x, maxit))) return rc;
    Scal h;
    if ((rc = read_scal(c, h))) return rc;
    st->iters = h.fin.iter;
    st->last_rec_res = h.hist_den > 0 ? std::sqrt(h.fin.rtr / h.hist_den) : 0.0;
    const int status = finish_status(h.fin, tol);
    if (status >= 0 && (rc = true_residual(c, x, h.hist_den, &st->true_rel_res))) return rc;
    return status;
}

int ensure_mixed_work(nek_ctx *c)
{
    int rc;
    if ((rc = ensure_fp64_work(c)) || (rc = ensure_g(c, c->prec))) return rc;
    if ((c->opts.corr_fp32 ? dalloc(c->d32, c->nl) : dalloc(c->d64, c->nl)) || dalloc(c->r32, c->nl) ||
        dalloc(c->p32, c->nl) || dalloc(c->w32, c->nl))
        return NEK_E_OOM;
    return NEK_OK;
}

// Iterative refinement: FP64 outer residual with FP64 g; inner CG with an
// FP32 operator (FP32 or BF16 g), FP64 reductions/scalars and a correction d
// accumulated in FP64 (or stored in FP32, each update d += alpha p formed in
// FP64 and rounded once), added to the FP64 x after the inner solve.
// The control below is shared by the solo and the batched solver.
void ir_init(const nek_ctx *c, IrCtl &s)
{
    s = IrCtl{};
    // Reliable updates by default: the inner CG keeps its search direction
    // when its residual is replaced by the FP64 true residual, so the solve
    // keeps the Krylov space that a restart would discard (16^3 N=9: 875
    // FP32-operator iterations against 1020 restarted and 861 in FP64).  The
    // replacement threshold is a residual reduction of 1e-2 with FP32 g; BF16
    // g's ~2^-9 operator error needs replacements every 0.3.
    const bool bf16 = c->prec == NEK_PREC_BF16G;
    s.keep_p = c->opts.refine_mode != 1;
    s.tau = c->opts.inner_tol > 0 ? c->opts.inner_tol : s.keep_p ? (bf16 ? 0.3 : 1e-2) : (bf16 ? 1e-2 : 1e-4);
    s.inner_cap = c->opts.inner_maxit > 0 ? c->opts.inner_maxit : 4000;
    s.max_outer = c->opts.max_outer > 0 ? c->opts.max_outer : 30;
}

// after cg_prologue: red[0] = b.b, red[1] = r.r
void ir_start(IrCtl &s, const Scal &h)
{
    s.bb = h.red[0];
    if (!std::isfinite(s.bb) || !std::isfinite(h.red[1])) {
        s.status = NEK_E_NONFINITE;
        s.finished = true;
        return;
    }
    s.rho = s.bb > 0 ? std::sqrt(h.red[1]) / std::sqrt(s.bb) : 0.0;
}

IrStep ir_decide(IrCtl &s, const nek_ctx *c, double tol, int maxit)
{
    if (s.finished || s.bb == 0.0 || s.rho <= tol) return IR_DONE;
    if (s.outer >= s.max_outer || s.total >= maxit) {
        s.status = NEK_NOCONV;
        return IR_DONE;
    }
    if (s.outer > 0 && s.rho > 0.5 * s.rho_prev) {
        if (!c->opts.fp64_fallback) {
            s.status = NEK_E_STAGNATION;
            return IR_DONE;
        }
        return IR_FALLBACK;
    }
    return IR_INNER;
}

// Finish in FP64 CG from the current x (restart of the Krylov space);
// synchronous.
int ir_fallback(nek_ctx *c, IrCtl &s, double tol, int maxit, double *x)
{
    int rc;
    Scal h;
    int rs = 1;
    if ((rc = pc_start64(c, c->r64, &rs))) return rc;
    if ((rc = start_launch(c, rs, s.total, tol, maxit - s.total, 0, 0.0, 1))) return rc;
    if ((rc = cg_fp64_iterations(c, x, maxit - s.total))) return rc;
    if ((rc = read_scal(c, h))) return rc;
    s.fp64_iters = h.fin.iter;
    s.total += h.fin.iter;
    s.last_rec = h.hist_den > 0 ? std::sqrt(h.fin.rtr / h.hist_den) : 0.0;
    if ((rc = ax_local_launch(c, x, c->w64, NEK_F64, NEK_PREC_FP64))) return rc;
    if ((rc = resid_launch(c, c->b, c->w64, c->r64, 1))) return rc;
    if ((rc = read_scal(c, h))) return rc;
    s.rho = std::sqrt(h.red[1]) / std::sqrt(s.bb);
    s.status = h.fin.status ? h.fin.status : (s.rho <= tol ? NEK_OK : NEK_NOCONV);
    ++s.outer;
    s.finished = true;
    return NEK_OK;
}

// Enqueue the start of an inner solve of A d = r; *cap = its iteration cap.
int ir_inner_launch(nek_ctx *c, IrCtl &s, double tol, int maxit, int *cap)
{
    int rc;
    if ((rc = ops(c)->inner_start(c, c->r64, c->r32, inner_x(c), !c->opts.corr_fp32))) return rc;
    if ((rc = red_final(c, 1))) return rc;
    int rs = 1;
    if ((rc = pc_start32(c, c->r32, &rs))) return rc;
    const double tau_k = std::min(0.5, std::max(s.tau, 0.3 * tol / s.rho));
    *cap = std::min(s.inner_cap, maxit - s.total);
    return start_launch(c, rs, s.total, tau_k, *cap, 1, s.keep_p ? s.rtz_last : 0.0, 1);
}

// After an inner run (h read back): count it, then enqueue x += d and the
// true FP64 residual.  Sets s.finished when the inner run failed.
int ir_inner_done(nek_ctx *c, IrCtl &s, const Scal &h, double *x)
{
    s.total += h.fin.iter;
    // A resumed run continues the search direction with beta = rtz(r_new) /
    // rtz(r_{K-1}), r_{K-1} the residual before the run's last one (the one
    // the true residual replaces); the stopping iteration's beta is
    // rtz(r_K) / rtz(r_{K-1}), so rtz(r_{K-1}) = rtz(r_K) / beta.  A run
    // that stopped at its start has no such residual and restarts.
    s.rtz_last = h.fin.beta > 0 ? h.fin.rtz / h.fin.beta : 0.0;
    s.last_rec = h.hist_den > 0 ? std::sqrt(h.fin.rtr / h.hist_den) : 0.0;
    if (h.fin.status) {
        s.status = h.fin.status;
        s.finished = true;
        return NEK_OK;
    }
    if (c->opts.corr_fp32)
        hipLaunchKernelGGL(k_axpy1<float>, dim3(4 * num_cu()), dim3(256), 0, c->stream, x, c->d32, (unsigned long)c->nl);
    else
        hipLaunchKernelGGL(k_axpy1<double>, dim3(4 * num_cu()), dim3(256), 0, c->stream, x, c->d64, (unsigned long)c->nl);
    HIP_TRY(hipGetLastError());
    int rc;
    if ((rc = ax_local_launch(c, x, c->w64, NEK_F64, NEK_PREC_FP64))) return rc;
    return resid_launch(c, c->b, c->w64, c->r64, 1);
}

// After the true residual (h read back).
void ir_outer_done(IrCtl &s, const Scal &h)
{
    s.rho_prev = s.rho;
    s.rho = std::sqrt(h.red[1]) / std::sqrt(s.bb);
    ++s.outer;
    if (!std::isfinite(s.rho)) {
        s.status = NEK_E_NONFINITE;
        s.finished = true;
    }
}

void ir_stats(const IrCtl &s, nek_stats *st)
{
    st->iters = s.total;
    st->outer_iters = s.outer;
    st->fp64_iters = s.fp64_iters;
    st->true_rel_res = s.rho;
    st->last_rec_res = s.last_rec;
}

int solve_mixed(nek_ctx *c, const double *f, const double *x0, double tol, int maxit, double *x, nek_stats *st)
{
    int rc;
    if ((rc = ensure_mixed_work(c))) return rc;
    IrCtl s;
    ir_init(c, s);
    if ((rc = cg_prologue(c, f, x0, x, c->r64))) return rc;
    Scal h;
    if ((rc = read_scal(c, h))) return rc;
    ir_start(s, h);
    while (!s.finished) {
        const IrStep step = ir_decide(s, c, tol, maxit);
        if (step == IR_DONE) break;
        if (step == IR_FALLBACK) {
            if ((rc = ir_fallback(c, s, tol, maxit, x))) return rc;
            break;
        }
        int cap = 0;
        if ((rc = ir_inner_launch(c, s, tol, maxit, &cap))) return rc;
        rc = run_cg(c, cap, [&](int it, bool final) -> int {
            return cg_iter(c, c->prec, c->variant[c->prec], it, final, inner_x(c));
        });
        if (rc) return rc;
        if ((rc = read_scal(c, h))) return rc;
        if ((rc = ir_inner_done(c, s, h, x))) return rc;
        if (s.finished) break;
        if ((rc = read_scal(c, h))) return rc;
        ir_outer_done(s, h);
    }
    ir_stats(s, st);
    return s.status;
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

namespace {

// Options check shared by nek_setup and setup_shared; *v_epw receives the
// kernel configuration that opts->elts_per_wg selects (0 if none).
int check_opts(int N, const nek_opts *opts, int *v_epw)
{
    *v_epw = 0;
    if (opts && (opts->prec < NEK_PREC_FP64 || opts->prec > NEK_PREC_BF16G || opts->elts_per_wg < -1 ||
                 opts->precond < NEK_PC_NONE || opts->precond > NEK_PC_SCHWARZ || opts->corr_fp32 < 0 ||
                 opts->corr_fp32 > 1))
        return NEK_E_ARG;
    if (opts && opts->elts_per_wg > 0 && (*v_epw = variant_for_epw(N + 1, opts->elts_per_wg)) < 0) return NEK_E_ARG;
    return NEK_OK;
}

void set_opts(nek_ctx *c, const nek_opts *opts, int v_epw)
{
    if (opts) c->opts = *opts;
    c->prec = c->opts.prec;
    if (c->opts.elts_per_wg != 0)
        for (int q = 0; q < 3; ++q) {
            c->variant[q] = v_epw;
            c->tuned[q] = true;
        }
}

// Per-context CG state: scalars, partials, the pinned done flag and its
// events, the static scratch address, g in the solve precision and the
// preconditioner.  Synchronises.
int setup_state(nek_ctx *c)
{
    int rc;
    if (dalloc(c->sc, 1) || dalloc(c->partials, 7 * MAXB)) return NEK_E_OOM;
    if (hipHostMalloc((void **)&c->hflags, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) return NEK_E_OOM;
    c->hflags[0] = c->hflags[1] = 0;
    int *hflag_dev = nullptr;
    if (hipHostGetDevicePointer((void **)&hflag_dev, c->hflags, 0) != hipSuccess) return NEK_E_HIP;
    for (auto &e : c->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return NEK_E_HIP;
    if (hipMemset(c->sc, 0, sizeof(Scal)) != hipSuccess ||
        hipMemcpy(&c->sc->host_done, &hflag_dev, sizeof(int *), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->partials, 0, 7 * MAXB * sizeof(double)) != hipSuccess)
        return NEK_E_HIP;
    if ((rc = noalloc_scratch_ptr(&c->noalloc_scratch))) return rc;
    if ((rc = ensure_g(c, c->prec))) return rc;
    if (c->opts.precond != NEK_PC_NONE) {
        if ((rc = ensure_precond(c, c->opts.precond))) return rc;
        c->precond = c->opts.precond;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return NEK_E_HIP;
    return NEK_OK;
}

}  // namespace

int setup_shared(nek_ctx *owner, const nek_opts *opts, void *stream, nek_ctx **out)
{
    if (!owner || !out || owner->mesh_owner) return NEK_E_ARG;
    *out = nullptr;
    int v_epw = 0, rc;
    if ((rc = check_opts(owner->N, opts, &v_epw))) return rc;
    nek_ctx *c = new (std::nothrow) nek_ctx;
    if (!c) return NEK_E_OOM;
    c->N = owner->N;
    c->NP = owner->NP;
    for (int d = 0; d < 3; ++d) c->nel[d] = owner->nel[d];
    c->box = owner->box;
    c->E = owner->E;
    c->nl = owner->nl;
    c->ng = owner->ng;
    c->nperm = owner->nperm;
    c->nseg = owner->nseg;
    c->stream = (hipStream_t)stream;
    set_opts(c, opts, v_epw);
    c->xi = owner->xi;
    c->w = owner->w;
    c->D = owner->D;
    c->vtx = owner->vtx;
    c->mesh_owner = owner;
    c->D64 = owner->D64;
    c->D32 = owner->D32;
    c->g64 = owner->g64;
    c->g32 = owner->g32;
    c->g16 = owner->g16;
    c->B = owner->B;
    c->perm = owner->perm;
    c->segptr = owner->segptr;
    c->segflag = owner->segflag;
    if ((rc = setup_state(c))) {
        nek_free(c);
        return rc;
    }
    *out = c;
    return NEK_OK;
}

}  // namespace nek

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
    case NEK_E_SCRATCH: return "vector larger than the static scratch of nek_ax_noalloc (32 MiB)";
    default: return "unknown status";
    }
}

void nek_free(nek_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->mesh_owner) {   // borrowed set-up data stays with its owner
        c->D64 = nullptr; c->D32 = nullptr; c->g64 = nullptr; c->g32 = nullptr; c->g16 = nullptr;
        c->B = nullptr; c->perm = nullptr; c->segptr = nullptr; c->segflag = nullptr;
    }
    dfree(c->D64); dfree(c->D32); dfree(c->g64); dfree(c->g32); dfree(c->g16); dfree(c->tri64); dfree(c->tri32); dfree(c->B);
    dfree(c->perm); dfree(c->segptr); dfree(c->segflag); dfree(c->sc); dfree(c->partials); dfree(c->hist);
    dfree(c->b); dfree(c->r64); dfree(c->p64); dfree(c->w64); dfree(c->d64); dfree(c->d32);
    dfree(c->r32); dfree(c->p32); dfree(c->w32); dfree(c->dg64); dfree(c->dg32);
    dfree(c->fdmS64); dfree(c->fdmL64); dfree(c->fdmC64); dfree(c->fdmS32); dfree(c->fdmL32); dfree(c->fdmC32);
    dfree(c->z64); dfree(c->z32);
    dfree(c->asmS64); dfree(c->asmL64); dfree(c->asmEll); dfree(c->asmCS); dfree(c->asmCL); dfree(c->asmS32);
    dfree(c->asmL32); dfree(c->asmU64); dfree(c->asmMom); dfree(c->asmEc); dfree(c->asmTmp); dfree(c->asmU32);
    dfree(c->xyz); dfree(c->gfeat); dfree(c->x0_X); dfree(c->x0_Y); dfree(c->x0_s);
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
    int v_epw = 0;
    if (const int rc0 = check_opts(N, opts, &v_epw)) return rc0;
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
    set_opts(c, opts, v_epw);

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
        dalloc(c->perm, perm.size()) || dalloc(c->segptr, segptr.size()) || dalloc(c->segflag, segflag.size()))
        return fail(NEK_E_OOM);
    // synchronous uploads: the host staging vectors die at return
    if (hipMemcpy(c->D64, c->D.data(), NP * NP * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->D32, D32.data(), NP * NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->g64, hg.data(), hg.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->B, hB.data(), hB.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->perm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->segptr, segptr.data(), segptr.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->segflag, segflag.data(), segflag.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(NEK_E_HIP);
    if ((rc = setup_state(c))) return fail(rc);
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
    case NEK_GET_DIAG: {
        const int rc = ensure_diag(c);
        return rc ? rc : d2h(o, c->dg64, (size_t)c->nl * sizeof(double));
    }
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

int nek_set_precond(nek_ctx *c, int precond)
{
    if (!c || precond < NEK_PC_NONE || precond > NEK_PC_SCHWARZ) return NEK_E_ARG;
    if (precond != NEK_PC_NONE) {
        const int rc = ensure_precond(c, precond);
        if (rc) return rc;
    }
    c->precond = precond;
    c->opts.precond = precond;
    return NEK_OK;
}

int nek_set_geometry(nek_ctx *c, int geom)
{
    if (!c || geom < NEK_GSRC_STORED || geom > NEK_GSRC_TRILINEAR) return NEK_E_ARG;
    if (geom == NEK_GSRC_TRILINEAR) {
        const int rc = ensure_tri(c);
        if (rc) return rc;
    }
    c->geom = geom;
    return NEK_OK;
}

int nek_set_max_workgroups(nek_ctx *c, int n)
{
    if (!c || n < 0 || n > MAXB || c->batch_member) return NEK_E_ARG;
    c->max_wg = n;
    return NEK_OK;
}

int nek_set_operator_kernel(nek_ctx *c, int kind)
{
    if (!c || (kind != NEK_OPERATOR_VALU && kind != NEK_OPERATOR_MFMA)) return NEK_E_ARG;
    if (kind == NEK_OPERATOR_MFMA && c->NP > 12) return NEK_E_ARG;
    c->op_kernel = kind;
    return NEK_OK;
}

int nek_set_schwarz_kernel(nek_ctx *c, int kind)
{
    if (!c || kind < NEK_SCHWARZ_AUTO || kind > NEK_SCHWARZ_VALU) return NEK_E_ARG;
    c->asm_kernel = kind;
    return NEK_OK;
}

int nek_set_update_kernel(nek_ctx *c, int kind)
{
    if (!c || kind < NEK_UPDATE_AUTO || kind > NEK_UPDATE_EXCHANGE) return NEK_E_ARG;
    c->upd_kernel = kind;
    return NEK_OK;
}

int nek_precond_apply(nek_ctx *c, const void *r, void *z, int dtype)
{
    if (!c || !r || !z || r == z || (dtype != NEK_F64 && dtype != NEK_F32)) return NEK_E_ARG;
    const size_t bytes = (size_t)c->nl * (dtype == NEK_F64 ? sizeof(double) : sizeof(float));
    if (c->precond == NEK_PC_FDM) {
        if (dtype == NEK_F64) return ops(c)->pc_fdm64(c, (const double *)r, (double *)z, c->P3(), red_grid(c), false, 0);
        return ops(c)->pc_fdm32(c, (const float *)r, (float *)z, c->P3(), red_grid(c), false, 0);
    }
    if (c->precond == NEK_PC_SCHWARZ) {
        if (dtype == NEK_F64) return ops(c)->pc_asm64(c, (const double *)r, (double *)z, c->P3(), red_grid(c), false, 0);
        return ops(c)->pc_asm32(c, (const float *)r, (float *)z, c->P3(), red_grid(c), false, 0);
    }
    HIP_TRY(hipMemcpyAsync(z, r, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (c->precond == NEK_PC_JACOBI) {
        if (dtype == NEK_F64) return ops(c)->pc_start64(c, (double *)z, c->dg64);
        return ops(c)->pc_start32(c, (float *)z, c->dg32);
    }
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
    if (!c || !u || !w || u == w || (dtype != NEK_F64 && dtype != NEK_F32)) return NEK_E_ARG;
    int rc;
    if (dtype == NEK_F64) {
        if ((rc = ensure_fp64_work(c))) return rc;
        return ops(c)->axa64(c, c->variant[NEK_PREC_FP64], (const double *)u, c->w64, (double *)w);
    }
    const int prec = c->prec == NEK_PREC_BF16G ? NEK_PREC_BF16G : NEK_PREC_FP32;
    if ((rc = ensure_g(c, prec))) return rc;
    if (dalloc(c->w32, c->nl)) return NEK_E_OOM;
    if (prec == NEK_PREC_BF16G) return ops(c)->axa16(c, c->variant[prec], (const float *)u, c->w32, (float *)w);
    return ops(c)->axa32(c, c->variant[prec], (const float *)u, c->w32, (float *)w);
}

int nek_ax_noalloc(nek_ctx *c, const void *u, void *w, int dtype)
{
    if (!c || !u || !w || u == w || (dtype != NEK_F64 && dtype != NEK_F32) || !c->noalloc_scratch) return NEK_E_ARG;
    const size_t bytes = (size_t)c->nl * (dtype == NEK_F64 ? sizeof(double) : sizeof(float));
    if (bytes > NEK_NOALLOC_SCRATCH_BYTES) return NEK_E_SCRATCH;
    if (dtype == NEK_F64) return ops(c)->axa64(c, c->variant[NEK_PREC_FP64], (const double *)u, (double *)c->noalloc_scratch,
                                               (double *)w);
    const int prec = c->prec == NEK_PREC_BF16G ? NEK_PREC_BF16G : NEK_PREC_FP32;
    const bool have = prec == NEK_PREC_BF16G ? c->g16 != nullptr
                    : c->geom == NEK_GSRC_TRILINEAR ? c->tri32 != nullptr : c->g32 != nullptr;
    if (!have) return NEK_E_ARG;   // the factor copy would have to be allocated
    float *sp = (float *)c->noalloc_scratch;
    if (prec == NEK_PREC_BF16G) return ops(c)->axa16(c, c->variant[prec], (const float *)u, sp, (float *)w);
    return ops(c)->axa32(c, c->variant[prec], (const float *)u, sp, (float *)w);
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

// Number of CG kernel configurations for this context's order.
int nek_num_variants(const nek_ctx *c)
{
    if (!c) return NEK_E_ARG;
    const NpOps *o = np_ops(c->NP);
    return o ? o->nvariants : NEK_E_ARG;
}

int nek_set_variant(nek_ctx *c, int prec, int variant)
{
    if (!c || prec < NEK_PREC_FP64 || prec > NEK_PREC_BF16G) return NEK_E_ARG;
    const int nv = nek_num_variants(c);
    if (variant < 0 || variant >= nv) return NEK_E_ARG;
    c->variant[prec] = variant;
    c->tuned[prec] = true;
    return NEK_OK;
}

int nek_get_variant(const nek_ctx *c, int prec, int *variant)
{
    if (!c || !variant || prec < NEK_PREC_FP64 || prec > NEK_PREC_BF16G) return NEK_E_ARG;
    *variant = c->variant[prec];
    return NEK_OK;
}

int nek_tune(nek_ctx *c, int prec, int iters, double *us_per_iter, int *best)
{
    if (!c || prec < NEK_PREC_FP64 || prec > NEK_PREC_BF16G || iters < 2) return NEK_E_ARG;
    int rc;
    if ((rc = ensure_fp64_work(c)) || (rc = ensure_g(c, prec)) || (rc = ensure_hist(c, iters + 1))) return rc;
    if (prec == NEK_PREC_FP64 ? dalloc(c->d64, c->nl)
                              : ((c->opts.corr_fp32 ? dalloc(c->d32, c->nl) : dalloc(c->d64, c->nl)) ||
                                 dalloc(c->r32, c->nl) || dalloc(c->p32, c->nl) || dalloc(c->w32, c->nl)))
        return NEK_E_OOM;
    void *xt = prec == NEK_PREC_FP64 ? (void *)c->d64 : inner_x(c);
    // synthetic SPD system: b = M dssum(1), x0 = 0
    if ((rc = fill<double>(c, c->w64, 1.0, c->nl)) || (rc = gather_launch(c, c->w64, c->b, false)) ||
        (rc = glsc3_to_slot(c, c->b, c->b, NEK_F64, 0)))
        return rc;
    const int nv = nek_num_variants(c);
    const int saved_prof = c->prof_every;
    c->prof_every = 0;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best_t = INFINITY;
    int best_v = c->variant[prec];
    for (int v = 0; v < nv && rc == NEK_OK; ++v) {
        float ms = 0;
        for (int rep = 0; rep < 2 && rc == NEK_OK; ++rep) {   // first pass warms up
            // the run starts as a solve does, through the preconditioner (if any)
            int rs = 1;
            if (prec == NEK_PREC_FP64) {
                HIP_TRY(hipMemcpyAsync(c->r64, c->b, c->nl * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
                if ((rc = glsc3_to_slot(c, c->r64, c->r64, NEK_F64, 1)) || (rc = fill<double>(c, c->d64, 0.0, c->nl)) ||
                    (rc = pc_start64(c, c->r64, &rs)))
                    break;
            } else {
                if ((rc = ops(c)->inner_start(c, c->b, c->r32, xt, !c->opts.corr_fp32))) break;
                if ((rc = red_final(c, 1)) || (rc = pc_start32(c, c->r32, &rs))) break;
            }
            if ((rc = start_launch(c, rs, 0, 0.0, iters, 0, 0.0, 1))) break;
            HIP_TRY(hipEventRecord(e0, c->stream));
            rc = run_cg(c, iters, [&](int it, bool final) -> int { return cg_iter(c, prec, v, it, final, xt); });
            HIP_TRY(hipEventRecord(e1, c->stream));
            HIP_TRY(hipEventSynchronize(e1));
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        }
        const double t = 1e3 * ms / iters;
        if (us_per_iter) us_per_iter[v] = t;
        if (t < best_t) {
            best_t = t;
            best_v = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof_every = saved_prof;
    if (rc) return rc;
    c->variant[prec] = best_v;
    c->tuned[prec] = true;
    if (best) *best = best_v;
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
    if ((rc = autotune_if_needed(c, c->prec))) return rc;
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
