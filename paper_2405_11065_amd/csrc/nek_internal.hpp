// Internal declarations shared by libnek's translation units: the context,
// launch-configuration rules, and the per-order function table through which
// the order-independent driver reaches the kernels instantiated for each
// N + 1 = NP in its own translation unit (nek_npNN.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <type_traits>
#include <vector>

#include "nek.h"
#include "nek_kernels.hpp"

namespace nek {

constexpr int MAX_NP = 16;        // N <= 15
constexpr int CHUNK_ITERS = 16;   // CG iterations enqueued between flag polls

#define HIP_TRY(expr)                                            \
    do {                                                         \
        if ((expr) != hipSuccess) return NEK_E_HIP;              \
    } while (0)


// Slices of geometric factors in flight per thread (register budget:
// 12 / 6 / 3 VGPRs per slice for FP64 / FP32 / BF16 storage).
template <typename GT> constexpr int pd_for() { return sizeof(GT) == 8 ? 2 : sizeof(GT) == 4 ? 4 : 6; }
template <typename GT> constexpr int pd_alt() { return sizeof(GT) == 8 ? 1 : sizeof(GT) == 4 ? 2 : 3; }

// Run-time configurations of the CG kernel pair (the autotuner's search
// space): variant v = 2 * ke + kp picks the ke-th EPW option and the default
// (kp = 0) or alternative (kp = 1) prefetch depth.  Orders used by the
// batched and benchmarked workloads (NP = 6, 8, 10, 12) have several EPW
// options; the others have one.
template <int NP> constexpr int n_epw_opts() { return NP == 6 || NP == 8 || NP == 10 ? 3 : NP == 12 ? 2 : 1; }
template <int NP> constexpr int epw_opt(int k)
{
    return k == 0 ? epw_for(NP)
         : NP == 6 ? (k == 1 ? 4 : 16)
         : NP == 8 ? (k == 1 ? 2 : 1)
         : NP == 10 ? (k == 1 ? 2 : 1)
         : NP == 12 ? 1 : epw_for(NP);
}
template <int NP> constexpr int n_variants() { return 2 * n_epw_opts<NP>(); }

template <int V> using IC = std::integral_constant<int, V>;

// Calls f(IC<EPW>, IC<PD>) for variant v of order NP and storage GT.
template <int NP, typename GT, typename F> int with_variant(int v, F &&f)
{
    constexpr int P0 = pd_for<GT>(), P1 = pd_alt<GT>();
    switch (v) {
    case 0: return f(IC<epw_opt<NP>(0)>{}, IC<P0>{});
    case 1: return f(IC<epw_opt<NP>(0)>{}, IC<P1>{});
    case 2: if constexpr (n_epw_opts<NP>() > 1) return f(IC<epw_opt<NP>(1)>{}, IC<P0>{}); break;
    case 3: if constexpr (n_epw_opts<NP>() > 1) return f(IC<epw_opt<NP>(1)>{}, IC<P1>{}); break;
    case 4: if constexpr (n_epw_opts<NP>() > 2) return f(IC<epw_opt<NP>(2)>{}, IC<P0>{}); break;
    case 5: if constexpr (n_epw_opts<NP>() > 2) return f(IC<epw_opt<NP>(2)>{}, IC<P1>{}); break;
    default: break;
    }
    return NEK_E_ARG;
}

int num_cu();

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

}  // namespace nek

struct nek_ctx {
    int N = 0, NP = 0;
    int nel[3] = {0, 0, 0};
    long E = 0, nl = 0, ng = 0, nperm = 0, nseg = 0;
    nek::Box box{};
    hipStream_t stream = nullptr;
    nek_opts opts{};
    int prec = NEK_PREC_FP64;
    int variant[3] = {0, 0, 0};   // CG kernel configuration per precision (nek_tune)
    bool tuned[3] = {false, false, false};   // configuration fixed (else the next solve autotunes)
    int max_wg = 0;               // cap on persistent / reduction workgroups (0: default)
    int ax_wg = 0;                // cap on the CG kernels' persistent grid alone (0: none): a batch
                                  // divides the grid among the problems on one mesh
    bool batch_member = false;    // owned by a batch, which lays out its grid once
    // set-up data borrowed from another context of the same mesh and order
    // (batch members with identical meshes): D*, g*, B and the segment maps
    // point into mesh_owner's buffers, which outlive this context
    nek_ctx *mesh_owner = nullptr;
    void *noalloc_scratch = nullptr;   // this device's static scratch of nek_ax_noalloc

    std::vector<double> xi, w, D, vtx;

    // device data; g* are stored per point: [E][NP^3][6]
    double *D64 = nullptr;
    float *D32 = nullptr;
    double *g64 = nullptr;
    float *g32 = nullptr;
    uint16_t *g16 = nullptr;
    // NEK_GSRC_TRILINEAR: the operator kernels recompute the factors from
    // per-element trilinear coefficients (header + [E][24], FP64 and FP32)
    int geom = 0;
    double *tri64 = nullptr;
    float *tri32 = nullptr;
    double *B = nullptr;
    int32_t *perm = nullptr, *segptr = nullptr;
    int8_t *segflag = nullptr;
    nek::Scal *sc = nullptr;
    double *partials = nullptr;   // 7 regions of MAXB doubles
    int precond = 0;              // 1: diagonal (Jacobi) preconditioner in the CG loop
    int asm_kernel = NEK_SCHWARZ_AUTO;   // Schwarz window solves: matrix cores or vector ALUs
    int op_kernel = NEK_OPERATOR_VALU;   // plain operator pass (nek_ax_local, nek_ax): D contractions
    int upd_kernel = NEK_UPDATE_AUTO;    // CG update kernel: x-face copies gathered or exchanged in LDS
    double *dg64 = nullptr;       // assembled diagonal, 1 on Dirichlet nodes
    float *dg32 = nullptr;        // its FP32 rounding (mixed inner solves)
    // fast-diagonalization preconditioner: 1-D interior modes S [(N-1)^2],
    // lambda [N-1], element factors [3 E]; the preconditioned residual z of
    // the FP64 loop and of the inner FP32 loop
    double *fdmS64 = nullptr, *fdmL64 = nullptr, *fdmC64 = nullptr;
    float *fdmS32 = nullptr, *fdmL32 = nullptr, *fdmC32 = nullptr;
    double *z64 = nullptr;
    float *z32 = nullptr;
    // two-level overlapping Schwarz: padded window modes [4][NW][NW], their
    // lambda [4][NW] (FP64 and FP32), GLL interpolation weights [2][NP], the
    // coarse modes per direction (FP64: S at asmCoff[d], lambda at asmCloff[d]),
    // the window solutions [E][NW^3], element moments [E][8], the coarse
    // correction on the vertex lattice and two coarse scratch vectors
    double *asmS64 = nullptr, *asmL64 = nullptr, *asmEll = nullptr, *asmCS = nullptr, *asmCL = nullptr;
    float *asmS32 = nullptr, *asmL32 = nullptr;
    int asmCoff[3] = {0, 0, 0}, asmCloff[3] = {0, 0, 0};
    double *asmU64 = nullptr, *asmMom = nullptr, *asmEc = nullptr, *asmTmp = nullptr;
    float *asmU32 = nullptr;
    double *hist = nullptr;
    long hist_cap = 0;
    // work vectors
    double *b = nullptr, *r64 = nullptr, *p64 = nullptr, *w64 = nullptr;
    double *d64 = nullptr;   // iterate of FP64 autotuning runs; FP64 correction of inner solves
    float *d32 = nullptr;    // FP32 correction of inner solves (opts.corr_fp32)
    float *r32 = nullptr, *p32 = nullptr, *w32 = nullptr;
    int *hflags = nullptr;   // pinned; [0] mirrors the run's done flag (written by its kernels)
    hipEvent_t ev[2] = {nullptr, nullptr};
    // learned initial guess (nek_x0_*, nek_grf): node coordinates [E][3][NP^3]
    // and per-element network buffers
    double *xyz = nullptr;
    double *gfeat = nullptr;
    int gfeat_cap = 0;
    uint16_t *x0_X = nullptr;
    float *x0_Y = nullptr;
    double *x0_s = nullptr;
    long x0_ldx = 0, x0_ldy = 0;
    // sampled kernel timing (nek_prof_*)
    int prof_every = 0;
    long prof_tick = 0;
    std::vector<hipEvent_t> prof_pool;
    std::vector<int> prof_pending;     // event triples awaiting resolution
    double prof_ms[2] = {0, 0};
    long prof_n[2] = {0, 0};

    // partials: operator pAp and update rtz (rtr without a preconditioner),
    // each double-buffered by iteration parity, one region for standalone
    // reductions, then the update's rtr of preconditioned runs
    double *P1(int it) { return partials + (it & 1) * nek::MAXB; }
    double *P2(int it) { return partials + (2 + (it & 1)) * nek::MAXB; }
    double *P3() { return partials + 4 * nek::MAXB; }
    double *P4(int it) { return partials + (5 + (it & 1)) * nek::MAXB; }
};

namespace nek {

inline unsigned red_grid(const nek_ctx *c)
{
    long want = (c->nl + UPD_BS - 1) / UPD_BS;
    long cap = std::min<long>(MAXB / 2, c->max_wg > 0 ? (long)c->max_wg : 4L * num_cu());
    return (unsigned)std::max<long>(1, std::min(want, cap));
}

inline int ax_groups(const nek_ctx *c, int epw) { return (int)((c->E + epw - 1) / epw); }

// When the update kernel (fewest element groups per workgroup) and the
// assembly pass of nek_ax (fewest elements per workgroup) take the exchange
// form (nek_set_update_kernel).
inline int upd_xmin(const nek_ctx *c, bool assembly = false)
{
    if (c->upd_kernel == NEK_UPDATE_GATHER) return INT_MAX;
    if (c->upd_kernel == NEK_UPDATE_EXCHANGE) return 0;
    return assembly ? ASM_X_MIN_ELEMENTS : UPD_X_MIN_GROUPS;
}

// Workgroups of `kernel` (block threads, static LDS only) resident on one
// compute unit at once, at least 1.
inline int resident_per_cu(const void *kernel, int threads)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

// Trilinear-coefficient buffer of the vectors' type, as the operator's tag type.
template <typename T> inline const TriG<T> *tri_ptr(const nek_ctx *c)
{
    if constexpr (sizeof(T) == 8) return reinterpret_cast<const TriG<T> *>(c->tri64);
    else return reinterpret_cast<const TriG<T> *>(c->tri32);
}

inline unsigned ax_grid(const nek_ctx *c, int epw, int vbytes)
{
    long want = ax_groups(c, epw);
    // FP64 with in-kernel factors: half the workgroups, each with twice the
    // groups (16^3 N=9 CG: 105 -> 95 us per iteration; FP32 is slower so)
    const bool half = c->geom == NEK_GSRC_TRILINEAR && vbytes == 8;
    long cap = std::min<long>(MAXB, c->max_wg > 0 ? (long)c->max_wg : (half ? 4L : 8L) * num_cu());
    if (c->ax_wg > 0) cap = std::min<long>(cap, c->ax_wg);
    return (unsigned)std::max<long>(1, std::min(want, cap));
}

// Index of a free event triple for sampled timing (creates events as needed).
int prof_take(nek_ctx *c);

// Kernels instantiated for one order; every entry enqueues on c->stream and
// returns a nek_status.  Reductions leave per-workgroup partials in c->P3().
struct NpOps {
    int nvariants;
    // one CG iteration (final: only the closing operator launch); the
    // iterate x has the type of the vectors
    int (*cg_iter64)(nek_ctx *, int variant, int it, bool final, double *x, double *r, double *p, double *w,
                     const double *g, const double *D);
    // 4-byte vectors: x is the inner correction, FP64 (x64) or FP32
    int (*cg_iter32)(nek_ctx *, int variant, int it, bool final, void *x, bool x64, float *r, float *p, float *w,
                     const float *g, const float *D);
    int (*cg_iter16)(nek_ctx *, int variant, int it, bool final, void *x, bool x64, float *r, float *p, float *w,
                     const uint16_t *g, const float *D);
    // w = A_L u
    int (*ax64)(nek_ctx *, const double *u, double *w);
    int (*ax32)(nek_ctx *, const float *u, float *w);
    int (*ax16)(nek_ctx *, const float *u, float *w);
    // w = M dssum(A_L u) through scratch, in configuration v
    int (*axa64)(nek_ctx *, int v, const double *u, double *scratch, double *w);
    int (*axa32)(nek_ctx *, int v, const float *u, float *scratch, float *w);
    int (*axa16)(nek_ctx *, int v, const float *u, float *scratch, float *w);
    // out = M o sum of copies (weighted by c when weighted)
    int (*gather64)(nek_ctx *, const double *in, double *out, bool weighted);
    // partials of glsc3(a, c, b)
    int (*glsc3_64)(nek_ctx *, const double *a, const double *b);
    int (*glsc3_32)(nek_ctx *, const float *a, const float *b);
    // r = b - M dssum(w), partials of glsc3(r, c, r)
    int (*resid)(nek_ctx *, const double *b, const double *w, double *r);
    // r -> z = r / m in place, partials of glsc3(r, c, z)
    int (*pc_start64)(nek_ctx *, double *r, const double *m);
    int (*pc_start32)(nek_ctx *, float *r, const float *m);
    // z = M^-1 r (fast diagonalization), partials of glsc3(r, c, z) in P;
    // with step set, as the third kernel of CG iteration it
    int (*pc_fdm64)(nek_ctx *, const double *r, double *z, double *P, unsigned grid, bool step, int it);
    int (*pc_fdm32)(nek_ctx *, const float *r, float *z, double *P, unsigned grid, bool step, int it);
    // z = M^-1 r (two-level overlapping Schwarz), partials of glsc3(r, c, z)
    // in P over `grid` workgroups; with step set, as a CG step of iteration it
    int (*pc_asm64)(nek_ctx *, const double *r, double *z, double *P, unsigned grid, bool step, int it);
    int (*pc_asm32)(nek_ctx *, const float *r, float *z, double *P, unsigned grid, bool step, int it);
    // r32 = (float) r64, d = 0 (FP64 when d64, else FP32), partials of glsc3(r32, c, r32)
    int (*inner_start)(nek_ctx *, const double *r64, float *r32, void *d, bool d64);
    // elements per workgroup of a CG variant
    int (*variant_epw)(int variant);
    // Batched CG iteration base + it_local of every active problem in tab
    // (operator, then gather/update unless final) on stream s; with prepare
    // set, only configures the kernels (call before any graph capture).
    // x64: the iterates of 4-byte runs are FP64 corrections.
    int (*batch_iter)(hipStream_t s, int prec, int variant, bool x64, const BatchProb *tab, const int2 *owner,
                      unsigned grid, const void *D, int it_local, const int *base, bool final, bool prepare);
};

const NpOps *np_ops(int NP);
const NpOps *ops(const nek_ctx *c);

// ---------------------------------------------- driver steps (nek_lib.hip)

int ensure_hist(nek_ctx *c, long need);
int ensure_g(nek_ctx *c, int prec);
// A context on owner's mesh and order that shares its read-only set-up data
// (the options validated as nek_setup does); its own CG state and vectors.
int setup_shared(nek_ctx *owner, const nek_opts *opts, void *stream, nek_ctx **out);
int ensure_fp64_work(nek_ctx *c);
int ensure_mixed_work(nek_ctx *c);
int fill_f64(nek_ctx *c, double *p, double v, unsigned long n);
int red_final(nek_ctx *c, int slot);
int glsc3_to_slot(nek_ctx *c, const void *a, const void *b, int dtype, int slot);
int gather_launch(nek_ctx *c, const double *in, double *out, bool weighted);
int start_launch(nek_ctx *c, int rslot, int hist_off, double stop_tol, int maxit, int stop_on_initial,
                 double rtz_prev = 0.0, int rtr_slot = -1);
// Preconditioned runs: red[2] = glsc3(r, c, z) with z = M^-1 r, in place
// (diagonal: r64 with the FP64 diagonal, r32 with the FP32 one) or into z64
// / z32 (fast diagonalization); no-op without a preconditioner.  Returns the
// red slot of the run's rtz (2, or 1).
int pc_start64(nek_ctx *c, double *r, int *rtz_slot);
int pc_start32(nek_ctx *c, float *r, int *rtz_slot);
int ensure_diag(nek_ctx *c);
int ensure_fdm(nek_ctx *c);
int ensure_schwarz(nek_ctx *c);
// the coarse solve of the Schwarz preconditioner (one workgroup), from the
// element moments to the correction on the vertex lattice
int asm_coarse_launch(nek_ctx *c, const Scal *sc, int it);
int ensure_tri(nek_ctx *c);
// the inner correction of a mixed solve (FP64 unless opts.corr_fp32)
inline void *inner_x(nek_ctx *c) { return c->opts.corr_fp32 ? (void *)c->d32 : (void *)c->d64; }
// configuration of the CG pair for opts.elts_per_wg > 0 (-1 if none)
int variant_for_epw(int NP, int epw);
// opts.elts_per_wg == 0 and no configuration fixed yet at prec: autotune
int autotune_if_needed(nek_ctx *c, int prec);
// true relative residual of x (FP64 operator and gather); red[1] = its r.r
int true_residual(nek_ctx *c, const double *x, double bb, double *rho);
int cg_prologue(nek_ctx *c, const double *f, const double *x0, double *x, double *r);
int ax_local_launch(nek_ctx *c, const void *u, void *w, int dtype, int prec);
int resid_launch(nek_ctx *c, const double *b, const double *w, double *r, int slot);
int read_scal(nek_ctx *c, Scal &h);
int finish_status(const IterState &s, double tol);
int batch_advance_launch(hipStream_t s, int *base, int step);
int batch_alldone_launch(hipStream_t s, Scal *const *scs, int nprob, int *out);
int fill_i32(hipStream_t s, int *p, int v, unsigned long n);

// Control state of one mixed-precision (iterative refinement) solve; the
// solo and batched solvers drive it through the same steps.
struct IrCtl {
    // rtz_last: rtz of the residual before the last one of the previous inner
    // run (denominator of the resumed beta in reliable-update mode)
    double bb = 0, rho = 0, rho_prev = 0, tau = 0, rtz_last = 0, last_rec = 0;
    int total = 0, outer = 0, fp64_iters = 0, status = NEK_OK, inner_cap = 0, max_outer = 0;
    bool keep_p = false, finished = false;
};
enum IrStep { IR_DONE, IR_FALLBACK, IR_INNER };
void ir_init(const nek_ctx *c, IrCtl &s);
void ir_start(IrCtl &s, const Scal &h);
IrStep ir_decide(IrCtl &s, const nek_ctx *c, double tol, int maxit);
int ir_fallback(nek_ctx *c, IrCtl &s, double tol, int maxit, double *x);
int ir_inner_launch(nek_ctx *c, IrCtl &s, double tol, int maxit, int *cap);
int ir_inner_done(nek_ctx *c, IrCtl &s, const Scal &h, double *x);
void ir_outer_done(IrCtl &s, const Scal &h);
void ir_stats(const IrCtl &s, nek_stats *st);

}  // namespace nek
