// Launchers of the order-dependent kernels, instantiated once per order in
// nek_npNN.hip.  Internal header.
#pragma once
#include "nek_internal.hpp"

namespace nek {

template <int NP> struct OpsImpl {
    template <int EPW, int PD, typename T, typename GT, bool CG, typename XT = T, bool PC = false>
    static int launch_ax(nek_ctx *c, const T *src, T *p, T *w, const GT *g, const T *D, int it, XT *x = nullptr)
    {
        if constexpr (!CG && !TriOf<GT>::value && NP <= 12)
            if (c->op_kernel == NEK_OPERATOR_MFMA) {   // the D contractions on the matrix cores
                static const int occ = resident_per_cu((const void *)k_ax_mfma<NP, T, GT>, 256);
                const unsigned grid = (unsigned)std::min<long>(c->E, (long)occ * num_cu());
                hipLaunchKernelGGL((k_ax_mfma<NP, T, GT>), dim3(grid), dim3(256), 0, c->stream, src, w, g, D,
                                   (int)c->E);
                HIP_TRY(hipGetLastError());
                return NEK_OK;
            }
        constexpr int BS = EPW * NP * NP;
        const size_t shm = ax_lds_bytes<NP, EPW, T>();
        static bool attr_done = false;
        if (!attr_done) {
            if (shm > 65536)
                HIP_TRY(hipFuncSetAttribute((const void *)k_ax<NP, EPW, PD, T, GT, CG, XT, PC>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
            attr_done = true;
        }
        // the CG form writes one partial per workgroup, read by every workgroup
        // of the next kernel: a capped grid of persistent workgroups; the plain
        // operator reduces nothing and takes one element group per workgroup
        const unsigned grid = CG ? ax_grid(c, EPW, (int)sizeof(T)) : (unsigned)ax_groups(c, EPW);
        hipLaunchKernelGGL((k_ax<NP, EPW, PD, T, GT, CG, XT, PC>), dim3(grid), dim3(BS), shm, c->stream, src, p, w, g,
                           D, x, c->sc, c->P1(it), c->P1(it - 1), c->P2(it - 1), (int)grid, it, c->hist, (int)c->E,
                           ax_groups(c, EPW), c->P4(it - 1));
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }

    // CG iteration it (1-based): operator (+ the pending x update) and pAp
    // partials, then gather/update and rtr partials.  With final set, only
    // the operator kernel runs: it applies the last x update and publishes
    // the final state.  Sampled timing brackets every prof_every-th
    // iteration with events.
    template <typename T, typename GT, bool PC, typename XT>
    static int cg_iter_pc(nek_ctx *c, int variant, int it, bool final, XT *x, T *r, T *p, T *w, const GT *g,
                          const T *D, const T *dg)
    {
        return with_variant<NP, GT>(variant, [&](auto epw_c, auto pd_c) -> int {
            constexpr int EPW = decltype(epw_c)::value, PD = decltype(pd_c)::value;
            if (final) return launch_ax<EPW, PD, T, GT, true, XT, PC>(c, r, p, w, g, D, it, x);
            int slot = -1;
            if (c->prof_every > 0 && (c->prof_tick++ % c->prof_every) == 0) {
                if ((slot = prof_take(c)) < 0) return NEK_E_HIP;
                HIP_TRY(hipEventRecord(c->prof_pool[3 * slot], c->stream));
            }
            int rc = launch_ax<EPW, PD, T, GT, true, XT, PC>(c, r, p, w, g, D, it, x);
            if (rc) return rc;
            if (slot >= 0) HIP_TRY(hipEventRecord(c->prof_pool[3 * slot + 1], c->stream));
            const unsigned grid = ax_grid(c, EPW, (int)sizeof(T));
            if constexpr (PC)
                hipLaunchKernelGGL((k_cg_update_pc<NP, EPW, T>), dim3(grid), dim3(EPW * NP * NP), 0, c->stream, r, w,
                                   c->sc, c->P1(it), (int)grid, c->P2(it), it, c->box, (int)c->E, ax_groups(c, EPW), dg,
                                   c->P4(it));
            else
                hipLaunchKernelGGL((k_cg_update<NP, EPW, T>), dim3(grid), dim3(EPW * NP * NP), 0, c->stream, r, w,
                                   c->sc, c->P1(it), (int)grid, c->P2(it), it, c->box, (int)c->E, ax_groups(c, EPW),
                                   upd_xmin(c));
            HIP_TRY(hipGetLastError());
            if (slot >= 0) HIP_TRY(hipEventRecord(c->prof_pool[3 * slot + 2], c->stream));
            return NEK_OK;
        });
    }

    template <typename T>
    static int pc_fdm(nek_ctx *c, const T *r, T *z, double *P, unsigned grid, bool step, int it)
    {
        const T *m, *S, *L, *C;
        if constexpr (sizeof(T) == 8) {
            m = c->dg64; S = c->fdmS64; L = c->fdmL64; C = c->fdmC64;
        } else {
            m = c->dg32; S = c->fdmS32; L = c->fdmL32; C = c->fdmC32;
        }
        if (!m || !S || !L || !C) return NEK_E_ARG;
        hipLaunchKernelGGL((k_pc_fdm<NP, T>), dim3(grid), dim3(NP * NP), 0, c->stream, r, z, m, S, L, C, P, c->box,
                           (int)c->E, step ? c->sc : nullptr, it);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }
    static int pc_fdm64(nek_ctx *c, const double *r, double *z, double *P, unsigned grid, bool step, int it)
    {
        return pc_fdm<double>(c, r, z, P, grid, step, it);
    }
    static int pc_fdm32(nek_ctx *c, const float *r, float *z, double *P, unsigned grid, bool step, int it)
    {
        return pc_fdm<float>(c, r, z, P, grid, step, it);
    }

    // Two-level overlapping Schwarz: local window solves and element moments,
    // the coarse solve (one workgroup), then the gather of z with the
    // partials of glsc3(r, c, z) over `grid` workgroups.
    template <typename T>
    static int pc_asm(nek_ctx *c, const T *r, T *z, double *P, unsigned grid, bool step, int it)
    {
        constexpr int NW = NP + 2;
        const T *S, *L, *C;
        T *U;
        if constexpr (sizeof(T) == 8) {
            S = c->asmS64; L = c->asmL64; C = c->fdmC64; U = c->asmU64;
        } else {
            S = c->asmS32; L = c->asmL32; C = c->fdmC32; U = c->asmU32;
        }
        if (NP < 3 || !S || !L || !C || !U || !c->asmMom || !c->asmEc || !c->asmTmp) return NEK_E_ARG;
        const Scal *scp = step ? c->sc : nullptr;
        // persistent grid of exactly the workgroups that are resident at once
        // (a second, partial round would double the walk of the first)
        static const int occ_valu = resident_per_cu((const void *)k_asm_local<NP, T>, NW * NW);
        static const int occ_mfma = resident_per_cu((const void *)k_asm_local_mfma<NP, T>, 256);
        // measured on MI355X (16^3 and 32^3, N = 9): the matrix-core form is
        // 1.12-1.16x faster per application in FP64 and 0.92-0.95x in FP32
        const bool valu = c->asm_kernel == NEK_SCHWARZ_VALU || (c->asm_kernel == NEK_SCHWARZ_AUTO && sizeof(T) == 4);
        const unsigned lgrid = (unsigned)std::min<long>(c->E, (long)(valu ? occ_valu : occ_mfma) * num_cu());
        if (valu)
            hipLaunchKernelGGL((k_asm_local<NP, T>), dim3(lgrid), dim3(NW * NW), 0, c->stream, r, U, c->asmMom, S,
                               L, C, c->asmEll, c->box, (int)c->E, scp, it);
        else
            hipLaunchKernelGGL((k_asm_local_mfma<NP, T>), dim3(lgrid), dim3(256), 0, c->stream, r, U, c->asmMom, S,
                               L, C, c->asmEll, c->box, (int)c->E, scp, it);
        HIP_TRY(hipGetLastError());
        int rc = asm_coarse_launch(c, scp, it);
        if (rc) return rc;
        hipLaunchKernelGGL((k_asm_gather<NP, T>), dim3(grid), dim3(NP * NP), 0, c->stream, r, z, U, c->asmEc,
                           c->asmEll, P, c->box, (int)c->E, scp, it);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }
    static int pc_asm64(nek_ctx *c, const double *r, double *z, double *P, unsigned grid, bool step, int it)
    {
        return pc_asm<double>(c, r, z, P, grid, step, it);
    }
    static int pc_asm32(nek_ctx *c, const float *r, float *z, double *P, unsigned grid, bool step, int it)
    {
        return pc_asm<float>(c, r, z, P, grid, step, it);
    }

    // block preconditioner of the three-kernel iteration
    template <typename T>
    static int pc_block(nek_ctx *c, const T *r, T *z, double *P, unsigned grid, bool step, int it)
    {
        if (c->precond == NEK_PC_SCHWARZ) return pc_asm<T>(c, r, z, P, grid, step, it);
        return pc_fdm<T>(c, r, z, P, grid, step, it);
    }

    // Fast-diagonalization iteration: the operator kernel forms p = z + beta p
    // from the z vector, the gather/update kernel updates r and writes the
    // r.r partials to P4, the block-solve kernel forms z = M^-1 r and writes
    // the r.z partials to P2 (the prologue of the next operator kernel sums
    // both, as for the diagonal preconditioner).
    template <typename T, typename GT, typename XT>
    static int cg_iter_fdm(nek_ctx *c, int variant, int it, bool final, XT *x, T *r, T *p, T *w, const GT *g,
                           const T *D)
    {
        T *zb;
        if constexpr (sizeof(T) == 8) zb = c->z64;
        else zb = c->z32;
        if (!zb) return NEK_E_ARG;
        return with_variant<NP, GT>(variant, [&](auto epw_c, auto pd_c) -> int {
            constexpr int EPW = decltype(epw_c)::value, PD = decltype(pd_c)::value;
            if (final) return launch_ax<EPW, PD, T, GT, true, XT, true>(c, zb, p, w, g, D, it, x);
            int slot = -1;
            if (c->prof_every > 0 && (c->prof_tick++ % c->prof_every) == 0) {
                if ((slot = prof_take(c)) < 0) return NEK_E_HIP;
                HIP_TRY(hipEventRecord(c->prof_pool[3 * slot], c->stream));
            }
            int rc = launch_ax<EPW, PD, T, GT, true, XT, true>(c, zb, p, w, g, D, it, x);
            if (rc) return rc;
            if (slot >= 0) HIP_TRY(hipEventRecord(c->prof_pool[3 * slot + 1], c->stream));
            const unsigned grid = ax_grid(c, EPW, (int)sizeof(T));
            hipLaunchKernelGGL((k_cg_update<NP, EPW, T>), dim3(grid), dim3(EPW * NP * NP), 0, c->stream, r, w, c->sc,
                               c->P1(it), (int)grid, c->P4(it), it, c->box, (int)c->E, ax_groups(c, EPW), upd_xmin(c));
            HIP_TRY(hipGetLastError());
            if ((rc = pc_block<T>(c, r, zb, c->P2(it), grid, true, it))) return rc;
            if (slot >= 0) HIP_TRY(hipEventRecord(c->prof_pool[3 * slot + 2], c->stream));
            return NEK_OK;
        });
    }

    // With the diagonal preconditioner on, r holds z = M^-1 r and the update
    // kernel reads the diagonal of the vectors' precision.
    template <typename T, typename GT, typename XT>
    static int cg_iter(nek_ctx *c, int variant, int it, bool final, XT *x, T *r, T *p, T *w, const GT *g,
                       const T *D)
    {
        if (c->precond == NEK_PC_FDM || c->precond == NEK_PC_SCHWARZ)
            return cg_iter_fdm<T, GT, XT>(c, variant, it, final, x, r, p, w, g, D);
        if (c->precond) {
            const T *dg;
            if constexpr (sizeof(T) == 8) dg = c->dg64;
            else dg = c->dg32;
            if (!dg) return NEK_E_ARG;
            return cg_iter_pc<T, GT, true, XT>(c, variant, it, final, x, r, p, w, g, D, dg);
        }
        return cg_iter_pc<T, GT, false, XT>(c, variant, it, final, x, r, p, w, g, D, nullptr);
    }

    // 4-byte vectors with an FP64 (x64) or FP32 inner correction x
    template <typename GT>
    static int cg_iter4(nek_ctx *c, int v, int it, bool final, void *x, bool x64, float *r, float *p, float *w,
                        const GT *g, const float *D)
    {
        if (x64) return cg_iter<float, GT, double>(c, v, it, final, (double *)x, r, p, w, g, D);
        return cg_iter<float, GT, float>(c, v, it, final, (float *)x, r, p, w, g, D);
    }

    // FP64 and FP32 operators read the stored factors, or recompute them in
    // the kernel from the elements' trilinear coefficients (c->geom).
    static int cg_iter64(nek_ctx *c, int v, int it, bool final, double *x, double *r, double *p, double *w,
                         const double *g, const double *D)
    {
        if (c->geom == NEK_GSRC_TRILINEAR)
            return cg_iter<double, TriG<double>, double>(c, v, it, final, x, r, p, w, tri_ptr<double>(c), D);
        return cg_iter<double, double, double>(c, v, it, final, x, r, p, w, g, D);
    }
    static int cg_iter32(nek_ctx *c, int v, int it, bool final, void *x, bool x64, float *r, float *p, float *w,
                         const float *g, const float *D)
    {
        if (c->geom == NEK_GSRC_TRILINEAR)
            return cg_iter4<TriG<float>>(c, v, it, final, x, x64, r, p, w, tri_ptr<float>(c), D);
        return cg_iter4<float>(c, v, it, final, x, x64, r, p, w, g, D);
    }
    static int cg_iter16(nek_ctx *c, int v, int it, bool final, void *x, bool x64, float *r, float *p, float *w,
                         const uint16_t *g, const float *D)
    {
        return cg_iter4<uint16_t>(c, v, it, final, x, x64, r, p, w, g, D);
    }

    static int ax64(nek_ctx *c, const double *u, double *w)
    {
        if (c->geom == NEK_GSRC_TRILINEAR)
            return launch_ax<epw_for(NP), pd_for<double>(), double, TriG<double>, false>(c, u, nullptr, w,
                                                                                         tri_ptr<double>(c), c->D64, 0);
        return launch_ax<epw_for(NP), pd_for<double>(), double, double, false>(c, u, nullptr, w, c->g64, c->D64, 0);
    }
    static int ax32(nek_ctx *c, const float *u, float *w)
    {
        if (c->geom == NEK_GSRC_TRILINEAR)
            return launch_ax<epw_for(NP), pd_for<float>(), float, TriG<float>, false>(c, u, nullptr, w,
                                                                                      tri_ptr<float>(c), c->D32, 0);
        return launch_ax<epw_for(NP), pd_for<float>(), float, float, false>(c, u, nullptr, w, c->g32, c->D32, 0);
    }
    static int ax16(nek_ctx *c, const float *u, float *w)
    {
        return launch_ax<epw_for(NP), pd_for<uint16_t>(), float, uint16_t, false>(c, u, nullptr, w, c->g16, c->D32,
                                                                                  0);
    }

    // w = M dssum(A_L u): operator into scratch, then the out-of-place
    // column assembly, both in the configuration `variant`.
    template <typename T, typename GT>
    static int ax_assembled(nek_ctx *c, int variant, const T *u, T *scratch, T *w, const GT *g, const T *D)
    {
        return with_variant<NP, GT>(variant, [&](auto epw_c, auto pd_c) -> int {
            constexpr int EPW = decltype(epw_c)::value, PD = decltype(pd_c)::value;
            int rc = launch_ax<EPW, PD, T, GT, false>(c, u, nullptr, scratch, g, D, 0);
            if (rc) return rc;
            // the assembly in its own element groups; the exchange form on a
            // capped grid when every workgroup walks enough elements (the
            // choice of nek_set_update_kernel)
            constexpr int EA = asm_epw(NP);
            const int groups = ax_groups(c, EA);
            const unsigned cap = ax_grid(c, EA, (int)sizeof(T));
            if ((long)c->E >= (long)upd_xmin(c, true) * cap) {
                hipLaunchKernelGGL((k_assemble_x<NP, EA, T>), dim3(cap), dim3(EA * NP * NP), 0, c->stream, scratch,
                                   w, c->box, (int)c->E, groups);
                HIP_TRY(hipGetLastError());
                return NEK_OK;
            }
            hipLaunchKernelGGL((k_assemble<NP, EA, T>), dim3(groups), dim3(EA * NP * NP), 0, c->stream, scratch, w,
                               c->box, (int)c->E, groups);
            HIP_TRY(hipGetLastError());
            return NEK_OK;
        });
    }
    static int axa64(nek_ctx *c, int v, const double *u, double *scratch, double *w)
    {
        if (c->geom == NEK_GSRC_TRILINEAR)
            return ax_assembled<double, TriG<double>>(c, v, u, scratch, w, tri_ptr<double>(c), c->D64);
        return ax_assembled<double, double>(c, v, u, scratch, w, c->g64, c->D64);
    }
    static int axa32(nek_ctx *c, int v, const float *u, float *scratch, float *w)
    {
        if (c->geom == NEK_GSRC_TRILINEAR)
            return ax_assembled<float, TriG<float>>(c, v, u, scratch, w, tri_ptr<float>(c), c->D32);
        return ax_assembled<float, float>(c, v, u, scratch, w, c->g32, c->D32);
    }
    static int axa16(nek_ctx *c, int v, const float *u, float *scratch, float *w)
    {
        return ax_assembled<float, uint16_t>(c, v, u, scratch, w, c->g16, c->D32);
    }

    static int gather64(nek_ctx *c, const double *in, double *out, bool weighted)
    {
        if (weighted)
            hipLaunchKernelGGL((k_gather<NP, double, true>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, in, out,
                               c->box, (unsigned)c->nl);
        else
            hipLaunchKernelGGL((k_gather<NP, double, false>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, in, out,
                               c->box, (unsigned)c->nl);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }

    static int glsc3_64(nek_ctx *c, const double *a, const double *b)
    {
        hipLaunchKernelGGL((k_glsc3<NP, double, double>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, a, b,
                           c->P3(), c->box, (unsigned)c->nl);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }
    static int glsc3_32(nek_ctx *c, const float *a, const float *b)
    {
        hipLaunchKernelGGL((k_glsc3<NP, float, float>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, a, b, c->P3(),
                           c->box, (unsigned)c->nl);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }

    static int resid(nek_ctx *c, const double *b, const double *w, double *r)
    {
        hipLaunchKernelGGL((k_resid<NP>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, b, w, r, c->P3(), c->box,
                           (unsigned)c->nl);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }

    template <typename T> static int pc_start(nek_ctx *c, T *r, const T *m)
    {
        hipLaunchKernelGGL((k_pc_start<NP, T>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, r, m, c->P3(), c->box,
                           (unsigned)c->nl);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }
    static int pc_start64(nek_ctx *c, double *r, const double *m) { return pc_start<double>(c, r, m); }
    static int pc_start32(nek_ctx *c, float *r, const float *m) { return pc_start<float>(c, r, m); }

    static int inner_start(nek_ctx *c, const double *r64, float *r32, void *d, bool d64)
    {
        if (d64)
            hipLaunchKernelGGL((k_inner_start<NP, double>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, r64, r32,
                               (double *)d, c->P3(), c->box, (unsigned)c->nl);
        else
            hipLaunchKernelGGL((k_inner_start<NP, float>), dim3(red_grid(c)), dim3(UPD_BS), 0, c->stream, r64, r32,
                               (float *)d, c->P3(), c->box, (unsigned)c->nl);
        HIP_TRY(hipGetLastError());
        return NEK_OK;
    }

    static int variant_epw(int v)
    {
        return with_variant<NP, double>(v, [](auto epw_c, auto) -> int { return decltype(epw_c)::value; });
    }

    template <typename T, typename GT, typename XT>
    static int batch_iter_t(hipStream_t s, int v, const BatchProb *tab, const int2 *owner, unsigned grid, const T *D,
                            int it_local, const int *base, bool final, bool prepare)
    {
        return with_variant<NP, GT>(v, [&](auto epw_c, auto pd_c) -> int {
            constexpr int EPW = decltype(epw_c)::value, PD = decltype(pd_c)::value, BS = EPW * NP * NP;
            const size_t shm = ax_lds_bytes<NP, EPW, T>();
            if (prepare) {
                if (shm > 65536)
                    HIP_TRY(hipFuncSetAttribute((const void *)k_ax_batch<NP, EPW, PD, T, GT, XT>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
                return NEK_OK;
            }
            hipLaunchKernelGGL((k_ax_batch<NP, EPW, PD, T, GT, XT>), dim3(grid), dim3(BS), shm, s, tab, owner, D,
                               it_local, base);
            HIP_TRY(hipGetLastError());
            if (!final) {
                hipLaunchKernelGGL((k_cg_update_batch<NP, EPW, T>), dim3(grid), dim3(BS), 0, s, tab, owner, it_local,
                                   base);
                HIP_TRY(hipGetLastError());
            }
            return NEK_OK;
        });
    }

    static int batch_iter(hipStream_t s, int prec, int v, bool x64, const BatchProb *tab, const int2 *owner,
                          unsigned grid, const void *D, int it_local, const int *base, bool final, bool prepare)
    {
        const float *D32 = (const float *)D;
        if (prec == NEK_PREC_FP64)
            return batch_iter_t<double, double, double>(s, v, tab, owner, grid, (const double *)D, it_local, base,
                                                        final, prepare);
        if (prec == NEK_PREC_BF16G)
            return x64 ? batch_iter_t<float, uint16_t, double>(s, v, tab, owner, grid, D32, it_local, base, final,
                                                               prepare)
                       : batch_iter_t<float, uint16_t, float>(s, v, tab, owner, grid, D32, it_local, base, final,
                                                              prepare);
        return x64 ? batch_iter_t<float, float, double>(s, v, tab, owner, grid, D32, it_local, base, final, prepare)
                   : batch_iter_t<float, float, float>(s, v, tab, owner, grid, D32, it_local, base, final, prepare);
    }
};

template <int NP> const NpOps *make_np_ops()
{
    using I = OpsImpl<NP>;
    static const NpOps ops{n_variants<NP>(), &I::cg_iter64, &I::cg_iter32, &I::cg_iter16, &I::ax64, &I::ax32,
                           &I::ax16, &I::axa64, &I::axa32, &I::axa16, &I::gather64, &I::glsc3_64, &I::glsc3_32, &I::resid, &I::pc_start64, &I::pc_start32, &I::pc_fdm64, &I::pc_fdm32, &I::pc_asm64, &I::pc_asm32,
                           &I::inner_start,
                           &I::variant_epw, &I::batch_iter};
    return &ops;
}

}  // namespace nek

// One translation unit per order: nek_npNN.hip expands this.
#define NEK_DEFINE_NP_OPS(NPV) \
    namespace nek { const NpOps *np_ops_##NPV() { return make_np_ops<NPV>(); } }
