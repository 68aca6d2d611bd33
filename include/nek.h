/*
 * nek.h -- C ABI of libnek, an MI355X (gfx950) implementation of the
 * conjugate-gradient solve of the spectral-element Poisson problem that the
 * Nekbone mini-app runs (Chen, de Oliveira Castro, Bientinesi, Iakymchuk,
 * "Enabling mixed-precision with the help of tools: A Nekbone case study").
 *
 * Problem.  A box of nel[0] x nel[1] x nel[2] trilinear hexahedra, polynomial
 * order N on Gauss-Lobatto-Legendre (GLL) points, homogeneous Dirichlet
 * conditions on the six outer faces.  The matrix-free operator is the one the
 * paper's Fig. 2 call graph evaluates: local_grad3 (derivatives along r, s, t
 * with the 1-D GLL matrix D), the six geometric factors g1..g6, local_grad3_t,
 * followed by gather-scatter (dssum) and the Dirichlet mask.
 *
 * Vector layout.  Every vector is an element-local ("duplicated") vector of
 * n_local = E (N+1)^3 entries, index l = e (N+1)^3 + i + (N+1)(j + (N+1) k),
 * e = ex + nel0 (ey + nel1 ez).  Copies of a shared node hold equal values
 * in a continuous vector.
 *
 * Pointers.  Vector arguments are DEVICE pointers owned by the caller; the
 * library never frees them and keeps none after a call returns.  Scalars,
 * statistics, histories and nek_get outputs are HOST pointers.
 *
 * Streams.  All work of a context is enqueued on the hipStream_t given to
 * nek_setup (NULL = the default stream).  nek_ax, nek_ax_local and nek_dssum
 * return without synchronising; nek_glsc3, nek_get and the solvers
 * synchronise before they return.
 *
 * Errors.  Every call returns a nek_status; nothing throws across the ABI.
 * Negative values are errors (the context stays usable unless the value is
 * NEK_E_HIP); NEK_NOCONV is a warning (x holds the last iterate).
 * nek_strerror gives a static message.  Calls on one context must not
 * overlap (one host thread at a time per context).
 */
#ifndef NEK_H
#define NEK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nek_ctx nek_ctx;

typedef enum {
    NEK_OK = 0,
    NEK_NOCONV = 1,          /* warning: maxit reached before tol           */
    NEK_E_ARG = -1,          /* bad argument (NULL, size, unsupported N)    */
    NEK_E_HIP = -2,          /* a HIP runtime call failed                   */
    NEK_E_OOM = -3,          /* device or host allocation failed            */
    NEK_E_JACOBIAN = -4,     /* det J <= 0 somewhere: inverted element      */
    NEK_E_BREAKDOWN = -5,    /* CG breakdown: p.Ap <= 0                     */
    NEK_E_NONFINITE = -6,    /* a NaN or Inf reached a reduction            */
    NEK_E_STAGNATION = -7,   /* mixed refinement stopped reducing and the
                                FP64 fallback was disabled                  */
    NEK_E_SCRATCH = -8       /* nek_ax_noalloc: the vector exceeds the static
                                scratch (NEK_NOALLOC_SCRATCH_BYTES)          */
} nek_status;

/* Operator precision of a context's solves. */
typedef enum {
    NEK_PREC_FP64 = 0,       /* FP64 vectors, FP64 g                                   */
    NEK_PREC_FP32 = 1,       /* mixed: FP32 p/w/r and FP32 g inside FP64 refinement    */
    NEK_PREC_BF16G = 2       /* mixed: as FP32, g1..g6 stored as BF16 (RNE from FP64)  */
} nek_prec;

/* Element type of the vectors passed to nek_ax / nek_ax_local / nek_dssum /
 * nek_glsc3. */
typedef enum { NEK_F64 = 0, NEK_F32 = 1 } nek_dtype;

typedef struct {
    int nel[3];              /* elements per direction, each >= 1             */
    double lo[3], hi[3];     /* box corners, used when vtx == NULL            */
    const double *vtx;       /* optional host array [(nel0+1)(nel1+1)(nel2+1)][3],
                                vertex lattice, x-index fastest; NULL = uniform
                                lattice on [lo, hi]                           */
} nek_mesh;

typedef struct {
    int prec;                /* nek_prec of nek_cg_solve                                */
    double inner_tol;        /* mixed: residual reduction of each inner run before the
                                next FP64 true-residual update; 0 = the default of
                                the refinement mode: reliable update 1e-2 (FP32 g) or
                                0.3 (BF16 g); restarted 1e-4 (FP32 g) or 1e-2 (BF16 g) */
    int inner_maxit;         /* mixed: inner iteration cap per refinement step; 0 = 4000 */
    int max_outer;           /* mixed: refinement steps cap; 0 = 30                      */
    int fp64_fallback;       /* mixed: 1 = when a refinement step fails to halve the
                                true residual, finish with FP64 CG from the current x  */
    int elts_per_wg;         /* configuration of the CG kernel pair:
                                 0 = autotune: the first solve at each precision times
                                     every configuration on the context's mesh (as
                                     nek_tune with 20 iterations) and keeps the fastest;
                                > 0 = the configuration with that many elements per
                                     workgroup and the default prefetch depth
                                     (NEK_E_ARG when the order has none);
                                -1 = the order's default configuration, untuned.
                                nek_tune and nek_set_variant override it.              */
    int refine_mode;         /* mixed: 0 = default (2);
                                1 = restart CG after each true-residual update;
                                2 = reliable update: replace r by the FP64 true
                                    residual and continue the search direction
                                    (beta from the replaced residual and the one
                                    before the run's last)                      */
    int precond;             /* solveM of Table 1: NEK_PC_NONE (z = r), NEK_PC_JACOBI,
                                NEK_PC_FDM or NEK_PC_SCHWARZ                            */
    int corr_fp32;           /* mixed: 0 = the inner correction d is FP64 (each
                                d += alpha p in FP64); 1 = d stored in FP32 (each
                                update formed in FP64 and rounded once: 8 B per point
                                and inner iteration less)                               */
} nek_opts;

/* Preconditioner of the CG loop (the solveM step of the paper's Table 1). */
typedef enum {
    NEK_PC_NONE = 0,         /* z = r: the unpreconditioned loop                        */
    NEK_PC_JACOBI = 1,       /* z = r / m, m = diagonal of the assembled masked operator
                                (FP64 in FP64 solves, its FP32 rounding in the inner
                                solves of mixed ones); 1 on Dirichlet nodes             */
    NEK_PC_FDM = 2,          /* element-interior block solve by fast diagonalization on
                                each element's (N-1)^3 interior nodes (the element's
                                separable stiffness block with factors from its mean
                                edge lengths: exact for axis-aligned boxes), z = r / m
                                on the other nodes: the non-overlapping Schwarz stage  */
    NEK_PC_SCHWARZ = 3       /* two-level overlapping Schwarz (N >= 2): z = sum_e R_e^T
                                A~_e^-1 R_e r + P A~_c^-1 P^T r.  Each element's
                                subdomain is extruded one GLL node into every face
                                neighbour ((N+3)^3 window, clipped at Dirichlet faces)
                                and solved by fast diagonalization of the separable
                                operator with the element's mean edge lengths; the
                                coarse space is the trilinear functions on the vertex
                                lattice, solved by fast diagonalization of the
                                separable Q1 operator of the slab-mean lattice (FP64).
                                Exact subdomain and coarse solves on uniform box
                                meshes; symmetric positive definite on any mesh       */
} nek_pc;

/* Source of the geometric factors g1..g6 in the operator kernels. */
typedef enum {
    NEK_GSRC_STORED = 0,     /* read per point from memory: the FP64 array, or its
                                FP32 / BF16 copy                                        */
    NEK_GSRC_TRILINEAR = 1   /* recomputed in the kernel, in the vectors' precision,
                                from each element's trilinear map (21 coefficients per
                                element): FP64 and FP32 operators; BF16-g solves keep
                                their stored factors                                   */
} nek_geom_src;

typedef struct {
    int iters;               /* CG iterations (mixed: sum of inner iterations)          */
    int outer_iters;         /* mixed: refinement steps (true-residual checks)          */
    int fp64_iters;          /* mixed: iterations of the FP64 fallback, if used         */
    int status;              /* nek_status of the solve                                 */
    double true_rel_res;     /* sqrt(glsc3(r*,c,r*) / glsc3(b,b)) with r* = b - A x
                                formed in FP64 (FP64 g) from the returned x; 0 if b = 0 */
    double last_rec_res;     /* the CG loop's last recursive residual relative to |b|
                                (mixed: of the last inner or fallback run)              */
    double t_solve_s;        /* wall time of the solve on the context's stream          */
} nek_stats;

/* nek_get selectors (host output sizes in parentheses). */
typedef enum {
    NEK_GET_GLL = 0,         /* double xi[N+1]                                   */
    NEK_GET_W = 1,           /* double w[N+1] (GLL weights)                      */
    NEK_GET_D = 2,           /* double D[(N+1)^2], row-major, D[i][j] = l_j'(x_i) */
    NEK_GET_G = 3,           /* double g[E][6][(N+1)^3]: G_rr, G_ss, G_tt, G_rs,
                                G_rt, G_st (FP64)                                 */
    NEK_GET_B = 4,           /* double B[n_local] (diagonal mass)                */
    NEK_GET_GID = 5,         /* int64 gid[n_local]                               */
    NEK_GET_MULT = 6,        /* int32 mult[n_local]                              */
    NEK_GET_MASK = 7,        /* int8 mask[n_local], 0 on the Dirichlet boundary  */
    NEK_GET_PERM = 8,        /* int32 perm[n_perm]                               */
    NEK_GET_SEGPTR = 9,      /* int32 seg_ptr[n_seg+1]                           */
    NEK_GET_SEGFLAG = 10,    /* int8 seg_flag[n_seg], 1 = masked segment         */
    NEK_GET_XYZ = 11,        /* double X[E][3][(N+1)^3] node coordinates         */
    NEK_GET_DIAG = 12        /* double m[n_local]: diagonal of the assembled masked
                                operator, 1 on Dirichlet nodes (the Jacobi
                                preconditioner; built on first use)              */
} nek_get_what;

/* nek_size selectors. */
typedef enum {
    NEK_SIZE_NLOCAL = 0, NEK_SIZE_NGLOBAL = 1, NEK_SIZE_E = 2,
    NEK_SIZE_NPERM = 3, NEK_SIZE_NSEG = 4, NEK_SIZE_N = 5
} nek_size_what;

/*
 * nek_setup -- build a context for one box mesh of order N (1 <= N <= 15).
 * On the host, in FP64: GLL nodes and weights, D, geometry (trilinear map,
 * J = D X, G, B), global numbering and the sorted-segment gather-scatter maps
 * (the initialisation that the paper's mixed build keeps in double, Sect. 6).
 * These are uploaded once; the FP32 / BF16 copies of g that opts->prec needs
 * are rounded on the device.
 * opts may be NULL (FP64 defaults).  stream is a hipStream_t or NULL.
 * Returns NEK_E_JACOBIAN for an inverted element, NEK_E_ARG for bad sizes.
 */
int nek_setup(const nek_mesh *mesh, int N, const nek_opts *opts, void *stream, nek_ctx **out);

/* nek_free -- release everything the context allocated.  NULL is a no-op. */
void nek_free(nek_ctx *ctx);

/* nek_size -- *out = the size selected by what (nek_size_what). */
int nek_size(const nek_ctx *ctx, int what, int64_t *out);

/* nek_get -- copy a setup array (nek_get_what) to host memory (synchronous). */
int nek_get(nek_ctx *ctx, int what, void *host_out);

/*
 * nek_set_prec -- switch the precision of later nek_cg_solve calls.  Builds
 * the FP32 or BF16 copy of g on first use.
 */
int nek_set_prec(nek_ctx *ctx, int prec);

/*
 * nek_set_precond -- preconditioner (nek_pc) of later nek_cg_solve calls.
 * NEK_PC_JACOBI builds the diagonal on first use (host FP64, from the
 * geometric factors; then an FP32 copy); the loop's work vector then holds
 * z = r / m, updated as z -= alpha S / m, and the gather/update kernel
 * reduces both r.z and r.r (r = m z).  NEK_PC_FDM builds the diagonal, the
 * 1-D interior modes and the element factors; NEK_PC_SCHWARZ (N >= 2) the
 * window and coarse modes and the window-solution buffer (E (N+3)^3 entries
 * per precision); both run each iteration as the operator kernel, the
 * gather/update kernel and the preconditioner kernels (one block-solve
 * kernel; or the window solves, the one-workgroup coarse solve and the
 * gather of z), with z in its own vector.  Solves follow Table 1 with
 * solveM; the stopping test and the reported residuals stay those of r.
 * Batches (nek_batch_*) run unpreconditioned and refuse members with a
 * preconditioner (NEK_E_ARG).  NEK_E_ARG for NEK_PC_SCHWARZ at N = 1.
 */
int nek_set_precond(nek_ctx *ctx, int precond);

/*
 * nek_set_geometry -- source (nek_geom_src) of the geometric factors of the
 * element operator ax_e (Fig. 2: g1..g6 between local_grad3 and
 * local_grad3_t) in every later operator call and solve of the context.
 * By default (NEK_GSRC_STORED) the factors computed at set-up are read per
 * point; with NEK_GSRC_TRILINEAR the kernels compute the same quantities
 * per point from each element's trilinear map (J from the map's
 * coefficients, G = w det(J) J^-1 J^-T), trading six loads per point for
 * about 60 arithmetic operations.  Builds the coefficients on first use
 * (host FP64; an FP32 copy for FP32 operators).  Returns NEK_E_JACOBIAN if
 * an element's map is not orientation-preserving at a GLL node, NEK_E_ARG
 * for an unknown mode.  Batches refuse member contexts with
 * NEK_GSRC_TRILINEAR (NEK_E_ARG).
 */
int nek_set_geometry(nek_ctx *ctx, int geom);

/*
 * nek_set_max_workgroups -- cap on the workgroups of the context's
 * persistent CG kernels and of its reduction kernels (1 <= n <= 2048;
 * 0 restores the default of 8 per compute unit, 4 for FP64 operators with
 * in-kernel factors).  Each workgroup then walks a contiguous share of the
 * element groups, so a low cap makes every workgroup walk several groups
 * even on a small mesh, or leaves compute units to concurrent work.  The
 * per-workgroup partials of the reductions follow the grid, so results at
 * different caps agree to rounding, not bit for bit.  NEK_E_ARG for n out of
 * range or a batch member context (a batch lays out its grid once).
 */
int nek_set_max_workgroups(nek_ctx *ctx, int n);

/* Kernel of the plain operator pass (nek_ax_local, nek_ax). */
typedef enum {
    NEK_OPERATOR_VALU = 0,   /* D contractions on the vector ALUs, u staged in LDS
                                (the kernel of every CG iteration; the default)   */
    NEK_OPERATOR_MFMA = 1    /* each D contraction as 16x16x4 matrix-core products
                                (v_mfma_f32 / v_mfma_f64), N + 1 <= 12            */
} nek_operator_kernel;

/*
 * nek_set_operator_kernel -- choose how the plain local operator A_L u of
 * nek_ax_local and nek_ax computes the D contractions of local_grad3 and
 * local_grad3_t (Fig. 2).  Both apply the same factors and products in a
 * different summation order (results agree to rounding); the CG kernels
 * always use the vector-ALU form, which measured faster on MI355X at
 * N + 1 = 10 and 12 in both precisions (NEK_OPERATOR_MFMA is the measured
 * alternative).  NEK_E_ARG for an unknown kind, or MFMA with N + 1 > 12.
 */
int nek_set_operator_kernel(nek_ctx *ctx, int kind);

/* Kernel of the Schwarz window solves (NEK_PC_SCHWARZ). */
typedef enum {
    NEK_SCHWARZ_AUTO = 0,    /* the faster of the two on MI355X per vector type:
                                matrix cores for FP64, vector ALUs for FP32 (the
                                default)                                          */
    NEK_SCHWARZ_MFMA = 1,    /* each fast-diagonalization pass as 16x16x4 matrix-core
                                products (v_mfma_f32 / v_mfma_f64)               */
    NEK_SCHWARZ_VALU = 2     /* one window line per thread on the vector ALUs    */
} nek_schwarz_kernel;

/*
 * nek_set_schwarz_kernel -- choose the kernel of the overlapping Schwarz
 * window solves (the local solves of solveM in Table 1, Fig. 3's
 * fast-diagonalization smoother); both compute the same products in a
 * different summation order, so results agree to rounding.  Takes effect at
 * the next preconditioner application.  NEK_E_ARG for an unknown kind.
 */
int nek_set_schwarz_kernel(nek_ctx *ctx, int kind);

/* Kernel of the CG update step (dssum of w_L, mask, r -= alpha w, glsc3 of r). */
typedef enum {
    NEK_UPDATE_AUTO = 0,      /* the default: exchange in the CG update kernel; in
                                 nek_ax's assembly, exchange when the mesh has at
                                 least six elements per workgroup of the capped
                                 grid (problems beyond the caches), gather
                                 otherwise                                        */
    NEK_UPDATE_GATHER = 1,    /* every copy of a face node read from memory      */
    NEK_UPDATE_EXCHANGE = 2   /* x-face copies of elements walked by one workgroup
                                 swapped through LDS                              */
} nek_update_kernel;

/*
 * nek_set_update_kernel -- choose how the kernels that sum the copies of each
 * face node for dssum (Table 1) collect them: the update kernel of the
 * unpreconditioned and fast-diagonalization / Schwarz CG iterations, and the
 * assembly pass of nek_ax and nek_ax_noalloc.  Both forms add the same
 * copies in the same fixed order (the CG update with the same workgroups and
 * partials), so solves and nek_ax results are bit-identical under every
 * choice; only the time differs.  Batched solves always use NEK_UPDATE_AUTO.
 * NEK_E_ARG for an unknown kind.
 */
int nek_set_update_kernel(nek_ctx *ctx, int kind);

/*
 * nek_precond_apply -- z = M^-1 r with the context's preconditioner (a copy
 * without one); r and z are device vectors of n_local entries of dtype
 * (NEK_F64: the FP64 data, NEK_F32: the FP32 copies), not overlapping.
 * Asynchronous on the context's stream.
 */
int nek_precond_apply(nek_ctx *ctx, const void *r, void *z, int dtype);

/*
 * nek_ax_local -- w = A_L u, the unassembled element operator ax_e of the
 * paper's Fig. 2 for every element (local_grad3, g1..g6, local_grad3_t).
 * dtype NEK_F64 uses FP64 g; NEK_F32 uses the context's FP32 or BF16 g.
 * u and w are device vectors of n_local entries and must not overlap.
 */
int nek_ax_local(nek_ctx *ctx, const void *u, void *w, int dtype);

/*
 * nek_ax -- w = M o dssum(A_L u): the assembled, masked operator (the ax call
 * of Table 1 with its gather-scatter).  Same arguments as nek_ax_local.
 * A_L u goes to a work vector of the context, then every node's copies are
 * summed in FP64 in the fixed order of the CG update kernel (within a plane
 * of constant k: (own + x-neighbour) + (y + xy-neighbour); the planes below
 * and above added in turn), identical for every copy, and rounded once to
 * dtype.  Runs in the context's CG kernel configuration for the precision.
 */
int nek_ax(nek_ctx *ctx, const void *u, void *w, int dtype);

/*
 * nek_ax_noalloc -- nek_ax that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and result as nek_ax, the
 * same kernels and configuration (bit-identical output), but the
 * unassembled A_L u goes to a static device array of the library instead of
 * a work vector of the context (which nek_ax allocates on its first call).
 * The array holds NEK_NOALLOC_SCRATCH_BYTES (32 MiB: n_local up to 4,194,304
 * for NEK_F64, 8,388,608 for NEK_F32); a larger vector returns
 * NEK_E_SCRATCH.  Each GPU the library runs on holds one such array until
 * the process ends, shared by every call on that GPU: calls that overlap on
 * one GPU (on different streams, or from different host threads) race on
 * it, so serialise them.  Every entry it reads is written earlier in the
 * same call, so nothing needs clearing between calls.  The factor copy the
 * dtype needs must already exist (NEK_E_ARG otherwise): FP64 always; for
 * NEK_F32 the FP32 or BF16 copy that nek_setup (opts->prec) or
 * nek_set_prec built.  No hipMalloc, hipFree or allocating library call is
 * made; asynchronous on the context's stream.
 */
#define NEK_NOALLOC_SCRATCH_BYTES (32u << 20)
int nek_ax_noalloc(nek_ctx *ctx, const void *u, void *w, int dtype);

/*
 * nek_dssum -- in place: every local copy of a global node receives the sum
 * of all copies, taken in ascending local index (gather-scatter, gslib's
 * gs_op in the paper); with apply_mask != 0 the Dirichlet nodes are then
 * zeroed.  FP64 sums are bit-identical to a serial ascending-order sum; FP32
 * copies are summed in FP64 and rounded once.
 */
int nek_dssum(nek_ctx *ctx, void *w, int dtype, int apply_mask);

/*
 * nek_glsc3 -- *out = sum_l a_l c_l b_l with c_l = 1 / multiplicity (glsc3 of
 * Table 1), accumulated in FP64 in a fixed order (deterministic).
 */
int nek_glsc3(nek_ctx *ctx, const void *a, const void *b, int dtype, double *out);

/*
 * nek_cg_solve -- solve A x = b, b = M o dssum(f), by CG in the order of the
 * paper's Table 1 (unpreconditioned, or with the preconditioner set by
 * opts->precond / nek_set_precond), in the context's precision:
 *  - NEK_PREC_FP64: FP64 CG; stops when the recursive relative residual
 *    sqrt(glsc3(r,r)/glsc3(b,b)) <= tol; tol <= 0 runs exactly maxit
 *    iterations.  The true residual of the returned x is formed once at
 *    exit (one FP64 operator application, inside t_solve_s).
 *  - NEK_PREC_FP32 / NEK_PREC_BF16G: iterative refinement (Sect. 6 lowers
 *    the CG loop, here wrapped in FP64 refinement).  The outer loop forms
 *    r = b - A x in FP64 (FP64 g) and stops when the true relative residual
 *    <= tol; each inner solve is CG with an FP32 operator, FP64 reductions
 *    and scalars, and a correction d accumulated in FP64 (opts->corr_fp32:
 *    stored in FP32, each update formed in FP64 and rounded once); x += d
 *    in FP64.
 * With opts->elts_per_wg == 0 the first solve at a precision autotunes the
 * CG kernel pair first (nek_tune; its time is inside t_solve_s).
 * f (load vector), x0 (optional, projected as M o dssum(c o x0)) and x are
 * FP64 device vectors of n_local entries; x may alias x0.  maxit caps the
 * total CG iterations.  stats and res_hist (host, length maxit+1: entry 0 is
 * the initial residual, entry k the residual after iteration k) may be NULL.
 * Returns NEK_OK, NEK_NOCONV, or an error; stats->status repeats it.
 */
int nek_cg_solve(nek_ctx *ctx, const double *f, const double *x0, double tol, int maxit,
                 double *x, nek_stats *stats, double *res_hist);

/*
 * Sampled kernel timing with HIP events on the context's stream, for
 * roofline reporting.  nek_prof_enable(ctx, k): every k-th CG iteration of
 * later solves is bracketed by events (k = 0 turns sampling off).
 * nek_prof_read(ctx, kernel, &ms, &count, reset) returns the summed duration
 * and number of sampled launches of kernel 0 (the fused add2s1 + operator
 * kernel) or kernel 1 (the fused gather-scatter + update kernel); it
 * synchronises the stream.  reset != 0 clears that kernel's totals.
 */
int nek_prof_enable(nek_ctx *ctx, int every);
int nek_prof_read(nek_ctx *ctx, int kernel, double *total_ms, int64_t *count, int reset);

/*
 * Autotuning of the CG kernel pair.  The operator and gather/update kernels
 * of each order N exist in several configurations (elements per workgroup,
 * slices of geometric factors in flight).  nek_num_variants returns their
 * number for the context's N (or a negative status).  nek_tune times
 * `iters` (>= 2) CG iterations of every configuration on a synthetic SPD
 * system of the context's mesh at precision prec (nek_prec), with the
 * context's preconditioner (the kernels of a preconditioned loop differ),
 * after one warm-up pass each; it fills us_per_iter[v] (may be NULL, else at least
 * nek_num_variants entries), selects the fastest for later solves at that
 * precision and returns its index in *best (may be NULL).  It overwrites the
 * context's work vectors, not caller memory; it synchronises the stream.
 * nek_set_variant / nek_get_variant set or read the configuration directly
 * (e.g. from a cache of earlier tuning).
 */
int nek_num_variants(const nek_ctx *ctx);
int nek_tune(nek_ctx *ctx, int prec, int iters, double *us_per_iter, int *best);
int nek_set_variant(nek_ctx *ctx, int prec, int variant);
int nek_get_variant(const nek_ctx *ctx, int prec, int *variant);

/* ------------------------------------------------------------------ batches
 *
 * A batch holds many independent problems, each with its own box mesh and
 * order N, solved together: every CG iteration advances all of them with one
 * launch of the operator kernel and one of the gather/update kernel per
 * distinct order (one stream per order), a chunk of iterations is recorded
 * once as a HIP graph and replayed, and each problem stops at its own
 * tolerance or cap while the others continue.  Each problem computes exactly
 * what nek_cg_solve computes on a context of the same mesh, order, options
 * and kernel configuration: with equal configurations the results are
 * bit-identical.
 */
typedef struct nek_batch nek_batch;

#define NEK_MAX_VARIANTS 6       /* bound on nek_num_variants for any N          */
#define NEK_BATCH_NO_GRAPH 1     /* nek_cg_solve_batch flag: plain launches, no graph */

/*
 * nek_setup_batch -- one context per problem i (meshes[i], order N[i], the
 * common opts, whose prec applies to every problem).  The batch creates and
 * owns its streams; member contexts run on the batch's main stream.  stream
 * is the caller's stream: setup and every solve wait for the work already
 * enqueued on it.  1 <= nprob <= 4096.  opts->elts_per_wg applies per
 * order: 0 autotunes every order's configuration at the first batched solve
 * of each precision (nek_batch_tune with 20 iterations), > 0 selects that
 * many elements per workgroup (NEK_E_ARG if some order has no such
 * configuration), -1 keeps the defaults.  Member contexts take the batch's
 * configuration and do not tune on their own.  Errors as nek_setup (nothing
 * is left allocated).
 *
 * Many right-hand sides on one mesh: a problem whose order and mesh repeat
 * an earlier problem's (equal nel and, with vtx NULL, equal lo and hi, else
 * identical vertex values) shares that problem's set-up data on the device
 * (geometric factors in every precision, D, mass, maps) instead of holding
 * a copy, and its context reads them from there.  In the batched solve the
 * workgroups of the problems on one mesh are interleaved block by block on
 * the same XCD, so that their reads of the shared factors are served by
 * that XCD's L2 after the first.  Results are bit-identical to separate
 * meshes (the kernels and their summation order do not change).
 */
int nek_setup_batch(int nprob, const nek_mesh *meshes, const int *N, const nek_opts *opts, void *stream,
                    nek_batch **out);

/* nek_batch_free -- release the batch, its member contexts and streams. */
void nek_batch_free(nek_batch *batch);

/* Number of problems (or a negative status). */
int nek_batch_size(const nek_batch *batch);

/*
 * nek_batch_ctx -- the member context of problem i, owned by the batch (do
 * not free it).  It may be used with every nek_* call; its work runs on the
 * batch's stream, and calls that do not synchronise need a
 * hipDeviceSynchronize (or a later synchronising call) before the caller's
 * stream reads their output.
 */
int nek_batch_ctx(nek_batch *batch, int i, nek_ctx **out);

/*
 * nek_batch_mesh_of -- index of the problem whose set-up data problem i
 * uses (i itself when it holds its own; an earlier problem on the same mesh
 * and order otherwise), or NEK_E_ARG.
 */
int nek_batch_mesh_of(const nek_batch *batch, int i);

/*
 * nek_batch_orders -- number of distinct orders in the batch; N_out (may be
 * NULL, else at least 15 entries) receives them in ascending order.
 */
int nek_batch_orders(const nek_batch *batch, int *N_out);

/*
 * nek_batch_tune -- per order, time `iters` (>= 2) batched CG iterations of
 * all problems of that order under every kernel configuration (synthetic
 * SPD systems, one warm-up pass each) and keep the fastest for later batched
 * solves at precision prec; the member contexts get the same configuration.
 * us_per_iter (may be NULL) receives NEK_MAX_VARIANTS entries per order, in
 * the order of nek_batch_orders (unused entries 0).  Overwrites the members'
 * work vectors, not caller memory; synchronises.
 */
int nek_batch_tune(nek_batch *batch, int prec, int iters, double *us_per_iter);

/* Set the configuration of all problems of order N, or read problem i's. */
int nek_batch_set_variant(nek_batch *batch, int prec, int N, int variant);
int nek_batch_get_variant(const nek_batch *batch, int prec, int i, int *variant);

/*
 * nek_cg_solve_batch -- solve every problem i as nek_cg_solve(ctx_i, f[i],
 * x0 ? x0[i] : NULL, tol, maxit, x[i], &stats[i], NULL) would, together.
 * f, x0, x are HOST arrays of nprob DEVICE pointers (x0 itself or any entry
 * may be NULL); stats (may be NULL) is a host array of nprob entries, each
 * with its problem's status; t_solve_s is the wall time of the whole batch.
 * flags: NEK_BATCH_NO_GRAPH enqueues every launch instead of replaying the
 * recorded chunk.  Returns the most negative status of any problem, else
 * NEK_NOCONV if any problem did not converge, else NEK_OK.  Synchronises.
 */
int nek_cg_solve_batch(nek_batch *batch, const double *const *f, const double *const *x0, double tol, int maxit,
                       double *const *x, nek_stats *stats, int flags);

/* Totals since setup: chunks of iterations launched, graphs recorded. */
int nek_batch_counters(const nek_batch *batch, int64_t *chunks, int64_t *captures);

/* nek_strerror -- static description of a status code. */
const char *nek_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* NEK_H */
