/*
 * Sanitizer driver for the host code: every nek_host_* set-up routine of
 * libnek (paper_2405_11065_amd/csrc/nek_setup.cpp) and every routine of the
 * oracle (oracle/nek_oracle.c, oracle/nek_vprec.c), called on box meshes of
 * several shapes and orders with each buffer allocated at exactly the size
 * its header states, so that an AddressSanitizer build reports any read or
 * write past it and an UndefinedBehaviorSanitizer build any overflow, bad
 * shift or misaligned access.  A few cross-checks between the two
 * independent implementations keep the calls honest (they must agree, as the
 * Python tests also check).  Exit status 0 when everything ran and agreed.
 * Test infrastructure: built and run by tests/test_sanitizers.py only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nek_host.h"

/* oracle entry points (oracle/nek_oracle.c, oracle/nek_vprec.c) */
int or_gll(int N, double *xi, double *w);
int or_deriv(int N, const double *xi, double *D);
int or_numbering(int N, const int *nel, int64_t *gid, int32_t *mult, int8_t *mask);
int or_segments(int N, const int *nel, const int64_t *gid, const int8_t *mask, int32_t *perm, int32_t *seg_ptr,
                int8_t *seg_flag, int64_t *nperm, int64_t *nseg);
int or_geometry(int N, const int *nel, const double *vtx, double *g, double *B, double *X);
void or_ax_local(int N, int64_t E, const double *D, const double *g, const double *u, double *w);
void or_dssum(int64_t nl, int64_t ng, const int64_t *gid, double *w, double *acc);
void or_mask(int64_t nl, const int8_t *mask, double *w);
double or_glsc3(int64_t nl, const double *a, const double *c, const double *b);
int or_apply_A(int N, const int *nel, const double *D, const double *g, const int64_t *gid, const int8_t *mask,
               const double *u, double *w);
int or_cg(int N, const int *nel, const double *D, const double *g, const int64_t *gid, const int32_t *mult,
          const int8_t *mask, const double *f, const double *x0, double tol, int maxit, double *x, double *res_hist);
int or_diag(int N, const int *nel, const double *D, const double *g, const int64_t *gid, const int8_t *mask,
            double *m);
int or_pcg(int N, const int *nel, const double *D, const double *g, const int64_t *gid, const int32_t *mult,
           const int8_t *mask, const double *m, const double *f, const double *x0, double tol, int maxit, double *x,
           double *res_hist);
double vp_round(double x, int t);
int vp_cg(int N, const int *nel, const double *vtx, const double *f, const int *t, int mode, uint64_t seed,
          double tol, int maxit, double *x, double *hist, double *g_out, const double *m);

static int fails = 0;

#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                 \
            fputc('\n', stderr);                          \
            ++fails;                                      \
        }                                                 \
    } while (0)

static void *xalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* Box vertex lattice [nz+1][ny+1][nx+1][3] on [0,1]^3, interior vertices
 * moved by up to pert of a cell by a fixed linear congruential sequence. */
static double *box_vertices(const int nel[3], double pert, uint64_t seed)
{
    size_t nv = (size_t)(nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1);
    double *v = (double *)xalloc(3 * nv * sizeof(double));
    uint64_t s = seed * 2862933555777941757ull + 3037000493ull;
    for (int k = 0; k <= nel[2]; ++k)
        for (int j = 0; j <= nel[1]; ++j)
            for (int i = 0; i <= nel[0]; ++i) {
                size_t a = 3 * ((size_t)i + (nel[0] + 1) * ((size_t)j + (nel[1] + 1) * k));
                int idx[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    s = s * 6364136223846793005ull + 1442695040888963407ull;
                    double u = (double)(s >> 11) / 9007199254740992.0 - 0.5;
                    int inner = idx[d] > 0 && idx[d] < nel[d];
                    v[a + d] = ((double)idx[d] + (inner ? pert * u : 0.0)) / nel[d];
                }
            }
    return v;
}

static void check_rules(void)
{
    for (int N = 1; N <= 15; ++N) {
        int n = N + 1;
        double *xh = xalloc(n * sizeof(double)), *wh = xalloc(n * sizeof(double));
        double *xo = xalloc(n * sizeof(double)), *wo = xalloc(n * sizeof(double));
        double *Dh = xalloc((size_t)n * n * sizeof(double)), *Do = xalloc((size_t)n * n * sizeof(double));
        CHECK(nek_host_gll(N, xh, wh) == 0, "nek_host_gll N=%d", N);
        CHECK(nek_host_deriv(N, Dh) == 0, "nek_host_deriv N=%d", N);
        CHECK(or_gll(N, xo, wo) == 0, "or_gll N=%d", N);
        CHECK(or_deriv(N, xo, Do) == 0, "or_deriv N=%d", N);
        for (int i = 0; i < n; ++i) {
            CHECK(fabs(xh[i] - xo[i]) <= 1e-14 && fabs(wh[i] - wo[i]) <= 1e-14, "GLL N=%d i=%d", N, i);
            for (int j = 0; j < n; ++j)
                CHECK(fabs(Dh[i * n + j] - Do[i * n + j]) <= 1e-10 * (1.0 + fabs(Do[i * n + j])),
                      "D N=%d (%d,%d)", N, i, j);
        }
        free(xh); free(wh); free(xo); free(wo); free(Dh); free(Do);
    }
    /* argument rejection */
    double a[20];
    CHECK(nek_host_gll(0, a, a) == -1 && nek_host_gll(16, a, a) == -1, "gll range");
    int bad[3] = {0, 1, 1};
    CHECK(nek_host_numbering(3, bad, NULL, NULL, NULL) == -1, "numbering bad nel");
    for (int t = 1; t <= 52; ++t) {
        double r = vp_round(1.0 / 3.0, t);
        CHECK(fabs(r - 1.0 / 3.0) <= ldexp(1.0 / 3.0, -t), "vp_round t=%d", t);
    }
}

static void check_mesh(int N, const int nel[3], double pert, uint64_t seed)
{
    const int n = N + 1, n3 = n * n * n;
    const int64_t E = (int64_t)nel[0] * nel[1] * nel[2], nl = E * n3;
    const int64_t ng = (int64_t)(nel[0] * N + 1) * (nel[1] * N + 1) * (nel[2] * N + 1);
    double *vtx = box_vertices(nel, pert, seed);

    /* numbering and segments, both sides */
    int64_t *gid = xalloc(nl * sizeof(int64_t)), *gid_o = xalloc(nl * sizeof(int64_t));
    int32_t *mult = xalloc(nl * sizeof(int32_t)), *mult_o = xalloc(nl * sizeof(int32_t));
    int8_t *mask = xalloc(nl), *mask_o = xalloc(nl);
    CHECK(nek_host_numbering(N, nel, gid, mult, mask) == 0, "numbering");
    CHECK(or_numbering(N, nel, gid_o, mult_o, mask_o) == 0, "or_numbering");
    CHECK(!memcmp(gid, gid_o, nl * sizeof(int64_t)) && !memcmp(mult, mult_o, nl * sizeof(int32_t)) &&
              !memcmp(mask, mask_o, nl),
          "numbering differs N=%d", N);
    CHECK(nek_host_numbering(N, nel, NULL, mult, NULL) == 0, "numbering with NULL outputs");

    int64_t np = 0, ns = 0;
    CHECK(nek_host_segment_sizes(N, nel, &np, &ns) == 0, "segment sizes");
    int32_t *perm = xalloc(np * sizeof(int32_t)), *ptr = xalloc((ns + 1) * sizeof(int32_t));
    int8_t *flag = xalloc(ns);
    CHECK(nek_host_segments(N, nel, perm, ptr, flag) == 0, "segments");
    /* the oracle writes at most every local node into perm and a segment per copy */
    int32_t *perm_o = xalloc(nl * sizeof(int32_t)), *ptr_o = xalloc((nl + 1) * sizeof(int32_t));
    int8_t *flag_o = xalloc(nl);
    int64_t np_o = -1, ns_o = -1;
    CHECK(or_segments(N, nel, gid_o, mask_o, perm_o, ptr_o, flag_o, &np_o, &ns_o) == 0, "or_segments");
    CHECK(np == np_o && ns == ns_o, "segment sizes differ");
    if (np == np_o && ns == ns_o)
        CHECK(!memcmp(perm, perm_o, np * sizeof(int32_t)) && !memcmp(ptr, ptr_o, (ns + 1) * sizeof(int32_t)) &&
                  !memcmp(flag, flag_o, ns),
              "segment maps differ");

    /* geometry, both sides */
    double *g = xalloc((size_t)E * 6 * n3 * sizeof(double)), *B = xalloc(nl * sizeof(double));
    double *X = xalloc((size_t)E * 3 * n3 * sizeof(double));
    double *g_o = xalloc((size_t)E * 6 * n3 * sizeof(double)), *B_o = xalloc(nl * sizeof(double));
    double *X_o = xalloc((size_t)E * 3 * n3 * sizeof(double));
    CHECK(nek_host_geometry(N, nel, vtx, g, B, X) == 0, "geometry");
    CHECK(nek_host_geometry(N, nel, vtx, g, B, NULL) == 0, "geometry without X");
    CHECK(or_geometry(N, nel, vtx, g_o, B_o, X_o) == 0, "or_geometry");
    double gmax = 0.0, gerr = 0.0;
    for (int64_t q = 0; q < E * 6 * n3; ++q) {
        gmax = fmax(gmax, fabs(g_o[q]));
        gerr = fmax(gerr, fabs(g[q] - g_o[q]));
    }
    CHECK(gerr <= 1e-12 * gmax, "geometry differs %.3e", gerr / gmax);

    double *coef = xalloc((size_t)E * 24 * sizeof(double));
    CHECK(nek_host_trilinear(N, nel, vtx, coef) == 0, "trilinear");
    if (N >= 2) {
        int nm = N - 1;
        double *S = xalloc((size_t)nm * nm * sizeof(double)), *lam = xalloc(nm * sizeof(double));
        double *cf = xalloc((size_t)3 * E * sizeof(double));
        CHECK(nek_host_fdm(N, nel, vtx, S, lam, cf) == 0, "fdm");
        int w = N + 3;
        double *Sw = xalloc((size_t)4 * w * w * sizeof(double)), *lamw = xalloc((size_t)4 * w * sizeof(double));
        size_t nsc = 0, nlc = 0;
        for (int d = 0; d < 3; ++d) {
            nsc += (size_t)(nel[d] - 1) * (nel[d] - 1);
            nlc += (size_t)(nel[d] - 1);
        }
        double *Sc = xalloc(nsc * sizeof(double)), *lamc = xalloc(nlc * sizeof(double));
        CHECK(nek_host_schwarz(N, nel, vtx, Sw, lamw, Sc, lamc) == 0, "schwarz");
        free(S); free(lam); free(cf); free(Sw); free(lamw); free(Sc); free(lamc);
    }

    /* operator, dssum, mask, dot, CG, PCG, emulated CG */
    double *xi = xalloc(n * sizeof(double)), *wq = xalloc(n * sizeof(double));
    double *D = xalloc((size_t)n * n * sizeof(double));
    or_gll(N, xi, wq);
    or_deriv(N, xi, D);
    double *u = xalloc(nl * sizeof(double)), *w = xalloc(nl * sizeof(double)), *acc = xalloc(ng * sizeof(double));
    double *c = xalloc(nl * sizeof(double));
    for (int64_t l = 0; l < nl; ++l) {
        u[l] = (double)((l * 7919) % 1000) / 1000.0;
        c[l] = 1.0 / mult_o[l];
    }
    or_ax_local(N, E, D, g_o, u, w);
    or_dssum(nl, ng, gid_o, w, acc);
    or_mask(nl, mask_o, w);
    double *w2 = xalloc(nl * sizeof(double));
    CHECK(or_apply_A(N, nel, D, g_o, gid_o, mask_o, u, w2) == 0, "or_apply_A");
    CHECK(!memcmp(w, w2, nl * sizeof(double)), "apply_A differs from its steps");
    double dot = or_glsc3(nl, u, c, w);
    CHECK(isfinite(dot), "glsc3");

    double *f = xalloc(nl * sizeof(double)), *x = xalloc(nl * sizeof(double)), *x2 = xalloc(nl * sizeof(double));
    double *m = xalloc(nl * sizeof(double));
    const int maxit = 40;
    double *h = xalloc((maxit + 1) * sizeof(double)), *h2 = xalloc((maxit + 1) * sizeof(double));
    for (int64_t l = 0; l < nl; ++l) f[l] = (double)((l * 104729) % 997) / 997.0;
    int it = or_cg(N, nel, D, g_o, gid_o, mult_o, mask_o, f, NULL, 1e-10, maxit, x, h);
    CHECK(it >= 0, "or_cg %d", it);
    CHECK(or_diag(N, nel, D, g_o, gid_o, mask_o, m) == 0, "or_diag");
    int itp = or_pcg(N, nel, D, g_o, gid_o, mult_o, mask_o, m, f, NULL, 1e-10, maxit, x2, h2);
    CHECK(itp >= 0, "or_pcg %d", itp);
    for (int64_t l = 0; l < nl; ++l) m[l] = 1.0;
    itp = or_pcg(N, nel, D, g_o, gid_o, mult_o, mask_o, m, f, NULL, 1e-10, maxit, x2, h2);
    CHECK(itp == it && !memcmp(x, x2, nl * sizeof(double)), "pcg with m = 1 differs from cg");
    int t52[4] = {52, 52, 52, 52};
    double *gv = xalloc((size_t)E * 6 * n3 * sizeof(double));
    int itv = vp_cg(N, nel, vtx, f, t52, 0, 1, 1e-10, maxit, x2, h2, gv, NULL);
    CHECK(itv == it && !memcmp(x, x2, nl * sizeof(double)), "vp_cg at 52 bits differs from or_cg");
    int t23[4] = {52, 23, 23, 52};
    /* Monte Carlo arithmetic at 23 bits: a run may also end in breakdown
     * (-5) once the noise floor is reached on a mesh with a handful of
     * unknowns, a valid outcome */
    itv = vp_cg(N, nel, vtx, f, t23, 3, 7, 1e-10, maxit, x2, h2, NULL, NULL);
    CHECK(itv >= 0 || itv == -5, "vp_cg mca %d", itv);

    printf("N=%d nel=%dx%dx%d: %lld local points, cg %d its\n", N, nel[0], nel[1], nel[2], (long long)nl, it);
    free(vtx); free(gid); free(gid_o); free(mult); free(mult_o); free(mask); free(mask_o);
    free(perm); free(ptr); free(flag); free(perm_o); free(ptr_o); free(flag_o);
    free(g); free(B); free(X); free(g_o); free(B_o); free(X_o); free(coef);
    free(xi); free(wq); free(D); free(u); free(w); free(acc); free(c); free(w2);
    free(f); free(x); free(x2); free(m); free(h); free(h2); free(gv);
}

int main(void)
{
    check_rules();
    static const int meshes[][4] = {
        /* N, nx, ny, nz */
        {1, 2, 2, 2}, {2, 3, 1, 2}, {3, 1, 1, 1}, {4, 2, 3, 1}, {5, 3, 2, 2}, {7, 2, 2, 2}, {9, 1, 2, 3}, {15, 2, 1, 1},
    };
    for (size_t k = 0; k < sizeof(meshes) / sizeof(meshes[0]); ++k) {
        int nel[3] = {meshes[k][1], meshes[k][2], meshes[k][3]};
        check_mesh(meshes[k][0], nel, k % 2 ? 0.2 : 0.0, 11 + k);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("all host checks passed\n");
    return 0;
}
