/*
 * Precision-emulation harness for the oracle (the accuracy-check method of
 * Sect. 4 of Chen, de Oliveira Castro, Bientinesi, Iakymchuk, "Enabling
 * mixed-precision with the help of tools: A Nekbone case study": lower
 * precision emulated per floating-point operation, then Monte Carlo
 * arithmetic to test how sensitive the result is).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/: the product library
 * never links, loads or calls it, and it shares nothing with the GPU path.
 *
 * The FP64 initialisation (GLL rule, D, trilinear geometry), the assembled
 * operator and the CG loop of the paper's Table 1 are written here once more,
 * in the same operation order as nek_oracle.c, with every floating-point
 * result (and, in one mode, every operand) passed through a hook.  With the
 * hook off the results are bit-identical to nek_oracle.c (a CPU test checks
 * this), so the harness computes the oracle's arithmetic and nothing else.
 *
 * Hook modes, applied at a virtual precision of t explicit mantissa bits
 * (t >= 52: the value passes unchanged):
 *   VP_IEEE  -- none: plain binary64.
 *   VP_RNE   -- round the result to t bits, nearest, ties to even (what the
 *               paper's variable-precision backend does; the exponent range
 *               of binary64 is kept, so only the mantissa is narrowed).
 *   VP_RR    -- Monte Carlo random rounding: result x -> x + 2^(e_x - t) xi,
 *               e_x = floor(log2 |x|) + 1, xi ~ U(-1/2, 1/2), zero left alone.
 *   VP_MCA   -- the same perturbation on both operands and on the result.
 * xi comes from splitmix64 of (seed, running counter), so a sample is
 * reproducible from its seed.
 *
 * Each operation belongs to one of four regions, each with its own t:
 *   VP_INIT  GLL nodes and weights, D, geometry, b = M dssum(f);
 *   VP_OP    the element operator (local_grad3, g1..g6, local_grad3_t) and
 *            the dssum additions;
 *   VP_VEC   the vector updates p = r + beta p, x += alpha p, r -= alpha w,
 *            r = b - A x;
 *   VP_DOT   glsc3 (with its compensation terms), alpha, beta, the residual
 *            norm.
 * "Only CG" in the paper's sense instruments OP, VEC and DOT; "whole
 * program" instruments INIT as well.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int or_numbering(int N, const int *nel, int64_t *gid, int32_t *mult, int8_t *mask);

enum { VP_IEEE = 0, VP_RNE = 1, VP_RR = 2, VP_MCA = 3 };
enum { VP_INIT = 0, VP_OP = 1, VP_VEC = 2, VP_DOT = 3, VP_NREG = 4 };

static int vp_mode = VP_IEEE;
static int vp_t[VP_NREG] = {52, 52, 52, 52};
static int vp_reg = VP_INIT;
static uint64_t vp_seed = 0, vp_ctr = 0;

/* splitmix64 (Steele, Lea, Flood 2014) of seed + counter step: 64 uniform bits */
static uint64_t vp_bits(void)
{
    uint64_t z = vp_seed + (++vp_ctr) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* x rounded to t explicit mantissa bits, nearest, ties to even. */
double vp_round(double x, int t)
{
    if (t >= 52 || x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                            /* x = m 2^e, 1/2 <= |m| < 1 */
    double y = ldexp(x, t + 1 - e);          /* 2^t <= |y| < 2^(t+1): exact scaling */
    return ldexp(nearbyint(y), e - t - 1);   /* default rounding mode: ties to even */
}

/* x + 2^(e_x - t) xi, e_x = floor(log2|x|) + 1, xi ~ U(-1/2, 1/2). */
double vp_perturb(double x, int t)
{
    if (t >= 52 || x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);
    double xi = (double)(vp_bits() >> 11) * 0x1p-53 - 0.5;
    return x + ldexp(xi, e - t);
}

static double O(double x)
{
    int t = vp_t[vp_reg];
    if (vp_mode == VP_RNE) return vp_round(x, t);
    if (vp_mode == VP_RR || vp_mode == VP_MCA) return vp_perturb(x, t);
    return x;
}

static double I(double x) { return vp_mode == VP_MCA ? vp_perturb(x, vp_t[vp_reg]) : x; }

static double add(double a, double b) { double x = I(a), y = I(b); return O(x + y); }
static double sub(double a, double b) { double x = I(a), y = I(b); return O(x - y); }
static double mul(double a, double b) { double x = I(a), y = I(b); return O(x * y); }
static double dvd(double a, double b) { double x = I(a), y = I(b); return O(x / y); }
static double vsqrt(double a) { return O(sqrt(I(a))); }
static double vcos(double a) { return O(cos(I(a))); }

/* ---------------------------------------------------------------- init */

static void vp_legendre_pair(int N, double x, double *pN, double *pNm1)
{
    double pm = 1.0, p = x;
    if (N == 0) { *pN = 1.0; *pNm1 = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double pp = dvd(sub(mul(mul(add(mul(2.0, k), 1.0), x), p), mul(k, pm)), add(k, 1.0));
        pm = p;
        p = pp;
    }
    *pN = p;
    *pNm1 = pm;
}

static void vp_gll(int N, double *xi, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i <= N; ++i) {
        double x = -vcos(dvd(mul(pi, i), N));
        for (int it = 0; it < 100; ++it) {
            double pN, pNm1;
            vp_legendre_pair(N, x, &pN, &pNm1);
            double dx = dvd(sub(mul(x, pN), pNm1), mul(add(N, 1.0), pN));
            x = sub(x, dx);
            if (fabs(dx) < 1e-17) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i <= N / 2; ++i) {
        double a = mul(0.5, sub(xi[N - i], xi[i]));
        xi[i] = -a;
        xi[N - i] = a;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 0; i <= N; ++i) {
        double pN, pNm1;
        vp_legendre_pair(N, xi[i], &pN, &pNm1);
        w[i] = dvd(2.0, mul(mul(mul(N, add(N, 1.0)), pN), pN));
    }
}

static void vp_deriv(int N, const double *xi, double *D)
{
    int n = N + 1;
    double pn[64];
    for (int i = 0; i < n; ++i) {
        double a, b;
        vp_legendre_pair(N, xi[i], &a, &b);
        pn[i] = a;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d;
            if (i != j) d = dvd(pn[i], mul(pn[j], sub(xi[i], xi[j])));
            else if (i == 0) d = dvd(mul(-N, add(N, 1.0)), 4.0);
            else if (i == N) d = dvd(mul(N, add(N, 1.0)), 4.0);
            else d = 0.0;
            D[i * n + j] = d;
        }
}

static int vp_geometry(int N, const int *nel, const double *vtx, const double *xi, const double *w, double *g)
{
    int n = N + 1, n3 = n * n * n;
    int64_t vx = nel[0] + 1, vy = nel[1] + 1;
    int bad = 0;
    for (int ez = 0; ez < nel[2]; ++ez)
        for (int ey = 0; ey < nel[1]; ++ey)
            for (int ex = 0; ex < nel[0]; ++ex) {
                int64_t e = ex + (int64_t)nel[0] * (ey + (int64_t)nel[1] * ez);
                double V[2][2][2][3];
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            for (int d = 0; d < 3; ++d)
                                V[c][b][a][d] = vtx[3 * ((ex + a) + vx * ((ey + b) + vy * (ez + c))) + d];
                for (int k = 0; k < n; ++k)
                    for (int j = 0; j < n; ++j)
                        for (int i = 0; i < n; ++i) {
                            double r = xi[i], s = xi[j], t = xi[k];
                            double ph[3][2] = {{dvd(sub(1, r), 2), dvd(add(1, r), 2)},
                                               {dvd(sub(1, s), 2), dvd(add(1, s), 2)},
                                               {dvd(sub(1, t), 2), dvd(add(1, t), 2)}};
                            double dph[2] = {-0.5, 0.5};
                            double J[3][3] = {{0}};
                            for (int c = 0; c < 2; ++c)
                                for (int b = 0; b < 2; ++b)
                                    for (int a = 0; a < 2; ++a)
                                        for (int d = 0; d < 3; ++d) {
                                            double v = V[c][b][a][d];
                                            J[d][0] = add(J[d][0], mul(mul(mul(dph[a], ph[1][b]), ph[2][c]), v));
                                            J[d][1] = add(J[d][1], mul(mul(mul(ph[0][a], dph[b]), ph[2][c]), v));
                                            J[d][2] = add(J[d][2], mul(mul(mul(ph[0][a], ph[1][b]), dph[c]), v));
                                        }
                            double det = add(sub(mul(J[0][0], sub(mul(J[1][1], J[2][2]), mul(J[1][2], J[2][1]))),
                                                 mul(J[0][1], sub(mul(J[1][0], J[2][2]), mul(J[1][2], J[2][0])))),
                                             mul(J[0][2], sub(mul(J[1][0], J[2][1]), mul(J[1][1], J[2][0]))));
                            if (!(det > 0)) bad = 1;
                            double Ji[3][3];
                            Ji[0][0] = dvd(sub(mul(J[1][1], J[2][2]), mul(J[1][2], J[2][1])), det);
                            Ji[0][1] = dvd(sub(mul(J[0][2], J[2][1]), mul(J[0][1], J[2][2])), det);
                            Ji[0][2] = dvd(sub(mul(J[0][1], J[1][2]), mul(J[0][2], J[1][1])), det);
                            Ji[1][0] = dvd(sub(mul(J[1][2], J[2][0]), mul(J[1][0], J[2][2])), det);
                            Ji[1][1] = dvd(sub(mul(J[0][0], J[2][2]), mul(J[0][2], J[2][0])), det);
                            Ji[1][2] = dvd(sub(mul(J[0][2], J[1][0]), mul(J[0][0], J[1][2])), det);
                            Ji[2][0] = dvd(sub(mul(J[1][0], J[2][1]), mul(J[1][1], J[2][0])), det);
                            Ji[2][1] = dvd(sub(mul(J[0][1], J[2][0]), mul(J[0][0], J[2][1])), det);
                            Ji[2][2] = dvd(sub(mul(J[0][0], J[1][1]), mul(J[0][1], J[1][0])), det);
                            double W = mul(mul(w[i], w[j]), w[k]);
                            double Gm[3][3];
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b) {
                                    double acc = 0;
                                    for (int d = 0; d < 3; ++d) acc = add(acc, mul(Ji[a][d], Ji[b][d]));
                                    Gm[a][b] = mul(mul(W, det), acc);
                                }
                            int64_t q = i + n * (j + n * k);
                            double *ge = g + e * 6 * n3;
                            ge[0 * n3 + q] = Gm[0][0];
                            ge[1 * n3 + q] = Gm[1][1];
                            ge[2 * n3 + q] = Gm[2][2];
                            ge[3 * n3 + q] = Gm[0][1];
                            ge[4 * n3 + q] = Gm[0][2];
                            ge[5 * n3 + q] = Gm[1][2];
                        }
            }
    return bad ? -4 : 0;
}

/* ------------------------------------------------------------ operator */

typedef struct {
    int N;
    int64_t E, nl, ng;
    const double *D, *g;
    const int64_t *gid;
    const int8_t *mask;
    double *acc, *wr;
} vp_opd;

static void vp_ax_local(const vp_opd *op, const double *u, double *w)
{
    int n = op->N + 1, n3 = n * n * n;
    const double *D = op->D;
    double *wr = op->wr, *ws = wr + n3, *wt = wr + 2 * n3;
    for (int64_t e = 0; e < op->E; ++e) {
        const double *ue = u + e * n3;
        const double *ge = op->g + e * 6 * n3;
        double *we = w + e * n3;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double ur = 0, us = 0, ut = 0;
                    for (int l = 0; l < n; ++l) {
                        ur = add(ur, mul(D[i * n + l], ue[l + n * (j + n * k)]));
                        us = add(us, mul(D[j * n + l], ue[i + n * (l + n * k)]));
                        ut = add(ut, mul(D[k * n + l], ue[i + n * (j + n * l)]));
                    }
                    int q = i + n * (j + n * k);
                    double g1 = ge[q], g2 = ge[n3 + q], g3 = ge[2 * n3 + q];
                    double g4 = ge[3 * n3 + q], g5 = ge[4 * n3 + q], g6 = ge[5 * n3 + q];
                    wr[q] = add(add(mul(g1, ur), mul(g4, us)), mul(g5, ut));
                    ws[q] = add(add(mul(g4, ur), mul(g2, us)), mul(g6, ut));
                    wt[q] = add(add(mul(g5, ur), mul(g6, us)), mul(g3, ut));
                }
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double acc = 0;
                    for (int l = 0; l < n; ++l) acc = add(acc, mul(D[l * n + i], wr[l + n * (j + n * k)]));
                    for (int l = 0; l < n; ++l) acc = add(acc, mul(D[l * n + j], ws[i + n * (l + n * k)]));
                    for (int l = 0; l < n; ++l) acc = add(acc, mul(D[l * n + k], wt[i + n * (j + n * l)]));
                    we[i + n * (j + n * k)] = acc;
                }
    }
}

static void vp_dssum(const vp_opd *op, double *w)
{
    for (int64_t a = 0; a < op->ng; ++a) op->acc[a] = 0.0;
    for (int64_t l = 0; l < op->nl; ++l) op->acc[op->gid[l]] = add(op->acc[op->gid[l]], w[l]);
    for (int64_t l = 0; l < op->nl; ++l) w[l] = op->acc[op->gid[l]];
}

static void vp_mask(const vp_opd *op, double *w)
{
    for (int64_t l = 0; l < op->nl; ++l)
        if (!op->mask[l]) w[l] = 0.0;
}

static void vp_apply(const vp_opd *op, const double *u, double *w)
{
    vp_reg = VP_OP;
    vp_ax_local(op, u, w);
    vp_dssum(op, w);
    vp_mask(op, w);
}

/* glsc3 with Neumaier's compensation, every operation instrumented */
static double vp_glsc3(int64_t nl, const double *a, const double *c, const double *b)
{
    double s = 0.0, comp = 0.0;
    for (int64_t l = 0; l < nl; ++l) {
        double t = mul(mul(a[l], c[l]), b[l]);
        double y = add(s, t);
        if (fabs(s) >= fabs(t)) comp = add(comp, add(sub(s, y), t));
        else comp = add(comp, add(sub(t, y), s));
        s = y;
    }
    return add(s, comp);
}

/*
 * The whole oracle pipeline under the hook: init (GLL, D, geometry,
 * b = M o dssum(f)) in region INIT, then CG from x = 0 in the order of
 * Table 1 (as or_cg), each step in its region.
 *   t[4]   precision per region (INIT, OP, VEC, DOT); mode one of VP_*;
 *   seed   stream of the random perturbations;
 *   tol    relative residual to stop at (<= 0: exactly maxit iterations).
 * m (optional): a diagonal preconditioner per local node; the loop is then
 * or_pcg's (solveM z = r / m, the division in region VEC).
 * Outputs: x (n_local), hist (maxit+1 recursive relative residuals, entry 0
 * the initial one), g_out (optional, E*6*n^3 geometric factors as the hook
 * left them) and the iteration count as return value (-4 inverted element,
 * -5 breakdown, -6 non-finite, -1 allocation).  The residual of the
 * returned x is left to the exact oracle.
 */
int vp_cg(int N, const int *nel, const double *vtx, const double *f, const int *t, int mode, uint64_t seed,
          double tol, int maxit, double *x, double *hist, double *g_out, const double *m)
{
    if (N < 1 || N > 63) return -1;
    for (int q = 0; q < VP_NREG; ++q) vp_t[q] = t[q];
    vp_mode = mode;
    vp_seed = seed;
    vp_ctr = 0;
    int n = N + 1, n3 = n * n * n;
    int64_t E = (int64_t)nel[0] * nel[1] * nel[2], nl = E * n3;
    int64_t ng = ((int64_t)nel[0] * N + 1) * ((int64_t)nel[1] * N + 1) * ((int64_t)nel[2] * N + 1);
    double xi[64], w[64], D[64 * 64];
    double *g = (double *)malloc(sizeof(double) * 6 * nl);
    int64_t *gid = (int64_t *)malloc(sizeof(int64_t) * nl);
    int32_t *mult = (int32_t *)malloc(sizeof(int32_t) * nl);
    int8_t *mask = (int8_t *)malloc(nl);
    double *acc = (double *)malloc(sizeof(double) * ng);
    double *wr = (double *)malloc(sizeof(double) * 3 * n3);
    double *c = (double *)malloc(sizeof(double) * nl);
    double *b = (double *)malloc(sizeof(double) * nl);
    double *r = (double *)malloc(sizeof(double) * nl);
    double *p = (double *)malloc(sizeof(double) * nl);
    double *wv = (double *)malloc(sizeof(double) * nl);
    double *z = m ? (double *)malloc(sizeof(double) * nl) : r;
    int status = 0, it = 0;
    if (!g || !gid || !mult || !mask || !acc || !wr || !c || !b || !r || !p || !wv || !z ||
        or_numbering(N, nel, gid, mult, mask)) {
        status = -1;
        goto out;
    }
    vp_reg = VP_INIT;
    vp_gll(N, xi, w);
    vp_deriv(N, xi, D);
    if (vp_geometry(N, nel, vtx, xi, w, g)) { status = -4; goto out; }
    if (g_out) memcpy(g_out, g, sizeof(double) * 6 * nl);
    vp_opd op = {N, E, nl, ng, D, g, gid, mask, acc, wr};
    for (int64_t l = 0; l < nl; ++l) c[l] = 1.0 / mult[l];   /* exact: 1, 1/2, 1/4, 1/8 */
    for (int64_t l = 0; l < nl; ++l) b[l] = f[l];
    vp_reg = VP_INIT;
    for (int64_t a = 0; a < ng; ++a) acc[a] = 0.0;
    for (int64_t l = 0; l < nl; ++l) acc[gid[l]] = add(acc[gid[l]], b[l]);
    for (int64_t l = 0; l < nl; ++l) b[l] = acc[gid[l]];
    vp_mask(&op, b);

    for (int64_t l = 0; l < nl; ++l) x[l] = 0.0;
    vp_apply(&op, x, wv);
    vp_reg = VP_VEC;
    for (int64_t l = 0; l < nl; ++l) r[l] = sub(b[l], wv[l]);
    vp_reg = VP_DOT;
    double bb = vp_glsc3(nl, b, c, b);
    double rnorm0 = vp_glsc3(nl, r, c, r);
    if (hist) hist[0] = bb > 0 ? dvd(vsqrt(rnorm0), vsqrt(bb)) : 0.0;
    int converged0 = rnorm0 == 0.0 || (tol > 0 && dvd(vsqrt(rnorm0), vsqrt(bb)) <= tol);
    if (bb > 0 && !converged0) {
        double rtz1 = 1.0, rtz2;
        for (int64_t l = 0; l < nl; ++l) p[l] = 0.0;
        for (it = 1; it <= maxit; ++it) {
            if (m) {
                vp_reg = VP_VEC;
                for (int64_t l = 0; l < nl; ++l) z[l] = dvd(r[l], m[l]);
            }
            vp_reg = VP_DOT;
            rtz2 = rtz1;
            rtz1 = vp_glsc3(nl, r, c, z);
            if (rtz1 == 0.0) { --it; break; }
            double beta = it == 1 ? 0.0 : dvd(rtz1, rtz2);
            vp_reg = VP_VEC;
            for (int64_t l = 0; l < nl; ++l) p[l] = add(mul(beta, p[l]), z[l]);
            vp_apply(&op, p, wv);
            vp_reg = VP_DOT;
            double pap = vp_glsc3(nl, wv, c, p);
            if (!isfinite(pap) || !isfinite(rtz1)) { status = -6; break; }
            if (!(pap > 0)) { status = -5; break; }
            double alpha = dvd(rtz1, pap);
            vp_reg = VP_VEC;
            for (int64_t l = 0; l < nl; ++l) x[l] = add(x[l], mul(alpha, p[l]));
            for (int64_t l = 0; l < nl; ++l) r[l] = add(r[l], mul(-alpha, wv[l]));
            vp_reg = VP_DOT;
            double rtr = vp_glsc3(nl, r, c, r);
            double res = dvd(vsqrt(rtr), vsqrt(bb));
            if (hist) hist[it] = res;
            if (!isfinite(res)) { status = -6; break; }
            if (tol > 0 && res <= tol) break;
        }
        if (it > maxit) it = maxit;
    }
out:
    free(g); free(gid); free(mult); free(mask); free(acc); free(wr);
    free(c); free(b); free(r); free(p); free(wv);
    if (m) free(z);
    vp_mode = VP_IEEE;
    return status ? status : it;
}
