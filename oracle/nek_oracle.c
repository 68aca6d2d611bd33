/*
 * Serial FP64 CPU oracle for the spectral-element Poisson CG solve that
 * Nekbone runs (Chen, de Oliveira Castro, Bientinesi, Iakymchuk,
 * "Enabling mixed-precision with the help of tools: A Nekbone case study").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * Every routine is the plain definition of what it computes, in FP64, with
 * no blocking, fusion or reordering.  Build with -ffp-contract=off so that
 * every product and sum is rounded separately (IEEE round-to-nearest-even).
 *
 * Local ("element-duplicated") layout used everywhere, as in the CG loop of
 * the paper's Table 1, whose vectors have length n = E (N+1)^3:
 *     l = e*(N+1)^3 + i + (N+1)*(j + (N+1)*k),   e = ex + nx*(ey + ny*ez).
 * Geometric factors: g[e][q][i,j,k] with q = 0..5 holding
 *     G_rr, G_ss, G_tt, G_rs, G_rt, G_st   (the six factors g1..g6).
 *
 * The paper never writes the discretisation down.  The operator here is the
 * standard spectral-element stiffness matrix that the call graph of its
 * Fig. 2 evaluates (local_grad3 -> six geometric factors -> local_grad3_t on
 * Gauss-Lobatto-Legendre points), with homogeneous Dirichlet conditions on the
 * outer faces of a box of hexahedra.  Parity is pinned by closed forms and
 * invariants in the CPU tests, not by the paper.
 *
 * The same file also builds with OpenMP (the all-core timing of the CPU
 * baseline): the element loop of or_ax_local and the element-wise vector
 * updates of or_cg then run on several threads.  Every reduction and the
 * gather-scatter stay serial in their fixed order, so that build returns
 * results bit-identical to the serial one.
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* P_N(x) and P_{N-1}(x) from (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static void legendre_pair(int N, double x, double *pN, double *pNm1)
{
    double pm = 1.0, p = x;
    if (N == 0) { *pN = 1.0; *pNm1 = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double pp = ((2.0 * k + 1.0) * x * p - k * pm) / (k + 1.0);
        pm = p;
        p = pp;
    }
    *pN = p;
    *pNm1 = pm;
}

/*
 * Gauss-Lobatto-Legendre nodes and weights of order N (N+1 points).
 * Nodes: -1, the N-1 roots of P'_N, +1.  Found as the roots of
 * f(x) = x P_N(x) - P_{N-1}(x), which equals -(1-x^2) P'_N(x) / N; its
 * derivative is (N+1) P_N(x), so Newton's step is f / ((N+1) P_N).
 * Start: Chebyshev-Gauss-Lobatto points -cos(pi i / N).
 * Weights: w_i = 2 / (N (N+1) P_N(x_i)^2).
 * Returns 0, or -1 for N < 1.
 */
int or_gll(int N, double *xi, double *w)
{
    if (N < 1) return -1;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i <= N; ++i) {
        double x = -cos(pi * i / N);
        for (int it = 0; it < 100; ++it) {
            double pN, pNm1;
            legendre_pair(N, x, &pN, &pNm1);
            double dx = (x * pN - pNm1) / ((N + 1.0) * pN);
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        xi[i] = x;
    }
    /* the node set is symmetric about 0 */
    for (int i = 0; i <= N / 2; ++i) {
        double a = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -a;
        xi[N - i] = a;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 0; i <= N; ++i) {
        double pN, pNm1;
        legendre_pair(N, xi[i], &pN, &pNm1);
        w[i] = 2.0 / (N * (N + 1.0) * pN * pN);
    }
    return 0;
}

/*
 * Differentiation matrix on the GLL nodes, row-major D[i*(N+1)+j] = l_j'(x_i),
 * l_j the Lagrange polynomial of node j:
 *   D_ij = P_N(x_i) / (P_N(x_j) (x_i - x_j))   (i != j)
 *   D_00 = -N(N+1)/4,  D_NN = N(N+1)/4,  otherwise D_ii = 0.
 */
int or_deriv(int N, const double *xi, double *D)
{
    if (N < 1) return -1;
    int n = N + 1;
    double *pn = (double *)malloc(sizeof(double) * n);
    if (!pn) return -1;
    for (int i = 0; i < n; ++i) {
        double a, b;
        legendre_pair(N, xi[i], &a, &b);
        pn[i] = a;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d;
            if (i != j) d = pn[i] / (pn[j] * (xi[i] - xi[j]));
            else if (i == 0) d = -N * (N + 1.0) / 4.0;
            else if (i == N) d = N * (N + 1.0) / 4.0;
            else d = 0.0;
            D[i * n + j] = d;
        }
    free(pn);
    return 0;
}

/*
 * Global numbering of a box of nel[0] x nel[1] x nel[2] elements of order N.
 * Global lattice coordinates (ex*N+i, ey*N+j, ez*N+k) in a lattice of
 * G_d = nel[d]*N + 1 points per direction; gid = gi + Gx*(gj + Gy*gk).
 * mult[l] = number of local copies of gid[l];  mask[l] = 0 on the outer
 * faces of the box (homogeneous Dirichlet), 1 elsewhere.
 */
int or_numbering(int N, const int *nel, int64_t *gid, int32_t *mult, int8_t *mask)
{
    int n = N + 1;
    int64_t Gx = (int64_t)nel[0] * N + 1, Gy = (int64_t)nel[1] * N + 1, Gz = (int64_t)nel[2] * N + 1;
    int64_t E = (int64_t)nel[0] * nel[1] * nel[2];
    int64_t nl = E * n * n * n;
    int64_t ng = Gx * Gy * Gz;
    int32_t *count = (int32_t *)calloc((size_t)ng, sizeof(int32_t));
    if (!count) return -1;
    for (int ez = 0; ez < nel[2]; ++ez)
        for (int ey = 0; ey < nel[1]; ++ey)
            for (int ex = 0; ex < nel[0]; ++ex) {
                int64_t e = ex + (int64_t)nel[0] * (ey + (int64_t)nel[1] * ez);
                for (int k = 0; k < n; ++k)
                    for (int j = 0; j < n; ++j)
                        for (int i = 0; i < n; ++i) {
                            int64_t l = e * n * n * n + i + n * (j + n * k);
                            int64_t gi = (int64_t)ex * N + i, gj = (int64_t)ey * N + j, gk = (int64_t)ez * N + k;
                            gid[l] = gi + Gx * (gj + Gy * gk);
                            int bnd = gi == 0 || gi == Gx - 1 || gj == 0 || gj == Gy - 1 || gk == 0 || gk == Gz - 1;
                            mask[l] = bnd ? 0 : 1;
                            count[gid[l]] += 1;
                        }
            }
    for (int64_t l = 0; l < nl; ++l) mult[l] = count[gid[l]];
    free(count);
    return 0;
}

typedef struct { int64_t g, l; } or_pair;

static int or_pair_cmp(const void *a, const void *b)
{
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    if (x->g != y->g) return x->g < y->g ? -1 : 1;
    if (x->l != y->l) return x->l < y->l ? -1 : 1;
    return 0;
}

/*
 * Gather-scatter segments: every local node on an element surface (i, j or k
 * equal to 0 or N) sorted by (gid, local index).  perm lists the local
 * indices in that order; segment s covers perm[seg_ptr[s] .. seg_ptr[s+1]);
 * seg_flag[s] = 1 when the segment's global node is masked.
 * Output sizes: *nperm local surface nodes, *nseg segments.
 */
int or_segments(int N, const int *nel, const int64_t *gid, const int8_t *mask,
                int32_t *perm, int32_t *seg_ptr, int8_t *seg_flag,
                int64_t *nperm, int64_t *nseg)
{
    int n = N + 1;
    int64_t E = (int64_t)nel[0] * nel[1] * nel[2];
    int64_t nl = E * n * n * n;
    or_pair *pr = (or_pair *)malloc(sizeof(or_pair) * (size_t)nl);
    if (!pr) return -1;
    int64_t m = 0;
    for (int64_t l = 0; l < nl; ++l) {
        int64_t q = l % ((int64_t)n * n * n);
        int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((int64_t)n * n));
        int surf = i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
        if (surf) { pr[m].g = gid[l]; pr[m].l = l; ++m; }
    }
    qsort(pr, (size_t)m, sizeof(or_pair), or_pair_cmp);
    int64_t s = 0;
    for (int64_t a = 0; a < m; ++a) {
        perm[a] = (int32_t)pr[a].l;
        if (a == 0 || pr[a].g != pr[a - 1].g) {
            seg_ptr[s] = (int32_t)a;
            seg_flag[s] = mask[pr[a].l] ? 0 : 1;
            ++s;
        }
    }
    seg_ptr[s] = (int32_t)m;
    *nperm = m;
    *nseg = s;
    free(pr);
    return 0;
}

/*
 * Geometry of trilinear hexahedra.  vtx holds the (nel0+1)(nel1+1)(nel2+1)
 * vertices of the element lattice, x-index fastest, 3 coordinates each.
 * Element e maps (r,s,t) in [-1,1]^3 by
 *     X(r,s,t) = sum_{a,b,c in {0,1}} phi_a(r) phi_b(s) phi_c(t) V_abc,
 *     phi_0 = (1-r)/2, phi_1 = (1+r)/2.
 * J[d][a] = dX_d / dr_a is the exact derivative of that map.  At each GLL
 * node with tensor weight W = w_i w_j w_k:
 *     G = W det(J) J^{-1} J^{-T},   B = W det(J).
 * Outputs g[e][6][n^3] (rr, ss, tt, rs, rt, st), B[e][n^3], and, when X is
 * non-NULL, the node coordinates X[e][3][n^3].
 * Returns 0, or -4 if some det(J) <= 0 (inverted element).
 */
int or_geometry(int N, const int *nel, const double *vtx, double *g, double *B, double *X)
{
    int n = N + 1, n3 = n * n * n;
    double xi[64], w[64];
    if (n > 64 || or_gll(N, xi, w)) return -1;
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
                            double ph[3][2] = {{(1 - r) / 2, (1 + r) / 2}, {(1 - s) / 2, (1 + s) / 2}, {(1 - t) / 2, (1 + t) / 2}};
                            double dph[2] = {-0.5, 0.5};
                            double Xp[3] = {0, 0, 0}, J[3][3] = {{0}};
                            for (int c = 0; c < 2; ++c)
                                for (int b = 0; b < 2; ++b)
                                    for (int a = 0; a < 2; ++a)
                                        for (int d = 0; d < 3; ++d) {
                                            double v = V[c][b][a][d];
                                            Xp[d] += ph[0][a] * ph[1][b] * ph[2][c] * v;
                                            J[d][0] += dph[a] * ph[1][b] * ph[2][c] * v;
                                            J[d][1] += ph[0][a] * dph[b] * ph[2][c] * v;
                                            J[d][2] += ph[0][a] * ph[1][b] * dph[c] * v;
                                        }
                            double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                                       - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                                       + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                            if (!(det > 0)) bad = 1;
                            /* inverse by the adjugate: Ji[a][d] = dr_a / dx_d */
                            double Ji[3][3];
                            Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                            Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                            Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                            Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                            Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                            Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                            Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                            Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                            Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                            double W = w[i] * w[j] * w[k];
                            double Gm[3][3];
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b) {
                                    double acc = 0;
                                    for (int d = 0; d < 3; ++d) acc += Ji[a][d] * Ji[b][d];
                                    Gm[a][b] = W * det * acc;
                                }
                            int64_t q = i + n * (j + n * k);
                            double *ge = g + e * 6 * n3;
                            ge[0 * n3 + q] = Gm[0][0];
                            ge[1 * n3 + q] = Gm[1][1];
                            ge[2 * n3 + q] = Gm[2][2];
                            ge[3 * n3 + q] = Gm[0][1];
                            ge[4 * n3 + q] = Gm[0][2];
                            ge[5 * n3 + q] = Gm[1][2];
                            B[e * n3 + q] = W * det;
                            if (X)
                                for (int d = 0; d < 3; ++d) X[e * 3 * n3 + d * n3 + q] = Xp[d];
                        }
            }
    return bad ? -4 : 0;
}

/*
 * Element-local stiffness action w_L = A_L u, element by element (the ax_e
 * of Fig. 2):
 *   local_grad3:   ur = D_r u, us = D_s u, ut = D_t u,
 *                  (D_r u)_ijk = sum_l D_il u_ljk   (and likewise along j, k)
 *   geometry:      (wr,ws,wt) = G (ur,us,ut), G symmetric with g1..g6
 *   local_grad3_t: w = D_r^T wr + D_s^T ws + D_t^T wt.
 * No assembly, no mask.
 */
void or_ax_local(int N, int64_t E, const double *D, const double *g, const double *u, double *w)
{
    int n = N + 1, n3 = n * n * n;
    /* elements are independent: an OpenMP build splits them over threads
       (each with its own scratch); the arithmetic per element is unchanged */
#pragma omp parallel
    {
    double *wr = (double *)malloc(sizeof(double) * 3 * n3);
    double *ws = wr + n3, *wt = wr + 2 * n3;
#pragma omp for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double *ue = u + e * n3;
        const double *ge = g + e * 6 * n3;
        double *we = w + e * n3;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double ur = 0, us = 0, ut = 0;
                    for (int l = 0; l < n; ++l) {
                        ur += D[i * n + l] * ue[l + n * (j + n * k)];
                        us += D[j * n + l] * ue[i + n * (l + n * k)];
                        ut += D[k * n + l] * ue[i + n * (j + n * l)];
                    }
                    int q = i + n * (j + n * k);
                    double g1 = ge[q], g2 = ge[n3 + q], g3 = ge[2 * n3 + q];
                    double g4 = ge[3 * n3 + q], g5 = ge[4 * n3 + q], g6 = ge[5 * n3 + q];
                    wr[q] = g1 * ur + g4 * us + g5 * ut;
                    ws[q] = g4 * ur + g2 * us + g6 * ut;
                    wt[q] = g5 * ur + g6 * us + g3 * ut;
                }
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double acc = 0;
                    for (int l = 0; l < n; ++l) acc += D[l * n + i] * wr[l + n * (j + n * k)];
                    for (int l = 0; l < n; ++l) acc += D[l * n + j] * ws[i + n * (l + n * k)];
                    for (int l = 0; l < n; ++l) acc += D[l * n + k] * wt[i + n * (j + n * l)];
                    we[i + n * (j + n * k)] = acc;
                }
    }
    free(wr);
    }
}

/* Threads an OpenMP build runs the element loop on (1 without OpenMP);
   or_set_threads(n) changes it (no effect without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Direct-stiffness summation: for every global node, S = sum of its local
 * copies taken in ascending local index (starting from 0.0); every copy is
 * then overwritten with S.  acc must hold ng doubles.
 */
void or_dssum(int64_t nl, int64_t ng, const int64_t *gid, double *w, double *acc)
{
    for (int64_t a = 0; a < ng; ++a) acc[a] = 0.0;
    for (int64_t l = 0; l < nl; ++l) acc[gid[l]] += w[l];
    for (int64_t l = 0; l < nl; ++l) w[l] = acc[gid[l]];
}

/* Dirichlet mask: zero every local copy of a boundary node. */
void or_mask(int64_t nl, const int8_t *mask, double *w)
{
    for (int64_t l = 0; l < nl; ++l)
        if (!mask[l]) w[l] = 0.0;
}

/*
 * glsc3(a, c, b) = sum_l a_l c_l b_l (Table 1 of the paper, with the
 * multiplicity weights c), summed serially with Neumaier's compensation.
 */
double or_glsc3(int64_t nl, const double *a, const double *c, const double *b)
{
    double s = 0.0, comp = 0.0;
    for (int64_t l = 0; l < nl; ++l) {
        double t = a[l] * c[l] * b[l];
        double y = s + t;
        if (fabs(s) >= fabs(t)) comp += (s - y) + t;
        else comp += (t - y) + s;
        s = y;
    }
    return s + comp;
}

/* The same sum, plain serial order, no compensation (reported beside it). */
double or_glsc3_plain(int64_t nl, const double *a, const double *c, const double *b)
{
    double s = 0.0;
    for (int64_t l = 0; l < nl; ++l) s += a[l] * c[l] * b[l];
    return s;
}

typedef struct {
    int N;
    int nel[3];
    int64_t nl, ng, E;
    const double *D, *g;
    const int64_t *gid;
    const int8_t *mask;
    double *acc;
} or_op;

/* A u = M o dssum(A_L u): the assembled, masked operator applied to u. */
static void or_apply(const or_op *op, const double *u, double *w)
{
    or_ax_local(op->N, op->E, op->D, op->g, u, w);
    or_dssum(op->nl, op->ng, op->gid, w, op->acc);
    or_mask(op->nl, op->mask, w);
}

static int or_op_init(or_op *op, int N, const int *nel, const double *D, const double *g,
                      const int64_t *gid, const int8_t *mask)
{
    op->N = N;
    for (int d = 0; d < 3; ++d) op->nel[d] = nel[d];
    op->E = (int64_t)nel[0] * nel[1] * nel[2];
    op->nl = op->E * (N + 1) * (N + 1) * (N + 1);
    op->ng = ((int64_t)nel[0] * N + 1) * ((int64_t)nel[1] * N + 1) * ((int64_t)nel[2] * N + 1);
    op->D = D;
    op->g = g;
    op->gid = gid;
    op->mask = mask;
    op->acc = (double *)malloc(sizeof(double) * (size_t)op->ng);
    return op->acc ? 0 : -1;
}

/* w = M o dssum(A_L u). */
int or_apply_A(int N, const int *nel, const double *D, const double *g, const int64_t *gid,
               const int8_t *mask, const double *u, double *w)
{
    or_op op;
    if (or_op_init(&op, N, nel, D, g, gid, mask)) return -1;
    or_apply(&op, u, w);
    free(op.acc);
    return 0;
}

/*
 * Unpreconditioned CG in the order of the paper's Table 1 (solveM is a copy,
 * so z = r):
 *   b = M o dssum(f);  x = M o dssum(c o x0) (or 0);  r = b - A x
 *   rtz1 = 1;  p = 0
 *   per iteration:
 *     rtz2 = rtz1;  rtz1 = glsc3(r,c,r);  beta = rtz1/rtz2 (0 on the first)
 *     p = beta p + r                        (add2s1)
 *     w = A p;  pap = glsc3(w,c,p);  alpha = rtz1/pap
 *     x = x + alpha p;  r = r - alpha w     (add2s2, twice)
 *     rtr = glsc3(r,c,r)
 *   stop when sqrt(rtr)/sqrt(glsc3(b,c,b)) <= tol (tol <= 0: run maxit).
 * Before the first iteration the initial residual is tested the same way;
 * a residual of exactly zero also ends the loop (no division by zero).
 * res_hist (length maxit+1, may be NULL) receives the recursive relative
 * residual, entry 0 being the initial one.  Returns the iteration count, or
 * -5 on breakdown (pap <= 0), -6 on a non-finite value.
 */
int or_cg(int N, const int *nel, const double *D, const double *g, const int64_t *gid,
          const int32_t *mult, const int8_t *mask, const double *f, const double *x0,
          double tol, int maxit, double *x, double *res_hist)
{
    or_op op;
    if (or_op_init(&op, N, nel, D, g, gid, mask)) return -1;
    int64_t nl = op.nl;
    double *c = (double *)malloc(sizeof(double) * nl);
    double *b = (double *)malloc(sizeof(double) * nl);
    double *r = (double *)malloc(sizeof(double) * nl);
    double *p = (double *)malloc(sizeof(double) * nl);
    double *w = (double *)malloc(sizeof(double) * nl);
    for (int64_t l = 0; l < nl; ++l) c[l] = 1.0 / mult[l];

    for (int64_t l = 0; l < nl; ++l) b[l] = f[l];
    or_dssum(nl, op.ng, gid, b, op.acc);
    or_mask(nl, mask, b);

    if (x0) {
        for (int64_t l = 0; l < nl; ++l) x[l] = c[l] * x0[l];
        or_dssum(nl, op.ng, gid, x, op.acc);
        or_mask(nl, mask, x);
    } else {
        for (int64_t l = 0; l < nl; ++l) x[l] = 0.0;
    }
    or_apply(&op, x, w);
    for (int64_t l = 0; l < nl; ++l) r[l] = b[l] - w[l];

    double bb = or_glsc3(nl, b, c, b);
    double rnorm0 = or_glsc3(nl, r, c, r);
    int status = 0, it = 0;
    if (res_hist) res_hist[0] = bb > 0 ? sqrt(rnorm0) / sqrt(bb) : 0.0;
    /* Table 1 has no test before the first iteration; here a residual that
       already meets tol (or is exactly zero) ends the solve with 0 iterations. */
    int converged0 = rnorm0 == 0.0 || (tol > 0 && sqrt(rnorm0) / sqrt(bb) <= tol);
    if (bb > 0 && !converged0) {
        double rtz1 = 1.0, rtz2;
        for (int64_t l = 0; l < nl; ++l) p[l] = 0.0;
        for (it = 1; it <= maxit; ++it) {
            rtz2 = rtz1;
            rtz1 = or_glsc3(nl, r, c, r);
            if (rtz1 == 0.0) { --it; break; }   /* exact solution reached */
            double beta = it == 1 ? 0.0 : rtz1 / rtz2;
#pragma omp parallel for schedule(static)
            for (int64_t l = 0; l < nl; ++l) p[l] = beta * p[l] + r[l];
            or_apply(&op, p, w);
            double pap = or_glsc3(nl, w, c, p);
            if (!isfinite(pap) || !isfinite(rtz1)) { status = -6; break; }
            if (!(pap > 0)) { status = -5; break; }
            double alpha = rtz1 / pap;
#pragma omp parallel for schedule(static)
            for (int64_t l = 0; l < nl; ++l) {
                x[l] = x[l] + alpha * p[l];
                r[l] = r[l] + (-alpha) * w[l];
            }
            double rtr = or_glsc3(nl, r, c, r);
            double res = sqrt(rtr) / sqrt(bb);
            if (res_hist) res_hist[it] = res;
            if (!isfinite(res)) { status = -6; break; }
            if (tol > 0 && res <= tol) break;
        }
        if (it > maxit) it = maxit;
    }
    free(c); free(b); free(r); free(p); free(w);
    free(op.acc);
    return status ? status : it;
}

/*
 * Diagonal of the assembled masked operator, the Jacobi preconditioner of
 * the solveM step of Table 1.  For A_L = sum_{a,b in r,s,t} D_a^T G_ab D_b the
 * entry at node p = (i,j,k) of an element is
 *     sum_l D_li^2 G_rr(l,j,k) + sum_l D_lj^2 G_ss(i,l,k) + sum_l D_lk^2 G_tt(i,j,l)
 *   + 2 D_ii D_jj G_rs(p) + 2 D_ii D_kk G_rt(p) + 2 D_jj D_kk G_st(p),
 * because (D_r)_{q,p} = D_{q_i, i} when q shares j and k with p (0 otherwise),
 * so a cross term survives only at q = p.  The element values are summed
 * over the copies of each node (ascending local index); nodes on the
 * Dirichlet boundary get 1 (their residual is 0, so z = r / m is 0 there).
 */
int or_diag(int N, const int *nel, const double *D, const double *g, const int64_t *gid, const int8_t *mask,
            double *m)
{
    int n = N + 1, n3 = n * n * n;
    int64_t E = (int64_t)nel[0] * nel[1] * nel[2], nl = E * n3;
    int64_t ng = ((int64_t)nel[0] * N + 1) * ((int64_t)nel[1] * N + 1) * ((int64_t)nel[2] * N + 1);
    double *acc = (double *)malloc(sizeof(double) * (size_t)ng);
    if (!acc) return -1;
    for (int64_t e = 0; e < E; ++e) {
        const double *ge = g + e * 6 * n3;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double d = 0.0;
                    for (int l = 0; l < n; ++l) d += D[l * n + i] * D[l * n + i] * ge[0 * n3 + l + n * (j + n * k)];
                    for (int l = 0; l < n; ++l) d += D[l * n + j] * D[l * n + j] * ge[1 * n3 + i + n * (l + n * k)];
                    for (int l = 0; l < n; ++l) d += D[l * n + k] * D[l * n + k] * ge[2 * n3 + i + n * (j + n * l)];
                    int q = i + n * (j + n * k);
                    double di = D[i * n + i], dj = D[j * n + j], dk = D[k * n + k];
                    d += 2.0 * di * dj * ge[3 * n3 + q];
                    d += 2.0 * di * dk * ge[4 * n3 + q];
                    d += 2.0 * dj * dk * ge[5 * n3 + q];
                    m[e * n3 + q] = d;
                }
    }
    or_dssum(nl, ng, gid, m, acc);
    for (int64_t l = 0; l < nl; ++l)
        if (!mask[l]) m[l] = 1.0;
    free(acc);
    return 0;
}

/*
 * Preconditioned CG in the order of Table 1 with solveM: z = r / m
 * (diagonal preconditioner m > 0, given per local node, equal on copies):
 *   per iteration:
 *     z = r / m                              (solveM)
 *     rtz2 = rtz1;  rtz1 = glsc3(r,c,z);  beta = rtz1/rtz2 (0 on the first)
 *     p = beta p + z                         (add2s1)
 *     w = A p;  pap = glsc3(w,c,p);  alpha = rtz1/pap
 *     x = x + alpha p;  r = r - alpha w
 *     rtr = glsc3(r,c,r)
 * The stopping test, the start and the outputs are those of or_cg (the
 * residual r itself is tested, not z).  With m = 1 every value equals
 * or_cg's bit for bit.
 */
int or_pcg(int N, const int *nel, const double *D, const double *g, const int64_t *gid,
           const int32_t *mult, const int8_t *mask, const double *m, const double *f, const double *x0,
           double tol, int maxit, double *x, double *res_hist)
{
    or_op op;
    if (or_op_init(&op, N, nel, D, g, gid, mask)) return -1;
    int64_t nl = op.nl;
    double *c = (double *)malloc(sizeof(double) * nl);
    double *b = (double *)malloc(sizeof(double) * nl);
    double *r = (double *)malloc(sizeof(double) * nl);
    double *z = (double *)malloc(sizeof(double) * nl);
    double *p = (double *)malloc(sizeof(double) * nl);
    double *w = (double *)malloc(sizeof(double) * nl);
    for (int64_t l = 0; l < nl; ++l) c[l] = 1.0 / mult[l];

    for (int64_t l = 0; l < nl; ++l) b[l] = f[l];
    or_dssum(nl, op.ng, gid, b, op.acc);
    or_mask(nl, mask, b);

    if (x0) {
        for (int64_t l = 0; l < nl; ++l) x[l] = c[l] * x0[l];
        or_dssum(nl, op.ng, gid, x, op.acc);
        or_mask(nl, mask, x);
    } else {
        for (int64_t l = 0; l < nl; ++l) x[l] = 0.0;
    }
    or_apply(&op, x, w);
    for (int64_t l = 0; l < nl; ++l) r[l] = b[l] - w[l];

    double bb = or_glsc3(nl, b, c, b);
    double rnorm0 = or_glsc3(nl, r, c, r);
    int status = 0, it = 0;
    if (res_hist) res_hist[0] = bb > 0 ? sqrt(rnorm0) / sqrt(bb) : 0.0;
    int converged0 = rnorm0 == 0.0 || (tol > 0 && sqrt(rnorm0) / sqrt(bb) <= tol);
    if (bb > 0 && !converged0) {
        double rtz1 = 1.0, rtz2;
        for (int64_t l = 0; l < nl; ++l) p[l] = 0.0;
        for (it = 1; it <= maxit; ++it) {
            for (int64_t l = 0; l < nl; ++l) z[l] = r[l] / m[l];
            rtz2 = rtz1;
            rtz1 = or_glsc3(nl, r, c, z);
            if (rtz1 == 0.0) { --it; break; }
            double beta = it == 1 ? 0.0 : rtz1 / rtz2;
            for (int64_t l = 0; l < nl; ++l) p[l] = beta * p[l] + z[l];
            or_apply(&op, p, w);
            double pap = or_glsc3(nl, w, c, p);
            if (!isfinite(pap) || !isfinite(rtz1)) { status = -6; break; }
            if (!(pap > 0)) { status = -5; break; }
            double alpha = rtz1 / pap;
#pragma omp parallel for schedule(static)
            for (int64_t l = 0; l < nl; ++l) {
                x[l] = x[l] + alpha * p[l];
                r[l] = r[l] + (-alpha) * w[l];
            }
            double rtr = or_glsc3(nl, r, c, r);
            double res = sqrt(rtr) / sqrt(bb);
            if (res_hist) res_hist[it] = res;
            if (!isfinite(res)) { status = -6; break; }
            if (tol > 0 && res <= tol) break;
        }
        if (it > maxit) it = maxit;
    }
    free(c); free(b); free(r); free(z); free(p); free(w);
    free(op.acc);
    return status ? status : it;
}
