// Host-side FP64 initialisation for libnek: GLL rule, differentiation
// matrix, trilinear geometry and the sorted-segment gather-scatter maps.
// The paper's mixed build leaves all of this set-up in double precision and
// lowers only the CG loop (Sect. 6).
#include "nek_setup.hpp"

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace nek {

// Legendre P_N, P_N' at x by the three-term recurrence and
// P'_{k+1} = P'_{k-1} + (2k+1) P_k.
static void legendre_with_deriv(int N, double x, double &p, double &dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (N == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        double d2 = d0 + (2 * k + 1) * p1;
        p0 = p1; p1 = p2;
        d0 = d1; d1 = d2;
    }
    p = p1;
    dp = d1;
}

// GLL points: +-1 and the zeros of P_N'.  Newton on P_N' with P_N'' taken
// from Legendre's equation (1-x^2) P'' = 2x P' - N(N+1) P.
void gll_rule(int N, std::vector<double> &x, std::vector<double> &w)
{
    const int n = N + 1;
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    x[0] = -1.0;
    x[N] = 1.0;
    const double pi = std::acos(-1.0);
    for (int i = 1; i < N; ++i) {
        // interior Chebyshev-Lobatto guess, refined by Newton
        double t = -std::cos(pi * i / N);
        for (int it = 0; it < 60; ++it) {
            double p, dp;
            legendre_with_deriv(N, t, p, dp);
            double ddp = (2.0 * t * dp - N * (N + 1.0) * p) / (1.0 - t * t);
            double step = dp / ddp;
            t -= step;
            if (std::fabs(step) <= 1e-16 * std::max(1.0, std::fabs(t))) break;
        }
        x[i] = t;
    }
    for (int i = 0; i < n / 2; ++i) {   // symmetric node set
        double m = 0.5 * (x[N - i] - x[i]);
        x[i] = -m;
        x[N - i] = m;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    for (int i = 0; i < n; ++i) {
        double p, dp;
        legendre_with_deriv(N, x[i], p, dp);
        w[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
}

// Derivative of the Lagrange interpolant in barycentric form:
// D_ij = (lam_j / lam_i) / (x_i - x_j), lam_j = 1 / prod_{k != j} (x_j - x_k),
// and D_ii = -sum_{j != i} D_ij so that constants are differentiated to zero.
void deriv_matrix(const std::vector<double> &x, std::vector<double> &D)
{
    const int n = (int)x.size();
    std::vector<double> lam(n, 1.0);
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) prod *= (x[j] - x[k]);
        lam[j] = 1.0 / prod;
    }
    D.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double v = (lam[j] / lam[i]) / (x[i] - x[j]);
            D[(size_t)i * n + j] = v;
            diag -= v;
        }
        D[(size_t)i * n + i] = diag;
    }
}

void uniform_vertices(const int nel[3], const double lo[3], const double hi[3], std::vector<double> &vtx)
{
    const long vx = nel[0] + 1, vy = nel[1] + 1, vz = nel[2] + 1;
    vtx.resize((size_t)vx * vy * vz * 3);
    for (long c = 0; c < vz; ++c)
        for (long b = 0; b < vy; ++b)
            for (long a = 0; a < vx; ++a) {
                long v = a + vx * (b + vy * c);
                long idx[3] = {a, b, c};
                for (int d = 0; d < 3; ++d) {
                    double t = (double)idx[d] / nel[d];
                    vtx[3 * v + d] = idx[d] == nel[d] ? hi[d] : lo[d] + (hi[d] - lo[d]) * t;
                }
            }
}

// One element: X at the GLL nodes from the 8 vertices, J = D X along r, s, t
// (exact for a trilinear map), then G = W det(J) J^-1 J^-T and B = W det(J).
static int element_geometry(int N, const std::vector<double> &x, const std::vector<double> &w,
                            const std::vector<double> &D, const double V[8][3], double *g, double *B,
                            double *X, long n3)
{
    const int n = N + 1;
    std::vector<double> Xe(3 * (size_t)n3);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double hr[2] = {0.5 * (1 - x[i]), 0.5 * (1 + x[i])};
                double hs[2] = {0.5 * (1 - x[j]), 0.5 * (1 + x[j])};
                double ht[2] = {0.5 * (1 - x[k]), 0.5 * (1 + x[k])};
                long q = i + n * (j + (long)n * k);
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int v = 0; v < 8; ++v)
                        s += hr[v & 1] * hs[(v >> 1) & 1] * ht[v >> 2] * V[v][d];
                    Xe[d * n3 + q] = s;
                }
            }
    int bad = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long q = i + n * (j + (long)n * k);
                double J[3][3];   // J[d][a] = dx_d / dr_a
                for (int d = 0; d < 3; ++d) {
                    const double *Xd = &Xe[d * n3];
                    double a0 = 0, a1 = 0, a2 = 0;
                    for (int m = 0; m < n; ++m) {
                        a0 += D[(size_t)i * n + m] * Xd[m + n * (j + (long)n * k)];
                        a1 += D[(size_t)j * n + m] * Xd[i + n * (m + (long)n * k)];
                        a2 += D[(size_t)k * n + m] * Xd[i + n * (j + (long)n * m)];
                    }
                    J[d][0] = a0; J[d][1] = a1; J[d][2] = a2;
                }
                double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
                if (!(det > 0)) { bad = 1; det = 1.0; }
                // rows of the inverse: R[a][d] = dr_a / dx_d = cofactor(d,a) / det
                double R[3][3];
                R[0][0] = c00 / det; R[1][0] = c01 / det; R[2][0] = c02 / det;
                R[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                R[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                R[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                R[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                R[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                R[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                double wdet = w[i] * w[j] * w[k] * det;
                auto dot = [&](int a, int b) { return R[a][0] * R[b][0] + R[a][1] * R[b][1] + R[a][2] * R[b][2]; };
                g[0 * n3 + q] = wdet * dot(0, 0);
                g[1 * n3 + q] = wdet * dot(1, 1);
                g[2 * n3 + q] = wdet * dot(2, 2);
                g[3 * n3 + q] = wdet * dot(0, 1);
                g[4 * n3 + q] = wdet * dot(0, 2);
                g[5 * n3 + q] = wdet * dot(1, 2);
                B[q] = wdet;
                if (X)
                    for (int d = 0; d < 3; ++d) X[d * n3 + q] = Xe[d * n3 + q];
            }
    return bad;
}

// A[d][m]: coefficient m of x_d(r,s,t) = a0 + a1 r + a2 s + a3 t + a4 rs
// + a5 rt + a6 st + a7 rst for element e; a_m = 1/8 sum over the 8 vertices
// of (the product of the vertex's +-1 coordinates in m's variables) X_v.
// Returns nonzero if det(J) is not positive at some GLL node x^3.
static int element_trilinear(const int nel[3], const std::vector<double> &vtx, const std::vector<double> &x, long e,
                             double A[3][8])
{
    const long vx = nel[0] + 1, vy = nel[1] + 1;
    const long ex = e % nel[0], ey = (e / nel[0]) % nel[1], ez = e / ((long)nel[0] * nel[1]);
    for (int d = 0; d < 3; ++d) {
        double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int v = 0; v < 8; ++v) {
            const long ia = ex + (v & 1), ib = ey + ((v >> 1) & 1), ic = ez + (v >> 2);
            const double X = vtx[3 * (ia + vx * (ib + vy * ic)) + d];
            const double sr = (v & 1) ? 1.0 : -1.0, ss = (v & 2) ? 1.0 : -1.0, st = (v & 4) ? 1.0 : -1.0;
            a[0] += X;
            a[1] += sr * X;
            a[2] += ss * X;
            a[3] += st * X;
            a[4] += sr * ss * X;
            a[5] += sr * st * X;
            a[6] += ss * st * X;
            a[7] += sr * ss * st * X;
        }
        for (int m = 0; m < 8; ++m) A[d][m] = 0.125 * a[m];
    }
    const int n = (int)x.size();
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const double r = x[i], s = x[j], t = x[k];
                double J[3][3];
                for (int d = 0; d < 3; ++d) {
                    const double *a = A[d];
                    J[d][0] = a[1] + a[4] * s + a[5] * t + a[7] * s * t;
                    J[d][1] = a[2] + a[4] * r + a[6] * t + a[7] * r * t;
                    J[d][2] = a[3] + a[5] * r + a[6] * s + a[7] * r * s;
                }
                const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                   J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                   J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                if (!(det > 0)) return 1;
            }
    return 0;
}

int trilinear_all(int N, const int nel[3], const std::vector<double> &vtx, double *coef)
{
    std::vector<double> x, w;
    gll_rule(N, x, w);
    const long E = (long)nel[0] * nel[1] * nel[2];
    int bad = 0;
    for (long e = 0; e < E; ++e) {
        double A[3][8];
        bad |= element_trilinear(nel, vtx, x, e, A);
        for (int d = 0; d < 3; ++d)
            for (int m = 0; m < 8; ++m) coef[(e * 3 + d) * 8 + m] = A[d][m];
    }
    return bad;
}

int trilinear_coefs(int N, const int nel[3], const std::vector<double> &vtx, const std::vector<double> &x,
                    const std::vector<double> &w, int hdr, std::vector<double> &out)
{
    const int n = N + 1;
    const long E = (long)nel[0] * nel[1] * nel[2];
    out.assign((size_t)hdr + (size_t)E * 24, 0.0);
    for (int i = 0; i < n; ++i) {
        out[i] = x[i];
        out[n + i] = w[i];
    }
    int bad = 0;
    for (long e = 0; e < E; ++e) {
        double A[3][8];
        bad |= element_trilinear(nel, vtx, x, e, A);
        double *rec = &out[hdr + (size_t)e * 24];
        for (int d = 0; d < 3; ++d)
            for (int m = 0; m < 7; ++m) rec[8 * d + m] = A[d][m + 1];
    }
    return bad;
}

int geometry(int N, const int nel[3], const std::vector<double> &vtx, const std::vector<double> &x,
             const std::vector<double> &w, const std::vector<double> &D, double *g, double *B, double *X)
{
    const int n = N + 1;
    const long n3 = (long)n * n * n;
    const long E = (long)nel[0] * nel[1] * nel[2];
    const long vx = nel[0] + 1, vy = nel[1] + 1;
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (E < 64) nt = 1;
    std::vector<int> bad(nt, 0);
    auto work = [&](unsigned tid) {
        for (long e = tid; e < E; e += nt) {
            long ex = e % nel[0], ey = (e / nel[0]) % nel[1], ez = e / ((long)nel[0] * nel[1]);
            double V[8][3];
            for (int v = 0; v < 8; ++v) {
                long a = ex + (v & 1), b = ey + ((v >> 1) & 1), c = ez + (v >> 2);
                for (int d = 0; d < 3; ++d) V[v][d] = vtx[3 * (a + vx * (b + vy * c)) + d];
            }
            bad[tid] |= element_geometry(N, x, w, D, V, g + e * 6 * n3, B + e * n3, X ? X + e * 3 * n3 : nullptr, n3);
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &t : th) t.join();
    for (int b : bad)
        if (b) return 1;
    return 0;
}

// Local node l -> (element coords, i, j, k) -> global lattice id.
static inline long global_id(long l, int N, const int nel[3], long Gx, long Gy)
{
    const long n = N + 1, n3 = n * n * n;
    long e = l / n3, q = l - e * n3;
    long i = q % n, j = (q / n) % n, k = q / (n * n);
    long ex = e % nel[0], ey = (e / nel[0]) % nel[1], ez = e / ((long)nel[0] * nel[1]);
    return (ex * N + i) + Gx * ((ey * N + j) + Gy * (ez * N + k));
}

// Segments by counting sort over global ids: walk the local nodes in
// ascending order, so the copies of each node come out in ascending local
// index and the segments in ascending global id.
void segment_maps(int N, const int nel[3], std::vector<int32_t> &perm, std::vector<int32_t> &seg_ptr,
                  std::vector<int8_t> &seg_flag)
{
    const long n = N + 1, n3 = n * n * n;
    const long E = (long)nel[0] * nel[1] * nel[2];
    const long nl = E * n3;
    const long Gx = (long)nel[0] * N + 1, Gy = (long)nel[1] * N + 1, Gz = (long)nel[2] * N + 1;
    const long ng = Gx * Gy * Gz;
    auto on_surface = [&](long l) {
        long q = l % n3;
        long i = q % n, j = (q / n) % n, k = q / (n * n);
        return i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
    };
    std::vector<int32_t> count(ng, 0);
    long m = 0;
    for (long l = 0; l < nl; ++l)
        if (on_surface(l)) { ++count[global_id(l, N, nel, Gx, Gy)]; ++m; }
    std::vector<int32_t> start(ng, -1);
    seg_ptr.clear();
    seg_flag.clear();
    long pos = 0;
    for (long gidx = 0; gidx < ng; ++gidx) {
        if (!count[gidx]) continue;
        start[gidx] = (int32_t)pos;
        seg_ptr.push_back((int32_t)pos);
        long gi = gidx % Gx, gj = (gidx / Gx) % Gy, gk = gidx / (Gx * Gy);
        bool bnd = gi == 0 || gi == Gx - 1 || gj == 0 || gj == Gy - 1 || gk == 0 || gk == Gz - 1;
        seg_flag.push_back(bnd ? 1 : 0);
        pos += count[gidx];
    }
    seg_ptr.push_back((int32_t)pos);
    perm.assign(m, 0);
    for (long l = 0; l < nl; ++l)
        if (on_surface(l)) perm[start[global_id(l, N, nel, Gx, Gy)]++] = (int32_t)l;
}

void numbering(int N, const int nel[3], int64_t *gid, int32_t *mult, int8_t *mask)
{
    const long n = N + 1, n3 = n * n * n;
    const long E = (long)nel[0] * nel[1] * nel[2];
    const long Gx = (long)nel[0] * N + 1, Gy = (long)nel[1] * N + 1;
    for (long l = 0; l < E * n3; ++l) {
        long e = l / n3, q = l - e * n3;
        long i = q % n, j = (q / n) % n, k = q / (n * n);
        long ex = e % nel[0], ey = (e / nel[0]) % nel[1], ez = e / ((long)nel[0] * nel[1]);
        long c[3] = {i, j, k}, el[3] = {ex, ey, ez};
        int m = 1, bnd = 0;
        for (int d = 0; d < 3; ++d) {
            bool lo = c[d] == 0, hi = c[d] == N;
            if ((lo && el[d] == 0) || (hi && el[d] == nel[d] - 1)) bnd = 1;
            if ((lo && el[d] > 0) || (hi && el[d] < nel[d] - 1)) m *= 2;
        }
        if (gid) gid[l] = global_id(l, N, nel, Gx, Gy);
        if (mult) mult[l] = m;
        if (mask) mask[l] = bnd ? 0 : 1;
    }
}

// Interior modes of the 1-D GLL stiffness for the fast-diagonalization
// block solve: K_I S = W_I S Lambda with S^T W_I S = I, where K = D^T W D and
// the subscript I keeps the N-1 interior nodes.  W_I is diagonal, so this is
// the symmetric eigenproblem of C = W_I^-1/2 K_I W_I^-1/2, solved by cyclic
// Jacobi rotations; S = W_I^-1/2 V.  S is row-major S[i * (N-1) + a] (node i,
// mode a).
// Eigen-decomposition of the symmetric m x m matrix C (row-major, destroyed)
// by cyclic Jacobi rotations: C = V diag(lam) V^T, V row-major [row][mode].
void sym_eig(int m, std::vector<double> &C, std::vector<double> &V, std::vector<double> &lam)
{
    V.assign((size_t)m * m, 0.0);
    lam.assign(m, 0.0);
    for (int a = 0; a < m; ++a) V[a * m + a] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) (a == b ? diag : off) += C[a * m + b] * C[a * m + b];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = C[p * m + q];
                if (apq == 0.0) continue;
                // rotation that zeroes C[p][q]: tan(2 theta) = 2 apq / (aqq - app)
                const double theta = 0.5 * std::atan2(2.0 * apq, C[q * m + q] - C[p * m + p]);
                const double c = std::cos(theta), sn = std::sin(theta);
                for (int k = 0; k < m; ++k) {   // C <- C G (columns p, q)
                    const double ckp = C[k * m + p], ckq = C[k * m + q];
                    C[k * m + p] = c * ckp - sn * ckq;
                    C[k * m + q] = sn * ckp + c * ckq;
                }
                for (int k = 0; k < m; ++k) {   // C <- G^T C (rows p, q)
                    const double cpk = C[p * m + k], cqk = C[q * m + k];
                    C[p * m + k] = c * cpk - sn * cqk;
                    C[q * m + k] = sn * cpk + c * cqk;
                }
                for (int k = 0; k < m; ++k) {   // V <- V G
                    const double vkp = V[k * m + p], vkq = V[k * m + q];
                    V[k * m + p] = c * vkp - sn * vkq;
                    V[k * m + q] = sn * vkp + c * vkq;
                }
            }
    }
    for (int a = 0; a < m; ++a) lam[a] = C[a * m + a];
}

void fdm_modes(int N, const std::vector<double> &w, const std::vector<double> &D, std::vector<double> &S,
               std::vector<double> &lam)
{
    const int n = N + 1, m = N - 1;
    S.assign((size_t)std::max(m, 0) * std::max(m, 0), 0.0);
    lam.assign(std::max(m, 0), 0.0);
    if (m <= 0) return;
    std::vector<double> C((size_t)m * m), V, s(m);
    for (int a = 0; a < m; ++a) s[a] = 1.0 / std::sqrt(w[a + 1]);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double k = 0.0;   // K[a+1][b+1] = sum_l D[l][a+1] w[l] D[l][b+1]
            for (int l = 0; l < n; ++l) k += D[l * n + a + 1] * w[l] * D[l * n + b + 1];
            C[a * m + b] = s[a] * k * s[b];
        }
    sym_eig(m, C, V, lam);
    for (int a = 0; a < m; ++a)
        for (int i = 0; i < m; ++i) S[i * m + a] = s[i] * V[i * m + a];
}

// Overlapping Schwarz windows.  The window of an element along one direction
// holds NW = N + 3 nodes: the left neighbour's node N-1, the element's nodes
// 0..N and the right neighbour's node 1.  Kw, Ww: the 1-D GLL stiffness
// D^T W D and the mass W of three reference elements assembled along the line
// and restricted to the window.  Variant v = lo + 2 hi drops the two nodes on
// the left (lo: the element's left face is the Dirichlet boundary, the node
// beyond it does not exist) and / or the two on the right.  For each variant
// K S = W S Lambda (S^T W S = I) on the kept nodes; S is stored padded to
// NW x NW (row = window node, column = mode; rows of dropped nodes and
// columns past the kept count are 0, their lambda 1).  S[v][a][m] =
// S[(v * NW + a) * NW + m], lam[v * NW + m].
void schwarz_windows(int N, const std::vector<double> &w, const std::vector<double> &D, std::vector<double> &S,
                     std::vector<double> &lam)
{
    const int n = N + 1, NW = N + 3, L = 3 * N + 1;
    std::vector<double> K((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            for (int l = 0; l < n; ++l) K[a * n + b] += D[l * n + a] * w[l] * D[l * n + b];
    std::vector<double> Ka((size_t)L * L, 0.0), Wa(L, 0.0);
    for (int q = 0; q < 3; ++q)
        for (int a = 0; a < n; ++a) {
            Wa[q * N + a] += w[a];
            for (int b = 0; b < n; ++b) Ka[(q * N + a) * L + q * N + b] += K[a * n + b];
        }
    S.assign((size_t)4 * NW * NW, 0.0);
    lam.assign((size_t)4 * NW, 1.0);
    for (int v = 0; v < 4; ++v) {
        const int a0 = (v & 1) ? 2 : 0, a1 = (v & 2) ? N + 1 : N + 3;   // kept window nodes [a0, a1)
        const int m = a1 - a0;
        std::vector<double> C((size_t)m * m), V, l, s(m);
        for (int a = 0; a < m; ++a) s[a] = 1.0 / std::sqrt(Wa[N - 1 + a0 + a]);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) C[a * m + b] = s[a] * Ka[(N - 1 + a0 + a) * L + N - 1 + a0 + b] * s[b];
        sym_eig(m, C, V, l);
        for (int md = 0; md < m; ++md) {
            lam[v * NW + md] = l[md];
            for (int a = 0; a < m; ++a) S[((size_t)v * NW + a0 + a) * NW + md] = s[a] * V[a * m + md];
        }
    }
}

// Coarse level of the Schwarz preconditioner along each direction d: the
// trilinear (Q1) functions on the vertex lattice, on the rectilinear
// lattice whose spacing in slab q is the mean of the element lengths h_d
// over the slab (h_d per element: mean of its four edges along d).  The 1-D
// stiffness is assembled from (1/h) [[1,-1],[-1,1]] and the mass from
// (h/2) [sum_q w_q l_a(x_q) l_b(x_q)] (the GLL rule of order N; l_0 = (1-x)/2,
// l_1 = (1+x)/2), both restricted to the n_d - 1 interior vertices; then
// K S = M S Lambda with S^T M S = I (Cholesky M = L L^T, C = L^-1 K L^-T =
// V Lambda V^T, S = L^-T V).  Out: per direction, S row-major [vertex][mode]
// at offset off[d] of S (size (n_d - 1)^2) and lambda at offset loff[d].
void schwarz_coarse(int N, const int nel[3], const std::vector<double> &vtx, const std::vector<double> &x,
                    const std::vector<double> &w, std::vector<double> &S, std::vector<double> &lam, int off[3],
                    int loff[3])
{
    // element mean lengths: the mean of each element's four edges along d
    const long vx = nel[0] + 1, vy = nel[1] + 1;
    auto V = [&](long a, long b, long c, int d) { return vtx[3 * (a + vx * (b + vy * c)) + d]; };
    auto len = [&](long a0, long b0, long c0, long a1, long b1, long c1) {
        double s2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double t = V(a1, b1, c1, d) - V(a0, b0, c0, d);
            s2 += t * t;
        }
        return std::sqrt(s2);
    };
    std::vector<double> slab[3];
    for (int d = 0; d < 3; ++d) slab[d].assign(nel[d], 0.0);
    for (long ez = 0; ez < nel[2]; ++ez)
        for (long ey = 0; ey < nel[1]; ++ey)
            for (long ex = 0; ex < nel[0]; ++ex) {
                double h[3] = {0.0, 0.0, 0.0};
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v) {
                        h[0] += len(ex, ey + u, ez + v, ex + 1, ey + u, ez + v);
                        h[1] += len(ex + u, ey, ez + v, ex + u, ey + 1, ez + v);
                        h[2] += len(ex + u, ey + v, ez, ex + u, ey + v, ez + 1);
                    }
                slab[0][ex] += 0.25 * h[0];
                slab[1][ey] += 0.25 * h[1];
                slab[2][ez] += 0.25 * h[2];
            }
    const double cnt[3] = {(double)nel[1] * nel[2], (double)nel[0] * nel[2], (double)nel[0] * nel[1]};
    double me[2][2] = {{0, 0}, {0, 0}};
    for (size_t q = 0; q < x.size(); ++q) {
        const double l[2] = {(1.0 - x[q]) / 2.0, (1.0 + x[q]) / 2.0};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) me[a][b] += w[q] * l[a] * l[b];
    }
    S.clear();
    lam.clear();
    for (int d = 0; d < 3; ++d) {
        const int n = nel[d], m = n - 1;
        off[d] = (int)S.size();
        loff[d] = (int)lam.size();
        if (m <= 0) continue;
        std::vector<double> Kf((size_t)(n + 1) * (n + 1), 0.0), Mf((size_t)(n + 1) * (n + 1), 0.0);
        for (int e = 0; e < n; ++e) {
            const double h = slab[d][e] / cnt[d];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    Kf[(e + a) * (n + 1) + e + b] += (a == b ? 1.0 : -1.0) / h;
                    Mf[(e + a) * (n + 1) + e + b] += me[a][b] * h / 2.0;
                }
        }
        // interior block, Cholesky of M
        std::vector<double> K((size_t)m * m), M((size_t)m * m), Lc((size_t)m * m, 0.0);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) {
                K[a * m + b] = Kf[(a + 1) * (n + 1) + b + 1];
                M[a * m + b] = Mf[(a + 1) * (n + 1) + b + 1];
            }
        for (int a = 0; a < m; ++a)
            for (int b = 0; b <= a; ++b) {
                double t = M[a * m + b];
                for (int q = 0; q < b; ++q) t -= Lc[a * m + q] * Lc[b * m + q];
                Lc[a * m + b] = a == b ? std::sqrt(t) : t / Lc[b * m + b];
            }
        // Li = L^-1 (lower triangular)
        std::vector<double> Li((size_t)m * m, 0.0);
        for (int col = 0; col < m; ++col)
            for (int a = col; a < m; ++a) {
                double t = a == col ? 1.0 : 0.0;
                for (int q = col; q < a; ++q) t -= Lc[a * m + q] * Li[q * m + col];
                Li[a * m + col] = t / Lc[a * m + a];
            }
        std::vector<double> T((size_t)m * m, 0.0), C((size_t)m * m, 0.0), Vv, l;
        for (int a = 0; a < m; ++a)   // T = Li K
            for (int b = 0; b < m; ++b) {
                double t = 0.0;
                for (int q = 0; q <= a; ++q) t += Li[a * m + q] * K[q * m + b];
                T[a * m + b] = t;
            }
        for (int a = 0; a < m; ++a)   // C = T Li^T, symmetrised
            for (int b = 0; b < m; ++b) {
                double t = 0.0;
                for (int q = 0; q <= b; ++q) t += T[a * m + q] * Li[b * m + q];
                C[a * m + b] = t;
            }
        for (int a = 0; a < m; ++a)
            for (int b = a + 1; b < m; ++b) C[a * m + b] = C[b * m + a] = 0.5 * (C[a * m + b] + C[b * m + a]);
        sym_eig(m, C, Vv, l);
        const size_t base = S.size();
        S.resize(base + (size_t)m * m, 0.0);
        for (int a = 0; a < m; ++a)   // S = Li^T V
            for (int md = 0; md < m; ++md) {
                double t = 0.0;
                for (int q = a; q < m; ++q) t += Li[q * m + a] * Vv[q * m + md];
                S[base + (size_t)a * m + md] = t;
            }
        lam.insert(lam.end(), l.begin(), l.end());
    }
}

// Per element (cx, cy, cz) = (hy hz / hx, hx hz / hy, hx hy / hz), h_d the
// mean length of the element's four edges along direction d, from the vertex
// lattice (x-index fastest).  cf has 3 E entries.
void fdm_scales(const int nel[3], const std::vector<double> &vtx, double *cf)
{
    const long vx = nel[0] + 1, vy = nel[1] + 1;
    auto V = [&](long a, long b, long c, int d) { return vtx[3 * (a + vx * (b + vy * c)) + d]; };
    auto len = [&](long a0, long b0, long c0, long a1, long b1, long c1) {
        double s2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double t = V(a1, b1, c1, d) - V(a0, b0, c0, d);
            s2 += t * t;
        }
        return std::sqrt(s2);
    };
    for (long ez = 0; ez < nel[2]; ++ez)
        for (long ey = 0; ey < nel[1]; ++ey)
            for (long ex = 0; ex < nel[0]; ++ex) {
                double h[3] = {0.0, 0.0, 0.0};
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v) {
                        h[0] += len(ex, ey + u, ez + v, ex + 1, ey + u, ez + v);
                        h[1] += len(ex + u, ey, ez + v, ex + u, ey + 1, ez + v);
                        h[2] += len(ex + u, ey + v, ez, ex + u, ey + v, ez + 1);
                    }
                for (double &t : h) t *= 0.25;
                double *c = cf + 3 * (ex + nel[0] * (ey + nel[1] * ez));
                c[0] = h[1] * h[2] / h[0];
                c[1] = h[0] * h[2] / h[1];
                c[2] = h[0] * h[1] / h[2];
            }
}

// Diagonal of the assembled masked operator M o dssum(A_L), the Jacobi
// preconditioner of Table 1's solveM step.  Per element node (i,j,k), with
// A_L = sum_{a,b} D_a^T G_ab D_b: the squared entries of D's columns i, j, k
// against G_rr, G_ss, G_tt along the node's three lines, plus 2 D_ii D_jj
// G_rs + 2 D_ii D_kk G_rt + 2 D_jj D_kk G_st at the node (the only place a
// mixed term survives).  Copies of a node are summed in ascending local
// index; Dirichlet nodes get 1.  g is [E][6][n^3]; m has E n^3 entries.
void assembled_diagonal(int N, const int nel[3], const std::vector<double> &D, const double *g, double *m)
{
    const long n = N + 1, n2 = n * n, n3 = n2 * n;
    const long E = (long)nel[0] * nel[1] * nel[2], nl = E * n3;
    std::vector<double> sq(n * n), dd(n);   // sq[a*n + i] = D[a][i]^2
    for (long a = 0; a < n; ++a) {
        dd[a] = D[a * n + a];
        for (long i = 0; i < n; ++i) sq[a * n + i] = D[a * n + i] * D[a * n + i];
    }
    for (long e = 0; e < E; ++e) {
        const double *grr = g + e * 6 * n3, *gss = grr + n3, *gtt = gss + n3;
        const double *grs = gtt + n3, *grt = grs + n3, *gst = grt + n3;
        double *me = m + e * n3;
        for (long k = 0; k < n; ++k)
            for (long j = 0; j < n; ++j)
                for (long i = 0; i < n; ++i) {
                    const long q = i + n * j + n2 * k;
                    double v = 0.0;
                    for (long a = 0; a < n; ++a) v += sq[a * n + i] * grr[a + n * j + n2 * k];
                    for (long a = 0; a < n; ++a) v += sq[a * n + j] * gss[i + n * a + n2 * k];
                    for (long a = 0; a < n; ++a) v += sq[a * n + k] * gtt[i + n * j + n2 * a];
                    v += 2.0 * dd[i] * dd[j] * grs[q] + 2.0 * dd[i] * dd[k] * grt[q] + 2.0 * dd[j] * dd[k] * gst[q];
                    me[q] = v;
                }
    }
    std::vector<int64_t> gid(nl);
    std::vector<int8_t> mask(nl);
    numbering(N, nel, gid.data(), nullptr, mask.data());
    const long ng = ((long)nel[0] * N + 1) * ((long)nel[1] * N + 1) * ((long)nel[2] * N + 1);
    std::vector<double> acc(ng, 0.0);
    for (long l = 0; l < nl; ++l) acc[gid[l]] += m[l];
    for (long l = 0; l < nl; ++l) m[l] = mask[l] ? acc[gid[l]] : 1.0;
}

}  // namespace nek

// ------------------------------------------------------------ host C ABI
#include <cstring>

#include "nek_host.h"

namespace {
bool host_args_ok(int N, const int nel[3])
{
    if (N < 1 || N > 15 || !nel) return false;
    for (int d = 0; d < 3; ++d)
        if (nel[d] < 1) return false;
    const long np = N + 1;
    return (long)nel[0] * nel[1] * nel[2] * np * np * np < (1L << 31);
}
}  // namespace

extern "C" {

int nek_host_gll(int N, double *xi, double *w)
{
    if (N < 1 || N > 15 || !xi || !w) return -1;
    std::vector<double> x, ww;
    nek::gll_rule(N, x, ww);
    std::memcpy(xi, x.data(), x.size() * sizeof(double));
    std::memcpy(w, ww.data(), ww.size() * sizeof(double));
    return 0;
}

int nek_host_deriv(int N, double *D)
{
    if (N < 1 || N > 15 || !D) return -1;
    std::vector<double> x, w, d;
    nek::gll_rule(N, x, w);
    nek::deriv_matrix(x, d);
    std::memcpy(D, d.data(), d.size() * sizeof(double));
    return 0;
}

int nek_host_geometry(int N, const int nel[3], const double *vtx, double *g, double *B, double *X)
{
    if (!host_args_ok(N, nel) || !vtx || !g || !B) return -1;
    std::vector<double> x, w, d;
    nek::gll_rule(N, x, w);
    nek::deriv_matrix(x, d);
    const size_t nv = 3 * (size_t)(nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1);
    std::vector<double> v(vtx, vtx + nv);
    return nek::geometry(N, nel, v, x, w, d, g, B, X) ? -4 : 0;
}

int nek_host_numbering(int N, const int nel[3], int64_t *gid, int32_t *mult, int8_t *mask)
{
    if (!host_args_ok(N, nel)) return -1;
    nek::numbering(N, nel, gid, mult, mask);
    return 0;
}

int nek_host_segment_sizes(int N, const int nel[3], int64_t *n_perm, int64_t *n_seg)
{
    if (!host_args_ok(N, nel) || !n_perm || !n_seg) return -1;
    std::vector<int32_t> perm, ptr;
    std::vector<int8_t> flag;
    nek::segment_maps(N, nel, perm, ptr, flag);
    *n_perm = (int64_t)perm.size();
    *n_seg = (int64_t)flag.size();
    return 0;
}

int nek_host_segments(int N, const int nel[3], int32_t *perm, int32_t *seg_ptr, int8_t *seg_flag)
{
    if (!host_args_ok(N, nel) || !perm || !seg_ptr || !seg_flag) return -1;
    std::vector<int32_t> p, ptr;
    std::vector<int8_t> flag;
    nek::segment_maps(N, nel, p, ptr, flag);
    std::memcpy(perm, p.data(), p.size() * sizeof(int32_t));
    std::memcpy(seg_ptr, ptr.data(), ptr.size() * sizeof(int32_t));
    std::memcpy(seg_flag, flag.data(), flag.size());
    return 0;
}

int nek_host_fdm(int N, const int nel[3], const double *vtx, double *S, double *lam, double *cf)
{
    if (!host_args_ok(N, nel) || N < 2 || !vtx || !S || !lam || !cf) return -1;
    std::vector<double> x, w, d, s, l;
    nek::gll_rule(N, x, w);
    nek::deriv_matrix(x, d);
    nek::fdm_modes(N, w, d, s, l);
    std::memcpy(S, s.data(), s.size() * sizeof(double));
    std::memcpy(lam, l.data(), l.size() * sizeof(double));
    const size_t nv = 3 * (size_t)(nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1);
    std::vector<double> v(vtx, vtx + nv);
    nek::fdm_scales(nel, v, cf);
    return 0;
}

int nek_host_schwarz(int N, const int nel[3], const double *vtx, double *Sw, double *lamw, double *Sc,
                     double *lamc)
{
    if (!host_args_ok(N, nel) || N < 2 || !vtx || !Sw || !lamw || !Sc || !lamc) return -1;
    std::vector<double> x, w, d, s, l;
    nek::gll_rule(N, x, w);
    nek::deriv_matrix(x, d);
    nek::schwarz_windows(N, w, d, s, l);
    std::memcpy(Sw, s.data(), s.size() * sizeof(double));
    std::memcpy(lamw, l.data(), l.size() * sizeof(double));
    const size_t nv = 3 * (size_t)(nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1);
    std::vector<double> v(vtx, vtx + nv), sc, lc;
    int off[3], loff[3];
    nek::schwarz_coarse(N, nel, v, x, w, sc, lc, off, loff);
    if (!sc.empty()) std::memcpy(Sc, sc.data(), sc.size() * sizeof(double));
    if (!lc.empty()) std::memcpy(lamc, lc.data(), lc.size() * sizeof(double));
    return 0;
}

int nek_host_trilinear(int N, const int nel[3], const double *vtx, double *coef)
{
    if (!host_args_ok(N, nel) || !vtx || !coef) return -1;
    const size_t nv = 3 * (size_t)(nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1);
    std::vector<double> v(vtx, vtx + nv);
    return nek::trilinear_all(N, nel, v, coef) ? -4 : 0;
}

}  // extern "C"
