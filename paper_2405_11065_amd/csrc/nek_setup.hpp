// Host-side FP64 initialisation used by libnek (internal header).
#pragma once
#include <cstdint>
#include <vector>

namespace nek {

// GLL nodes x[0..N] (ascending, x0 = -1, xN = 1) and weights w.
void gll_rule(int N, std::vector<double> &x, std::vector<double> &w);

// D[i*(N+1)+j] = derivative at x_i of the Lagrange polynomial of node j.
void deriv_matrix(const std::vector<double> &x, std::vector<double> &D);

// Uniform vertex lattice on [lo, hi], x-index fastest, 3 doubles per vertex.
void uniform_vertices(const int nel[3], const double lo[3], const double hi[3], std::vector<double> &vtx);

// g[E][6][n^3] = (G_rr, G_ss, G_tt, G_rs, G_rt, G_st), B[E][n^3] and, when X
// is non-null, X[E][3][n^3].  Returns nonzero if any det(J) <= 0.
int geometry(int N, const int nel[3], const std::vector<double> &vtx, const std::vector<double> &x,
             const std::vector<double> &w, const std::vector<double> &D, double *g, double *B, double *X);

// Sorted-segment gather-scatter maps over the element-surface local nodes.
void segment_maps(int N, const int nel[3], std::vector<int32_t> &perm, std::vector<int32_t> &seg_ptr,
                  std::vector<int8_t> &seg_flag);

// Diagonal of the assembled masked operator (1 on Dirichlet nodes) from
// g[E][6][n^3]: the Jacobi preconditioner.
void assembled_diagonal(int N, const int nel[3], const std::vector<double> &D, const double *g, double *m);

// Fast-diagonalization data of the element-interior block solve: the 1-D
// interior modes (K_I S = W_I S Lambda, S^T W_I S = I; S row-major [node][mode])
// and per-element factors (cx, cy, cz) = (hy hz/hx, hx hz/hy, hx hy/hz).
void fdm_modes(int N, const std::vector<double> &w, const std::vector<double> &D, std::vector<double> &S,
               std::vector<double> &lam);
void fdm_scales(const int nel[3], const std::vector<double> &vtx, double *cf);

// Symmetric eigen-decomposition by cyclic Jacobi rotations (C destroyed):
// C = V diag(lam) V^T, V row-major [row][mode].
void sym_eig(int m, std::vector<double> &C, std::vector<double> &V, std::vector<double> &lam);

// Two-level overlapping Schwarz preconditioner: the window modes of the four
// clipping variants, padded to (N+3) x (N+3) (S[v][node][mode], lam[v][mode]),
// and the coarse modes per direction (S at off[d], (n_d-1)^2 entries
// [vertex][mode]; lambda at loff[d]).
void schwarz_windows(int N, const std::vector<double> &w, const std::vector<double> &D, std::vector<double> &S,
                     std::vector<double> &lam);
void schwarz_coarse(int N, const int nel[3], const std::vector<double> &vtx, const std::vector<double> &x,
                    const std::vector<double> &w, std::vector<double> &S, std::vector<double> &lam, int off[3],
                    int loff[3]);

// Coefficients of every element's trilinear map for the in-kernel factors:
// out = [hdr entries: x[0..N], w[0..N], zeros] then per element, per
// coordinate d, (a1..a7, 0) of x_d(r,s,t) = a0 + a1 r + a2 s + a3 t + a4 rs
// + a5 rt + a6 st + a7 rst.  Returns nonzero if any element's Jacobian
// determinant is not positive at a GLL node.
int trilinear_coefs(int N, const int nel[3], const std::vector<double> &vtx, const std::vector<double> &x,
                    const std::vector<double> &w, int hdr, std::vector<double> &out);
// The same maps with a0, as coef[E][3][8] (a0..a7 per coordinate).
int trilinear_all(int N, const int nel[3], const std::vector<double> &vtx, double *coef);

// Per-local-node global id, multiplicity and Dirichlet mask (any may be null).
void numbering(int N, const int nel[3], int64_t *gid, int32_t *mult, int8_t *mask);

}  // namespace nek
