/*
 * nek_host.h -- host-only setup routines of libnek, callable without a GPU.
 *
 * They compute the FP64 initialisation that nek_setup uploads to the device
 * (the part the paper keeps in double precision, Sect. 6): the GLL rule, the
 * differentiation matrix, trilinear geometry, global numbering and the
 * sorted-segment gather-scatter maps.  All pointers are HOST pointers owned
 * by the caller and sized as stated; nothing is retained.  Each returns
 * NEK_OK (0) or a negative nek_status from nek.h.
 */
#ifndef NEK_HOST_H
#define NEK_HOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* GLL nodes xi[N+1] (ascending, -1 .. 1) and weights w[N+1]; 1 <= N <= 15. */
int nek_host_gll(int N, double *xi, double *w);

/* D[(N+1)^2], row-major, D[i][j] = derivative at xi_i of the Lagrange
 * polynomial of node j (barycentric form, rows summing to zero). */
int nek_host_deriv(int N, double *D);

/* Geometry of the box nel[3] from the vertex lattice vtx (as in nek_mesh):
 * g[E][6][(N+1)^3], B[E][(N+1)^3], X[E][3][(N+1)^3] (X may be NULL).
 * Returns NEK_E_JACOBIAN (-4) for an inverted element. */
int nek_host_geometry(int N, const int nel[3], const double *vtx, double *g, double *B, double *X);

/* Per local node: gid (int64), multiplicity (int32), mask (int8); any may be
 * NULL. */
int nek_host_numbering(int N, const int nel[3], int64_t *gid, int32_t *mult, int8_t *mask);

/* Segment sizes, then the maps: perm[n_perm], seg_ptr[n_seg+1], seg_flag[n_seg]. */
int nek_host_segment_sizes(int N, const int nel[3], int64_t *n_perm, int64_t *n_seg);
int nek_host_segments(int N, const int nel[3], int32_t *perm, int32_t *seg_ptr, int8_t *seg_flag);

/* Fast-diagonalization data of the element-interior block solve (the
 * non-overlapping Schwarz stage of the solveM step): S[(N-1)^2] row-major
 * [node][mode] and lam[N-1] with K_I S = W_I S diag(lam), S^T W_I S = I
 * (K = D^T W D, interior nodes only); cf[3 E] = (hy hz/hx, hx hz/hy,
 * hx hy/hz) per element from the mean edge lengths of the vertex lattice vtx.
 * N >= 2. */
int nek_host_fdm(int N, const int nel[3], const double *vtx, double *S, double *lam, double *cf);

/*
 * nek_host_schwarz -- set-up data of the two-level overlapping Schwarz
 * preconditioner (NEK_PC_SCHWARZ; solveM of Table 1, the Schwarz smoother by
 * fast diagonalization of the Fig. 3 call graph), N >= 2.
 * Sw [4][N+3][N+3], lamw [4][N+3]: per clipping variant v = lo + 2 hi (lo:
 * the element's left face is on the Dirichlet boundary, hi: its right face),
 * the 1-D modes of the window (the left neighbour's node N-1, the element's
 * nodes 0..N, the right neighbour's node 1; the two nodes past a Dirichlet
 * face dropped): K S = W S Lambda, S^T W S = I, with K, W the GLL stiffness
 * and mass of three reference elements assembled and restricted to the
 * window; S padded with zero rows (dropped nodes) and columns (missing
 * modes, lambda 1).  Sc, lamc: the coarse modes per direction d = x, y, z in
 * turn, (nel[d]-1)^2 and nel[d]-1 entries, of the Q1 stiffness and
 * GLL-integrated mass on the slab-mean lattice restricted to the interior
 * vertices (S^T M S = I).  Host pointers sized by the caller.  0, or -1 for
 * bad arguments.
 */
int nek_host_schwarz(int N, const int nel[3], const double *vtx, double *Sw, double *lamw, double *Sc,
                     double *lamc);

/* Trilinear map of every element, the input of the in-kernel geometric
 * factors (nek_set_geometry): coef[E][3][8] = (a0..a7) of
 * x_d(r,s,t) = a0 + a1 r + a2 s + a3 t + a4 rs + a5 rt + a6 st + a7 rst on
 * [-1,1]^3, d = 0..2, from the vertex lattice vtx (as in nek_mesh).  Returns
 * NEK_E_JACOBIAN (-4) when det(J) is not positive at some GLL node of order
 * N (coef is still filled). */
int nek_host_trilinear(int N, const int nel[3], const double *vtx, double *coef);

#ifdef __cplusplus
}
#endif

#endif /* NEK_HOST_H */
