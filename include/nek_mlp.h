/*
 * nek_mlp.h -- C ABI of libnek's learned initial guess for nek_cg_solve.
 *
 * A small per-element network predicts the solution on each element from
 * the element's load and shape; its local predictions are made continuous,
 * scaled by the best multiple in the operator's energy norm, and handed to
 * nek_cg_solve as x0, with plain CG from zero as the fallback when the guess
 * does not reduce the residual.  This is an addition to the solver of the
 * Nekbone paper (which always starts CG from zero); the CG solve itself is
 * unchanged.
 *
 * Network.  A perceptron with two hidden layers of width n_hidden and the
 * SiLU activation silu(z) = z / (1 + exp(-z)):
 *     Y = W3 silu(W2 silu(W1 X + b1) + b2) + b3
 * trained on the mean squared error with Adam.  On the device, the matrix
 * products take bfloat16 operands with FP32 accumulation (gfx950 matrix
 * cores); pre-activations, outputs, gradients, the Adam state and the master
 * parameters are FP32.
 *
 * Row layouts (device).  Network inputs are bfloat16 rows of ldx >= n_in
 * entries (ldx a multiple of 8; entries n_in..ldx-1 must be 0); targets and
 * outputs are FP32 rows of ldt / ldy >= n_out entries.
 *
 * Parameters (host, FP32, this order, dense):
 *     W1[n_hidden][n_in], b1[n_hidden], W2[n_hidden][n_hidden], b2[n_hidden],
 *     W3[n_out][n_hidden], b3[n_out].
 *
 * Per-element inputs of the initial guess (nek_x0_features), for an order-N
 * context, n3 = (N+1)^3, F = f / B pointwise (f = B o F for a forcing F):
 *     X_e = [F_e / s_e (local point order), six geometric numbers],
 *     so n_in = n3 + 6 and n_out = n3; elements with s_e = 0 get zero
 *     forcing inputs.  Targets for a solution x: T_e = x_e / (s_e kappa).
 * The scale s_e and the geometric numbers depend on the feature mode:
 *     mode 0: s_e = sqrt(mean of F^2 over the element's points); geometric
 *             numbers q = (sum over the element of G) / (sum of B) divided
 *             by the mean of its first three entries (G in the order rr, ss,
 *             tt, rs, rt, st): the element's volume average of J^-1 J^-T
 *             normalised to its mean diagonal (its shape, not its size);
 *     mode 1: s_e = S = sqrt(mean of F^2 over all local points), the same
 *             for every element; geometric numbers as in mode 0;
 *     mode 2: s_e = S as in mode 1; geometric numbers: the element's
 *             centroid (sum B x / sum B, for x, y, z) and the three
 *             off-diagonal numbers q_rs, q_rt, q_st of mode 0.
 *
 * Streams and errors as in nek.h: a network runs on the stream given to
 * nek_mlp_create; every call returns a nek_status.
 */
#ifndef NEK_MLP_H
#define NEK_MLP_H

#include <stdint.h>

#include "nek.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nek_mlp nek_mlp;

/*
 * nek_mlp_create -- a network n_in -> n_hidden -> n_hidden -> n_out (each
 * between 1 and 4096) with the given host parameters (NULL = all zero) and
 * zero Adam state, on stream (a hipStream_t or NULL).
 */
int nek_mlp_create(int n_in, int n_hidden, int n_out, const float *params, void *stream, nek_mlp **out);
void nek_mlp_free(nek_mlp *mlp);

/* Number of parameters (or a negative status). */
int64_t nek_mlp_num_params(const nek_mlp *mlp);

/* Copy the FP32 master parameters to / from host memory (synchronous);
 * setting them also clears the Adam state and step count. */
int nek_mlp_get_params(nek_mlp *mlp, float *host);
int nek_mlp_set_params(nek_mlp *mlp, const float *host);

/*
 * nek_mlp_forward -- Y[r] = network(X[r]) for rows r < rows (device X, Y).
 * Asynchronous.
 */
int nek_mlp_forward(nek_mlp *mlp, const uint16_t *X, int ldx, int64_t rows, float *Y, int ldy);

/*
 * nek_mlp_loss_grad -- mean squared error over rows x n_out entries of the
 * network on (X, T) and its gradient, kept for nek_mlp_adam.  *loss (host,
 * may be NULL) and grad (host, nek_mlp_num_params entries in the parameter
 * order, may be NULL) are filled; synchronises when either is requested.
 */
int nek_mlp_loss_grad(nek_mlp *mlp, const uint16_t *X, int ldx, const float *T, int ldt, int64_t rows,
                      double *loss, float *grad);

/* nek_mlp_adam -- one Adam step (bias-corrected) with the last gradient. */
int nek_mlp_adam(nek_mlp *mlp, float lr, float beta1, float beta2, float eps);

/*
 * nek_mlp_train -- `steps` Adam steps (beta 0.9 / 0.999, eps 1e-8) on
 * minibatches of `batch` rows drawn without replacement from the nsamples
 * rows of (X, T): each pass over the data visits them in a fresh random order
 * (Fisher-Yates with a 64-bit Mersenne Twister seeded by seed).  loss_hist
 * (host, may be NULL) receives the loss of every step.  Synchronises.
 */
int nek_mlp_train(nek_mlp *mlp, const uint16_t *X, int ldx, const float *T, int ldt, int64_t nsamples, int batch,
                  int steps, float lr, uint64_t seed, float *loss_hist);

/*
 * nek_x0_features -- network inputs X[e] (bfloat16 rows, ldx >= n3 + 6, the
 * padding written as 0) and scales s[e] (FP64) of the load vector f (FP64
 * local vector) on the context's mesh, in feature mode 0, 1 or 2.  Device
 * pointers; asynchronous.
 */
int nek_x0_features(nek_ctx *ctx, const double *f, int mode, uint16_t *X, int ldx, double *s);

/* nek_x0_targets -- T[e] = x_e / (s_e kappa) (FP32 rows, 0 where s_e = 0). */
int nek_x0_targets(nek_ctx *ctx, const double *x, const double *s, double kappa, float *T, int ldt);

/* nek_x0_predict policies: when to keep the guess. */
#define NEK_X0_RESIDUAL 0  /* keep it only if rho0 < 1 (its residual is below that of zero)      */
#define NEK_X0_ENERGY 1    /* keep the energy-scaled guess whenever alpha is finite: its error in
                              the energy norm never exceeds that of zero, which its residual may */

/*
 * nek_x0_predict -- initial guess for nek_cg_solve(ctx, f, x0, ...):
 *     x0_e = y_e s_e kappa with y = network(features of f in mode `mode`,
 *            the mode the network was trained with);
 *     x0 <- M o dssum(c o x0)  (continuity, Dirichlet mask);
 *     alpha = glsc3(x0, b) / glsc3(x0, A x0), b = M o dssum(f);
 *     x0 <- alpha x0, rho0 = |b - A x0|_c / |b|_c.
 * alpha minimises the energy-norm error |x - alpha x0|_A over multiples of
 * x0, so that error is never above |x|_A (the error of starting from zero).
 * When glsc3(x0, A x0) <= 0 or alpha is not finite, or under
 * NEK_X0_RESIDUAL when rho0 >= 1, x0 is set to zero (plain CG from zero) and
 * *used = 0; else *used = 1.  The network must have n_in = (N+1)^3 + 6 and
 * n_out = (N+1)^3.  f, x0: FP64 device vectors of n_local entries; alpha,
 * rho0, used: host (may be NULL).  Runs on the context's stream;
 * synchronises.
 */
int nek_x0_predict(nek_ctx *ctx, nek_mlp *mlp, const double *f, int mode, double kappa, int policy, double *x0,
                   double *alpha, double *rho0, int *used);

/*
 * nek_grf -- a forcing sample on the context's nodes:
 *     out = scale * sum_m amp[m] cos(omega[m] . x + phi[m])   (times B if times_B)
 * (a Gaussian random field by random Fourier features when omega, phi and
 * amp are drawn accordingly).  omega (host, [nfeat][3]), phi, amp (host,
 * nfeat entries), 1 <= nfeat <= 4096; out: FP64 device vector of n_local
 * entries.  The node coordinates are built on the device at the first call.
 * Asynchronous.
 */
int nek_grf(nek_ctx *ctx, int nfeat, const double *omega, const double *phi, const double *amp, double scale,
            int times_B, double *out);

#ifdef __cplusplus
}
#endif

#endif /* NEK_MLP_H */
