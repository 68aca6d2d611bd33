// libnek: inputs, targets and assembly of the learned initial guess, and the
// random-field forcing generator (include/nek_mlp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "nek.h"
#include "nek_bf16.hpp"
#include "nek_mlp.h"
#include "nek_mlp_internal.hpp"
#include "nek_setup.hpp"

using namespace nek;

namespace nek {
namespace {

constexpr int XB = 256;   // threads per element of the per-element kernels

// Fixed-order block sum of NV values per thread; results valid in v[] of every thread.
template <int NV> __device__ __forceinline__ void block_sum(double v[NV], double (*sb)[XB])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) sb[q][t] = v[q];
    __syncthreads();
    for (int w = XB / 2; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < NV; ++q) sb[q][t] += sb[q][t + w];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = sb[q][0];
    __syncthreads();
}

// Global forcing scale: q[e] = sum over element e of F^2 (first pass) ...
__global__ __launch_bounds__(XB) void k_x0_fsq(const double *__restrict__ f, const double *__restrict__ B, int n3,
                                               double *__restrict__ q)
{
    __shared__ double sb[1][XB];
    const long e = blockIdx.x;
    double v[1] = {0.0};
    for (int p = threadIdx.x; p < n3; p += XB) {
        const double F = f[e * n3 + p] / B[e * n3 + p];
        v[0] += F * F;
    }
    block_sum<1>(v, sb);
    if (threadIdx.x == 0) q[e] = v[0];
}

// ... then S = sqrt(sum_e q[e] / (E n3)) in a fixed order, written to every q[e].
__global__ __launch_bounds__(XB) void k_x0_gscale(double *__restrict__ q, long E, int n3)
{
    __shared__ double sb[1][XB];
    double v[1] = {0.0};
    for (long e = threadIdx.x; e < E; e += XB) v[0] += q[e];
    block_sum<1>(v, sb);
    const double S = sqrt(v[0] / ((double)E * n3));
    for (long e = threadIdx.x; e < E; e += XB) q[e] = S;
}

// One workgroup per element: F = f / B; the element scale s_e (its own RMS
// of F in mode 0; given, the global RMS, in modes 1 and 2); inputs F / s_e
// and six geometric numbers: the normalised shape numbers (modes 0, 1), or
// the element's centroid and its three normalised off-diagonal shape numbers
// (mode 2); zero padding up to ldx.
__global__ __launch_bounds__(XB) void k_x0_features(const double *__restrict__ f, const double *__restrict__ B,
                                                    const double *__restrict__ g, const double *__restrict__ xyz,
                                                    int n3, int mode, uint16_t *__restrict__ X, int ldx,
                                                    double *__restrict__ s)
{
    __shared__ double sb[11][XB];
    const long e = blockIdx.x;
    const double *fe = f + e * n3, *Be = B + e * n3, *ge = g + e * n3 * 6;
    // sum F^2, sum B, sum G_k (6), sum B x, sum B y, sum B z
    double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int p = threadIdx.x; p < n3; p += XB) {
        const double F = fe[p] / Be[p];
        v[0] += F * F;
        v[1] += Be[p];
#pragma unroll
        for (int k = 0; k < 6; ++k) v[2 + k] += ge[p * 6 + k];
        if (mode == 2) {
            const double *xe = xyz + e * 3 * n3;
            v[8] += Be[p] * xe[p];
            v[9] += Be[p] * xe[n3 + p];
            v[10] += Be[p] * xe[2 * n3 + p];
        }
    }
    block_sum<11>(v, sb);
    const double se = mode == 0 ? sqrt(v[0] / n3) : s[e];
    uint16_t *Xe = X + e * ldx;
    for (int p = threadIdx.x; p < n3; p += XB) Xe[p] = se > 0 ? f64_to_bf16_rne((fe[p] / Be[p]) / se) : (uint16_t)0;
    if (threadIdx.x < 6) {
        double q[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = v[2 + k] / v[1];
        const double tr = (q[0] + q[1] + q[2]) / 3.0;
        const int k = threadIdx.x;
        const double val = mode == 2 ? (k < 3 ? v[8 + k] / v[1] : q[k] / tr) : q[k] / tr;
        Xe[n3 + k] = f64_to_bf16_rne(val);
    }
    for (int c = n3 + 6 + threadIdx.x; c < ldx; c += XB) Xe[c] = 0;
    if (threadIdx.x == 0) s[e] = se;
}

__global__ __launch_bounds__(XB) void k_x0_targets(const double *__restrict__ x, const double *__restrict__ s,
                                                   double kappa, int n3, float *__restrict__ T, int ldt)
{
    const long e = blockIdx.x;
    const double se = s[e];
    for (int p = threadIdx.x; p < ldt; p += XB)
        T[e * ldt + p] = (p < n3 && se > 0) ? (float)(x[e * n3 + p] / (se * kappa)) : 0.0f;
}

// Local prediction x0_e = y_e s_e kappa (FP64).
__global__ __launch_bounds__(XB) void k_x0_local(const float *__restrict__ Y, int ldy, const double *__restrict__ s,
                                                 double kappa, int n3, double *__restrict__ x0)
{
    const long e = blockIdx.x;
    const double f = s[e] * kappa;
    for (int p = threadIdx.x; p < n3; p += XB) x0[e * n3 + p] = (double)Y[e * ldy + p] * f;
}

__global__ void k_scale(double *__restrict__ x, double a, unsigned long n)
{
    for (unsigned long t = blockIdx.x * (unsigned long)blockDim.x + threadIdx.x; t < n;
         t += (unsigned long)gridDim.x * blockDim.x)
        x[t] *= a;
}

// out = scale sum_m amp_m cos(omega_m . x + phi_m) (times B), one thread per
// point; feature m at feat[5 m + 0..4] = omega (3), phi, amp.
__global__ __launch_bounds__(256) void k_grf(const double *__restrict__ xyz, int n3, long nl,
                                             const double *__restrict__ feat, int nfeat, double scale,
                                             const double *__restrict__ B, double *__restrict__ out)
{
    for (long t = blockIdx.x * 256L + threadIdx.x; t < nl; t += (long)gridDim.x * 256) {
        const long e = t / n3, p = t - e * n3;
        const double *xe = xyz + e * 3 * n3;
        const double x = xe[p], y = xe[n3 + p], z = xe[2 * n3 + p];
        double acc = 0.0;
        for (int m = 0; m < nfeat; ++m) {
            const double *q = feat + 5 * m;
            acc += q[4] * cos(q[0] * x + q[1] * y + q[2] * z + q[3]);
        }
        acc *= scale;
        out[t] = B ? acc * B[t] : acc;
    }
}

int ensure_xyz(nek_ctx *c)
{
    if (c->xyz) return NEK_OK;
    const size_t n3 = (size_t)c->NP * c->NP * c->NP;
    std::vector<double> g((size_t)c->E * 6 * n3), B((size_t)c->nl), X((size_t)c->E * 3 * n3);
    if (geometry(c->N, c->nel, c->vtx, c->xi, c->w, c->D, g.data(), B.data(), X.data())) return NEK_E_JACOBIAN;
    if (dalloc(c->xyz, X.size())) return NEK_E_OOM;
    HIP_TRY(hipMemcpy(c->xyz, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice));
    return NEK_OK;
}

int n3_of(const nek_ctx *c) { return c->NP * c->NP * c->NP; }

}  // namespace
}  // namespace nek

extern "C" {

int nek_x0_features(nek_ctx *c, const double *f, int mode, uint16_t *X, int ldx, double *s)
{
    if (!c || !f || !X || !s || ldx < n3_of(c) + 6 || mode < 0 || mode > 2) return NEK_E_ARG;
    int rc;
    if (mode == 2 && (rc = ensure_xyz(c))) return rc;
    if (mode > 0) {
        hipLaunchKernelGGL(k_x0_fsq, dim3((unsigned)c->E), dim3(XB), 0, c->stream, f, c->B, n3_of(c), s);
        hipLaunchKernelGGL(k_x0_gscale, dim3(1), dim3(XB), 0, c->stream, s, c->E, n3_of(c));
    }
    hipLaunchKernelGGL(k_x0_features, dim3((unsigned)c->E), dim3(XB), 0, c->stream, f, c->B, c->g64,
                       mode == 2 ? c->xyz : nullptr, n3_of(c), mode, X, ldx, s);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int nek_x0_targets(nek_ctx *c, const double *x, const double *s, double kappa, float *T, int ldt)
{
    if (!c || !x || !s || !T || ldt < n3_of(c) || !(kappa > 0)) return NEK_E_ARG;
    hipLaunchKernelGGL(k_x0_targets, dim3((unsigned)c->E), dim3(XB), 0, c->stream, x, s, kappa, n3_of(c), T, ldt);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

int nek_x0_predict(nek_ctx *c, nek_mlp *m, const double *f, int mode, double kappa, int policy, double *x0,
                   double *alpha, double *rho0, int *used)
{
    if (!c || !m || !f || !x0 || f == x0 || !(kappa > 0) || (policy != NEK_X0_RESIDUAL && policy != NEK_X0_ENERGY))
        return NEK_E_ARG;
    const int n3 = n3_of(c);
    if (m->nin != n3 + 6 || m->nout != n3) return NEK_E_ARG;
    int rc;
    if ((rc = ensure_fp64_work(c))) return rc;
    if (!c->x0_X) {
        c->x0_ldx = m->ldin;
        c->x0_ldy = m->ldout;
        if (dalloc(c->x0_X, (size_t)c->E * c->x0_ldx) || dalloc(c->x0_Y, (size_t)c->E * c->x0_ldy) ||
            dalloc(c->x0_s, c->E))
            return NEK_E_OOM;
    }
    if (c->x0_ldx < n3 + 6 || c->x0_ldy < n3) return NEK_E_ARG;
    // network on the element inputs (the network may run on another stream)
    if ((rc = nek_x0_features(c, f, mode, c->x0_X, (int)c->x0_ldx, c->x0_s))) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if ((rc = nek_mlp_forward(m, c->x0_X, (int)c->x0_ldx, c->E, c->x0_Y, (int)c->x0_ldy))) return rc;
    HIP_TRY(hipStreamSynchronize(m->stream));
    // continuous prediction and its energy-norm scaling
    hipLaunchKernelGGL(k_x0_local, dim3((unsigned)c->E), dim3(XB), 0, c->stream, c->x0_Y, (int)c->x0_ldy, c->x0_s,
                       kappa, n3, c->w64);
    HIP_TRY(hipGetLastError());
    if ((rc = gather_launch(c, c->w64, x0, true)) || (rc = gather_launch(c, f, c->b, false)) ||
        (rc = ax_local_launch(c, x0, c->w64, NEK_F64, NEK_PREC_FP64)) ||
        (rc = gather_launch(c, c->w64, c->r64, false)) || (rc = glsc3_to_slot(c, x0, c->r64, NEK_F64, 2)) ||
        (rc = glsc3_to_slot(c, x0, c->b, NEK_F64, 3)) || (rc = glsc3_to_slot(c, c->b, c->b, NEK_F64, 0)))
        return rc;
    Scal h;
    if ((rc = read_scal(c, h))) return rc;
    const double den = h.red[2], a = den > 0 ? h.red[3] / den : NAN, bb = h.red[0];
    double r0 = 1.0;
    bool ok = std::isfinite(a) && bb > 0;
    if (ok) {
        hipLaunchKernelGGL(k_scale, dim3(4 * num_cu()), dim3(256), 0, c->stream, x0, a, (unsigned long)c->nl);
        HIP_TRY(hipGetLastError());
        if ((rc = ax_local_launch(c, x0, c->w64, NEK_F64, NEK_PREC_FP64)) ||
            (rc = resid_launch(c, c->b, c->w64, c->r64, 1)) || (rc = read_scal(c, h)))
            return rc;
        r0 = std::sqrt(h.red[1]) / std::sqrt(bb);
        ok = policy == NEK_X0_ENERGY || r0 < 1.0;
    }
    if (!ok && (rc = fill_f64(c, x0, 0.0, c->nl))) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (alpha) *alpha = a;
    if (rho0) *rho0 = r0;
    if (used) *used = ok ? 1 : 0;
    return NEK_OK;
}

int nek_grf(nek_ctx *c, int nfeat, const double *omega, const double *phi, const double *amp, double scale,
            int times_B, double *out)
{
    if (!c || !omega || !phi || !amp || !out || nfeat < 1 || nfeat > 4096) return NEK_E_ARG;
    int rc = ensure_xyz(c);
    if (rc) return rc;
    if (nfeat > c->gfeat_cap) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        dfree(c->gfeat);
        if (dalloc(c->gfeat, 5 * (size_t)nfeat)) return NEK_E_OOM;
        c->gfeat_cap = nfeat;
    }
    std::vector<double> feat(5 * (size_t)nfeat);
    for (int m = 0; m < nfeat; ++m) {
        feat[5 * m + 0] = omega[3 * m + 0];
        feat[5 * m + 1] = omega[3 * m + 1];
        feat[5 * m + 2] = omega[3 * m + 2];
        feat[5 * m + 3] = phi[m];
        feat[5 * m + 4] = amp[m];
    }
    // the previous call's kernel may still read the feature buffer
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->gfeat, feat.data(), feat.size() * sizeof(double), hipMemcpyHostToDevice));
    const long want = (c->nl + 255) / 256;
    const unsigned grid = (unsigned)std::max<long>(1, std::min<long>(want, 16L * num_cu()));
    hipLaunchKernelGGL(k_grf, dim3(grid), dim3(256), 0, c->stream, c->xyz, n3_of(c), c->nl, c->gfeat, nfeat, scale,
                       times_B ? c->B : nullptr, out);
    HIP_TRY(hipGetLastError());
    return NEK_OK;
}

}  // extern "C"
