// libnek: the initial-guess network (include/nek_mlp.h) -- bfloat16 matrix
// products on the gfx950 matrix cores with FP32 accumulation and fused
// epilogues, FP32 elementwise kernels, Adam, and the minibatch training loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "nek.h"
#include "nek_bf16.hpp"
#include "nek_mlp.h"
#include "nek_mlp_internal.hpp"

namespace nek {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GB = 256;                 // threads of the GEMM workgroup (4 waves)
constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDT = BK + 8;             // LDS row pitch (bfloat16 entries, 80 bytes)

enum Epi { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_PLAIN = 2, EPI_DSILU = 3 };

// C(m, n) = sum_k A(m, k) B(n, k).  A(m, k) sits at A[m lda + k] when AKC
// (k contiguous) else at A[k lda + m]; likewise B.  Contiguous extents (lda,
// ldb) are multiples of 8 and every entry between the logical extent and the
// pitch is 0, so tiles are read in 16-byte pieces without masking inside a
// row.
struct GemmArgs {
    const uint16_t *A;
    const uint16_t *B;
    int lda, ldb, M, N, K;
    float *C;                 // FP32 result (pre-activation, output or gradient)
    int ldc;
    uint16_t *Cb;             // bfloat16 copy (HIDDEN: silu(z), DSILU: the product)
    int ldcb;
    const float *bias;        // HIDDEN, OUT
    const float *Z;           // DSILU: pre-activation of the layer
    int ldz;
    int kchunk;               // split K: workgroup z covers [z kchunk, (z+1) kchunk) (0: all of K)
    long cstride;             // split K: C of split z at C + z cstride
};

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }

// A BM x BK (or BN x BK) tile, staged into LDS as [row][k]: each thread
// fetches one 16-byte piece into registers, and stores it once the LDS
// buffer it goes to is free, so the fetch of the next tile overlaps the
// products of the current one.
template <bool KC>
__device__ __forceinline__ uint4 fetch_tile(const uint16_t *__restrict__ P, int ld, int rows, int K, int r0, int k0,
                                            int tid)
{
    uint4 v = make_uint4(0, 0, 0, 0);
    if constexpr (KC) {
        const int r = tid >> 2, kc = (tid & 3) * 8;
        if (r0 + r < rows && k0 + kc < ld) v = *reinterpret_cast<const uint4 *>(P + (size_t)(r0 + r) * ld + k0 + kc);
    } else {
        const int k = tid >> 3, mc = (tid & 7) * 8;
        if (k0 + k < K && r0 + mc < ld) v = *reinterpret_cast<const uint4 *>(P + (size_t)(k0 + k) * ld + r0 + mc);
    }
    return v;
}

template <bool KC> __device__ __forceinline__ void store_tile(uint4 v, uint16_t *__restrict__ S, int tid)
{
    if constexpr (KC) {
        const int r = tid >> 2, kc = (tid & 3) * 8;
        *reinterpret_cast<uint4 *>(S + r * LDT + kc) = v;
    } else {
        const int k = tid >> 3, mc = (tid & 7) * 8;
        const uint16_t e[8] = {(uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16), (uint16_t)(v.y & 0xffff),
                               (uint16_t)(v.y >> 16),    (uint16_t)(v.z & 0xffff), (uint16_t)(v.z >> 16),
                               (uint16_t)(v.w & 0xffff), (uint16_t)(v.w >> 16)};
#pragma unroll
        for (int q = 0; q < 8; ++q) S[(mc + q) * LDT + k] = e[q];
    }
}

// 64 x 64 output tile per workgroup; wave w owns the 32 x 32 quadrant
// (w >> 1, w & 1) as 2 x 2 blocks of gfx950's 16x16x32 bfloat16 MFMA, one
// instruction per block and K tile.  Operand lanes: A row (lane & 15),
// k = 8 (lane >> 4) + 0..7; B column (lane & 15), same k; result element r
// of a block is row 4 (lane >> 4) + r, column (lane & 15).  Two LDS buffers
// per operand: tile t + 1 is fetched while tile t is multiplied.
template <bool AKC, bool BKC, int EPI>
__global__ __launch_bounds__(GB) void k_gemm(GemmArgs a)
{
    __shared__ __align__(16) uint16_t As[2][BM * LDT];
    __shared__ __align__(16) uint16_t Bs[2][BN * LDT];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kb = a.kchunk ? blockIdx.z * a.kchunk : 0;
    const int ke = a.kchunk ? min(a.K, kb + a.kchunk) : a.K;
    float *C = a.C + (a.kchunk ? blockIdx.z * a.cstride : 0);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = 4 * (lane >> 4), lk8 = 8 * (lane >> 4);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (kb < ke) {
        store_tile<AKC>(fetch_tile<AKC>(a.A, a.lda, a.M, ke, m0, kb, tid), As[0], tid);
        store_tile<BKC>(fetch_tile<BKC>(a.B, a.ldb, a.N, ke, n0, kb, tid), Bs[0], tid);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
        const bool more = k0 + BK < ke;
        uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
        if (more) {
            va = fetch_tile<AKC>(a.A, a.lda, a.M, ke, m0, k0 + BK, tid);
            vb = fetch_tile<BKC>(a.B, a.ldb, a.N, ke, n0, k0 + BK, tid);
        }
        bf16x8 af[2], bfv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            af[i] = *reinterpret_cast<const bf16x8 *>(As[buf] + (wm + 16 * i + lr) * LDT + lk8);
            bfv[i] = *reinterpret_cast<const bf16x8 *>(Bs[buf] + (wn + 16 * i + lr) * LDT + lk8);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfv[j], acc[i][j], 0, 0, 0);
        if (more) {
            store_tile<AKC>(va, As[buf ^ 1], tid);
            store_tile<BKC>(vb, Bs[buf ^ 1], tid);
        }
        __syncthreads();
        buf ^= 1;
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + lk + r, n = n0 + wn + 16 * j + lr;
                if (m >= a.M || n >= a.N) continue;
                const float v = acc[i][j][r];
                if constexpr (EPI == EPI_HIDDEN) {
                    const float z = v + a.bias[n];
                    C[(size_t)m * a.ldc + n] = z;
                    a.Cb[(size_t)m * a.ldcb + n] = f32_to_bf16_rne(z * sigmoidf_(z));
                } else if constexpr (EPI == EPI_OUT) {
                    C[(size_t)m * a.ldc + n] = v + a.bias[n];
                } else if constexpr (EPI == EPI_PLAIN) {
                    C[(size_t)m * a.ldc + n] = v;
                } else {
                    const float z = a.Z[(size_t)m * a.ldz + n];
                    const float s = sigmoidf_(z);
                    const float d = v * (s * (1.0f + z * (1.0f - s)));
                    C[(size_t)m * a.ldc + n] = d;
                    a.Cb[(size_t)m * a.ldcb + n] = f32_to_bf16_rne(d);
                }
            }
}

template <bool AKC, bool BKC, int EPI> int gemm(hipStream_t s, const GemmArgs &a, int splits = 1)
{
    if (a.M <= 0 || a.N <= 0 || a.K <= 0) return NEK_OK;
    const dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, splits);
    hipLaunchKernelGGL((k_gemm<AKC, BKC, EPI>), grid, dim3(GB), 0, s, a);
    return hipGetLastError() == hipSuccess ? NEK_OK : NEK_E_HIP;
}

// out[m][n] = sum over splits z (in order) of part[z][m][n] (pitch ld, split stride cs).
__global__ __launch_bounds__(256) void k_sum_splits(const float *__restrict__ part, int nsplit, long cs, int M,
                                                    int N, int ld, float *__restrict__ out)
{
    const long total = (long)M * N;
    for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        const int m = (int)(t / N), n = (int)(t - (long)m * N);
        float acc = 0.0f;
        for (int z = 0; z < nsplit; ++z) acc += part[z * cs + (size_t)m * ld + n];
        out[(size_t)m * ld + n] = acc;
    }
}

// dY = 2 (Y - T) / (rows n_out) (FP32 and bfloat16), partial sums of
// (Y - T)^2 per workgroup.
__global__ __launch_bounds__(256) void k_loss_dy(const float *__restrict__ Y, int ldy, const float *__restrict__ T,
                                                 int ldt, int rows, int nout, float *__restrict__ dY,
                                                 uint16_t *__restrict__ dYb, int ldd, double *__restrict__ part)
{
    __shared__ double sb[256];
    const float inv = 2.0f / ((float)rows * (float)nout);
    double acc = 0.0;
    const long total = (long)rows * nout;
    for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        const int r = (int)(t / nout), c = (int)(t - (long)r * nout);
        const float d = Y[(size_t)r * ldy + c] - T[(size_t)r * ldt + c];
        acc += (double)d * (double)d;
        const float g = d * inv;
        dY[(size_t)r * ldd + c] = g;
        dYb[(size_t)r * ldd + c] = f32_to_bf16_rne(g);
    }
    sb[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sb[threadIdx.x] += sb[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sb[0];
}

// Sum of n partials in a fixed order; out[0] = sum * scale.
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ part, int n, double scale,
                                                      double *__restrict__ out)
{
    __shared__ double sb[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    sb[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sb[threadIdx.x] += sb[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sb[0] * scale;
}

// Bias gradient: column sums of D (rows x ncol, pitch ld) in two fixed-order
// passes.  Pass 1: workgroup (x, y) sums rows [y CR, (y+1) CR) of 64 columns,
// four row lanes per column combined in order; pass 2 adds the chunks in order.
constexpr int CR = 128;   // rows per chunk
__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ D, int ld, int rows, int ncol,
                                                     float *__restrict__ part)
{
    __shared__ float sb[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), rl = threadIdx.x >> 6;
    const int r0 = blockIdx.y * CR, r1 = min(rows, r0 + CR);
    float acc = 0.0f;
    if (c < ncol)
        for (int r = r0 + rl; r < r1; r += 4) acc += D[(size_t)r * ld + c];
    sb[rl][threadIdx.x & 63] = acc;
    __syncthreads();
    if (rl == 0 && c < ncol) {
        const int q = threadIdx.x & 63;
        part[(size_t)blockIdx.y * ncol + c] = (sb[0][q] + sb[1][q]) + (sb[2][q] + sb[3][q]);
    }
}

__global__ __launch_bounds__(256) void k_colsum_final(const float *__restrict__ part, int nchunk, int ncol,
                                                      float *__restrict__ out)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ncol) return;
    float acc = 0.0f;
    for (int q = 0; q < nchunk; ++q) acc += part[(size_t)q * ncol + c];
    out[c] = acc;
}

// Adam over n parameters; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ P, const float *__restrict__ G,
                                              float *__restrict__ M, float *__restrict__ V, long n, float lr,
                                              float b1, float b2, float eps, float bc1, float bc2)
{
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const float g = G[i];
        const float m = b1 * M[i] + (1.0f - b1) * g;
        const float v = b2 * V[i] + (1.0f - b2) * g * g;
        M[i] = m;
        V[i] = v;
        P[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    }
}

// bfloat16 copy of a weight matrix (rows x cols) into a pitch-ld buffer.
__global__ __launch_bounds__(256) void k_weight_bf16(const float *__restrict__ W, int rows, int cols,
                                                     uint16_t *__restrict__ Wb, int ld)
{
    const long total = (long)rows * cols;
    for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        const int r = (int)(t / cols), c = (int)(t - (long)r * cols);
        Wb[(size_t)r * ld + c] = f32_to_bf16_rne(W[t]);
    }
}

// Minibatch assembly: rows idx[0..rows) of (X, T).
__global__ __launch_bounds__(256) void k_gather_rows(const uint16_t *__restrict__ X, int ldx,
                                                     const float *__restrict__ T, int ldt,
                                                     const int64_t *__restrict__ idx, int rows,
                                                     uint16_t *__restrict__ Xb, int ldxb, float *__restrict__ Tb,
                                                     int ldtb, int nin, int nout)
{
    const int r = blockIdx.x;
    if (r >= rows) return;
    const int64_t s = idx[r];
    for (int c = threadIdx.x; c < ldxb; c += 256) Xb[(size_t)r * ldxb + c] = c < nin ? X[s * ldx + c] : (uint16_t)0;
    for (int c = threadIdx.x; c < nout; c += 256) Tb[(size_t)r * ldtb + c] = T[s * ldt + c];
}

int round8(int v) { return (v + 7) / 8 * 8; }

}  // namespace
}  // namespace nek

using namespace nek;


namespace nek {
namespace {

constexpr int LOSS_BLOCKS = 1024;
constexpr int MAX_SPLITS = 16;   // split-K pieces of a weight gradient

int refresh_bf16(nek_mlp *m)
{
    const int grid = 4 * num_cu();
    hipLaunchKernelGGL(k_weight_bf16, dim3(grid), dim3(256), 0, m->stream, m->P + m->oW1, m->nh, m->nin, m->W1b,
                       m->ldin);
    hipLaunchKernelGGL(k_weight_bf16, dim3(grid), dim3(256), 0, m->stream, m->P + m->oW2, m->nh, m->nh, m->W2b,
                       m->ldh);
    hipLaunchKernelGGL(k_weight_bf16, dim3(grid), dim3(256), 0, m->stream, m->P + m->oW3, m->nout, m->nh, m->W3b,
                       m->ldh);
    return hipGetLastError() == hipSuccess ? NEK_OK : NEK_E_HIP;
}

// Zero-filled allocation; complete before the call returns (the network's
// stream may not be ordered after the null stream).
template <typename T> int zalloc(T *&p, size_t count)
{
    if (dalloc(p, count)) return NEK_E_OOM;
    if (hipMemset(p, 0, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return NEK_E_HIP;
    return hipDeviceSynchronize() == hipSuccess ? NEK_OK : NEK_E_HIP;
}

// Activation buffers for `rows` rows (padding entries stay 0).
int ensure_rows(nek_mlp *m, long rows)
{
    if (rows <= m->cap) return NEK_OK;
    HIP_TRY(hipStreamSynchronize(m->stream));
    dfree(m->Z1); dfree(m->Z2); dfree(m->Y); dfree(m->dY); dfree(m->dZ2); dfree(m->dZ1);
    dfree(m->H1); dfree(m->H2); dfree(m->dYb); dfree(m->dZ2b); dfree(m->dZ1b);
    const long cap = std::max<long>(rows, 256);
    const size_t nh = (size_t)cap * m->ldh, no = (size_t)cap * m->ldout;
    int rc;
    if ((rc = zalloc(m->Z1, nh)) || (rc = zalloc(m->Z2, nh)) || (rc = zalloc(m->Y, no)) || (rc = zalloc(m->dY, no)) ||
        (rc = zalloc(m->dZ2, nh)) || (rc = zalloc(m->dZ1, nh)) || (rc = zalloc(m->H1, nh)) ||
        (rc = zalloc(m->H2, nh)) || (rc = zalloc(m->dYb, no)) || (rc = zalloc(m->dZ2b, nh)) ||
        (rc = zalloc(m->dZ1b, nh)))
        return rc;
    m->cap = cap;
    // column-sum chunks and split-K partial products
    dfree(m->cpart);
    dfree(m->kpart);
    const long nchunk = (cap + CR - 1) / CR;
    const long wmax = std::max({(long)m->nout * m->nh, (long)m->nh * m->nh, (long)m->nh * m->nin});
    if ((rc = zalloc(m->cpart, nchunk * std::max(m->nout, m->nh))) || (rc = zalloc(m->kpart, MAX_SPLITS * wmax)))
        return rc;
    return NEK_OK;
}

// out[c] = sum over rows of D[r][c] (bias gradients), deterministic.
int colsum(nek_mlp *m, const float *D, int ld, int rows, int ncol, float *out)
{
    const int nchunk = (rows + CR - 1) / CR;
    hipLaunchKernelGGL(k_colsum_part, dim3((ncol + 63) / 64, nchunk), dim3(256), 0, m->stream, D, ld, rows, ncol,
                       m->cpart);
    hipLaunchKernelGGL(k_colsum_final, dim3((ncol + 255) / 256), dim3(256), 0, m->stream, m->cpart, nchunk, ncol, out);
    return hipGetLastError() == hipSuccess ? NEK_OK : NEK_E_HIP;
}

// Weight gradient C (M x N, pitch ldc) = A^T B over `rows` rows, split along
// the rows so that enough workgroups run, the splits added in order.
int gemm_wgrad(nek_mlp *m, GemmArgs a)
{
    const int rows = a.K;
    int splits = std::min(MAX_SPLITS, std::max(1, rows / 512));
    if (splits == 1) return gemm<false, false, EPI_PLAIN>(m->stream, a);
    const int kchunk = ((rows + splits - 1) / splits + BK - 1) / BK * BK;
    splits = (rows + kchunk - 1) / kchunk;
    float *out = a.C;
    a.C = m->kpart;
    a.kchunk = kchunk;
    a.cstride = (long)a.M * a.ldc;
    int rc = gemm<false, false, EPI_PLAIN>(m->stream, a, splits);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_splits, dim3(std::min<long>(1024, ((long)a.M * a.N + 255) / 256)), dim3(256), 0,
                       m->stream, m->kpart, splits, a.cstride, a.M, a.N, a.ldc, out);
    return hipGetLastError() == hipSuccess ? NEK_OK : NEK_E_HIP;
}

int check_rows(const nek_mlp *m, int ld, int need) { return ld >= need && ld % 8 == 0 ? NEK_OK : NEK_E_ARG; }

// Forward pass of rows rows of X into m->Y (and Z1, H1, Z2, H2).
int forward(nek_mlp *m, const uint16_t *X, int ldx, int rows, float *Y, int ldy)
{
    int rc;
    GemmArgs a{};
    a.A = X; a.lda = ldx; a.B = m->W1b; a.ldb = m->ldin; a.M = rows; a.N = m->nh; a.K = m->nin;
    a.C = m->Z1; a.ldc = m->ldh; a.Cb = m->H1; a.ldcb = m->ldh; a.bias = m->P + m->ob1;
    if ((rc = gemm<true, true, EPI_HIDDEN>(m->stream, a))) return rc;
    a = GemmArgs{};
    a.A = m->H1; a.lda = m->ldh; a.B = m->W2b; a.ldb = m->ldh; a.M = rows; a.N = m->nh; a.K = m->nh;
    a.C = m->Z2; a.ldc = m->ldh; a.Cb = m->H2; a.ldcb = m->ldh; a.bias = m->P + m->ob2;
    if ((rc = gemm<true, true, EPI_HIDDEN>(m->stream, a))) return rc;
    a = GemmArgs{};
    a.A = m->H2; a.lda = m->ldh; a.B = m->W3b; a.ldb = m->ldh; a.M = rows; a.N = m->nout; a.K = m->nh;
    a.C = Y; a.ldc = ldy; a.bias = m->P + m->ob3;
    return gemm<true, true, EPI_OUT>(m->stream, a);
}

// Loss and gradient (into m->G) of rows rows; the loss lands in m->dloss.
int loss_grad(nek_mlp *m, const uint16_t *X, int ldx, const float *T, int ldt, int rows)
{
    int rc;
    if ((rc = forward(m, X, ldx, rows, m->Y, m->ldout))) return rc;
    hipLaunchKernelGGL(k_loss_dy, dim3(LOSS_BLOCKS), dim3(256), 0, m->stream, m->Y, m->ldout, T, ldt, rows, m->nout,
                       m->dY, m->dYb, m->ldout, m->part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, m->stream, m->part, LOSS_BLOCKS,
                       1.0 / ((double)rows * m->nout), m->dloss);
    HIP_TRY(hipGetLastError());
    GemmArgs a{};
    // dW3 = dY^T H2
    a.A = m->dYb; a.lda = m->ldout; a.B = m->H2; a.ldb = m->ldh; a.M = m->nout; a.N = m->nh; a.K = rows;
    a.C = m->G + m->oW3; a.ldc = m->nh;
    if ((rc = gemm_wgrad(m, a)) || (rc = colsum(m, m->dY, m->ldout, rows, m->nout, m->G + m->ob3))) return rc;
    // dZ2 = (dY W3) o silu'(Z2)
    a = GemmArgs{};
    a.A = m->dYb; a.lda = m->ldout; a.B = m->W3b; a.ldb = m->ldh; a.M = rows; a.N = m->nh; a.K = m->nout;
    a.C = m->dZ2; a.ldc = m->ldh; a.Cb = m->dZ2b; a.ldcb = m->ldh; a.Z = m->Z2; a.ldz = m->ldh;
    if ((rc = gemm<true, false, EPI_DSILU>(m->stream, a))) return rc;
    // dW2 = dZ2^T H1, db2
    a = GemmArgs{};
    a.A = m->dZ2b; a.lda = m->ldh; a.B = m->H1; a.ldb = m->ldh; a.M = m->nh; a.N = m->nh; a.K = rows;
    a.C = m->G + m->oW2; a.ldc = m->nh;
    if ((rc = gemm_wgrad(m, a)) || (rc = colsum(m, m->dZ2, m->ldh, rows, m->nh, m->G + m->ob2))) return rc;
    // dZ1 = (dZ2 W2) o silu'(Z1)
    a = GemmArgs{};
    a.A = m->dZ2b; a.lda = m->ldh; a.B = m->W2b; a.ldb = m->ldh; a.M = rows; a.N = m->nh; a.K = m->nh;
    a.C = m->dZ1; a.ldc = m->ldh; a.Cb = m->dZ1b; a.ldcb = m->ldh; a.Z = m->Z1; a.ldz = m->ldh;
    if ((rc = gemm<true, false, EPI_DSILU>(m->stream, a))) return rc;
    // dW1 = dZ1^T X, db1
    a = GemmArgs{};
    a.A = m->dZ1b; a.lda = m->ldh; a.B = X; a.ldb = ldx; a.M = m->nh; a.N = m->nin; a.K = rows;
    a.C = m->G + m->oW1; a.ldc = m->nin;
    if ((rc = gemm_wgrad(m, a)) || (rc = colsum(m, m->dZ1, m->ldh, rows, m->nh, m->G + m->ob1))) return rc;
    return NEK_OK;
}

int adam(nek_mlp *m, float lr, float b1, float b2, float eps)
{
    m->t += 1;
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)m->t));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)m->t));
    hipLaunchKernelGGL(k_adam, dim3(4 * num_cu()), dim3(256), 0, m->stream, m->P, m->G, m->M, m->V, m->np, lr, b1,
                       b2, eps, bc1, bc2);
    HIP_TRY(hipGetLastError());
    return refresh_bf16(m);
}

}  // namespace
}  // namespace nek

extern "C" {

void nek_mlp_free(nek_mlp *m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    dfree(m->P); dfree(m->G); dfree(m->M); dfree(m->V); dfree(m->W1b); dfree(m->W2b); dfree(m->W3b);
    dfree(m->Z1); dfree(m->Z2); dfree(m->Y); dfree(m->dY); dfree(m->dZ2); dfree(m->dZ1);
    dfree(m->H1); dfree(m->H2); dfree(m->dYb); dfree(m->dZ2b); dfree(m->dZ1b);
    dfree(m->part); dfree(m->dloss); dfree(m->Xb); dfree(m->Tb); dfree(m->idx); dfree(m->cpart); dfree(m->kpart);
    delete m;
}

int nek_mlp_create(int nin, int nh, int nout, const float *params, void *stream, nek_mlp **out)
{
    if (!out || nin < 1 || nh < 1 || nout < 1 || nin > 4096 || nh > 4096 || nout > 4096) return NEK_E_ARG;
    *out = nullptr;
    nek_mlp *m = new (std::nothrow) nek_mlp;
    if (!m) return NEK_E_OOM;
    m->nin = nin; m->nh = nh; m->nout = nout;
    m->ldin = round8(nin); m->ldh = round8(nh); m->ldout = round8(nout);
    m->stream = (hipStream_t)stream;
    m->oW1 = 0; m->ob1 = m->oW1 + (long)nh * nin; m->oW2 = m->ob1 + nh; m->ob2 = m->oW2 + (long)nh * nh;
    m->oW3 = m->ob2 + nh; m->ob3 = m->oW3 + (long)nout * nh; m->np = m->ob3 + nout;
    int rc;
    if ((rc = zalloc(m->P, m->np)) || (rc = zalloc(m->G, m->np)) || (rc = zalloc(m->M, m->np)) ||
        (rc = zalloc(m->V, m->np)) || (rc = zalloc(m->W1b, (size_t)nh * m->ldin)) ||
        (rc = zalloc(m->W2b, (size_t)nh * m->ldh)) || (rc = zalloc(m->W3b, (size_t)nout * m->ldh)) ||
        (rc = zalloc(m->part, LOSS_BLOCKS)) || (rc = zalloc(m->dloss, 1))) {
        nek_mlp_free(m);
        return rc;
    }
    if (params && (rc = nek_mlp_set_params(m, params))) {
        nek_mlp_free(m);
        return rc;
    }
    *out = m;
    return NEK_OK;
}

int64_t nek_mlp_num_params(const nek_mlp *m) { return m ? m->np : NEK_E_ARG; }

int nek_mlp_get_params(nek_mlp *m, float *host)
{
    if (!m || !host) return NEK_E_ARG;
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(hipMemcpy(host, m->P, m->np * sizeof(float), hipMemcpyDeviceToHost));
    return NEK_OK;
}

int nek_mlp_set_params(nek_mlp *m, const float *host)
{
    if (!m || !host) return NEK_E_ARG;
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(hipMemcpy(m->P, host, m->np * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(m->M, 0, m->np * sizeof(float)));
    HIP_TRY(hipMemset(m->V, 0, m->np * sizeof(float)));
    m->t = 0;
    int rc = refresh_bf16(m);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(m->stream));
    return NEK_OK;
}

int nek_mlp_forward(nek_mlp *m, const uint16_t *X, int ldx, int64_t rows, float *Y, int ldy)
{
    if (!m || !X || !Y || rows < 0 || rows > (1L << 30) || check_rows(m, ldx, m->nin) || ldy < m->nout)
        return NEK_E_ARG;
    int rc = ensure_rows(m, rows);
    return rc ? rc : forward(m, X, ldx, (int)rows, Y, ldy);
}

int nek_mlp_loss_grad(nek_mlp *m, const uint16_t *X, int ldx, const float *T, int ldt, int64_t rows, double *loss,
                      float *grad)
{
    if (!m || !X || !T || rows < 1 || rows > (1L << 30) || check_rows(m, ldx, m->nin) || ldt < m->nout)
        return NEK_E_ARG;
    int rc = ensure_rows(m, rows);
    if (rc || (rc = loss_grad(m, X, ldx, T, ldt, (int)rows))) return rc;
    if (loss || grad) HIP_TRY(hipStreamSynchronize(m->stream));
    if (loss) HIP_TRY(hipMemcpy(loss, m->dloss, sizeof(double), hipMemcpyDeviceToHost));
    if (grad) HIP_TRY(hipMemcpy(grad, m->G, m->np * sizeof(float), hipMemcpyDeviceToHost));
    return NEK_OK;
}

int nek_mlp_adam(nek_mlp *m, float lr, float b1, float b2, float eps)
{
    if (!m || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0)) return NEK_E_ARG;
    return adam(m, lr, b1, b2, eps);
}

int nek_mlp_train(nek_mlp *m, const uint16_t *X, int ldx, const float *T, int ldt, int64_t ns, int batch, int steps,
                  float lr, uint64_t seed, float *loss_hist)
{
    if (!m || !X || !T || ns < 1 || batch < 1 || steps < 0 || !(lr > 0) || check_rows(m, ldx, m->nin) ||
        ldt < m->nout)
        return NEK_E_ARG;
    batch = (int)std::min<int64_t>(batch, ns);
    int rc = ensure_rows(m, batch);
    if (rc) return rc;
    if (batch > m->bcap) {
        HIP_TRY(hipStreamSynchronize(m->stream));
        dfree(m->Xb);
        dfree(m->Tb);
        if ((rc = zalloc(m->Xb, (size_t)batch * m->ldin)) || (rc = zalloc(m->Tb, (size_t)batch * m->ldout))) return rc;
        m->bcap = batch;
    }
    if (ns > m->idx_cap) {
        HIP_TRY(hipStreamSynchronize(m->stream));
        dfree(m->idx);
        if (dalloc(m->idx, ns)) return NEK_E_OOM;
        m->idx_cap = ns;
    }
    std::mt19937_64 gen(seed);
    std::vector<int64_t> perm(ns);
    std::vector<double> hl;
    double *dl = nullptr;
    if (loss_hist && dalloc(dl, std::max(steps, 1))) return NEK_E_OOM;
    long pos = ns;   // start a new pass at the first step
    for (int s = 0; s < steps && rc == NEK_OK; ++s) {
        if (pos + batch > ns) {
            for (int64_t i = 0; i < ns; ++i) perm[i] = i;
            for (int64_t i = ns - 1; i > 0; --i) {
                const int64_t j = (int64_t)(gen() % (uint64_t)(i + 1));
                std::swap(perm[i], perm[j]);
            }
            // the previous pass's steps have read the old order
            if (hipStreamSynchronize(m->stream) != hipSuccess ||
                hipMemcpy(m->idx, perm.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
                rc = NEK_E_HIP;
                break;
            }
            pos = 0;
        }
        hipLaunchKernelGGL(k_gather_rows, dim3(batch), dim3(256), 0, m->stream, X, ldx, T, ldt, m->idx + pos, batch,
                           m->Xb, m->ldin, m->Tb, m->ldout, m->nin, m->nout);
        if (hipGetLastError() != hipSuccess) { rc = NEK_E_HIP; break; }
        pos += batch;
        if ((rc = loss_grad(m, m->Xb, m->ldin, m->Tb, m->ldout, batch))) break;
        if (dl && hipMemcpyAsync(dl + s, m->dloss, sizeof(double), hipMemcpyDeviceToDevice, m->stream) != hipSuccess) {
            rc = NEK_E_HIP;
            break;
        }
        rc = adam(m, lr, 0.9f, 0.999f, 1e-8f);
    }
    if (hipStreamSynchronize(m->stream) != hipSuccess && rc == NEK_OK) rc = NEK_E_HIP;
    if (dl) {
        if (rc == NEK_OK) {
            hl.resize(steps);
            if (hipMemcpy(hl.data(), dl, steps * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) rc = NEK_E_HIP;
            for (int s = 0; s < steps && rc == NEK_OK; ++s) loss_hist[s] = (float)hl[s];
        }
        dfree(dl);
    }
    return rc;
}

}  // extern "C"
