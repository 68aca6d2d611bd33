// bfloat16 conversions (round to nearest even) used by the kernels that
// store geometric factors or network operands in bfloat16.  Internal header.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nek {

__device__ __forceinline__ uint16_t f64_to_bf16_rne(double x)
{
    // Round-to-nearest-even directly from binary64 (no double rounding via
    // binary32).  Values below the binary32 normal range flush to signed 0.
    const unsigned long long u = __double_as_longlong(x);
    const unsigned sign = (unsigned)(u >> 63);
    const int ex = (int)((u >> 52) & 0x7ff);
    const unsigned long long man = u & 0xfffffffffffffULL;
    if (ex == 0x7ff) return (uint16_t)((sign << 15) | 0x7f80u | (man ? 0x40u : 0u));
    const int eb = ex - 1023 + 127;
    if (ex == 0 || eb <= 0) return (uint16_t)(sign << 15);
    if (eb >= 0xff) return (uint16_t)((sign << 15) | 0x7f80u);
    unsigned bits = (sign << 15) | ((unsigned)eb << 7) | (unsigned)(man >> 45);
    const unsigned long long rest = man & ((1ULL << 45) - 1);
    const unsigned long long half = 1ULL << 44;
    if (rest > half || (rest == half && (bits & 1u))) bits += 1u;   // carries into the exponent correctly
    return (uint16_t)bits;
}

// Round-to-nearest-even from binary32: add half an ulp of the kept part
// (minus one when the kept part is even) and truncate; NaN stays NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

}  // namespace nek
