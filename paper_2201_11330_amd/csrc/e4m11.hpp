// A 16-bit floating-point storage format for shifted populations f - w:
// 1 sign bit, 4 exponent bits, 11 fraction bits.
//
// Lehmann et al. (Phys. Rev. E 106, 015308, 2022) observe that the shifted
// distributions f_a - w_a of the lattice Boltzmann method are bounded by 1
// in magnitude, so a 16-bit format needs few exponent bits, and they spend
// the spare bit on the significand (their FP16C).  This format follows that
// idea with IEEE-style semantics: exponent field E = 1..14 holds normal
// numbers 2^(E-15) (1 + M/2^11), E = 0 subnormal numbers 2^-14 (M/2^11) =
// M 2^-25, E = 15 infinities (M = 0) and NaN (M != 0).  The largest finite
// value is 2^-1 (2 - 2^-11) = 0.99976; |f_a - w_a| < 1 - min w_a holds for
// every physical state of D2Q9, D3Q19 and D3Q27 (1 - 1/216 = 0.99537).  Over
// the whole range it has twice the precision of IEEE half (11 vs 10 fraction
// bits, subnormal spacing 2^-25 vs 2^-24).  Values past the largest finite
// round to infinity, so an unstable run is still flagged as non-finite.
//
// Conversions: from FP32 with round-to-nearest-even, to FP32 exactly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace imexlbm {

struct e4m11 {
    uint16_t bits;
};

__host__ __device__ inline uint32_t e4m11_f32_bits(float v)
{
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    return u;
}

__host__ __device__ inline float e4m11_bits_f32(uint32_t u)
{
    float v;
    __builtin_memcpy(&v, &u, 4);
    return v;
}

// FP32 -> e4m11, round to nearest, ties to even, without branches (a
// conditional expression here was compiled into branches that serialised
// the loads of a kernel), in about 14 instructions.
__host__ __device__ inline e4m11 e4m11_from_float(float v)
{
    const uint32_t u = e4m11_f32_bits(v);
    const uint32_t a = u & 0x7FFFFFFFu;
    // Normal result (|v| >= 2^-14): the FP32 exponent 127 + k becomes field
    // 15 + k, and 12 fraction bits are dropped with round-to-nearest-even; a
    // carry out of the fraction moves into the exponent.  Below 2^-14 this
    // is negative.
    const int32_t rn = int32_t(a + 0x7FFu + ((a >> 12) & 1u) - (112u << 23)) >> 12;
    // Subnormal result: M = |v| 2^25 rounded to the nearest integer, ties to
    // even, by one fused multiply-add with 2^23 (the product is exact and the
    // sum rounds at units); |v| is capped at 2^-14, where M = 2^11 is the
    // code of 2^-14 itself, so for normal inputs rs <= rn.
    const float cap = e4m11_bits_f32(a) < 0x1p-14f ? e4m11_bits_f32(a) : 0x1p-14f;
    const int32_t rs = int32_t(e4m11_f32_bits(__builtin_fmaf(cap, 0x1p25f, 0x1p23f)) - 0x4B000000u);
    uint32_t r = uint32_t(rn > rs ? rn : rs);
    // Past the largest finite value (and for infinities): infinity; NaN
    // keeps a nonzero fraction.
    r = r < 0x7800u ? r : 0x7800u;
    r |= uint32_t(a > 0x7F800000u) << 10;
    return {uint16_t(((u >> 16) & 0x8000u) | r)};
}

// e4m11 -> FP32, exact.  The 15 low bits shifted into an FP32's exponent and
// fraction (E << 23 | M << 12), with the sign in place, make the FP32
// 2^(E-127) (1 + M/2^11) for E >= 1 and the denormal M 2^-137 for E = 0, so a
// product with 2^112 gives 2^(E-15) (1 + M/2^11) and M 2^-25 exactly (the
// kernels keep FP32 denormals); E = 15 becomes infinity or NaN.
__host__ __device__ inline float e4m11_to_float(e4m11 h)
{
    const uint32_t em = uint32_t(h.bits & 0x7FFFu);
    const uint32_t x = ((uint32_t(h.bits) & 0x8000u) << 16) | (em << 12);
    const float mag = e4m11_bits_f32(x) * 0x1p112f;
    return em >= 0x7800u ? e4m11_bits_f32(x | 0x7F800000u) : mag;
}

}  // namespace imexlbm
