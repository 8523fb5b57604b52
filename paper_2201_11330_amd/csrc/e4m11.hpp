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
// the loads of a kernel), in about 12 instructions.
__host__ __device__ inline e4m11 e4m11_from_float(float v)
{
    const uint32_t u = e4m11_f32_bits(v);
    // For |v| in [2^e, 2^(e+1)) let c = 2^(max(e, -14) + 12).  The sum |v| + c
    // lies in [c, 2c), where FP32's spacing is 2^(max(e, -14) - 11), the
    // spacing of the format at |v| (normal and subnormal alike); so the sum
    // rounds |v| to the format, to nearest with ties to even (c is a multiple
    // of twice that spacing), and subtracting c again is exact.  From
    // |v| >= 2^116 on c is the tiny negative FP32 0x8...; the sum leaves |v|
    // unchanged, and so do infinity and NaN.
    uint32_t ce = u & 0x7F800000u;
    ce = ce > 0x38800000u ? ce : 0x38800000u;  // 2^max(e, -14)
    const float c = e4m11_bits_f32(ce + (12u << 23));
    const float q = (__builtin_fabsf(v) + c) - c;
    // q 2^-112 has the FP32 exponent field E and fraction M << 12 for a
    // normal result, and is the FP32 denormal M 2^-137 for a subnormal one
    // (exact either way): its bits shifted right by 12 are the code.  Past
    // the largest finite value (and for infinity): the code of infinity; NaN
    // keeps a nonzero fraction.
    uint32_t r = e4m11_f32_bits(q * 0x1p-112f) >> 12;
    r = r < 0x7800u ? r : 0x7800u;
    r |= v != v ? 0x400u : 0u;
    return {uint16_t(((u >> 16) & 0x8000u) | r)};
}

// e4m11 -> FP32, exact.  The 15 low bits shifted into an FP32's exponent and
// fraction (E << 23 | M << 12), with the sign in place, make the FP32
// 2^(E-127) (1 + M/2^11) for E >= 1 and the denormal M 2^-137 for E = 0, so a
// product with 2^112 gives 2^(E-15) (1 + M/2^11) and M 2^-25 exactly (the
// kernels keep FP32 denormals); E = 15, the only codes whose product reaches
// 1, becomes infinity or NaN.
__host__ __device__ inline float e4m11_to_float(e4m11 h)
{
    // The code sign-extended and shifted left by 12 holds E and M in bits
    // 26..12 and the sign in bits 31..27; clearing bits 30..27 leaves
    // sign | E << 23 | M << 12.
    const uint32_t x = (uint32_t(int32_t(int16_t(h.bits))) << 12) & 0x87FFF000u;
    const float mag = e4m11_bits_f32(x) * 0x1p112f;
    return __builtin_fabsf(mag) >= 1.0f ? e4m11_bits_f32(x | 0x7F800000u) : mag;
}

}  // namespace imexlbm
