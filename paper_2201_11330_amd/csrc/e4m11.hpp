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

// FP32 -> e4m11, round to nearest, ties to even.  The normal, subnormal and
// non-finite results are all computed and one is selected by masks, with no
// branches (a conditional expression here was compiled into branches that
// serialised the loads of a kernel).
__host__ __device__ inline e4m11 e4m11_from_float(float v)
{
    const uint32_t u = e4m11_f32_bits(v);
    const uint32_t sign = (u >> 16) & 0x8000u;
    const uint32_t a = u & 0x7FFFFFFFu;
    // Normal (|v| >= 2^-14, FP32 biased exponent e32 >= 113): the FP32
    // exponent 127 + k becomes field 15 + k; 12 fraction bits are dropped
    // with round-to-nearest-even, a carry out of the fraction moves into the
    // exponent, and past field 14 the result is infinity.
    uint32_t rn = (a - (112u << 23) + 0x7FFu + ((a >> 12) & 1u)) >> 12;
    rn = rn > 0x7800u ? 0x7800u : rn;
    // Subnormal (|v| < 2^-14): M = |v| 2^25 rounded to the nearest integer,
    // ties to even (the FP32 product is exact, and rintf rounds to nearest
    // even); M = 2^11 is the smallest normal (field 1, fraction 0).  The
    // clamp keeps the product finite and small for the other inputs.
    const float av = e4m11_bits_f32(a);
    const uint32_t rs = uint32_t(__builtin_rintf((av < 0x1p-14f ? av : 0x1p-14f) * 0x1p25f));
    // Infinity, or NaN with a nonzero fraction.
    const uint32_t rx = 0x7800u | (uint32_t(a > 0x7F800000u) << 10);
    const uint32_t use_n = 0u - uint32_t(a >= (113u << 23));
    const uint32_t use_x = 0u - uint32_t(a >= 0x7F800000u);
    uint32_t r = rs ^ ((rs ^ rn) & use_n);
    r = r ^ ((r ^ rx) & use_x);
    return {uint16_t(sign | r)};
}

// e4m11 -> FP32, exact.  With the 15 low bits shifted into an FP32's
// exponent and fraction (E << 23 | M << 12), that FP32 is 2^(E-127)
// (1 + M/2^11) for E >= 1 and the denormal M 2^-137 for E = 0, so a product
// with 2^112 gives 2^(E-15) (1 + M/2^11) and M 2^-25 exactly (the kernels
// keep FP32 denormals); E = 15 is selected as infinity or NaN.
__host__ __device__ inline float e4m11_to_float(e4m11 h)
{
    const uint32_t sign = uint32_t(h.bits & 0x8000u) << 16;
    const uint32_t em = uint32_t(h.bits & 0x7FFFu) << 12;
    uint32_t r = e4m11_f32_bits(e4m11_bits_f32(em) * 0x1p112f);
    const uint32_t use_x = 0u - uint32_t(em >= (15u << 23));
    r = r ^ ((r ^ (0x7F800000u | (em & 0x7FFFFFu))) & use_x);
    return e4m11_bits_f32(sign | r);
}

}  // namespace imexlbm
