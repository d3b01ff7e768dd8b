// rng.hpp -- counter-based noise for the simulation kernels (gfx950).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 4x32-bit counter, 2x32-bit key,
// ten rounds; a round multiplies words 0 and 2 by the two round multipliers, keeps
// the low halves as the new words 3 and 1, and XORs the high halves with the other
// two words and the round key into the new words 0 and 2; the key advances by the
// two Weyl increments between rounds. Every draw in the trial is addressed by
// (index, patient, tag, sub-index) so any patient's stream can be replayed anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vct {

enum : uint32_t { kTagParam = 0u, kTagMeal = 1u, kTagDiff = 2u };

struct U4 {
    uint32_t x, y, z, w;
};

// The two three-way XORs of a round map to one v_bitop3_b32 each (LUT 0x96 = a ^ b ^ c);
// the 32x32 -> 64-bit products to one v_mad_u64_u32 each.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(b >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(a >> 32), c3, k1);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// The same function for a counter whose words 0, 2 and 3 and key are the same on every
// lane of the wave and whose word 1 differs (the per-sample noise blocks: sample pair,
// patient, tag, block). Until word 1 has reached both multiplied words, some products and
// XORs depend on wave-uniform values only: words 0 and 2 of round 1, word 2 of round 2 and
// word 0 of round 3. Written with plain XORs, grouped so that the uniform operands meet
// first, those stay on the scalar unit (the three-way XOR instruction is vector only and
// takes at most one scalar operand). The result is bit-identical to philox4x32_10.
__device__ __forceinline__ U4 philox4x32_10_lane1(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                  uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    // round 1: both products uniform; the new word 0 takes the lane's word 1
    uint64_t a = (uint64_t)M0 * c0, b = (uint64_t)M1 * c2;
    uint32_t n0 = c1 ^ ((uint32_t)(b >> 32) ^ k0);
    uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)b; c3 = (uint32_t)a; c0 = n0; c2 = n2;
    k0 += W0; k1 += W1;
    // round 2: word 2 (and so the product b) still uniform, and so are words 1 and 3
    a = (uint64_t)M0 * c0;
    b = (uint64_t)M1 * c2;
    n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
    n2 = (uint32_t)(a >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)b; c3 = (uint32_t)a; c0 = n0; c2 = n2;
    k0 += W0; k1 += W1;
    // round 3: word 0 (and so the product a) and word 1 uniform
    a = (uint64_t)M0 * c0;
    b = (uint64_t)M1 * c2;
    n0 = (uint32_t)(b >> 32) ^ (c1 ^ k0);
    n2 = c3 ^ ((uint32_t)(a >> 32) ^ k1);
    c1 = (uint32_t)b; c3 = (uint32_t)a; c0 = n0; c2 = n2;
    k0 += W0; k1 += W1;
    // round 4: only word 3 uniform
    a = (uint64_t)M0 * c0;
    b = (uint64_t)M1 * c2;
    n0 = xor3((uint32_t)(b >> 32), c1, k0);
    n2 = (uint32_t)(a >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)b; c3 = (uint32_t)a; c0 = n0; c2 = n2;
    k0 += W0; k1 += W1;
    // rounds 5..10: every word differs per lane
#pragma unroll
    for (int r = 4; r < 10; ++r) {
        a = (uint64_t)M0 * c0;
        b = (uint64_t)M1 * c2;
        n0 = xor3((uint32_t)(b >> 32), c1, k0);
        n2 = xor3((uint32_t)(a >> 32), c3, k1);
        c1 = (uint32_t)b; c3 = (uint32_t)a; c0 = n0; c2 = n2;
        k0 += W0; k1 += W1;
    }
    return U4{c0, c1, c2, c3};
}

// Uniform on (0, 1): (2m + 1) 2^-24 with m the top 23 bits -- exact in both precisions.
// FP32: the bit pattern 1 + m 2^-23 minus (1 - 2^-24) is that value, and the
// subtraction is exact because the result has at most 24 significant bits.
// The bit pattern 0x3F800000 | (x >> 9) is one funnel shift: ((0x7F << 32) | x) >> 9.
__device__ __forceinline__ float uniform_f32(uint32_t x)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0.99999994039535522f;
}

__device__ __forceinline__ double uniform_f64(uint32_t x)
{
    return (double)((x >> 8) | 1u) * 5.9604644775390625e-08;
}

// Box-Muller: r = sqrt(-2 ln u0), z0 = r cos(2 pi u1), z1 = r sin(2 pi u1).
// FP32 uses the hardware log2 / sqrt / sin / cos (the trigonometric instructions take
// their argument in revolutions, so 2 pi u1 is never formed).
__device__ __forceinline__ void box_muller_f32(float u0, float u1, float &z0, float &z1)
{
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
    z0 = r * __builtin_amdgcn_cosf(u1);
    z1 = r * __builtin_amdgcn_sinf(u1);
}

__device__ __forceinline__ void box_muller_f64(double u0, double u1, double &z0, double &z1)
{
    const double r = sqrt(-2.0 * log(u0));
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Radius-scaled variants: r = sqrt(-2 ln u0) s folded into one square root as
// sqrt(ln u0 * (-2 s^2)); neg2s2 = -2 s^2 is precomputed (FP32 uses log2, so its
// constant carries ln 2).
__device__ __forceinline__ void box_muller_scaled_f32(float u0, float u1, float neg2s2_ln2, float &z0, float &z1)
{
    const float r = __builtin_amdgcn_sqrtf(neg2s2_ln2 * __builtin_amdgcn_logf(u0));
    z0 = r * __builtin_amdgcn_cosf(u1);
    z1 = r * __builtin_amdgcn_sinf(u1);
}

__device__ __forceinline__ void box_muller_scaled_f64(double u0, double u1, double neg2s2, double &z0, double &z1)
{
    const double r = sqrt(neg2s2 * log(u0));
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

template <typename R> struct Rng;

template <> struct Rng<float> {
    static __device__ __forceinline__ float uniform(uint32_t x) { return uniform_f32(x); }
    static __device__ __forceinline__ void box_muller(float u0, float u1, float &z0, float &z1)
    {
        box_muller_f32(u0, u1, z0, z1);
    }
    // constant for box_muller_scaled: -2 s^2 (times ln 2 for the log2 instruction)
    static __host__ __device__ __forceinline__ float scaled_const(double s) { return (float)(-2.0 * s * s * 0.69314718055994530942); }
    static __device__ __forceinline__ void box_muller_scaled(float u0, float u1, float k, float &z0, float &z1)
    {
        box_muller_scaled_f32(u0, u1, k, z0, z1);
    }
};

template <> struct Rng<double> {
    static __device__ __forceinline__ double uniform(uint32_t x) { return uniform_f64(x); }
    static __device__ __forceinline__ void box_muller(double u0, double u1, double &z0, double &z1)
    {
        box_muller_f64(u0, u1, z0, z1);
    }
    static __host__ __device__ __forceinline__ double scaled_const(double s) { return -2.0 * s * s; }
    static __device__ __forceinline__ void box_muller_scaled(double u0, double u1, double k, double &z0, double &z1)
    {
        box_muller_scaled_f64(u0, u1, k, z0, z1);
    }
};

}  // namespace vct
