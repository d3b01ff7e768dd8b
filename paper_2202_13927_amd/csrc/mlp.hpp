// mlp.hpp -- the learned controller: a 12 -> 64 -> 64 -> 64 -> 1 ReLU network evaluated by one
// wave for 64 samples at a time on BF16 MFMA (v_mfma_f32_16x16x16_bf16, FP32 accumulation).
//
// Operand layouts of v_mfma_f32_16x16x16_bf16 (checked on the device against a CPU matmul):
//   A[i][k] -> lane i + 16 (k/4), element k % 4;  B[k][j] -> lane j + 16 (k/4), element k % 4;
//   C[i][j] -> lane j + 16 (i/4), element i % 4.
// Activations are staged through LDS as BF16 row-major [sample][unit] tiles; weights are
// BF16 [out][in] (so a B fragment is 4 consecutive BF16 of one weight row).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vct {

constexpr int kMlpIn = 12;    // features
constexpr int kMlpInP = 16;   // padded to one MFMA K block
constexpr int kMlpH = 64;     // hidden width
constexpr int kMlpOutP = 16;  // output rows padded to one MFMA tile (row 0 is the output)

// Inference blob (bytes): BF16 weights, FP32 biases, FP32 normalisation and OOD box.
constexpr int kOffW1 = 0;                                  // bf16 [64][16]
constexpr int kOffW2 = kOffW1 + kMlpH * kMlpInP * 2;       // bf16 [64][64]
constexpr int kOffW3 = kOffW2 + kMlpH * kMlpH * 2;         // bf16 [64][64]
constexpr int kOffW4 = kOffW3 + kMlpH * kMlpH * 2;         // bf16 [16][64]
constexpr int kOffB1 = kOffW4 + kMlpOutP * kMlpH * 2;      // f32 [64]
constexpr int kOffB2 = kOffB1 + kMlpH * 4;
constexpr int kOffB3 = kOffB2 + kMlpH * 4;
constexpr int kOffB4 = kOffB3 + kMlpH * 4;                 // f32 [16]
constexpr int kOffMean = kOffB4 + kMlpOutP * 4;            // f32 [16] feature means
constexpr int kOffIstd = kOffMean + 16 * 4;                // f32 [16] 1 / feature std
constexpr int kOffLo = kOffIstd + 16 * 4;                  // f32 [16] 0.1 % quantile (raw)
constexpr int kOffHi = kOffLo + 16 * 4;                    // f32 [16] 99.9 % quantile (raw)
constexpr int kMlpBlobBytes = kOffHi + 16 * 4;
constexpr int kMlpNetBytes = kOffMean;                     // weights + biases (staged into LDS)

// FP32 parameter vector (master weights, Adam moments, gradients): same order, FP32.
constexpr int kPW1 = 0, kPW2 = kPW1 + kMlpH * kMlpInP, kPW3 = kPW2 + kMlpH * kMlpH, kPW4 = kPW3 + kMlpH * kMlpH;
constexpr int kPB1 = kPW4 + kMlpOutP * kMlpH, kPB2 = kPB1 + kMlpH, kPB3 = kPB2 + kMlpH, kPB4 = kPB3 + kMlpH;
constexpr int kMlpParams = kPB4 + kMlpOutP;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Two FP32 values -> packed BF16 pair (one v_cvt_pk_bf16_f32, round to nearest even).
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

// A fragment of a row-major matrix M (row stride ld): rows r0..r0+15, columns k0..k0+15.
// Also the B fragment of W^T for W row-major [N][K] (rows j0.., columns k0..).
__device__ __forceinline__ bf16x4 frag_rows(const uint16_t *M, int ld, int r0, int k0, int lane)
{
    const uint16_t *p = M + (r0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
    return __builtin_bit_cast(bf16x4, *(const uint2 *)p);
}

// The same for v_mfma_f32_16x16x32_bf16 (K block of 32): A[i][k] -> lane i + 16 (k/8),
// element k % 8, i.e. 8 consecutive columns of one row per lane (one 16-byte read).
__device__ __forceinline__ bf16x8 frag8_rows(const uint16_t *M, int ld, int r0, int k0, int lane)
{
    const uint16_t *p = M + (r0 + (lane & 15)) * ld + k0 + 8 * (lane >> 4);
    return __builtin_bit_cast(bf16x8, *(const uint4 *)p);
}

// B fragment of a row-major K x N matrix M: rows (k) r0.., columns c0..; also the A
// fragment of M^T (rows of M^T = columns of M).
__device__ __forceinline__ bf16x4 frag_cols(const uint16_t *M, int ld, int r0, int c0, int lane)
{
    const uint16_t *p = M + (r0 + 4 * (lane >> 4)) * ld + c0 + (lane & 15);
    bf16x4 r;
    r[0] = (short)p[0];
    r[1] = (short)p[ld];
    r[2] = (short)p[2 * ld];
    r[3] = (short)p[3 * ld];
    return r;
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Strides (in BF16 elements) of the LDS copies of the inputs, weights and activations.
// Padded strides keep the 16 rows read by one fragment load on distinct LDS banks.
template <int LDI, int LDW1, int LDW, int LDH> struct MlpLayout {
    static constexpr int ldi = LDI, ldw1 = LDW1, ldw = LDW, ldh = LDH;
};
using DenseLayout = MlpLayout<kMlpInP, kMlpInP, kMlpH, kMlpH>;   // the blob's own layout
using PaddedLayout = MlpLayout<24, 24, 72, 72>;                 // 48- and 144-byte rows

// Y[64][64] = relu(X[64][K] W^T + b) for one wave; W row-major [64][K]. Computed as
// Y^T = W X^T (A = W, B = X^T) with the bias as the accumulators' initial value, so each
// lane ends with four consecutive units of one sample and writes them with one 8-byte
// store. K = 16 uses v_mfma_f32_16x16x16_bf16, K = 64 v_mfma_f32_16x16x32_bf16. The result
// is written as BF16 into `out` after `sync()` (so out may alias X); two passes of 32 units
// keep 32 accumulator registers live.
template <int K, int LDX, int LDW, int LDO, typename Sync>
__device__ __forceinline__ void dense64_relu(const uint16_t *X, const uint16_t *W, const float *bias, uint16_t *out,
                                             int lane, Sync sync)
{
    uint2 res[2][2][4];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        f32x4 acc[2][4];   // [unit tile][sample tile]
#pragma unroll
        for (int ut = 0; ut < 2; ++ut) {
            const float4 bb = *(const float4 *)(bias + 32 * half + 16 * ut + 4 * (lane >> 4));
#pragma unroll
            for (int st = 0; st < 4; ++st)
                acc[ut][st] = f32x4{bb.x, bb.y, bb.z, bb.w};
        }
        if (K == 16) {
            bf16x4 a[2], b[4];
#pragma unroll
            for (int ut = 0; ut < 2; ++ut)
                a[ut] = frag_rows(W, LDW, 32 * half + 16 * ut, 0, lane);
#pragma unroll
            for (int st = 0; st < 4; ++st)
                b[st] = frag_rows(X, LDX, 16 * st, 0, lane);
#pragma unroll
            for (int ut = 0; ut < 2; ++ut)
#pragma unroll
                for (int st = 0; st < 4; ++st)
                    acc[ut][st] = mfma16(a[ut], b[st], acc[ut][st]);
        } else {
#pragma unroll
            for (int kb = 0; kb < K / 32; ++kb) {
                bf16x8 a[2], b[4];
#pragma unroll
                for (int ut = 0; ut < 2; ++ut)
                    a[ut] = frag8_rows(W, LDW, 32 * half + 16 * ut, 32 * kb, lane);
#pragma unroll
                for (int st = 0; st < 4; ++st)
                    b[st] = frag8_rows(X, LDX, 16 * st, 32 * kb, lane);
#pragma unroll
                for (int ut = 0; ut < 2; ++ut)
#pragma unroll
                    for (int st = 0; st < 4; ++st)
                        acc[ut][st] = mfma32(a[ut], b[st], acc[ut][st]);
            }
        }
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
#pragma unroll
            for (int st = 0; st < 4; ++st)
                res[half][ut][st] = uint2{pack_bf16(fmaxf(acc[ut][st][0], 0.f), fmaxf(acc[ut][st][1], 0.f)),
                                          pack_bf16(fmaxf(acc[ut][st][2], 0.f), fmaxf(acc[ut][st][3], 0.f))};
    }
    sync();
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
#pragma unroll
            for (int st = 0; st < 4; ++st)
                *(uint2 *)(out + (16 * st + (lane & 15)) * LDO + 32 * half + 16 * ut + 4 * (lane >> 4)) =
                    res[half][ut][st];
}

// Output layer: o[s] = H3[s][:] . W4[0][:] + b4[0] for the 64 samples, written to o (FP32).
// A = W4 (row 0 is the output unit), B = H3^T: row 0 of the product sits in element 0 of
// lanes 0..15.
template <int LDH, int LDW, typename Sync>
__device__ __forceinline__ void dense_out(const uint16_t *H, const uint16_t *W4, const float *b4, float *o, int lane,
                                          Sync sync)
{
    f32x4 acc[4];
    const float b = b4[0];
#pragma unroll
    for (int st = 0; st < 4; ++st)
        acc[st] = f32x4{b, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < kMlpH / 32; ++kb) {
        const bf16x8 a = frag8_rows(W4, LDW, 0, 32 * kb, lane);
#pragma unroll
        for (int st = 0; st < 4; ++st)
            acc[st] = mfma32(a, frag8_rows(H, LDH, 16 * st, 32 * kb, lane), acc[st]);
    }
    sync();
    if (lane < 16) {
#pragma unroll
        for (int st = 0; st < 4; ++st)
            o[16 * st + lane] = acc[st][0];
    }
}

// Network pointers into LDS (or global) memory.
struct MlpNet {
    const uint16_t *W1, *W2, *W3, *W4;
    const float *b1, *b2, *b3, *b4;
};

// Views of a blob (the unpadded layout).
__device__ __forceinline__ MlpNet mlp_net(const unsigned char *base)
{
    MlpNet n;
    n.W1 = (const uint16_t *)(base + kOffW1);
    n.W2 = (const uint16_t *)(base + kOffW2);
    n.W3 = (const uint16_t *)(base + kOffW3);
    n.W4 = (const uint16_t *)(base + kOffW4);
    n.b1 = (const float *)(base + kOffB1);
    n.b2 = (const float *)(base + kOffB2);
    n.b3 = (const float *)(base + kOffB3);
    n.b4 = (const float *)(base + kOffB4);
    return n;
}

// Forward pass of one wave: xs holds the 64 normalised samples (BF16 [64][L::ldi]); h1, h2,
// h3 receive the hidden activations (BF16 [64][L::ldh]; they may alias each other and xs
// when they are not needed later); o receives the outputs. sync() must order LDS writes
// before reads across the wave.
template <typename L, typename Sync>
__device__ __forceinline__ void mlp_forward(const MlpNet &n, const uint16_t *xs, uint16_t *h1, uint16_t *h2,
                                            uint16_t *h3, float *o, int lane, Sync sync)
{
    dense64_relu<kMlpInP, L::ldi, L::ldw1, L::ldh>(xs, n.W1, n.b1, h1, lane, sync);
    sync();
    dense64_relu<kMlpH, L::ldh, L::ldw, L::ldh>(h1, n.W2, n.b2, h2, lane, sync);
    sync();
    dense64_relu<kMlpH, L::ldh, L::ldw, L::ldh>(h2, n.W3, n.b3, h3, lane, sync);
    sync();
    dense_out<L::ldh, L::ldw>(h3, n.W4, n.b4, o, lane, sync);
    sync();
}

}  // namespace vct
