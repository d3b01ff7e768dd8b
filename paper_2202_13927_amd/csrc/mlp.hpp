// mlp.hpp -- the learned controller: a 12 -> 64 -> 64 -> 64 -> 1 ReLU network evaluated by one
// wave for 64 samples at a time on BF16 MFMA (v_mfma_f32_16x16x16_bf16 for the 16-wide input
// layer, v_mfma_f32_16x16x32_bf16 for the 64-wide layers; FP32 accumulation).
//
// Operand layouts (checked on the device against a CPU matmul), with K = 16 (x32: 8 and k/8):
//   A[i][k] -> lane i + 16 (k/4), element k % 4;  B[k][j] -> lane j + 16 (k/4), element k % 4;
//   C[i][j] -> lane j + 16 (i/4), element i % 4.
// Weights are BF16 [out][in]. Training stages activations through LDS as BF16 row-major
// [sample][unit] tiles (the backward pass needs them); inference keeps them in registers
// (mlp_forward_rf).
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

// FP32 parameter vector (master weights, Adam moments, gradients): same order, FP32.
constexpr int kPW1 = 0, kPW2 = kPW1 + kMlpH * kMlpInP, kPW3 = kPW2 + kMlpH * kMlpH, kPW4 = kPW3 + kMlpH * kMlpH;
constexpr int kPB1 = kPW4 + kMlpOutP * kMlpH, kPB2 = kPB1 + kMlpH, kPB3 = kPB2 + kMlpH, kPB4 = kPB3 + kMlpH;
constexpr int kMlpParams = kPB4 + kMlpOutP;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
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
using PaddedLayout = MlpLayout<24, 24, 72, 72>;                 // 48- and 144-byte rows

// ------------------------------------------------ register-resident inference ----
// The C fragment of Y^T = W X^T leaves lane j + 16 g holding units 4g..4g+3 of every 16-unit
// tile for sample j of every 16-sample tile. Two consecutive unit tiles 2t, 2t+1 thus give it
// eight units of its sample, which is exactly its B fragment for K block t of the next layer
// when that layer lists its inputs in the order of these fragments: K slot 8g + e of block t
// stands for unit 32t + 16 (e/4) + 4g + e % 4. The LDS image of the network stores the
// columns of W2, W3 and W4 in that order (a permutation of 4-column chunks inside each
// 32-column block), so a weight fragment stays one 16-byte read and the hidden activations
// never leave registers. Only the inputs (a transpose: each lane owns one sample) and the
// outputs (row 0 of the last product sits in lanes 0..15) pass through LDS.

// Source chunk (4 columns) of destination chunk q (0..7) of a 32-column block.
__host__ __device__ constexpr int hidden_chunk_src(int q) { return 4 * (q & 1) + (q >> 1); }

// Byte offsets of the LDS image of a blob: W1 [64][ldw1], W2 and W3 [64][ldw], W4 [16][ldw]
// (columns of W2..W4 permuted as above), then the biases, normalisation and box as in the blob.
template <typename L> struct NetImage {
    static constexpr int w1 = 0;
    static constexpr int w2 = w1 + kMlpH * L::ldw1 * 2;
    static constexpr int w3 = w2 + kMlpH * L::ldw * 2;
    static constexpr int w4 = w3 + kMlpH * L::ldw * 2;
    static constexpr int tail = w4 + kMlpOutP * L::ldw * 2;
    static constexpr int bytes = tail + (kMlpBlobBytes - kOffB1);
    static_assert(tail % 16 == 0, "16-byte aligned tail");
};

// Copies a blob into its LDS image (threads tid = 0..nthreads-1 of the block; the caller
// synchronises afterwards). 8-byte chunks: W1 256, W2 1024, W3 1024, W4 256, tail 136.
template <typename L>
__device__ __forceinline__ void stage_net(const unsigned char *blob, unsigned char *img, int tid, int nthreads)
{
    using I = NetImage<L>;
    constexpr int kTail = (kMlpBlobBytes - kOffB1) / 8;
    const uint2 *src = (const uint2 *)blob;
    for (int c = tid; c < 256 + 1024 + 1024 + 256 + kTail; c += nthreads) {
        int soff, doff;
        if (c < 256) {                       // W1: 4 chunks per row, natural order
            soff = kOffW1 + c * 8;
            doff = I::w1 + (c >> 2) * L::ldw1 * 2 + (c & 3) * 8;
        } else if (c < 256 + 2304) {          // W2, W3, W4: 16 chunks per row, permuted
            const int q = c - 256;
            const int layer = q < 1024 ? 0 : q < 2048 ? 1 : 2;
            const int qq = q - 1024 * layer;
            const int row = qq >> 4, blk = (qq >> 3) & 1, dq = qq & 7;
            const int sbase = layer == 0 ? kOffW2 : layer == 1 ? kOffW3 : kOffW4;
            const int dbase = layer == 0 ? I::w2 : layer == 1 ? I::w3 : I::w4;
            soff = sbase + (row * kMlpH + 32 * blk + 4 * hidden_chunk_src(dq)) * 2;
            doff = dbase + (row * L::ldw + 32 * blk + 4 * dq) * 2;
        } else {                              // biases, normalisation, box
            const int q = c - 256 - 2304;
            soff = kOffB1 + q * 8;
            doff = I::tail + q * 8;
        }
        *(uint2 *)(img + doff) = src[soff / 8];
    }
}

// ReLU of eight accumulators (units 4g..4g+3 of two unit tiles) rounded to BF16 (nearest,
// ties to even), as one B fragment. ReLU is taken on the rounded pairs as a signed 16-bit
// maximum with 0, which equals rounding the ReLU: rounding keeps the sign, and every negative
// BF16 (sign bit set) is a negative 16-bit integer.
__device__ __forceinline__ uint32_t relu_bf16x2(float lo, float hi)
{
    const s16x2 v = __builtin_bit_cast(s16x2, pack_bf16(lo, hi));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, s16x2{0, 0}));
}
__device__ __forceinline__ bf16x8 relu_frag(const f32x4 &a, const f32x4 &b)
{
    const uint4 w{relu_bf16x2(a[0], a[1]), relu_bf16x2(a[2], a[3]), relu_bf16x2(b[0], b[1]),
                  relu_bf16x2(b[2], b[3])};
    return __builtin_bit_cast(bf16x8, w);
}

// Weight and bias fragments of one 64 -> 64 layer for this lane: a[mt][kt] rows 16mt..,
// K block kt of the permuted LDS copy; b[mt] the biases of units 16mt + 4g .. +3.
struct HiddenFrags {
    bf16x8 a[4][2];
    f32x4 b[4];
};
template <typename L>
__device__ __forceinline__ HiddenFrags hidden_frags(const uint16_t *W, const float *bias, int lane)
{
    HiddenFrags f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f.b[mt] = *(const f32x4 *)(bias + 16 * mt + 4 * (lane >> 4));
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
            f.a[mt][kt] = frag8_rows(W, L::ldw, 16 * mt, 32 * kt, lane);
    }
    return f;
}

// One 64 -> 64 hidden layer on register fragments: h[t][s] (K block t, sample tile s) in,
// the next layer's fragments out.
__device__ __forceinline__ void hidden_rf(const HiddenFrags &f, bf16x8 h[2][4])
{
    bf16x8 out[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x4 acc[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[u][s] = f.b[2 * t + u];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc[u][s] = mfma32(f.a[2 * t + u][kt], h[kt][s], acc[u][s]);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
            out[t][s] = relu_frag(acc[0][s], acc[1][s]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s)
            h[t][s] = out[t][s];
}

// Forward pass of one wave on the LDS image `img` (layout L): xs holds the 64 normalised
// samples (BF16 [64][L::ldi], row = sample, columns 12..15 zero), o is 64 floats of LDS
// scratch; returns the output for sample `lane`. sync() must order the wave's LDS writes
// before its later reads. All 64 lanes must be active. Each layer's weight fragments are
// read one layer ahead, so the LDS latency overlaps the previous layer's MFMAs.
template <typename L, typename Sync>
__device__ __forceinline__ float mlp_forward_rf(const unsigned char *img, const uint16_t *xs, float *o, int lane,
                                                Sync sync)
{
    using I = NetImage<L>;
    const uint16_t *W1 = (const uint16_t *)(img + I::w1);
    const float *b1 = (const float *)(img + I::tail + (kOffB1 - kOffB1));
    const float *b2 = (const float *)(img + I::tail + (kOffB2 - kOffB1));
    const float *b3 = (const float *)(img + I::tail + (kOffB3 - kOffB1));
    const float *b4 = (const float *)(img + I::tail + (kOffB4 - kOffB1));
    bf16x4 a1[4], x[4];
    f32x4 bb1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        a1[mt] = frag_rows(W1, L::ldw1, 16 * mt, 0, lane);
        bb1[mt] = *(const f32x4 *)(b1 + 16 * mt + 4 * (lane >> 4));
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
        x[s] = frag_rows(xs, L::ldi, 16 * s, 0, lane);
    const HiddenFrags f2 = hidden_frags<L>((const uint16_t *)(img + I::w2), b2, lane);
    bf16x8 h[2][4];
    // input layer, K = 16: B = X^T read from the input tile
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x4 acc[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[u][s] = mfma16(a1[2 * t + u], x[s], bb1[2 * t + u]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
            h[t][s] = relu_frag(acc[0][s], acc[1][s]);
    }
    const HiddenFrags f3 = hidden_frags<L>((const uint16_t *)(img + I::w3), b3, lane);
    hidden_rf(f2, h);
    bf16x8 a4[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
        a4[kt] = frag8_rows((const uint16_t *)(img + I::w4), L::ldw, 0, 32 * kt, lane);
    const float bo = b4[0];
    hidden_rf(f3, h);
    f32x4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc[s] = f32x4{bo, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int s = 0; s < 4; ++s)
            acc[s] = mfma32(a4[kt], h[kt][s], acc[s]);
    if (lane < 16) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
            o[16 * s + lane] = acc[s][0];
    }
    sync();
    return o[lane];
}

// The same forward pass with a smaller register footprint, for kernels that keep much
// state of their own in registers: one layer's weight fragments are read from LDS just
// before the layer (not one layer ahead), and each 16-sample tile s goes through all 64
// units before the next, so its eight input fragments are replaced in place by its outputs
// (4 accumulator tiles live instead of 8, no second copy of the activations). The
// products, their order and the roundings are those of mlp_forward_rf: both return the
// same values bit for bit.
template <typename L, typename Sync>
__device__ __forceinline__ float mlp_forward_lean(const unsigned char *img, const uint16_t *xs, float *o, int lane,
                                                  Sync sync)
{
    using I = NetImage<L>;
    const float *b1 = (const float *)(img + I::tail + (kOffB1 - kOffB1));
    const float *b4 = (const float *)(img + I::tail + (kOffB4 - kOffB1));
    bf16x8 h[2][4];
    {   // input layer, K = 16: B = X^T read from the input tile
        const uint16_t *W1 = (const uint16_t *)(img + I::w1);
        bf16x4 a1[4];
        f32x4 bb1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            a1[mt] = frag_rows(W1, L::ldw1, 16 * mt, 0, lane);
            bb1[mt] = *(const f32x4 *)(b1 + 16 * mt + 4 * (lane >> 4));
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bf16x4 x = frag_rows(xs, L::ldi, 16 * s, 0, lane);
            f32x4 acc[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                acc[mt] = mfma16(a1[mt], x, bb1[mt]);
#pragma unroll
            for (int t = 0; t < 2; ++t)
                h[t][s] = relu_frag(acc[2 * t], acc[2 * t + 1]);
        }
    }
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {   // hidden layers 2 and 3
        const uint16_t *W = (const uint16_t *)(img + (layer == 0 ? I::w2 : I::w3));
        const float *bias = (const float *)(img + I::tail + ((layer == 0 ? kOffB2 : kOffB3) - kOffB1));
        const HiddenFrags f = hidden_frags<L>(W, bias, lane);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            f32x4 acc[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                acc[mt] = f.b[mt];
#pragma unroll
                for (int kt = 0; kt < 2; ++kt)
                    acc[mt] = mfma32(f.a[mt][kt], h[kt][s], acc[mt]);
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
                h[t][s] = relu_frag(acc[2 * t], acc[2 * t + 1]);
        }
    }
    bf16x8 a4[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
        a4[kt] = frag8_rows((const uint16_t *)(img + I::w4), L::ldw, 0, 32 * kt, lane);
    const float bo = b4[0];
    f32x4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        acc[s] = f32x4{bo, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
            acc[s] = mfma32(a4[kt], h[kt][s], acc[s]);
    }
    if (lane < 16) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
            o[16 * s + lane] = acc[s][0];
    }
    sync();
    return o[lane];
}

}  // namespace vct
