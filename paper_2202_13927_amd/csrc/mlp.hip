// mlp.hip -- training of the learned controller (behaviour cloning of the MPC) on BF16 MFMA.
//
// One training step over a minibatch of B rows (B a multiple of 64):
//  1. mlp_grad_kernel: one eight-wave workgroup per 64 rows draws its rows (Philox, with
//     replacement, or an explicit index list), normalises the 12 raw features, runs the
//     forward pass, and back-propagates the mean squared error sum (o - t)^2 / B through the
//     three hidden layers with MFMA GEMMs (activations and their gradients in BF16,
//     accumulation FP32), writing its partial gradient (all parameters) and partial loss;
//  2. mlp_update_kernel: sums the partials in a fixed order (deterministic), then applies
//     Adam to the FP32 master weights and refreshes the BF16 inference copy.
// Dataset rows are 13 FP32: the 12 features then the target u/u_b.
#include "internal.hpp"
#include "mlp.hpp"
#include "rng.hpp"

namespace vct {

constexpr int kRow = kMlpIn + 1;

__global__ void fill_u32_kernel_mlp(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

__device__ __forceinline__ bool padded_param(int p)
{
    if (p >= kPW1 && p < kPW2)
        return ((p - kPW1) % kMlpInP) >= kMlpIn;          // W1 columns 12..15
    if (p >= kPW4 && p < kPB1)
        return (p - kPW4) >= kMlpH;                         // W4 rows 1..15
    if (p >= kPB4)
        return p > kPB4;                                    // b4[1..15]
    return false;
}

// --------------------------------------------------------------------- init ----
// He-normal weights (std sqrt(2/fan_in); output row sqrt(1/64)), zero biases except the
// output bias 1 (the target u/u_b is 1 at the basal state). Normal p from Philox block
// (p/4, 0, 6, 0), Box-Muller. Adam moments zero.
__global__ void mlp_init_kernel(float *master, float *m, float *v, unsigned char *blob, uint32_t k0, uint32_t k1)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams)
        return;
    const U4 r = philox4x32_10((uint32_t)(p >> 2), 0u, 6u, 0u, k0, k1);
    double z0, z1, z2, z3;
    box_muller_f64(uniform_f64(r.x), uniform_f64(r.y), z0, z1);
    box_muller_f64(uniform_f64(r.z), uniform_f64(r.w), z2, z3);
    const double zz[4] = {z0, z1, z2, z3};
    const double z = zz[p & 3];
    double w = 0.0;
    if (p < kPW2)
        w = z * sqrt(2.0 / kMlpIn);
    else if (p < kPW4)
        w = z * sqrt(2.0 / kMlpH);
    else if (p < kPB1)
        w = z * sqrt(1.0 / kMlpH);
    else if (p == kPB4)
        w = 1.0;
    if (padded_param(p))
        w = 0.0;
    master[p] = (float)w;
    m[p] = 0.f;
    v[p] = 0.f;
    if (p < kPB1)
        ((uint16_t *)blob)[p] = f2bf((float)w);             // weights: same order, BF16
    else
        ((float *)(blob + kOffB1))[p - kPB1] = (float)w;    // biases: FP32
}

// ------------------------------------------------------------- normalisation ----
// Per-feature mean and standard deviation (FP64 sums) and the 0.1 % / 99.9 % quantiles of
// the raw features (nearest rank on a 4096-bin histogram between the min and max), which
// bound the inputs the network is trusted on.
constexpr int kHistBins = 4096;

struct StatPart {
    double sum[kMlpIn], sq[kMlpIn];
    float mn[kMlpIn], mx[kMlpIn];
};

__global__ __launch_bounds__(256) void mlp_stats_partial_kernel(const float *data, int64_t n, StatPart *parts)
{
    __shared__ StatPart sh[256];
    StatPart a;
    for (int f = 0; f < kMlpIn; ++f) {
        a.sum[f] = 0.0;
        a.sq[f] = 0.0;
        a.mn[f] = INFINITY;
        a.mx[f] = -INFINITY;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int f = 0; f < kMlpIn; ++f) {
            const float x = data[i * kRow + f];
            a.sum[f] += x;
            a.sq[f] += (double)x * x;
            a.mn[f] = fminf(a.mn[f], x);
            a.mx[f] = fmaxf(a.mx[f], x);
        }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int f = 0; f < kMlpIn; ++f) {
                sh[threadIdx.x].sum[f] += sh[threadIdx.x + w].sum[f];
                sh[threadIdx.x].sq[f] += sh[threadIdx.x + w].sq[f];
                sh[threadIdx.x].mn[f] = fminf(sh[threadIdx.x].mn[f], sh[threadIdx.x + w].mn[f]);
                sh[threadIdx.x].mx[f] = fmaxf(sh[threadIdx.x].mx[f], sh[threadIdx.x + w].mx[f]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        parts[blockIdx.x] = sh[0];
}

__global__ void mlp_stats_final_kernel(const StatPart *parts, int nparts, int64_t n, unsigned char *blob,
                                       float *range /* [2][12] min, max */)
{
    const int f = threadIdx.x;
    if (f >= 16)
        return;
    float *mean = (float *)(blob + kOffMean), *istd = (float *)(blob + kOffIstd);
    if (f >= kMlpIn) {
        mean[f] = 0.f;
        istd[f] = 0.f;
        ((float *)(blob + kOffLo))[f] = 0.f;
        ((float *)(blob + kOffHi))[f] = 0.f;
        return;
    }
    double s = 0.0, q = 0.0;
    float mn = INFINITY, mx = -INFINITY;
    for (int b = 0; b < nparts; ++b) {
        s += parts[b].sum[f];
        q += parts[b].sq[f];
        mn = fminf(mn, parts[b].mn[f]);
        mx = fmaxf(mx, parts[b].mx[f]);
    }
    const double mu = s / (double)n;
    const double var = fmax(q / (double)n - mu * mu, 0.0);
    mean[f] = (float)mu;
    istd[f] = (float)(1.0 / fmax(sqrt(var), 1e-6));
    range[f] = mn;
    range[kMlpIn + f] = mx;
}

__device__ __forceinline__ int hist_bin(float x, float mn, float mx)
{
    if (!(mx > mn))
        return 0;
    int b = (int)((x - mn) / (mx - mn) * (float)kHistBins);
    return b < 0 ? 0 : (b >= kHistBins ? kHistBins - 1 : b);
}

__global__ __launch_bounds__(256) void mlp_hist_kernel(const float *data, int64_t n, const float *range, uint32_t *hist)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int f = 0; f < kMlpIn; ++f)
            atomicAdd(&hist[f * kHistBins + hist_bin(data[i * kRow + f], range[f], range[kMlpIn + f])], 1u);
}

// Box edges: q = 0 -> [min, max]; else the nearest-rank q and 1 - q quantiles (rank
// ceil(q n), ceil((1 - q) n)), rounded outward to the histogram grid: lo = lower edge of the
// bin holding rank ceil(q n), hi = upper edge of the bin holding rank ceil((1 - q) n).
__global__ void mlp_quantile_kernel(const uint32_t *hist, const float *range, int64_t n, double q, unsigned char *blob)
{
    const int f = threadIdx.x;
    if (f >= kMlpIn)
        return;
    const float mn = range[f], mx = range[kMlpIn + f];
    float *lo = (float *)(blob + kOffLo), *hi = (float *)(blob + kOffHi);
    if (q <= 0.0) {
        lo[f] = mn;
        hi[f] = mx;
        return;
    }
    const float w = (mx - mn) / (float)kHistBins;
    const uint64_t r_lo = (uint64_t)ceil(q * (double)n);
    const uint64_t r_hi = (uint64_t)ceil((1.0 - q) * (double)n);
    uint64_t cum = 0;
    int b_lo = -1, b_hi = kHistBins - 1;
    for (int b = 0; b < kHistBins; ++b) {
        cum += hist[f * kHistBins + b];
        if (b_lo < 0 && cum >= r_lo)
            b_lo = b;
        if (cum >= r_hi) {
            b_hi = b;
            break;
        }
    }
    lo[f] = b_lo <= 0 ? mn : mn + w * (float)b_lo;
    hi[f] = b_hi >= kHistBins - 1 ? mx : mn + w * (float)(b_hi + 1);
}

// -------------------------------------------------------------- forward+backward ----
// One workgroup of eight waves per 64-row tile of the minibatch (two waves per SIMD). Wave
// (b, h) = (w % 4, w / 4) owns samples 16b..16b+15 and the half h of the units (32 of 64) in
// the forward pass and in the propagation of the gradient; the weight gradients, which
// contract over all 64 samples, are split by output tiles. Every MFMA operand is one 16-byte
// LDS read: activations and gradients are kept both as [sample][unit] and as [unit][sample]
// (the weight gradient contracts over samples), and the weights both as [out][in] and as
// [in][out] (the input gradient contracts over output units). Row strides are padded (72 and
// 24 elements) so the 16 rows a fragment reads fall on distinct banks.
constexpr int kGradThreads = 512;
constexpr int kLd = 72, kLd16 = 24;

struct TrainLds {
    uint16_t w1[64 * kLd16], w2[64 * kLd], w3[64 * kLd], w4[16 * kLd];   // [out][in]
    uint16_t w1t[16 * kLd], w2t[64 * kLd], w3t[64 * kLd];                // [in][out]
    alignas(16) float b1[64], b2[64], b3[64];
    uint16_t xs[64 * kLd16], xst[16 * kLd];                              // inputs [s][v], [v][s]
    uint16_t h[3][64 * kLd], ht[3][64 * kLd];                            // activations [s][u], [u][s]
    uint16_t g[2][64 * kLd], gt[2][64 * kLd];                            // gradients [s][u], [u][s]
    alignas(16) float o[64], target[64], dout[64], red[8][64];
};

// Workgroup barrier for LDS data only: waits for this wave's LDS operations, not for its
// global stores, so the partial gradients stream out while the next layer runs.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Stores the lane's four BF16 values (units u0..u0+3 of sample s, or samples s0..s0+3 of unit
// u; packed in pairs, low half first) of a C fragment in both layouts.
__device__ __forceinline__ void store_both(uint16_t *rowmajor, uint16_t *colmajor, int s, int u0, uint32_t p01,
                                           uint32_t p23)
{
    *(uint2 *)(rowmajor + s * kLd + u0) = uint2{p01, p23};
    colmajor[u0 * kLd + s] = (uint16_t)(p01 & 0xFFFFu);
    colmajor[(u0 + 1) * kLd + s] = (uint16_t)(p01 >> 16);
    colmajor[(u0 + 2) * kLd + s] = (uint16_t)(p23 & 0xFFFFu);
    colmajor[(u0 + 3) * kLd + s] = (uint16_t)(p23 >> 16);
}

// Keeps the low / high BF16 half of a packed pair where the flag is set, zero elsewhere.
__device__ __forceinline__ uint32_t keep_halves(uint32_t p, bool lo, bool hi)
{
    return p & ((lo ? 0x0000FFFFu : 0u) | (hi ? 0xFFFF0000u : 0u));
}

// Eight BF16 values at row-major (r, c0..c0+7) and transposed (c0..c0+7, r).
__device__ __forceinline__ void put8_both(uint16_t *rowmajor, int ldr, uint16_t *colmajor, int r, int c0, uint4 v)
{
    *(uint4 *)(rowmajor + r * ldr + c0) = v;
    const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        colmajor[(c0 + 2 * e) * kLd + r] = (uint16_t)(wd[e] & 0xFFFFu);
        colmajor[(c0 + 2 * e + 1) * kLd + r] = (uint16_t)(wd[e] >> 16);
    }
}

// Wave-local ordering of LDS accesses (the hardware keeps a wave's LDS operations in order;
// this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// H = relu(W X^T + b)^T for samples 16b..16b+15 and units 32h..32h+31 (K = 16 or 64): two
// 16-unit tiles, each element from the same MFMA operands and K order whichever wave
// computes it.
template <int K>
__device__ __forceinline__ void fwd_rows(const uint16_t *W, int ldw, const float *bias, const uint16_t *X, int ldx,
                                         uint16_t *H, uint16_t *HT, int b, int h, int lane)
{
    f32x4 acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float4 bb = *(const float4 *)(bias + 16 * (2 * h + i) + 4 * (lane >> 4));
        acc[i] = f32x4{bb.x, bb.y, bb.z, bb.w};
    }
    if (K == 16) {
        const bf16x4 x = frag_rows(X, ldx, 16 * b, 0, lane);
#pragma unroll
        for (int i = 0; i < 2; ++i)
            acc[i] = mfma16(frag_rows(W, ldw, 16 * (2 * h + i), 0, lane), x, acc[i]);
    } else {
#pragma unroll
        for (int kb = 0; kb < K / 32; ++kb) {
            const bf16x8 x = frag8_rows(X, ldx, 16 * b, 32 * kb, lane);
#pragma unroll
            for (int i = 0; i < 2; ++i)
                acc[i] = mfma32(frag8_rows(W, ldw, 16 * (2 * h + i), 32 * kb, lane), x, acc[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
        store_both(H, HT, 16 * b + (lane & 15), 16 * (2 * h + i) + 4 * (lane >> 4),
                   pack_bf16(fmaxf(acc[i][0], 0.f), fmaxf(acc[i][1], 0.f)),
                   pack_bf16(fmaxf(acc[i][2], 0.f), fmaxf(acc[i][3], 0.f)));
}

// Weight gradient of one hidden layer for output units 16ut..16ut+15 and input tiles
// vt0..vt0+NVT-1 (NV inputs in all), and with `bias` the bias gradient of those units. dHT:
// the layer's output gradient [u][s]; HinT: its input [v][s] (both over all 64 samples).
template <int NV, int NVT>
__device__ __forceinline__ void bwd_dw(const uint16_t *dHT, const uint16_t *HinT, float *gW, float *gb, int ut,
                                       int vt0, bool bias, int lane)
{
    // dW[u][v] = sum_s dH[s][u] Hin[s][v]: A = dH^T (rows u), B = Hin (K = samples)
#pragma unroll
    for (int i = 0; i < NVT; ++i) {
        const int vt = vt0 + i;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            acc = mfma32(frag8_rows(dHT, kLd, 16 * ut, 32 * kb, lane), frag8_rows(HinT, kLd, 16 * vt, 32 * kb, lane),
                         acc);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            gW[(16 * ut + 4 * (lane >> 4) + e) * NV + 16 * vt + (lane & 15)] = acc[e];
    }
    if (!bias)
        return;
    // db[u] = sum_s dH[s][u]: lane l sums samples 16q..16q+15 (q = l / 16) of unit 16ut + l % 16,
    // then the four quarters are added in a fixed order
    const uint16_t *p = dHT + (16 * ut + (lane & 15)) * kLd + 16 * (lane >> 4);
    const uint4 v0 = *(const uint4 *)p, v1 = *(const uint4 *)(p + 8);
    const uint32_t wd[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        acc += bf2f((uint16_t)(wd[q] & 0xFFFFu));
        acc += bf2f((uint16_t)(wd[q] >> 16));
    }
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    if (lane < 16)
        gb[16 * ut + lane] = acc;
}

// Input gradient of one hidden layer for samples 16b..16b+15 and inputs 32h..32h+31 through
// the previous ReLU: dHin[s][v] = sum_u dH[s][u] W[u][v] where Hin[s][v] > 0 (A = dH rows s,
// B = W^T rows v, K = all 64 units), in both layouts.
__device__ __forceinline__ void bwd_dh(const uint16_t *dH, const uint16_t *HinT, const uint16_t *WT, uint16_t *dHin,
                                       uint16_t *dHinT, int b, int h, int lane)
{
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int vt = 2 * h + i;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            acc = mfma32(frag8_rows(dH, kLd, 16 * b, 32 * kb, lane), frag8_rows(WT, kLd, 16 * vt, 32 * kb, lane), acc);
        // lane j + 16g holds samples 16b + 4g .. +3 of input unit 16vt + j
        const int v = 16 * vt + (lane & 15), s0 = 16 * b + 4 * (lane >> 4);
        const uint2 hin = *(const uint2 *)(HinT + v * kLd + s0);
        const uint32_t p01 = keep_halves(pack_bf16(acc[0], acc[1]), bf2f((uint16_t)(hin.x & 0xFFFFu)) > 0.f,
                                         bf2f((uint16_t)(hin.x >> 16)) > 0.f);
        const uint32_t p23 = keep_halves(pack_bf16(acc[2], acc[3]), bf2f((uint16_t)(hin.y & 0xFFFFu)) > 0.f,
                                         bf2f((uint16_t)(hin.y >> 16)) > 0.f);
        store_both(dHinT, dHin, v, s0, p01, p23);   // [v][s] takes the four consecutive samples
    }
}

// The raw features and the target of one minibatch row (thread s < 64 of a tile).
struct TileRow {
    float x[kMlpIn];
    float target;
};

__device__ __forceinline__ void fetch_row(const float *__restrict__ data, int64_t n_rows, const int32_t *idx,
                                          uint32_t k0, uint32_t k1, int32_t step, int64_t gi, TileRow &r)
{
    int64_t row;
    bool valid = true;
    if (idx) {
        row = idx[gi];
        valid = row >= 0 && row < n_rows;
        row = valid ? row : 0;   // an invalid index poisons the loss instead of reading outside
    } else {   // uniform with replacement: floor(x n / 2^32) for a Philox word x
        const U4 q = philox4x32_10((uint32_t)step, (uint32_t)gi, 5u, 0u, k0, k1);
        row = (int64_t)(((uint64_t)q.x * (uint64_t)n_rows) >> 32);
    }
#pragma unroll
    for (int f = 0; f < kMlpIn; ++f)
        r.x[f] = data[row * kRow + f];
    r.target = valid ? data[row * kRow + kMlpIn] : NAN;
}

// Gradient of one 64-row tile (kGradThreads threads): stages the network from the blob into
// LDS in both layouts (16-byte loads), normalises the tile's rows, runs the forward pass and
// back-propagates, writing the tile's partial gradient (all parameters) and partial loss.
__device__ __forceinline__ void grad_tile(TrainLds &L, const float *__restrict__ data, int64_t n_rows,
                                          const int32_t *idx, uint32_t k0, uint32_t k1, int32_t step, int32_t batch,
                                          int64_t tile, const unsigned char *blob, float *__restrict__ partial,
                                          float *__restrict__ loss_partial)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, b = w & 3, h = w >> 2;
    TileRow row;
    if (t < 64)
        fetch_row(data, n_rows, idx, k0, k1, step, tile * 64 + t, row);
    // weights: W2, W3 as 512 chunks of eight each, W1 and W4 as 128 each, b1..b3 as 48 float4
    const uint4 a0 = ((const uint4 *)(blob + kOffW2))[t], c0 = ((const uint4 *)(blob + kOffW3))[t];
    uint4 e0 = uint4{0u, 0u, 0u, 0u};
    if (t < 256)
        e0 = t < 128 ? ((const uint4 *)(blob + kOffW1))[t] : ((const uint4 *)(blob + kOffW4))[t - 128];
    float4 bb = float4{0.f, 0.f, 0.f, 0.f};
    if (t >= 256 && t < 256 + 48)
        bb = ((const float4 *)(blob + kOffB1))[t - 256];   // b1, b2, b3 are contiguous in the blob
    const float *mean = (const float *)(blob + kOffMean), *istd = (const float *)(blob + kOffIstd);
    put8_both(L.w2, kLd, L.w2t, t >> 3, (t & 7) * 8, a0);
    put8_both(L.w3, kLd, L.w3t, t >> 3, (t & 7) * 8, c0);
    if (t < 128)
        put8_both(L.w1, kLd16, L.w1t, t >> 1, (t & 1) * 8, e0);
    else if (t < 256)
        *(uint4 *)(L.w4 + ((t - 128) >> 3) * kLd + ((t - 128) & 7) * 8) = e0;
    else if (t < 256 + 48) {
        const int c = t - 256;
        float *dst = c < 16 ? L.b1 : (c < 32 ? L.b2 : L.b3);
        *(float4 *)(dst + 4 * (c & 15)) = bb;
    }
    if (t < 64) {
        static_assert(kMlpIn % 2 == 0 && kMlpInP == 16, "input pairs, one 16-element row");
        uint32_t xp[kMlpInP / 2];
#pragma unroll
        for (int f = 0; f < kMlpInP; f += 2)
            xp[f / 2] = f < kMlpIn ? pack_bf16((row.x[f] - mean[f]) * istd[f], (row.x[f + 1] - mean[f + 1]) * istd[f + 1])
                                   : 0u;
        *(uint4 *)(L.xs + t * kLd16) = uint4{xp[0], xp[1], xp[2], xp[3]};
        *(uint4 *)(L.xs + t * kLd16 + 8) = uint4{xp[4], xp[5], xp[6], xp[7]};
#pragma unroll
        for (int f = 0; f < kMlpInP; ++f)
            L.xst[f * kLd + t] = (uint16_t)(xp[f / 2] >> (16 * (f & 1)));
        L.target[t] = row.target;
    }
    lds_barrier();

    // Forward pass and the propagation of the gradient back to layer 1: wave (b, h) computes
    // samples 16b.. for the unit half h; a barrier before each layer that reads all 64 units
    // of the previous one. Activations h1..h3, gradients d3 (g[0]), d2 (g[1]) and d1 (into
    // h[2], whose h3 nobody reads any more by then), all in both layouts.
    fwd_rows<kMlpInP>(L.w1, kLd16, L.b1, L.xs, kLd16, L.h[0], L.ht[0], b, h, lane);
    lds_barrier();
    fwd_rows<kMlpH>(L.w2, kLd, L.b2, L.h[0], kLd, L.h[1], L.ht[1], b, h, lane);
    lds_barrier();
    fwd_rows<kMlpH>(L.w3, kLd, L.b3, L.h[1], kLd, L.h[2], L.ht[2], b, h, lane);
    lds_barrier();
    {   // output unit for samples 16b..16b+15 (row 0 of W4 H3^T in lanes 0..15); both waves of
        // the sample block compute it and store the same values, so each reads its own
        const float b4 = ((const float *)(blob + kOffB4))[0];
        f32x4 acc = f32x4{b4, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            acc = mfma32(frag8_rows(L.w4, kLd, 0, 32 * kb, lane), frag8_rows(L.h[2], kLd, 16 * b, 32 * kb, lane), acc);
        if (lane < 16) {
            const int s = 16 * b + lane;
            const float r = acc[0] - L.target[s];
            L.o[s] = acc[0];
            L.dout[s] = 2.f * r / (float)batch;
        }
    }
    wave_lds_order();
    {   // output layer for units 32h + l % 32 and samples 16b + 8(l / 32) .. +7: the partial
        // gW4[u] over those eight samples (in order) and d3 = dout w4 through the ReLU
        const int u = 32 * h + (lane & 31), s0 = 16 * b + 8 * (lane >> 5);
        const float w4u = bf2f(L.w4[u]);
        const uint4 hq = *(const uint4 *)(L.ht[2] + u * kLd + s0);
        const uint32_t hw[4] = {hq.x, hq.y, hq.z, hq.w};
        const float4 d0 = *(const float4 *)(L.dout + s0), d1 = *(const float4 *)(L.dout + s0 + 4);
        const float dv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
        float acc = 0.f;
        uint32_t dw[4];
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const float h0v = bf2f((uint16_t)(hw[i >> 1] & 0xFFFFu)), h1v = bf2f((uint16_t)(hw[i >> 1] >> 16));
            acc += dv[i] * h0v;
            acc += dv[i + 1] * h1v;
            dw[i >> 1] = keep_halves(pack_bf16(dv[i] * w4u, dv[i + 1] * w4u), h0v > 0.f, h1v > 0.f);
            L.g[0][(s0 + i) * kLd + u] = (uint16_t)(dw[i >> 1] & 0xFFFFu);
            L.g[0][(s0 + i + 1) * kLd + u] = (uint16_t)(dw[i >> 1] >> 16);
        }
        *(uint4 *)(L.gt[0] + u * kLd + s0) = uint4{dw[0], dw[1], dw[2], dw[3]};
        L.red[2 * b + (lane >> 5)][u] = acc;
    }
    lds_barrier();
    bwd_dh(L.g[0], L.ht[1], L.w3t, L.g[1], L.gt[1], b, h, lane);    // d2
    lds_barrier();
    bwd_dh(L.g[1], L.ht[0], L.w2t, L.h[2], L.ht[2], b, h, lane);    // d1
    float *g = partial + tile * kMlpParams;
    for (int i = t; i < (kMlpOutP - 1) * kMlpH; i += kGradThreads)   // output rows 1..15: padding
        g[kPW4 + kMlpH + i] = 0.f;
    lds_barrier();

    // Contractions over all 64 samples: wave w takes output tile w % 4 of each layer and half
    // w / 4 of its input tiles (the bias gradient with the first half)
    if (t < 64) {   // loss partial: sum over the 64 rows of r^2 / B (butterfly, fixed order)
        const float r = L.o[t] - L.target[t];
        float q = r * r / (float)batch;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            q += __shfl_xor(q, off);
        if (t == 0)
            loss_partial[tile] = q;
        g[kPW4 + t] = ((L.red[0][t] + L.red[1][t]) + (L.red[2][t] + L.red[3][t])) +
                      ((L.red[4][t] + L.red[5][t]) + (L.red[6][t] + L.red[7][t]));
    } else if (t < 64 + kMlpOutP) {
        float sb = 0.f;
        if (t == 64)
            for (int s = 0; s < 64; ++s)
                sb += L.dout[s];
        g[kPB4 + (t - 64)] = sb;
    }
    bwd_dw<kMlpH, 2>(L.gt[0], L.ht[1], g + kPW3, g + kPB3, b, 2 * h, h == 0, lane);
    bwd_dw<kMlpH, 2>(L.gt[1], L.ht[0], g + kPW2, g + kPB2, b, 2 * h, h == 0, lane);
    if (h == 0)
        bwd_dw<kMlpInP, 1>(L.ht[2], L.xst, g + kPW1, g + kPB1, b, 0, true, lane);
}

__global__ __launch_bounds__(kGradThreads) void mlp_grad_kernel(const float *__restrict__ data, int64_t n_rows,
                                                                const int32_t *__restrict__ idx, uint32_t k0,
                                                                uint32_t k1, int32_t step, int32_t batch,
                                                                const unsigned char *__restrict__ blob,
                                                                float *__restrict__ partial,
                                                                float *__restrict__ loss_partial)
{
    __shared__ __align__(16) TrainLds L;
    grad_tile(L, data, n_rows, idx, k0, k1, step, batch, blockIdx.x, blob, partial, loss_partial);
}

// ------------------------------------------------------------------ update ----
// Parameters 64 pb .. 64 pb + 63 (one block of 256 threads): thread (g, q) = (t / 16, t % 16)
// sums tiles q per .. (q + 1) per - 1 in order (per = ceil(tiles / 16)) for the four
// parameters 64 pb + 4g .., with 16-byte loads; the 16 parts are added by a butterfly over
// the lanes of the group (lane bits 0..3, the same sum in all 16 lanes), and lane q < 4 takes
// the Adam step of parameter 4g + q on the FP32 master weights and the BF16 / FP32 inference
// copy.
constexpr int kUpdParts = 16;
constexpr int kParamBlocks = (kMlpParams + 63) / 64;
static_assert(kMlpParams % 4 == 0, "parameters are summed four at a time");

__device__ __forceinline__ void update_block(int pb, int t, const float *__restrict__ partial, int n_parts,
                                             float *master, float *m, float *v, float *grad, unsigned char *blob,
                                             float lr, float bc1, float bc2, int apply)
{
    const int q = t & (kUpdParts - 1), p0 = pb * 64 + 4 * (t / kUpdParts);
    if (p0 >= kMlpParams)   // the 16 lanes of a group leave together
        return;
    const int p = p0 + (q & 3);
    const float m0 = m[p], v0 = v[p], w0 = master[p];   // in flight with the partials
    const int per = (n_parts + kUpdParts - 1) / kUpdParts;
    const int b0 = q * per, b1 = min(n_parts, b0 + per);
    float4 sum = float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int b = b0; b < b1; ++b) {
        const float4 x = *(const float4 *)(partial + (int64_t)b * kMlpParams + p0);
        sum.x += x.x;
        sum.y += x.y;
        sum.z += x.z;
        sum.w += x.w;
    }
    float s4[4] = {sum.x, sum.y, sum.z, sum.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int off = 1; off < kUpdParts; off <<= 1)
            s4[e] += __shfl_xor(s4[e], off);
    if (q >= 4)
        return;
    float gs = q == 0 ? s4[0] : (q == 1 ? s4[1] : (q == 2 ? s4[2] : s4[3]));
    if (padded_param(p))
        gs = 0.f;
    grad[p] = gs;
    if (!apply || padded_param(p))
        return;
    const float be1 = 0.9f, be2 = 0.999f, eps = 1e-8f;
    const float mm = be1 * m0 + (1.f - be1) * gs;
    const float vv = be2 * v0 + (1.f - be2) * gs * gs;
    m[p] = mm;
    v[p] = vv;
    const float wn = w0 - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    master[p] = wn;
    if (p < kPB1)
        ((uint16_t *)blob)[p] = f2bf(wn);
    else
        ((float *)(blob + kOffB1))[p - kPB1] = wn;
}

// Minibatch loss = the sum of the per-tile partials, by one wave: lane l adds tiles l, l + 64,
// .. in order (one round of loads for up to 64 tiles), then a butterfly in a fixed order.
__device__ __forceinline__ void sum_loss(const float *loss_partial, int n_parts, float *loss, int lane)
{
    float l = 0.f;
    for (int b = lane; b < n_parts; b += 64)
        l += loss_partial[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        l += __shfl_xor(l, off);
    if (lane == 0)
        *loss = l;
}

__global__ __launch_bounds__(256) void mlp_update_kernel(const float *__restrict__ partial, int n_parts,
                                                         const float *__restrict__ loss_partial, float *master,
                                                         float *m, float *v, float *grad, float *loss,
                                                         unsigned char *blob, float lr, float bc1, float bc2, int apply)
{
    if (blockIdx.x == 0 && threadIdx.x < 64)
        sum_loss(loss_partial, n_parts, loss, threadIdx.x);
    update_block(blockIdx.x, threadIdx.x, partial, n_parts, master, m, v, grad, blob, lr, bc1, bc2, apply);
}

// -------------------------------------------------------------- batched forward ----
// The learned controller's own evaluation (mlp_forward_rf on the padded LDS image), four
// waves per block sharing one staged copy of the network, 64 rows per wave.
constexpr int kFwdBlock = 256;
using FwdNet = NetImage<PaddedLayout>;
constexpr int kFwdWaveBytes = 64 * PaddedLayout::ldi * 2 + 64 * 4;

__global__ __launch_bounds__(kFwdBlock) void mlp_forward_kernel(const float *__restrict__ x, int64_t n,
                                                                const unsigned char *__restrict__ blob,
                                                                float *__restrict__ out)
{
    __shared__ __align__(16) unsigned char lds[FwdNet::bytes + (kFwdBlock / 64) * kFwdWaveBytes];
    stage_net<PaddedLayout>(blob, lds, threadIdx.x, kFwdBlock);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint16_t *xs = (uint16_t *)(lds + FwdNet::bytes + wave * kFwdWaveBytes);
    float *o = (float *)((unsigned char *)xs + 64 * PaddedLayout::ldi * 2);
    const int64_t gi = (int64_t)blockIdx.x * kFwdBlock + threadIdx.x;
    const int64_t row = gi < n ? gi : n - 1;
    const float *mean = (const float *)(blob + kOffMean), *istd = (const float *)(blob + kOffIstd);
    for (int f = 0; f < PaddedLayout::ldi; ++f)
        xs[lane * PaddedLayout::ldi + f] =
            f < kMlpIn ? f2bf((x[row * kMlpIn + f] - mean[f]) * istd[f]) : (uint16_t)0;
    __syncthreads();
    const float r = mlp_forward_rf<PaddedLayout>(lds, xs, o, lane, wave_sync);
    if (gi < n)
        out[gi] = r;
}

// ---------------------------------------------------------------- launchers ----
hipError_t launch_mlp_init(const MlpTrain &t, uint32_t k0, uint32_t k1, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_init_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, t.master, t.m, t.v, t.blob,
                       k0, k1);
    return hipGetLastError();
}

size_t mlp_stats_scratch_bytes() { return 256 * sizeof(StatPart) + 2 * kMlpIn * sizeof(float) + 12 * kHistBins * 4; }

hipError_t launch_mlp_stats(const float *data, int64_t n, double box_q, unsigned char *blob, void *scratch,
                            hipStream_t s)
{
    StatPart *parts = (StatPart *)scratch;
    float *range = (float *)((char *)scratch + 256 * sizeof(StatPart));
    uint32_t *hist = (uint32_t *)(range + 2 * kMlpIn);
    hipLaunchKernelGGL(mlp_stats_partial_kernel, dim3(256), dim3(256), 0, s, data, n, parts);
    hipLaunchKernelGGL(mlp_stats_final_kernel, dim3(1), dim3(64), 0, s, parts, 256, n, blob, range);
    hipLaunchKernelGGL(fill_u32_kernel_mlp, dim3(64), dim3(256), 0, s, hist, (int64_t)kMlpIn * kHistBins);
    hipLaunchKernelGGL(mlp_hist_kernel, dim3(512), dim3(256), 0, s, data, n, range, hist);
    hipLaunchKernelGGL(mlp_quantile_kernel, dim3(1), dim3(64), 0, s, hist, range, n, box_q, blob);
    return hipGetLastError();
}

hipError_t launch_mlp_step(const MlpTrain &t, const float *data, int64_t n_rows, const int32_t *idx, uint32_t k0,
                           uint32_t k1, int32_t step, int32_t batch, float lr, float bc1, float bc2, int apply,
                           hipStream_t s)
{
    const int parts = batch / 64;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(parts), dim3(kGradThreads), 0, s, data, n_rows, idx, k0, k1, step, batch, t.blob,
                       t.partial, t.loss_partial);
    hipLaunchKernelGGL(mlp_update_kernel, dim3(kParamBlocks), dim3(256), 0, s, t.partial, parts, t.loss_partial,
                       t.master, t.m, t.v, t.grad, t.loss, t.blob, lr, bc1, bc2, apply);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *x, int64_t n, const unsigned char *blob, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + kFwdBlock - 1) / kFwdBlock)), dim3(kFwdBlock), 0, s, x,
                       n, blob, out);
    return hipGetLastError();
}

}  // namespace vct
