// mlp.hip -- training of the learned controller (behaviour cloning of the MPC) on BF16 MFMA.
//
// One training step over a minibatch of B rows (B a multiple of 64):
//  1. mlp_grad_kernel: one four-wave workgroup per 64 rows draws its rows (Philox, with
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
// One workgroup of four waves per 64-row tile of the minibatch; each wave takes a quarter of
// every layer (16 output units in the forward pass and in the weight gradients, 16 samples in
// the input gradients), so the 64 tiles of a 4096-row step run as 256 waves. Every MFMA
// operand is one 16-byte LDS read: activations and gradients are kept both as [sample][unit]
// and as [unit][sample] (the weight gradient contracts over samples), and the weights both as
// [out][in] and as [in][out] (the input gradient contracts over output units). Row strides are
// padded (72 and 24 elements) so the 16 rows a fragment reads fall on distinct banks.
constexpr int kLd = 72, kLd16 = 24;

struct TrainLds {
    uint16_t w1[64 * kLd16], w2[64 * kLd], w3[64 * kLd], w4[16 * kLd];   // [out][in]
    uint16_t w1t[16 * kLd], w2t[64 * kLd], w3t[64 * kLd];                // [in][out]
    float b1[64], b2[64], b3[64];
    uint16_t xs[64 * kLd16], xst[16 * kLd];                              // inputs [s][v], [v][s]
    uint16_t h[3][64 * kLd], ht[3][64 * kLd];                            // activations [s][u], [u][s]
    uint16_t g[2][64 * kLd], gt[2][64 * kLd];                            // gradients [s][u], [u][s]
    float o[64], target[64], dout[64], red[4][64];
};

// Stores the lane's four values (units u0..u0+3 of sample s, or samples s0..s0+3 of unit u)
// of a C fragment in both layouts.
__device__ __forceinline__ void store_both(uint16_t *rowmajor, uint16_t *colmajor, int s, int u0, const uint16_t r[4])
{
    *(uint2 *)(rowmajor + s * kLd + u0) =
        uint2{(uint32_t)r[0] | ((uint32_t)r[1] << 16), (uint32_t)r[2] | ((uint32_t)r[3] << 16)};
#pragma unroll
    for (int e = 0; e < 4; ++e)
        colmajor[(u0 + e) * kLd + s] = r[e];
}

// Y^T = relu(W X^T + b) for units 16w..16w+15 and all 64 samples (K = 16 or 64).
template <int K>
__device__ __forceinline__ void fwd_quarter(const uint16_t *W, int ldw, const float *bias, const uint16_t *X, int ldx,
                                            uint16_t *H, uint16_t *HT, int w, int lane)
{
    const float4 bb = *(const float4 *)(bias + 16 * w + 4 * (lane >> 4));
    f32x4 acc[4];
#pragma unroll
    for (int st = 0; st < 4; ++st)
        acc[st] = f32x4{bb.x, bb.y, bb.z, bb.w};
    if (K == 16) {
        const bf16x4 a = frag_rows(W, ldw, 16 * w, 0, lane);
#pragma unroll
        for (int st = 0; st < 4; ++st)
            acc[st] = mfma16(a, frag_rows(X, ldx, 16 * st, 0, lane), acc[st]);
    } else {
#pragma unroll
        for (int kb = 0; kb < K / 32; ++kb) {
            const bf16x8 a = frag8_rows(W, ldw, 16 * w, 32 * kb, lane);
#pragma unroll
            for (int st = 0; st < 4; ++st)
                acc[st] = mfma32(a, frag8_rows(X, ldx, 16 * st, 32 * kb, lane), acc[st]);
        }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        uint16_t r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            r[e] = f2bf(fmaxf(acc[st][e], 0.f));
        store_both(H, HT, 16 * st + (lane & 15), 16 * w + 4 * (lane >> 4), r);
    }
}

// Gradients of one hidden layer, the wave's quarter: dW rows 16w.. (NV columns), db of units
// 16w.., and (dHin != null) the input gradient of samples 16w.. through the previous ReLU.
// dH / dHT: the layer's output gradient in both layouts; HinT: its input [v][s]; WT: its
// weights [v][u].
template <int NV>
__device__ __forceinline__ void bwd_quarter(const uint16_t *dH, const uint16_t *dHT, const uint16_t *HinT,
                                            const uint16_t *WT, float *gW, float *gb, uint16_t *dHin, uint16_t *dHinT,
                                            int w, int lane)
{
    // dW[u][v] = sum_s dH[s][u] Hin[s][v]: A = dH^T (rows u), B = Hin (K = samples)
#pragma unroll
    for (int vt = 0; vt < NV / 16; ++vt) {
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            acc = mfma32(frag8_rows(dHT, kLd, 16 * w, 32 * kb, lane), frag8_rows(HinT, kLd, 16 * vt, 32 * kb, lane),
                         acc);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            gW[(16 * w + 4 * (lane >> 4) + e) * NV + 16 * vt + (lane & 15)] = acc[e];
    }
    // db[u] = sum_s dH[s][u]: lane l sums samples 16q..16q+15 (q = l / 16) of unit 16w + l % 16,
    // then the four quarters are added in a fixed order
    {
        const uint16_t *p = dHT + (16 * w + (lane & 15)) * kLd + 16 * (lane >> 4);
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
            gb[16 * w + lane] = acc;
    }
    if (!dHin)
        return;
    // dHin[s][v] = sum_u dH[s][u] W[u][v] where Hin[s][v] > 0: A = dH (rows s), B = W (K = units)
#pragma unroll
    for (int vt = 0; vt < NV / 16; ++vt) {
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            acc = mfma32(frag8_rows(dH, kLd, 16 * w, 32 * kb, lane), frag8_rows(WT, kLd, 16 * vt, 32 * kb, lane), acc);
        // lane j + 16g holds samples 16w + 4g .. +3 of input unit 16vt + j
        const int v = 16 * vt + (lane & 15), s0 = 16 * w + 4 * (lane >> 4);
        const uint2 hin = *(const uint2 *)(HinT + v * kLd + s0);
        const uint16_t hv[4] = {(uint16_t)(hin.x & 0xFFFFu), (uint16_t)(hin.x >> 16), (uint16_t)(hin.y & 0xFFFFu),
                                (uint16_t)(hin.y >> 16)};
        uint16_t r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            r[e] = bf2f(hv[e]) > 0.f ? f2bf(acc[e]) : (uint16_t)0;
        store_both(dHinT, dHin, v, s0, r);   // [v][s] takes the four consecutive samples
    }
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float *__restrict__ data, int64_t n_rows,
                                                       const int32_t *__restrict__ idx, uint32_t k0, uint32_t k1,
                                                       int32_t step, int32_t batch,
                                                       const unsigned char *__restrict__ blob,
                                                       float *__restrict__ partial, float *__restrict__ loss_partial)
{
    __shared__ __align__(16) TrainLds L;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // weights in both layouts, biases
    const uint16_t *W1 = (const uint16_t *)(blob + kOffW1), *W2 = (const uint16_t *)(blob + kOffW2);
    const uint16_t *W3 = (const uint16_t *)(blob + kOffW3), *W4 = (const uint16_t *)(blob + kOffW4);
    for (int i = t; i < 64 * 64; i += 256) {
        const int u = i >> 6, v = i & 63;
        const uint16_t a = W2[i], b = W3[i];
        L.w2[u * kLd + v] = a;
        L.w2t[v * kLd + u] = a;
        L.w3[u * kLd + v] = b;
        L.w3t[v * kLd + u] = b;
    }
    for (int i = t; i < 64 * kMlpInP; i += 256) {
        const int u = i / kMlpInP, v = i % kMlpInP;
        L.w1[u * kLd16 + v] = W1[i];
        L.w1t[v * kLd + u] = W1[i];
    }
    for (int i = t; i < kMlpOutP * 64; i += 256)
        L.w4[(i >> 6) * kLd + (i & 63)] = W4[i];
    if (t < 64) {
        L.b1[t] = ((const float *)(blob + kOffB1))[t];
        L.b2[t] = ((const float *)(blob + kOffB2))[t];
        L.b3[t] = ((const float *)(blob + kOffB3))[t];
    }
    // the tile's rows: thread s < 64 takes sample s
    const int64_t tile = blockIdx.x;
    if (t < 64) {
        const int64_t gi = tile * 64 + t;
        int64_t row;
        bool valid = true;
        if (idx) {
            row = idx[gi];
            valid = row >= 0 && row < n_rows;
            row = valid ? row : 0;   // an invalid index poisons the loss instead of reading outside
        } else {   // uniform with replacement: floor(x n / 2^32) for a Philox word x
            const U4 r = philox4x32_10((uint32_t)step, (uint32_t)gi, 5u, 0u, k0, k1);
            row = (int64_t)(((uint64_t)r.x * (uint64_t)n_rows) >> 32);
        }
        const float *mean = (const float *)(blob + kOffMean), *istd = (const float *)(blob + kOffIstd);
        for (int f = 0; f < kMlpInP; ++f) {
            const uint16_t x = f < kMlpIn ? f2bf((data[row * kRow + f] - mean[f]) * istd[f]) : (uint16_t)0;
            L.xs[t * kLd16 + f] = x;
            L.xst[f * kLd + t] = x;
        }
        L.target[t] = valid ? data[row * kRow + kMlpIn] : NAN;
    }
    __syncthreads();

    // forward: each wave a quarter of the units of every layer
    fwd_quarter<kMlpInP>(L.w1, kLd16, L.b1, L.xs, kLd16, L.h[0], L.ht[0], w, lane);
    __syncthreads();
    fwd_quarter<kMlpH>(L.w2, kLd, L.b2, L.h[0], kLd, L.h[1], L.ht[1], w, lane);
    __syncthreads();
    fwd_quarter<kMlpH>(L.w3, kLd, L.b3, L.h[1], kLd, L.h[2], L.ht[2], w, lane);
    __syncthreads();
    {   // output unit for samples 16w..16w+15: row 0 of W4 H3^T sits in lanes 0..15
        const float b4 = ((const float *)(blob + kOffB4))[0];
        f32x4 acc = f32x4{b4, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            acc = mfma32(frag8_rows(L.w4, kLd, 0, 32 * kb, lane), frag8_rows(L.h[2], kLd, 16 * w, 32 * kb, lane), acc);
        if (lane < 16)
            L.o[16 * w + lane] = acc[0];
    }
    __syncthreads();

    float *g = partial + tile * kMlpParams;
    if (t < 64) {   // loss partial: sum over the 64 rows of r^2 / B (butterfly, fixed order)
        const float r = L.o[t] - L.target[t];
        L.dout[t] = 2.f * r / (float)batch;
        float q = r * r / (float)batch;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            q += __shfl_xor(q, off);
        if (t == 0)
            loss_partial[tile] = q;
    }
    __syncthreads();
    {   // output layer: gW4[u] = sum_s dout[s] h3[s][u] over four sample quarters; the gradient
        // of h3 through the ReLU, in both layouts
        const int u = t & 63, q = t >> 6;
        const float w4u = bf2f(L.w4[u]);
        float acc = 0.f;
        for (int s = 16 * q; s < 16 * q + 16; ++s) {
            const float hv = bf2f(L.h[2][s * kLd + u]);
            acc += L.dout[s] * hv;
            const uint16_t d = hv > 0.f ? f2bf(L.dout[s] * w4u) : (uint16_t)0;
            L.g[0][s * kLd + u] = d;
            L.gt[0][u * kLd + s] = d;
        }
        L.red[q][u] = acc;
    }
    for (int i = t; i < (kMlpOutP - 1) * kMlpH; i += 256)   // output rows 1..15: padding
        g[kPW4 + kMlpH + i] = 0.f;
    __syncthreads();
    if (t < 64)
        g[kPW4 + t] = (L.red[0][t] + L.red[1][t]) + (L.red[2][t] + L.red[3][t]);
    else if (t < 64 + kMlpOutP) {
        float sb = 0.f;
        if (t == 64)
            for (int s = 0; s < 64; ++s)
                sb += L.dout[s];
        g[kPB4 + (t - 64)] = sb;
    }
    bwd_quarter<kMlpH>(L.g[0], L.gt[0], L.ht[1], L.w3t, g + kPW3, g + kPB3, L.g[1], L.gt[1], w, lane);
    __syncthreads();
    bwd_quarter<kMlpH>(L.g[1], L.gt[1], L.ht[0], L.w2t, g + kPW2, g + kPB2, L.g[0], L.gt[0], w, lane);
    __syncthreads();
    bwd_quarter<kMlpInP>(L.g[0], L.gt[0], L.xst, L.w1t, g + kPW1, g + kPB1, nullptr, nullptr, w, lane);
}

// ------------------------------------------------------------------ update ----
// Sums the per-tile partials in a fixed order (four threads per parameter each add a quarter
// of the tiles in sequence, then the quarters are added pairwise), then Adam on the FP32
// master weights and the BF16 / FP32 inference copy.
constexpr int kUpdSplit = 4;

__global__ __launch_bounds__(256) void mlp_update_kernel(const float *__restrict__ partial, int n_parts,
                                                         const float *__restrict__ loss_partial, float *master,
                                                         float *m, float *v, float *grad, float *loss,
                                                         unsigned char *blob, float lr, float bc1, float bc2, int apply)
{
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = gt / kUpdSplit, part = gt % kUpdSplit;
    if (gt == 0) {
        float l = 0.f;
        for (int b = 0; b < n_parts; ++b)
            l += loss_partial[b];
        *loss = l;
    }
    const int per = (n_parts + kUpdSplit - 1) / kUpdSplit;
    const int b0 = part * per, b1 = min(n_parts, b0 + per);
    float gs = 0.f;
    if (p < kMlpParams) {
#pragma unroll 16
        for (int b = b0; b < b1; ++b)
            gs += partial[(int64_t)b * kMlpParams + p];
    }
    // (q0 + q1) + (q2 + q3) across the four consecutive lanes of a parameter
    gs += __shfl_xor(gs, 1);
    gs += __shfl_xor(gs, 2);
    if (p >= kMlpParams || part != 0)
        return;
    if (padded_param(p))
        gs = 0.f;
    grad[p] = gs;
    if (!apply || padded_param(p))
        return;
    const float be1 = 0.9f, be2 = 0.999f, eps = 1e-8f;
    const float mm = be1 * m[p] + (1.f - be1) * gs;
    const float vv = be2 * v[p] + (1.f - be2) * gs * gs;
    m[p] = mm;
    v[p] = vv;
    const float wn = master[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    master[p] = wn;
    if (p < kPB1)
        ((uint16_t *)blob)[p] = f2bf(wn);
    else
        ((float *)(blob + kOffB1))[p - kPB1] = wn;
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
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(parts), dim3(256), 0, s, data, n_rows, idx, k0, k1, step, batch, t.blob,
                       t.partial, t.loss_partial);
    hipLaunchKernelGGL(mlp_update_kernel, dim3((kMlpParams * kUpdSplit + 255) / 256), dim3(256), 0, s, t.partial,
                       parts, t.loss_partial, t.master, t.m, t.v, t.grad, t.loss, t.blob, lr, bc1, bc2, apply);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *x, int64_t n, const unsigned char *blob, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + kFwdBlock - 1) / kFwdBlock)), dim3(kFwdBlock), 0, s, x,
                       n, blob, out);
    return hipGetLastError();
}

}  // namespace vct
