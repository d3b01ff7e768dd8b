// mlp.hip -- training of the learned controller (behaviour cloning of the MPC) on BF16 MFMA.
//
// One training step over a minibatch of B rows (B a multiple of 64):
//  1. mlp_grad_kernel: one wave per 64 rows draws its rows (Philox, with replacement, or an
//     explicit index list), normalises the 12 raw features, runs the forward pass, and
//     back-propagates the mean squared error sum (o - t)^2 / B through the three hidden
//     layers with MFMA GEMMs (activations and their gradients in BF16, accumulation FP32),
//     writing its partial gradient (all parameters) and partial loss;
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
// dW[u][v] = sum_s dH[s][u] Hin[s][v]  (64 x NV, K = 64 samples), written to g (row stride NV);
// db[u] = sum_s dH[s][u]; dHin[s][v] = (sum_u dH[s][u] W[u][v]) [Hin[s][v] > 0] (if dHin).
template <int NV>
__device__ __forceinline__ void backprop_layer(const uint16_t *dH, const uint16_t *Hin, const uint16_t *W, float *gW,
                                               float *gb, uint16_t *dHin, int lane)
{
    // weight gradient
#pragma unroll
    for (int ut = 0; ut < 4; ++ut)
#pragma unroll
        for (int vt = 0; vt < NV / 16; ++vt) {
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int sb = 0; sb < 4; ++sb)
                acc = mfma16(frag_cols(dH, kMlpH, 16 * sb, 16 * ut, lane), frag_cols(Hin, NV, 16 * sb, 16 * vt, lane),
                             acc);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                gW[(16 * ut + 4 * (lane >> 4) + e) * NV + 16 * vt + (lane & 15)] = acc[e];
        }
    // bias gradient: lane u
    {
        float acc = 0.f;
        for (int s = 0; s < 64; ++s)
            acc += bf2f(dH[s * kMlpH + lane]);
        gb[lane] = acc;
    }
    if (!dHin)
        return;
    // gradient of the layer input (through the previous ReLU)
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int vt = 0; vt < NV / 16; ++vt) {
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ub = 0; ub < 4; ++ub)
                acc = mfma16(frag_rows(dH, kMlpH, 16 * st, 16 * ub, lane), frag_cols(W, NV, 16 * ub, 16 * vt, lane),
                             acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s = 16 * st + 4 * (lane >> 4) + e, v = 16 * vt + (lane & 15);
                dHin[s * NV + v] = bf2f(Hin[s * NV + v]) > 0.f ? f2bf(acc[e]) : (uint16_t)0;
            }
        }
}

__global__ __launch_bounds__(64) void mlp_grad_kernel(const float *__restrict__ data, int64_t n_rows,
                                                      const int32_t *__restrict__ idx, uint32_t k0, uint32_t k1,
                                                      int32_t step, int32_t batch,
                                                      const unsigned char *__restrict__ blob,
                                                      float *__restrict__ partial, float *__restrict__ loss_partial)
{
    __shared__ __align__(16) unsigned char net[kMlpNetBytes];
    __shared__ __align__(16) uint16_t xs[64 * kMlpInP];
    __shared__ __align__(16) uint16_t h1[64 * kMlpH], h2[64 * kMlpH], h3[64 * kMlpH], da[64 * kMlpH],
        db[64 * kMlpH];
    __shared__ float o[64], dout[64];
    const int lane = threadIdx.x;
    for (int i = lane; i < kMlpNetBytes / 16; i += 64)
        ((uint4 *)net)[i] = ((const uint4 *)blob)[i];

    const int64_t gi = (int64_t)blockIdx.x * 64 + lane;
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
    for (int f = 0; f < kMlpInP; ++f)
        xs[lane * kMlpInP + f] = f < kMlpIn ? f2bf((data[row * kRow + f] - mean[f]) * istd[f]) : (uint16_t)0;
    const float target = valid ? data[row * kRow + kMlpIn] : NAN;
    __syncthreads();

    const MlpNet n = mlp_net(net);
    mlp_forward<DenseLayout>(n, xs, h1, h2, h3, o, lane, wave_sync);

    float *g = partial + (int64_t)blockIdx.x * kMlpParams;
    const float r = o[lane] - target;
    dout[lane] = 2.f * r / (float)batch;
    // partial loss: sum over the 64 rows of r^2 / B (fixed tree through LDS)
    o[lane] = r * r / (float)batch;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (lane < w)
            o[lane] += o[lane + w];
        __syncthreads();
    }
    if (lane == 0)
        loss_partial[blockIdx.x] = o[0];

    // output layer: lane u
    {
        const float w4u = bf2f(n.W4[lane]);
        float acc = 0.f;
        for (int s = 0; s < 64; ++s) {
            const float hv = bf2f(h3[s * kMlpH + lane]);
            acc += dout[s] * hv;
            da[s * kMlpH + lane] = hv > 0.f ? f2bf(dout[s] * w4u) : (uint16_t)0;
        }
        g[kPW4 + lane] = acc;
        for (int q = 1; q < kMlpOutP; ++q)
            g[kPW4 + q * kMlpH + lane] = 0.f;
        if (lane < kMlpOutP) {
            float sb = 0.f;
            if (lane == 0)
                for (int s = 0; s < 64; ++s)
                    sb += dout[s];
            g[kPB4 + lane] = sb;
        }
    }
    __syncthreads();
    backprop_layer<kMlpH>(da, h2, n.W3, g + kPW3, g + kPB3, db, lane);
    __syncthreads();
    backprop_layer<kMlpH>(db, h1, n.W2, g + kPW2, g + kPB2, da, lane);
    __syncthreads();
    backprop_layer<kMlpInP>(da, xs, n.W1, g + kPW1, g + kPB1, nullptr, lane);
}

// ------------------------------------------------------------------ update ----
__global__ void mlp_update_kernel(const float *__restrict__ partial, int n_parts, const float *__restrict__ loss_partial,
                                  float *master, float *m, float *v, float *grad, float *loss, unsigned char *blob,
                                  float lr, float bc1, float bc2, int apply)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    // sequential sums (fixed order); unrolled so that the loads are issued ahead of the adds
    if (p == 0) {
        float l = 0.f;
#pragma unroll 16
        for (int b = 0; b < n_parts; ++b)
            l += loss_partial[b];
        *loss = l;
    }
    if (p >= kMlpParams)
        return;
    float gs = 0.f;
#pragma unroll 16
    for (int b = 0; b < n_parts; ++b)
        gs += partial[(int64_t)b * kMlpParams + p];
    if (padded_param(p))
        gs = 0.f;
    grad[p] = gs;
    if (!apply || padded_param(p))
        return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.f - b1) * gs;
    const float vv = b2 * v[p] + (1.f - b2) * gs * gs;
    m[p] = mm;
    v[p] = vv;
    const float w = master[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    master[p] = w;
    if (p < kPB1)
        ((uint16_t *)blob)[p] = f2bf(w);
    else
        ((float *)(blob + kOffB1))[p - kPB1] = w;
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
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(parts), dim3(64), 0, s, data, n_rows, idx, k0, k1, step, batch, t.blob,
                       t.partial, t.loss_partial);
    hipLaunchKernelGGL(mlp_update_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, t.partial, parts,
                       t.loss_partial, t.master, t.m, t.v, t.grad, t.loss, t.blob, lr, bc1, bc2, apply);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *x, int64_t n, const unsigned char *blob, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + kFwdBlock - 1) / kFwdBlock)), dim3(kFwdBlock), 0, s, x,
                       n, blob, out);
    return hipGetLastError();
}

}  // namespace vct
