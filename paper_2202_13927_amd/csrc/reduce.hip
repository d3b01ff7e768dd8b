// reduce.hip -- population reduction of the per-patient metric records (Sec. III-C).
//
// Pass 1 (grid of at most 1024 blocks, fixed for a given n so sums are reproducible):
// every thread strides over patients, accumulates integer totals and FP64 sums, tracks
// the lexicographic minimum (min G, patient) and adds the patient's in-range count to a
// histogram with integer atomics (exact, order-free); each block reduces its threads in
// a fixed tree and writes one partial. Pass 2 (one block) combines the partials in a
// fixed tree and finds the nearest-rank quantiles by a prefix sum over the histogram.
// Memory-bound: 64 B per patient read once.
#include "internal.hpp"

namespace vct {

struct Partial {
    uint64_t bins[5];
    uint64_t events[3];
    uint64_t st[3];
    double sum_g, sum_u;
    double min_v;
    int64_t min_i;
    int32_t min_k;
    int32_t pad;
};

__device__ __forceinline__ bool lex_less(double v1, int64_t i1, double v2, int64_t i2)
{
    return v1 < v2 || (v1 == v2 && i1 < i2);
}

__device__ __forceinline__ void combine(Partial &a, const Partial &b)
{
#pragma unroll
    for (int q = 0; q < 5; ++q) a.bins[q] += b.bins[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a.events[q] += b.events[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a.st[q] += b.st[q];
    a.sum_g += b.sum_g;
    a.sum_u += b.sum_u;
    if (lex_less(b.min_v, b.min_i, a.min_v, a.min_i)) {
        a.min_v = b.min_v;
        a.min_i = b.min_i;
        a.min_k = b.min_k;
    }
}

__device__ __forceinline__ void clear(Partial &a)
{
    for (int q = 0; q < 5; ++q) a.bins[q] = 0;
    for (int q = 0; q < 3; ++q) a.events[q] = 0;
    for (int q = 0; q < 3; ++q) a.st[q] = 0;
    a.sum_g = 0.0;
    a.sum_u = 0.0;
    a.min_v = INFINITY;
    a.min_i = INT64_MAX;
    a.min_k = -1;
    a.pad = 0;
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void reduce_partial_kernel(const double *sum_g, const double *min_g,
                                                             const double *sum_u, const int32_t *bins,
                                                             const int32_t *events, const int32_t *argmin_k,
                                                             const uint32_t *status, int64_t n, int64_t K,
                                                             uint32_t *hist, Partial *partials)
{
    __shared__ Partial sh[256];
    Partial acc;
    clear(acc);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int q = 0; q < 5; ++q) acc.bins[q] += (uint64_t)bins[q * n + i];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc.events[q] += (uint64_t)events[q * n + i];
        const uint32_t s = status[i];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc.st[q] += (s >> q) & 1u;
        acc.sum_g += sum_g[i];
        acc.sum_u += sum_u[i];
        const double m = min_g[i];
        if (m < INFINITY && lex_less(m, i, acc.min_v, acc.min_i)) {
            acc.min_v = m;
            acc.min_i = i;
            acc.min_k = argmin_k[i];
        }
        int64_t b = bins[2 * n + i];
        b = b < 0 ? 0 : (b > K ? K : b);
        atomicAdd(&hist[b], 1u);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            combine(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partials[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(1024) void reduce_final_kernel(const Partial *partials, int nparts,
                                                            const uint32_t *hist, int64_t n, int64_t K,
                                                            ReduceOut *out)
{
    __shared__ Partial sh[256];
    __shared__ uint64_t chunk_sum[1024];
    __shared__ int64_t qres[5];
    const int t = threadIdx.x;
    // combine partials: 256 lanes each fold a fixed subset, then a fixed tree
    if (t < 256) {
        Partial acc;
        clear(acc);
        for (int q = t; q < nparts; q += 256)
            combine(acc, partials[q]);
        sh[t] = acc;
    }
    if (t < 5)
        qres[t] = K;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            combine(sh[t], sh[t + w]);
        __syncthreads();
    }
    // nearest-rank quantiles: smallest c with #{count <= c} >= ceil(pct n / 100)
    const int64_t nb = K + 1;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = (int64_t)t * per, hi = lo + per < nb ? lo + per : nb;
    uint64_t s = 0;
    for (int64_t c = lo; c < hi; ++c) s += hist[c];
    chunk_sum[t] = s;
    __syncthreads();
    if (t == 0) {   // exclusive scan of 1024 chunk sums, fixed order
        uint64_t run = 0;
        for (int q = 0; q < 1024; ++q) {
            const uint64_t v = chunk_sum[q];
            chunk_sum[q] = run;
            run += v;
        }
    }
    __syncthreads();
    const int64_t pct[5] = {5, 25, 50, 75, 95};
    uint64_t run = chunk_sum[t];
    for (int64_t c = lo; c < hi; ++c) {
        const uint64_t nxt = run + hist[c];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const uint64_t rank = (uint64_t)((pct[q] * n + 99) / 100);
            if (run < rank && nxt >= rank)
                qres[q] = c;
        }
        run = nxt;
    }
    __syncthreads();
    if (t == 0) {
        const Partial &r = sh[0];
        for (int q = 0; q < 5; ++q) out->bins[q] = r.bins[q];
        for (int q = 0; q < 3; ++q) out->events[q] = r.events[q];
        for (int q = 0; q < 5; ++q) out->q_count[q] = qres[q];
        out->sum_g = r.sum_g;
        out->sum_u = r.sum_u;
        out->worst_min_g = r.min_v;
        out->worst_patient = r.min_i == INT64_MAX ? -1 : r.min_i;
        out->worst_k = r.min_k;
        out->pad = 0;
        for (int q = 0; q < 3; ++q) out->status_count[q] = (int64_t)r.st[q];
    }
}

static int partial_blocks(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t reduce_workspace_bytes(int64_t n, int64_t K)
{
    return align256((size_t)(K + 1) * sizeof(uint32_t)) + align256((size_t)partial_blocks(n) * sizeof(Partial));
}

hipError_t launch_reduce(const double *sum_g, const double *min_g, const double *sum_u, const int32_t *bins,
                         const int32_t *events, const int32_t *argmin_k, const uint32_t *status, int64_t n,
                         int64_t K, void *workspace, ReduceOut *dev_out, hipStream_t s)
{
    uint32_t *hist = (uint32_t *)workspace;
    Partial *parts = (Partial *)((char *)workspace + align256((size_t)(K + 1) * sizeof(uint32_t)));
    const int nb = partial_blocks(n);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(256), dim3(256), 0, s, hist, K + 1);
    hipLaunchKernelGGL(reduce_partial_kernel, dim3(nb), dim3(256), 0, s, sum_g, min_g, sum_u, bins, events,
                       argmin_k, status, n, K, hist, parts);
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(1024), 0, s, parts, nb, hist, n, K, dev_out);
    return hipGetLastError();
}

}  // namespace vct
