// reduce.hip -- population reduction of the per-patient metric records (Sec. III-C).
//
// The indicators of a trial are per-patient records written once at the end of each
// simulation; the population summary combines them. Four launches on the caller's stream:
//
//  clear   zero the two in-range-count histograms (all patients, unflagged patients).
//  pass 1  (<= 1024 blocks of 4 waves, the grid fixed for a given n so every FP64 sum is
//          reproducible): each lane strides over patients and accumulates integer totals,
//          FP64 sums and the lexicographic minimum (min G, patient); it adds the patient's
//          in-range count to the histograms with 32-bit atomics (exact, order-free). The
//          lanes of a wave are combined by a butterfly of lane exchanges (every lane ends
//          with the same value: IEEE addition is commutative), the 4 wave results in a
//          fixed order; one partial per block.
//  pass 2  per histogram chunk of 1024 bins, one block: the chunk's count (wave butterfly,
//          then the 4 waves in order).
//  pass 3  one block of 4 waves: the partials (each lane folds every 256th in order) by
//          wave butterflies and a fixed fold of the 4 wave results; the nearest-rank quantiles (smallest c with #{count <= c} >=
//          ceil(p n / 100)) by a wave prefix scan over the chunk counts that finds each
//          rank's chunk, then per rank one wave: lane l sums bins 16l..16l+15 of the chunk,
//          a wave prefix scan over the lane sums, and the lane holding the rank walks its 16.
//
// Memory-bound: 64 B per patient read once; the histograms (2 x 4 (K + 1) B) stay in L2.
#include "internal.hpp"

namespace vct {

constexpr int kChunk = 1024;        // histogram bins per chunk (pass 2)
constexpr int kMaxParts = 1024;     // pass-1 blocks

struct Partial {
    uint64_t bins[5];
    uint64_t bins_c[5];   // unflagged patients (status == 0)
    uint64_t events[3];
    uint64_t st[3];
    uint64_t n_c;
    double sum_g, sum_u, sum_g_c;
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
    for (int q = 0; q < 5; ++q) a.bins_c[q] += b.bins_c[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a.events[q] += b.events[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a.st[q] += b.st[q];
    a.n_c += b.n_c;
    a.sum_g += b.sum_g;
    a.sum_u += b.sum_u;
    a.sum_g_c += b.sum_g_c;
    if (lex_less(b.min_v, b.min_i, a.min_v, a.min_i)) {
        a.min_v = b.min_v;
        a.min_i = b.min_i;
        a.min_k = b.min_k;
    }
}

__device__ __forceinline__ void clear(Partial &a)
{
#pragma unroll
    for (int q = 0; q < 5; ++q) a.bins[q] = a.bins_c[q] = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) a.events[q] = a.st[q] = 0;
    a.n_c = 0;
    a.sum_g = a.sum_u = a.sum_g_c = 0.0;
    a.min_v = INFINITY;
    a.min_i = INT64_MAX;
    a.min_k = -1;
    a.pad = 0;
}

template <class T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Butterfly over the 64 lanes, one field at a time: afterwards every lane holds the wave's
// combination.
__device__ __forceinline__ void wave_combine(Partial &a)
{
#pragma unroll
    for (int q = 0; q < 5; ++q) a.bins[q] = wave_sum(a.bins[q]);
#pragma unroll
    for (int q = 0; q < 5; ++q) a.bins_c[q] = wave_sum(a.bins_c[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) a.events[q] = wave_sum(a.events[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) a.st[q] = wave_sum(a.st[q]);
    a.n_c = wave_sum(a.n_c);
    a.sum_g = wave_sum(a.sum_g);
    a.sum_u = wave_sum(a.sum_u);
    a.sum_g_c = wave_sum(a.sum_g_c);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double v = __shfl_xor(a.min_v, off);
        const int64_t i = __shfl_xor(a.min_i, off);
        const int32_t k = __shfl_xor(a.min_k, off);
        if (lex_less(v, i, a.min_v, a.min_i)) {
            a.min_v = v;
            a.min_i = i;
            a.min_k = k;
        }
    }
}

// Inclusive prefix sum over the lanes (Hillis-Steele).
__device__ __forceinline__ uint64_t wave_scan(uint64_t v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void reduce_partial_kernel(const double *sum_g, const double *min_g,
                                                             const double *sum_u, const int32_t *bins,
                                                             const int32_t *events, const int32_t *argmin_k,
                                                             const uint32_t *status, int64_t n, int64_t K,
                                                             uint32_t *hist, uint32_t *hist_c, Partial *partials)
{
    __shared__ Partial sh[4];
    Partial acc;
    clear(acc);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
#pragma unroll 1
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t s = status[i];
        const bool clean = s == 0u;
        int32_t bv[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            bv[q] = bins[q * n + i];
            acc.bins[q] += (uint64_t)bv[q];
            acc.bins_c[q] += clean ? (uint64_t)bv[q] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) acc.events[q] += (uint64_t)events[q * n + i];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc.st[q] += (s >> q) & 1u;
        const double g = sum_g[i];
        acc.n_c += clean ? 1u : 0u;
        acc.sum_g += g;
        acc.sum_g_c += clean ? g : 0.0;
        acc.sum_u += sum_u[i];
        const double m = min_g[i];
        if (m < INFINITY && lex_less(m, i, acc.min_v, acc.min_i)) {
            acc.min_v = m;
            acc.min_i = i;
            acc.min_k = argmin_k[i];
        }
        int64_t b = bv[2];
        b = b < 0 ? 0 : (b > K ? K : b);
        atomicAdd(&hist[b], 1u);
        if (clean)
            atomicAdd(&hist_c[b], 1u);
    }
    wave_combine(acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial r = sh[0];
        for (int q = 1; q < 4; ++q) combine(r, sh[q]);
        partials[blockIdx.x] = r;
    }
}

// Chunk counts: block (c, h) sums bins [c kChunk, (c + 1) kChunk) of histogram h (the
// histograms are zero-padded to a whole number of chunks).
__global__ __launch_bounds__(256) void hist_chunk_kernel(const uint32_t *hist, int64_t hstride, uint64_t *chunk,
                                                         int64_t n_chunks)
{
    __shared__ uint64_t sh[4];
    const uint32_t *h = hist + blockIdx.y * hstride + (int64_t)blockIdx.x * kChunk;
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kChunk / 256; ++j) s += h[threadIdx.x + 256 * j];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        chunk[blockIdx.y * n_chunks + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(256) void reduce_final_kernel(const Partial *partials, int nparts, const uint32_t *hist,
                                                           int64_t hstride, const uint64_t *chunk, int64_t n_chunks,
                                                           int64_t n, int64_t K, ReduceOut *out)
{
    __shared__ Partial sh[4];
    __shared__ uint64_t rank[10];        // 5 quantiles of all patients, then 5 of the unflagged
    __shared__ int64_t rank_chunk[10];   // chunk holding the rank
    __shared__ uint64_t rank_before[10]; // patients in the chunks before it
    __shared__ int64_t qres[10];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;

    // lane t folds partials t, t + 256, ... in order; then the wave butterflies and the
    // 4 wave results in order
    Partial acc;
    clear(acc);
    for (int q = t; q < nparts; q += 256)
        combine(acc, partials[q]);
    wave_combine(acc);
    if (lane == 0)
        sh[w] = acc;
    __syncthreads();
    if (t == 0) {
        for (int q = 1; q < 4; ++q) combine(sh[0], sh[q]);
        const int64_t pct[5] = {5, 25, 50, 75, 95};
        const int64_t nn[2] = {n, (int64_t)sh[0].n_c};
        for (int h = 0; h < 2; ++h)
            for (int q = 0; q < 5; ++q) {
                rank[5 * h + q] = (uint64_t)((pct[q] * nn[h] + 99) / 100);
                rank_chunk[5 * h + q] = -1;
                rank_before[5 * h + q] = 0;
                qres[5 * h + q] = 0;
            }
    }
    __syncthreads();

    // Wave h (0, 1) finds each rank's chunk in histogram h: the first chunk whose inclusive
    // running count reaches the rank.
    if (w < 2) {
        const uint64_t *cs = chunk + w * n_chunks;
        uint64_t base = 0;
        for (int64_t c0 = 0; c0 < n_chunks; c0 += 64) {
            const int64_t c = c0 + lane;
            const uint64_t v = c < n_chunks ? cs[c] : 0ull;
            const uint64_t incl = base + wave_scan(v, lane);
            const uint64_t excl = incl - v;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const uint64_t r = rank[5 * w + q];
                if (r > 0 && c < n_chunks && excl < r && incl >= r) {
                    rank_chunk[5 * w + q] = c;
                    rank_before[5 * w + q] = excl;
                }
            }
            base = __shfl(incl, 63);
        }
    }
    __syncthreads();

    // Wave w resolves ranks w, w + 4, w + 8 inside their chunks.
    for (int j = w; j < 10; j += 4) {
        if (rank_chunk[j] < 0)
            continue;
        const int h = j / 5;
        const uint4 *bp4 = (const uint4 *)(hist + h * hstride + rank_chunk[j] * kChunk + 16 * lane);
        uint32_t v[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 x = bp4[q];
            v[4 * q] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
        uint64_t s = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += v[q];
        const uint64_t incl = rank_before[j] + wave_scan(s, lane);
        uint64_t run = incl - s;
        const uint64_t r = rank[j];
        if (run < r && incl >= r) {
            int64_t c = rank_chunk[j] * kChunk + 16 * lane;
            for (int q = 0; q < 16; ++q) {
                run += v[q];
                if (run >= r) {
                    c += q;
                    break;
                }
            }
            qres[j] = c;
        }
    }
    __syncthreads();

    if (t == 0) {
        const Partial &r = sh[0];
        for (int q = 0; q < 5; ++q) out->bins[q] = r.bins[q];
        for (int q = 0; q < 5; ++q) out->bins_clean[q] = r.bins_c[q];
        for (int q = 0; q < 3; ++q) out->events[q] = r.events[q];
        for (int q = 0; q < 5; ++q) out->q_count[q] = qres[q];
        for (int q = 0; q < 5; ++q) out->q_count_clean[q] = qres[5 + q];
        out->n_clean = (int64_t)r.n_c;
        out->sum_g = r.sum_g;
        out->sum_g_clean = r.sum_g_c;
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
    return (int)(b < 1 ? 1 : (b > kMaxParts ? kMaxParts : b));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Histogram row length: K + 1 bins rounded up to whole chunks.
static int64_t hist_stride(int64_t K) { return (K + 1 + kChunk - 1) / kChunk * kChunk; }

size_t reduce_workspace_bytes(int64_t n, int64_t K)
{
    const int64_t hs = hist_stride(K);
    return align256((size_t)(2 * hs) * sizeof(uint32_t)) + align256((size_t)(2 * (hs / kChunk)) * sizeof(uint64_t)) +
           align256((size_t)partial_blocks(n) * sizeof(Partial)) + align256(sizeof(ReduceOut));
}

hipError_t launch_reduce(const double *sum_g, const double *min_g, const double *sum_u, const int32_t *bins,
                         const int32_t *events, const int32_t *argmin_k, const uint32_t *status, int64_t n,
                         int64_t K, void *workspace, ReduceOut **dev_out, hipStream_t s)
{
    const int64_t hs = hist_stride(K), n_chunks = hs / kChunk;
    char *p = (char *)workspace;
    uint32_t *hist = (uint32_t *)p;
    p += align256((size_t)(2 * hs) * sizeof(uint32_t));
    uint64_t *chunk = (uint64_t *)p;
    p += align256((size_t)(2 * n_chunks) * sizeof(uint64_t));
    Partial *parts = (Partial *)p;
    const int nb = partial_blocks(n);
    p += align256((size_t)nb * sizeof(Partial));
    *dev_out = (ReduceOut *)p;
    const int64_t fill_blocks = (2 * hs + 255) / 256;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)(fill_blocks < 1024 ? fill_blocks : 1024)), dim3(256), 0, s,
                       hist, 2 * hs);
    hipLaunchKernelGGL(reduce_partial_kernel, dim3(nb), dim3(256), 0, s, sum_g, min_g, sum_u, bins, events,
                       argmin_k, status, n, K, hist, hist + hs, parts);
    hipLaunchKernelGGL(hist_chunk_kernel, dim3((unsigned)n_chunks, 2), dim3(256), 0, s, hist, hs, chunk, n_chunks);
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, s, parts, nb, hist, hs, chunk, n_chunks, n, K,
                       *dev_out);
    return hipGetLastError();
}

}  // namespace vct
