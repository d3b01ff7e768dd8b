// kernels.hip -- population and closed-loop simulation kernels (gfx950 / CDNA4).
//
// One patient per lane, the whole horizon in one launch: the 11 states, ~25 derived
// constants, the controller state and the metric accumulators stay in VGPRs; a patient
// reads its 19 FP64 parameters once (coalesced SoA) and writes its 64-byte metric
// record once. Noise is drawn in the loop from Philox counters, never stored.
#include <algorithm>

#include "internal.hpp"
#include "mlp.hpp"
#include "model.hpp"
#include "mpc.hpp"
#include "rng.hpp"

namespace vct {

// ---------------------------------------------------------------- population ----
// Lognormal draws with median = nominal: p_j = nom_j exp(s z_j), z_j normal j of the
// Philox blocks (j/4, patient, PARAM, attempt). Kept iff the basal steady state at G*
// exists (Sec. IV-B keeps only parameter sets with a valid basal rate).
__device__ __forceinline__ bool basal_rate(const double *p, double g, double &I, double &ub)
{
    const double bw = p[kBW];
    const double egp0 = p[kEGP0] * bw, f01 = p[kF01] * bw, vg = p[kVG] * bw, vi = p[kVI] * bw;
    const double q1 = g * vg;
    const double f01c = f01 * fmin(1.0, g / 4.5);
    const double fr = g > 9.0 ? 0.003 * (g - 9.0) * vg : 0.0;
    // dQ1 = dQ2 = 0 with x_j = S_j I, multiplied by (k12 + SID I): a I^2 + b I + c = 0
    const double a = p[kSID] * (p[kSIT] * q1 + egp0 * p[kSIE]);
    const double b = p[kSID] * (f01c + fr - egp0) + egp0 * p[kSIE] * p[kK12];
    const double c = p[kK12] * (f01c + fr - egp0);
    if (!(c < 0.0) || !(a > 0.0))
        return false;
    const double sq = sqrt(b * b - 4.0 * a * c);
    // the positive root, in the form without cancellation
    I = b >= 0.0 ? (2.0 * c) / (-b - sq) : (-b + sq) / (2.0 * a);
    ub = I * p[kKe] * vi;
    return true;
}

__global__ __launch_bounds__(256) void population_kernel(const PopArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n)
        return;
    const uint32_t pid = (uint32_t)(a.patient_base + j);
    double p[15];
    double I = 0.0, ub = 0.0;
    uint32_t status = 0;
    int attempt = 0;
    for (; attempt < 32; ++attempt) {
        double z[16];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const U4 r = philox4x32_10((uint32_t)c, pid, kTagParam, (uint32_t)attempt, a.key0, a.key1);
            box_muller_f64(uniform_f64(r.x), uniform_f64(r.y), z[4 * c], z[4 * c + 1]);
            box_muller_f64(uniform_f64(r.z), uniform_f64(r.w), z[4 * c + 2], z[4 * c + 3]);
        }
#pragma unroll
        for (int q = 0; q < 15; ++q)
            p[q] = a.nominal[q] * exp(a.s * z[q]);
        if (basal_rate(p, a.g_target, I, ub) && (!(a.flags & 1u) || ub >= 400.0 / 60.0))
            break;
    }
    if (attempt == 32) {
#pragma unroll
        for (int q = 0; q < 15; ++q)
            p[q] = a.nominal[q];
        if (!basal_rate(p, a.g_target, I, ub)) {
            I = 0.0;
            ub = 0.0;
        }
        status |= kStResample;
    }
    double *out = a.params;
#pragma unroll
    for (int q = 0; q < 15; ++q)
        out[(int64_t)q * a.n + j] = p[q];
    out[(int64_t)kUb * a.n + j] = ub;
    out[(int64_t)kIstar * a.n + j] = I;
    out[(int64_t)kAttempts * a.n + j] = (double)(attempt < 32 ? attempt + 1 : 32);
    out[(int64_t)kStatus * a.n + j] = (double)status;
}

hipError_t launch_population(const PopArgs &a, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.n + 255) / 256);
    hipLaunchKernelGGL(population_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- simulation ----
// Controller codes of the kernels: those of vct.h (open loop, PID, MPC, learned, dual-hormone),
// and the PID and open loop on the extended model (glucagon and exercise states).
enum { kCtrlOpen = 0, kCtrlPid = 1, kCtrlMpc = 2, kCtrlMlp = 3, kCtrlDual = 4, kCtrlPidExt = 5, kCtrlOpenExt = 6 };
template <int CTRL> constexpr bool ctrl_ext() { return CTRL >= kCtrlDual; }
template <int CTRL> constexpr int ctrl_base()
{
    return CTRL == kCtrlPidExt ? kCtrlPid : (CTRL == kCtrlOpenExt ? kCtrlOpen : CTRL);
}
enum { kOutTraj = 1, kOutRecord = 2, kOutPop = 4 };   // optional per-sample outputs (template bits)

// Population BG as a function of time (Sec. III-C: mean, minimum and maximum BG over the
// patients at every sample): each wave reduces its live lanes' G(t_k) -- the sum of
// round(G 2^32) as a 64-bit integer (exact, so the total does not depend on the order of
// the atomics) and order-preserving keys of the FP64 value for min and max -- and one lane
// adds them with three 64-bit atomics. All 64 lanes of the wave must be active.
__device__ __forceinline__ unsigned long long order_key(double g)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(g);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
// The same order on FP32 values (a float and its FP64 conversion have the same rank).
__device__ __forceinline__ uint32_t order_key32(float g)
{
    const uint32_t b = __float_as_uint(g);
    return (b >> 31) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float order_key32_inv(uint32_t key)
{
    return __uint_as_float((key >> 31) ? (key & 0x7FFFFFFFu) : ~key);
}

// Wave reductions without LDS: two quad exchanges, the half-row and the row mirror leave
// every lane of a 16-lane row with the row's result (DPP moves, all source lanes inside the
// row); the four rows are read into scalar registers and combined there. All 64 lanes must
// be active. The result is the same on every lane.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v)
{
    const uint32_t lo = dpp32<CTRL>((uint32_t)v), hi = dpp32<CTRL>((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t rows32(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ unsigned long long rows64(unsigned long long v, int l)
{
    return ((unsigned long long)rows32((uint32_t)(v >> 32), l) << 32) | rows32((uint32_t)v, l);
}
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T x, Op op)
{
    if constexpr (sizeof(T) == 4) {
        x = op(x, dpp32<0xB1>(x));    // quad_perm [1,0,3,2]
        x = op(x, dpp32<0x4E>(x));    // quad_perm [2,3,0,1]
        x = op(x, dpp32<0x141>(x));   // row_half_mirror
        x = op(x, dpp32<0x140>(x));   // row_mirror
        return op(op(rows32(x, 0), rows32(x, 16)), op(rows32(x, 32), rows32(x, 48)));
    } else {
        x = op(x, dpp64<0xB1>(x));
        x = op(x, dpp64<0x4E>(x));
        x = op(x, dpp64<0x141>(x));
        x = op(x, dpp64<0x140>(x));
        return op(op(rows64(x, 0), rows64(x, 16)), op(rows64(x, 32), rows64(x, 48)));
    }
}

template <typename R>
__device__ __forceinline__ void pop_accumulate(const SimArgs &a, int32_t k, R G, bool live)
{
    using u64 = unsigned long long;
    const double g = (double)G;
    // a patient whose state is no longer finite (its status bit is set) leaves the sum and
    // the extremes; the count of such patients per sample is kept beside them
    const bool fin = live && __builtin_isfinite(g);
    const u64 nonfin = __ballot(live && !fin);
    const u64 q = fin ? (u64)__double2ll_rn(g * 4294967296.0) : 0ull;
    const u64 sum = wave_reduce(q, [](u64 x, u64 y) { return x + y; });
    u64 mn, mx;
    if constexpr (sizeof(R) == 4) {   // FP32 keys; the extremes converted once
        const uint32_t key = order_key32(G);
        const uint32_t kmn = wave_reduce(fin ? key : ~0u, [](uint32_t x, uint32_t y) { return x < y ? x : y; });
        const uint32_t kmx = wave_reduce(fin ? key : 0u, [](uint32_t x, uint32_t y) { return x > y ? x : y; });
        mn = kmn == ~0u ? ~0ull : order_key((double)order_key32_inv(kmn));
        mx = kmx == 0u ? 0ull : order_key((double)order_key32_inv(kmx));
    } else {
        const u64 key = order_key(g);
        mn = wave_reduce(fin ? key : ~0ull, [](u64 x, u64 y) { return x < y ? x : y; });
        mx = wave_reduce(fin ? key : 0ull, [](u64 x, u64 y) { return x > y ? x : y; });
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((u64 *)&a.pop_sum[k], sum);
        atomicMin((u64 *)&a.pop_min[k], mn);
        atomicMax((u64 *)&a.pop_max[k], mx);
        if (nonfin)
            atomicAdd((u64 *)&a.pop_nonfinite[k], (u64)__popcll(nonfin));
    }
}

// The pooled BG distribution (every patient and sample): bins of 0.1 mmol/L, bin 0 below
// 0 (and NaN), bin 1 + floor(10 G) for 0 <= G < 40, bin 401 at or above 40. Counted per wave
// in LDS, added to the 64-bit global bins when the wave ends.
constexpr int kPopBins = 402;

__device__ __forceinline__ int pop_bin(double g)
{
    return g >= 0.0 ? 1 + (int)fmin(g * 10.0, 400.5) : 0;
}

// Zeroes (start) or flushes (end) a wave's LDS bins; all lanes of the wave take part.
__device__ __forceinline__ void pop_hist_clear(uint32_t *h, int lane)
{
    for (int b = lane; b < kPopBins; b += 64)
        h[b] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ void pop_hist_flush(const SimArgs &a, uint32_t *h, int lane)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int b = lane; b < kPopBins; b += 64) {
        const uint32_t c = h[b];
        if (c)
            atomicAdd((unsigned long long *)&a.pop_hist[b], (unsigned long long)c);
    }
}

// The span of the patients' own BG distributions (Fig. 3's shaded area): each lane counts its
// patient's samples in bins of 0.5 mmol/L (bin floor(2 G), clamped to 0..49) in LDS laid out
// [bin][lane]; at the patient's end the cumulative counts (samples with G below
// (b + 1) / 2, all samples in the last bin) are reduced over the wave's live lanes to their
// minimum and maximum and added with 64-bit atomics. All lanes of the wave take part.
constexpr int kSpanBins = 50;

__device__ __forceinline__ int span_bin(double g)
{
    return g >= 0.0 ? (int)fmin(g * 2.0, 49.5) : 0;
}

__device__ __forceinline__ void span_flush(const SimArgs &a, uint32_t *cnt, int lane, bool live)
{
    uint32_t cum = 0;
    for (int b = 0; b < kSpanBins; ++b) {
        cum += cnt[b * 64 + lane];
        cnt[b * 64 + lane] = 0u;
        uint32_t mn = live ? cum : ~0u, mx = live ? cum : 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t omn = __shfl_xor(mn, off), omx = __shfl_xor(mx, off);
            mn = omn < mn ? omn : mn;
            mx = omx > mx ? omx : mx;
        }
        if (lane == 0) {
            atomicMin((unsigned long long *)&a.span_min[b], (unsigned long long)mn);
            atomicMax((unsigned long long *)&a.span_max[b], (unsigned long long)mx);
        }
    }
}

__global__ void popbg_init_kernel(int64_t *sum, uint64_t *mn, uint64_t *mx, uint64_t *hist, int64_t *nonfinite,
                                  int64_t K)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        sum[i] = 0;
        mn[i] = ~0ull;
        mx[i] = 0ull;
        nonfinite[i] = 0;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kPopBins; i += (int64_t)gridDim.x * blockDim.x)
        hist[i] = 0ull;
    // then the span: min[kSpanBins], max[kSpanBins]
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kSpanBins; i += (int64_t)gridDim.x * blockDim.x) {
        hist[kPopBins + i] = ~0ull;
        hist[kPopBins + kSpanBins + i] = 0ull;
    }
}

// Meals of one (patient, day) as a queue in time order: sample index within the day and
// the held glucose intake rate (mmol/min) of up to six meals; unused entries have k = -1.
template <typename R> struct DayMeals {
    int32_t k0, k1, k2, k3, k4, k5;
    R r0, r1, r2, r3, r4, r5;
};

// Takes the first meal off the queue and returns its intake rate.
template <typename R>
__device__ __forceinline__ R pop_front(DayMeals<R> &d)
{
    const R r = d.r0;
    d.k0 = d.k1; d.r0 = d.r1;
    d.k1 = d.k2; d.r1 = d.r2;
    d.k2 = d.k3; d.r2 = d.r3;
    d.k3 = d.k4; d.r3 = d.r4;
    d.k4 = d.k5; d.r4 = d.r5;
    d.k5 = -1;
    return r;
}

template <typename R>
__device__ __forceinline__ void push_front(DayMeals<R> &d, int32_t k, R r)
{
    d.k5 = d.k4; d.r5 = d.r4;
    d.k4 = d.k3; d.r4 = d.r3;
    d.k3 = d.k2; d.r3 = d.r2;
    d.k2 = d.k1; d.r2 = d.r1;
    d.k1 = d.k0; d.r1 = d.r0;
    d.k0 = k;
    d.r0 = r;
}

// Onset jitter from a Philox word: floor(u (2J + 1)) - J minutes, u the word's top 24 bits.
__device__ __forceinline__ int32_t meal_jitter(uint32_t x, int32_t J)
{
    return (int32_t)(((uint64_t)((x >> 8) | 1u) * (uint64_t)(2 * J + 1)) >> 24) - J;
}

// Slot protocol: Philox block (day, patient, MEAL, slot) gives carbs = max(0, mean + sd z)
// (cosine normal of u0, u1), the jitter from u2 and presence u3 < prob. The normal is
// drawn in the kernel's precision; jitter and presence are exact integer tests (u3 < prob
// is (2m + 1) < ceil(prob 2^24), precomputed on the host).
template <typename R>
__device__ __forceinline__ void draw_slot_meals(const SimArgs &a, uint32_t pid, int32_t day, DayMeals<R> &d)
{
#pragma unroll
    for (int m = 3; m >= 0; --m) {
        if (m < a.n_slots) {
            const U4 r = philox4x32_10((uint32_t)day, pid, kTagMeal, (uint32_t)m, a.key0, a.key1);
            const uint32_t odd3 = (r.w >> 8) | 1u;
            if (odd3 < a.prob_thresh[m]) {
                R z0, z1;
                Rng<R>::box_muller(Rng<R>::uniform(r.x), Rng<R>::uniform(r.y), z0, z1);
                const R carbs = vmax(R(0), R(a.carbs_mean[m]) + R(a.carbs_sd[m]) * z0);
                push_front(d, (a.minute_of_day[m] + meal_jitter(r.z, a.jitter)) / a.ts_min, carbs * R(a.rate_per_g));
            }
        }
    }
}

// ------------------------------------------------ Northern-European protocol ----
// Sec. II-B, Table I: a year of four 13-week seasons (winter, spring, summer, autumn) made of
// standard, active and vacation weeks; each week of standard days, active days, days with a
// movie night and days with a late night. Table II: meal sizes per kg of body weight.
// Each patient's year is a random arrangement of these compositions: at day d the season's
// 13 week types are shuffled (Fisher-Yates, i = 12..1 swapping slots i and
// floor(u_i (i + 1)), u_i the top 24 bits of word 12 - i of the Philox blocks
// (d / 91, patient, PROTO, 0..2)) from the order standard, active, vacation; the week's 7
// day types likewise (i = 6..1, blocks (d / 7, patient, PROTO, 4..5)) from the order
// standard, active, movie, late. Meals in time order (the figure with the clock times is
// not in the text; these are this implementation's choices): breakfast 07:00 small,
// snack 10:00 in spring and summer, lunch 12:00 medium, snack 15:00 in winter and autumn,
// dinner 18:00 large in winter and autumn and medium in spring and summer, one evening
// snack 21:00 on movie and late nights and a second at 22:30 on late nights. Vacation
// weeks ("they eat more") move breakfast, lunch and dinner one size up (large stays
// large). An active day has an exercise session, which this model has no input for: its
// meals are the standard day's. Meal kind q (0 breakfast, 1 morning snack, 2 lunch,
// 3 afternoon snack, 4 dinner, 5 and 6 evening snacks) draws Philox block (day, patient,
// MEAL, q): carbs = max(0, g BW (1 + meal_cv z)) with z the cosine normal of u0, u1, and
// the onset jitter from u2 as for the slot protocol.
enum : uint32_t { kTagProto = 8u };
constexpr int kDaysPerSeason = 91;
constexpr double kGramsLarge = 1.29, kGramsMedium = 0.86, kGramsSmall = 0.57, kGramsSnack = 0.29;

// Fisher-Yates on n 2-bit entries packed in a word, with 24-bit uniforms from the words w.
template <int N>
__device__ __forceinline__ uint32_t shuffle2(uint32_t arr, const uint32_t *w)
{
#pragma unroll
    for (int i = N - 1; i >= 1; --i) {
        const uint32_t j = (uint32_t)(((uint64_t)(w[N - 1 - i] >> 8) * (uint64_t)(i + 1)) >> 24);
        const uint32_t x = ((arr >> (2 * i)) ^ (arr >> (2 * j))) & 3u;
        arr ^= (x << (2 * i)) | (x << (2 * j));
    }
    return arr;
}

// n entries of value v appended from position p of a packed 2-bit array.
__device__ __forceinline__ uint32_t fill2(uint32_t arr, int &p, int n, uint32_t v)
{
    for (int e = 0; e < n; ++e, ++p)
        arr |= v << (2 * p);
    return arr;
}

// Season (0 winter .. 3 autumn), week type (0 standard, 1 active, 2 vacation) and day type
// (0 standard, 1 active, 2 movie night, 3 late night) of day d of a patient.
__device__ __forceinline__ void nordic_day(const SimArgs &a, uint32_t pid, int32_t d, int &season, int &wtype,
                                           int &dtype)
{
    season = (d / kDaysPerSeason) % 4;
    const int wk = (d % kDaysPerSeason) / 7;
    {   // Table I, top: standard / active / vacation weeks per season
        const int ns = season == 3 ? 9 : season == 2 ? 7 : 6;
        const int na = season == 1 ? 6 : season == 0 ? 4 : 3;
        const int nv = 13 - ns - na;
        int p = 0;
        uint32_t arr = fill2(0u, p, ns, 0u);
        arr = fill2(arr, p, na, 1u);
        arr = fill2(arr, p, nv, 2u);
        uint32_t w[12];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const U4 r = philox4x32_10((uint32_t)(d / kDaysPerSeason), pid, kTagProto, (uint32_t)b, a.key0, a.key1);
            w[4 * b] = r.x; w[4 * b + 1] = r.y; w[4 * b + 2] = r.z; w[4 * b + 3] = r.w;
        }
        wtype = (int)((shuffle2<13>(arr, w) >> (2 * wk)) & 3u);
    }
    {   // Table I, bottom: standard / active / movie / late days per week type
        const int n0 = wtype == 2 ? 5 : wtype == 1 ? 3 : 4;
        const int n1 = wtype == 2 ? 0 : wtype == 1 ? 3 : 1;
        const int n2 = wtype == 2 ? 0 : 1;
        const int n3 = 7 - n0 - n1 - n2;
        int p = 0;
        uint32_t arr = fill2(0u, p, n0, 0u);
        arr = fill2(arr, p, n1, 1u);
        arr = fill2(arr, p, n2, 2u);
        arr = fill2(arr, p, n3, 3u);
        uint32_t w[8];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const U4 r = philox4x32_10((uint32_t)(d / 7), pid, kTagProto, (uint32_t)(4 + b), a.key0, a.key1);
            w[4 * b] = r.x; w[4 * b + 1] = r.y; w[4 * b + 2] = r.z; w[4 * b + 3] = r.w;
        }
        dtype = (int)((shuffle2<7>(arr, w) >> (2 * (d % 7))) & 3u);
    }
}

template <typename R>
__device__ __forceinline__ void draw_nordic_meals(const SimArgs &a, uint32_t pid, int32_t day, R bw,
                                                  DayMeals<R> &d)
{
    int season, wtype, dtype;
    nordic_day(a, pid, day, season, wtype, dtype);
    const bool cold = season == 0 || season == 3, vac = wtype == 2;
    // meal kinds 6..0 pushed to the front (the queue ends in time order)
#pragma unroll
    for (int q = 6; q >= 0; --q) {
        double g;
        int minute;
        bool on;
        switch (q) {
        case 0: g = vac ? kGramsMedium : kGramsSmall; minute = 420; on = true; break;
        case 1: g = kGramsSnack; minute = 600; on = !cold; break;
        case 2: g = vac ? kGramsLarge : kGramsMedium; minute = 720; on = true; break;
        case 3: g = kGramsSnack; minute = 900; on = cold; break;
        case 4: g = (cold || vac) ? kGramsLarge : kGramsMedium; minute = 1080; on = true; break;
        case 5: g = kGramsSnack; minute = 1260; on = dtype >= 2; break;
        default: g = kGramsSnack; minute = 1350; on = dtype == 3; break;
        }
        if (on) {
            const U4 r = philox4x32_10((uint32_t)day, pid, kTagMeal, (uint32_t)q, a.key0, a.key1);
            R z0, z1;
            Rng<R>::box_muller(Rng<R>::uniform(r.x), Rng<R>::uniform(r.y), z0, z1);
            const R carbs = vmax(R(0), R(g) * bw * (R(1) + R(a.meal_cv) * z0));
            push_front(d, (minute + meal_jitter(r.z, a.jitter)) / a.ts_min, carbs * R(a.rate_per_g));
        }
    }
}

template <typename R>
__device__ __forceinline__ DayMeals<R> draw_meals(const SimArgs &a, uint32_t pid, int32_t day, R bw)
{
    DayMeals<R> d{-1, -1, -1, -1, -1, -1, R(0), R(0), R(0), R(0), R(0), R(0)};
    if (a.proto == kProtoNordic)
        draw_nordic_meals<R>(a, pid, day, bw, d);
    else
        draw_slot_meals<R>(a, pid, day, d);
    return d;
}

// Sec. II-B: each active day of the Northern-European protocol has one exercise session, from
// the sampling interval that contains ex_minute + a jitter (word 2 of Philox block (day,
// patient, EXER, 0), as for a meal) for ex_samples intervals. Returns the onset's sample
// index within the day, or -1 (other days, or no sessions).
enum : uint32_t { kTagExer = 9u };
__device__ __forceinline__ int32_t exercise_onset(const SimArgs &a, uint32_t pid, int32_t day)
{
    if (!a.exercise)
        return -1;
    int season, wtype, dtype;
    nordic_day(a, pid, day, season, wtype, dtype);
    if (dtype != 1)
        return -1;
    const U4 r = philox4x32_10((uint32_t)day, pid, kTagExer, 0u, a.key0, a.key1);
    return (a.ex_minute + meal_jitter(r.z, a.jitter)) / a.ts_min;
}

template <typename R>
__device__ __forceinline__ bool all_finite(const State<R> &s)
{
    return isfinite(s.D1s) && isfinite(s.D2) && isfinite(s.S1s) && isfinite(s.S2s) && isfinite(s.I) &&
           isfinite(s.x1h) && isfinite(s.x2s) && isfinite(s.e3) && isfinite(s.Q1) && isfinite(s.Q2) &&
           isfinite(s.GIs);
}

// Loop-carried state of one patient besides the model state: controller, meal queue,
// metric accumulators.
template <typename R> struct Lane {
    R pid_b, y_prev;   // PID: the part of the unclamped output fixed before y_k (below), y_k-1
    int32_t c30, c39, c100, c139;                 // cumulative edge counters (bins by differences)
    int32_t r_hypo, r_sev, r_hyper, e_hypo, e_sev, e_hyper;
    double sum_g, sum_u;
    R min_g;
    int32_t argmin;
    uint32_t status;
};

// Per-patient constants of the controller and of the sampled inputs.
template <typename R> struct CtrlConst {
    R kpd, kd_ts, kits, kits_sp, umax, ub, u_open;   // PID in the form below; output bounds; open loop
    R k_sig;          // Box-Muller constant giving normals scaled by sqrt(h) sigma
    R sig_sqh, sqrt_r;
    double ts_d;
};

// Loop-carried state of the extended model (glucagon depot, exercise) and of the
// dual-hormone AP, per lane.
template <typename R> struct ExtLane {
    ExtState<R> x;
    ExtConst<R> c;
    int32_t ex_k;            // this day's exercise onset (sample within the day), -1 if none
    int32_t glu;             // dual-hormone AP: 1 in glucagon mode
    R bolus_per_rate;        // meal bolus (mU) per unit of announced intake (mmol/min)
    R iob_s1, iob_s2, iob0;  // insulin on board above basal = S1s iob_s1 + S2s iob_s2 - iob0 (mU)
    double basal, bolus, glucagon;   // delivered over the horizon: mU, mU, ug
};

// Inputs of the learned controller (and of the recorded behaviour-cloning rows), per lane:
//   f0..f5  y_k, y_k-1, ..., y_k-5 (sensor history; y_0 repeated before the first sample),
//   f6      insulin on board, as the mean change of G over the MPC's prediction horizon that
//           the insulin states' deviation from basal (S1, S2, I, x1, x2, x3) still causes:
//           Fbar_ins . (x_ins - x_ins*), mmol/L,
//   f7      the announced meals, likewise: Fbar_D1 D1 + Fbar_D2 D2 + wbar dhat_k, mmol/L,
//   f8..f11 the patient: u_b; the insulin response over the horizon, sum of the MPC's Markov
//           parameters h_1..h_24 (mmol/L per mU/min held for one sample); its mean delay
//           sum m h_m / sum h_m (samples); BW.
// Fbar and wbar are the horizon means of the MPC's prediction rows and intake response. The
// insulin and meal states are those of a controller-side replica of the insulin and
// absorption subsystems driven by the delivered doses and the announced meals; both are
// deterministic and the announcements exact, so the replica equals the plant's states and
// is read from them (the coefficients below undo the state scaling).
//
// Rows of the per-lane coefficients: f6 (insulin), f7 (meals), f8..f11; the learned
// controller also keeps its Kalman gain and the linearised step of the time update there.
enum : int { kPcIns = 0, kPcIns0 = 6, kPcMealD1 = 7, kPcMealD2 = 8, kPcWbar = 9, kPcSt = 10, kPcFeat = 14,
             kPcKg = 14, kPcLin = kPcKg + kNx, kPcRows = kPcLin + 11 };

// Coefficients of one lane in registers (the MPC kernel's recording path: the input rows
// only) or in the wave's LDS block [kPcRows][64] (the learned controller: read when used,
// so they take no registers across the network's evaluation).
template <typename R, bool kLds> struct PolicyCoefs {
    R v[kPcFeat];
    __device__ __forceinline__ R get(int r) const { return v[r]; }
    __device__ __forceinline__ void set(int r, R x) { v[r] = x; }
};
template <typename R> struct PolicyCoefs<R, true> {
    R *p;
    int lane;
    __device__ __forceinline__ R get(int r) const { return p[r * 64 + lane]; }
    __device__ __forceinline__ void set(int r, R x) { p[r * 64 + lane] = x; }
};

template <typename R, bool kLds> struct PolicyLane {
    R yh[5];                 // y_k-1 .. y_k-5
    PolicyCoefs<R, kLds> co; // f6 = ins . (S1s, S2s, I, x1h, x2s, e3) + ins0,
                             // f7 = D1s meal_d1 + D2 meal_d2 + dhat wbar, f8..f11 = st
    int32_t fallbacks;       // samples on which the MPC acted instead of the network
};

// The four patient inputs f8..f11 (see PolicyLane), from the population and MPC buffers.
template <typename R>
__device__ __forceinline__ void patient_inputs(const SimArgs &a, int64_t j, R out[4])
{
    const auto M = as_global((const R *)a.mpc);
    double hs = 0.0, hm = 0.0;
    for (int q = 0; q < kMpcN; ++q) {
        const double v = (double)M[(int64_t)(kMh + q) * a.n + j];
        hs += v;
        hm += (double)(q + 1) * v;
    }
    out[0] = R(a.params[(int64_t)kUb * a.n + j]);
    out[1] = R(hs);
    out[2] = R(hm / hs);
    out[3] = R(a.params[(int64_t)kBW * a.n + j]);
}

// LDS views of the learned controller (simulate_policy_kernel only): the staged network and
// the wave's input tile.
struct PolicyShared {
    const unsigned char *img;   // LDS image of the blob (NetImage<PaddedLayout>), staged once per workgroup
    uint16_t *xs;               // [64][PaddedLayout::ldi] BF16 normalised inputs, row = lane
    float *o;                   // [64] network outputs
    const float *mean, *istd, *lo, *hi;
    uint32_t *hist;             // population BG bins of this wave (kOutPop)
    uint32_t *span;             // [kSpanBins][64] per-lane BG bins of this wave (kOutPop)
    void *pc;                   // [kPcRows][64] per-lane coefficients of this wave (working precision)
    int lane;
    bool rest;                  // this wave's patient is outside the box: the MPC acts on every sample
};

// Orders this wave's LDS writes before its later LDS reads (LDS operations of one wave
// complete in order; the fences keep the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R, bool kLds>
__device__ __forceinline__ void policy_features(const PolicyLane<R, kLds> &P, const State<R> &s, R y, R dr,
                                                R f[kMlpIn])
{
    f[0] = y;
#pragma unroll
    for (int q = 0; q < 5; ++q)
        f[1 + q] = P.yh[q];
    R a6 = P.co.get(kPcIns0);
    a6 = fmaf_t(P.co.get(kPcIns + 0), s.S1s, a6);
    a6 = fmaf_t(P.co.get(kPcIns + 1), s.S2s, a6);
    a6 = fmaf_t(P.co.get(kPcIns + 2), s.I, a6);
    a6 = fmaf_t(P.co.get(kPcIns + 3), s.x1h, a6);
    a6 = fmaf_t(P.co.get(kPcIns + 4), s.x2s, a6);
    f[6] = fmaf_t(P.co.get(kPcIns + 5), s.e3, a6);
    f[7] = fmaf_t(s.D1s, P.co.get(kPcMealD1), fmaf_t(s.D2, P.co.get(kPcMealD2), dr * P.co.get(kPcWbar)));
#pragma unroll
    for (int q = 0; q < 4; ++q)
        f[8 + q] = P.co.get(kPcSt + q);
}

// The linearised time-update constants of the learned controller, from its LDS block.
template <typename R>
__device__ __forceinline__ LinStep<R> lin_from(const PolicyCoefs<R, true> &co)
{
    LinStep<R> m;
    m.s2s1 = co.get(kPcLin + 0);
    m.is2 = co.get(kPcLin + 1);
    m.x1i = co.get(kPcLin + 2);
    m.x2i = co.get(kPcLin + 3);
    m.x3i = co.get(kPcLin + 4);
    m.hq1 = co.get(kPcLin + 5);
    m.q1x3 = co.get(kPcLin + 6);
    m.q1q1 = co.get(kPcLin + 7);
    m.q2x2 = co.get(kPcLin + 8);
    m.q2q1 = co.get(kPcLin + 9);
    m.q2q2 = co.get(kPcLin + 10);
    return m;
}

// Writes the lane's normalised fixed inputs f8..f11 (BF16, columns 8..11 of its row of the
// input tile) and zeros in the padding columns 12..15, once per patient; each sample then
// writes columns 0..7 only.
template <typename R>
__device__ __forceinline__ void policy_fixed_inputs(const PolicyShared &ps, const R st[4])
{
    uint32_t w[2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
        w[q] = pack_bf16(((float)st[2 * q] - ps.mean[8 + 2 * q]) * ps.istd[8 + 2 * q],
                         ((float)st[2 * q + 1] - ps.mean[9 + 2 * q]) * ps.istd[9 + 2 * q]);
    uint4 *dst = (uint4 *)(ps.xs + ps.lane * PaddedLayout::ldi);
    dst[1] = uint4{w[0], w[1], 0u, 0u};
}

// Network output o_k for the 64 lanes of the wave (all lanes must be active): normalise the
// time-varying inputs f0..f7, round them to BF16, stage them in row `lane` of the input tile
// (columns 8..15 hold the patient's fixed inputs), run the MFMA chain.
template <typename R>
__device__ __forceinline__ float policy_forward(const PolicyShared &ps, const R f[kMlpIn])
{
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        w[q] = pack_bf16(((float)f[2 * q] - ps.mean[2 * q]) * ps.istd[2 * q],
                         ((float)f[2 * q + 1] - ps.mean[2 * q + 1]) * ps.istd[2 * q + 1]);
    uint4 *dst = (uint4 *)(ps.xs + ps.lane * PaddedLayout::ldi);
    dst[0] = uint4{w[0], w[1], w[2], w[3]};
    wave_lds_sync();
    return mlp_forward_lean<PaddedLayout>(ps.img, ps.xs, ps.o, ps.lane, wave_lds_sync);
}

// ------------------------------------------------------ wave-cooperative QP ----
// The MPC's QP for one patient of the learned controller (its fallback, and the labels when
// recording), solved by the whole wave: lane i < 24 owns entry i of the plan and holds row i
// of Gamma (G[c] = h_(i-c)) and of Gamma^T (T[c] = h_(c-i)), zero outside the triangle.
// Each Toeplitz product of a projected-gradient step is then 24 FMAs of those rows with the
// broadcast entries of the vector (v_readlane to scalar registers). Pass 1 runs c downwards
// and pass 2 upwards, so each lane meets its zero entries first and then sums h_d terms in
// ascending d, the order of mpc_pg: both solvers give identical results. The plan lives in
// global memory, untouched while the network acts: the warm start at sample k is the plan
// computed at sample k_plan moved on k - k_plan samples (entries past the horizon repeat
// the last), exactly what shifting it once per sample would give.
__device__ __forceinline__ float lane_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_shl1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_shr1(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_shl1(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_read(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Solve the QP of the patient of lane L (all lanes must be active). Returns u_0 - u_b of
// that patient, uniform across the wave; stores its plan when it is a live lane.
// A real call (not inlined): falling back is rare on a tile wave, and its ~100 registers
// would otherwise add to the network's and the plant's at every sample; the caller saves
// its live registers around the call instead.
template <typename R>
__device__ __attribute__((noinline)) R coop_qp(const SimArgs &a, const R *__restrict__ M, int64_t j, bool live, int32_t k,
                                     const MpcState<R> &ms, R dhat, int L, int lane)
{
    const uint32_t jL = (uint32_t)lane_read((int)j, L);
    const bool liveL = lane_read((int)live, L) != 0;
    R xh[kNx];
#pragma unroll
    for (int c = 0; c < kNx; ++c)
        xh[c] = lane_read(ms.xh[c], L);
    const R dh = lane_read(dhat, L);
    // step, rho and bounds as mpc_load_state forms them
    const R step = soa<R>(M, a.n, jL, kMstep), rho = soa<R>(M, a.n, jL, kMrho), ubL = soa<R>(M, a.n, jL, kMub);
    const R lo = -ubL, hi = soa<R>(M, a.n, jL, kMumax) - ubL;
    const bool act = lane < kMpcN;
    const int i = act ? lane : 0;
    // linear term g_i (the order of mpc_linear_term)
    R g = fmaf_t(soa<R>(M, a.n, jL, kMgd + i), dh, soa<R>(M, a.n, jL, kMg1 + i) * R(a.g_target - a.setpoint));
#pragma unroll
    for (int c = 0; c < kNx; ++c)
        g = fmaf_t(soa<R>(M, a.n, jL, kMGx + i * kNx + c), xh[c], g);
    // rows of Gamma and Gamma^T from h (lane i: h_i) and its reverse (lane i: h_(23-i)),
    // both zero beyond lane 23, by one-lane shifts with zero fill
    R G[kMpcN], T[kMpcN];
    G[0] = act ? soa<R>(M, a.n, jL, kMh + i) : R(0);
    T[kMpcN - 1] = act ? soa<R>(M, a.n, jL, kMh + kMpcN - 1 - i) : R(0);
#pragma unroll
    for (int c = 1; c < kMpcN; ++c) {
        G[c] = lane_shr1(G[c - 1]);
        T[kMpcN - 1 - c] = lane_shl1(T[kMpcN - c]);
    }
    auto P = as_global((R *)a.plan);
    auto KP = as_global(a.kplan);
    const int32_t sh = min(max(k - KP[jL], 0), kMpcN - 1);
    R dU = act ? P[(int64_t)min(i + sh, kMpcN - 1) * a.n + jL] : R(0);
    for (int it = 0; it < a.mpc_iters; ++it) {
        // all broadcasts first (distinct scalar registers), then the FMA chain: a scalar
        // register written by v_readlane is read by VALU only after a wait, which the
        // batching pays once per product instead of once per term
        R v[kMpcN];
#pragma unroll
        for (int c = 0; c < kMpcN; ++c)
            v[c] = lane_read(dU, c);
        __builtin_amdgcn_sched_barrier(0);
        R r = R(0);
#pragma unroll
        for (int c = kMpcN - 1; c >= 0; --c)
            r = fmaf_t(G[c], v[c], r);
#pragma unroll
        for (int c = 0; c < kMpcN; ++c)
            v[c] = lane_read(r, c);
        __builtin_amdgcn_sched_barrier(0);
        R acc = fmaf_t(rho, dU, g);
#pragma unroll
        for (int c = 0; c < kMpcN; ++c)
            acc = fmaf_t(T[c], v[c], acc);
        dU = act ? vclamp(fmaf_t(-step, acc, dU), lo, hi) : R(0);
    }
    if (liveL && act)
        P[(int64_t)i * a.n + jL] = dU;
    if (liveL && lane == 0)
        KP[jL] = k;
    return lane_read(dU, 0);
}

// One sampling instant t_k: indicators on the true glucose, sensor value, controller,
// held inputs, then the EM steps of [t_k, t_k+1). dr is the held meal input of the
// interval (also the MPC's announcement). z[0..4] are the EM noise increments
// (sqrt(h) sigma xi), z[5] the sensor noise (sqrt(R) v). `live` is false for the padding
// lanes of the learned controller's last wave, which compute but write nothing.
template <typename R, int CTRL, int OUT>
__device__ __forceinline__ void sample_step(const SimArgs &a, int64_t j, bool live, int32_t k, int32_t kd, R dr,
                                            const R *z, State<R> &s, const StepConst<R> &c,
                                            const CtrlConst<R> &cc, Lane<R> &L, MpcState<R> &ms,
                                            MpcPlan<R> &mplan, const LinStep<R> &lin,
                                            PolicyLane<R, CTRL == kCtrlMlp> &pl, const PolicyShared &ps,
                                            ExtLane<R> &xl)
{
    constexpr int kBase = ctrl_base<CTRL>();
    // indicators (Sec. IV-A ranges) on G(t_k)
    const R G = s.Q1 * c.inv_vg;
    if (OUT & kOutPop) {
        pop_accumulate<R>(a, k, G, live);
        if (live)
            atomicAdd(&ps.hist[pop_bin((double)G)], 1u);
        atomicAdd(&ps.span[span_bin((double)G) * 64 + ps.lane], 1u);   // this lane's own counters
    }
    // one comparison per edge serves both the range count and the run: a run below an edge
    // continues while G is not at or above it, so a non-finite G (in the lowest range, with
    // its status bit) also continues the runs below 3.9 and 3.0
    const bool at30 = G >= R(3.0), at39 = G >= R(3.9), above139 = G > R(13.9);
    L.c30 += at30;
    L.c39 += at39;
    L.c100 += G > R(10.0);
    L.c139 += above139;
    L.r_hypo = at39 ? 0 : L.r_hypo + 1;
    L.r_sev = at30 ? 0 : L.r_sev + 1;
    L.r_hyper = above139 ? L.r_hyper + 1 : 0;
    L.e_hypo += L.r_hypo == 3;
    L.e_sev += L.r_sev == 3;
    L.e_hyper += L.r_hyper == 3;
    L.sum_g += (double)G;
    if (G < L.min_g) {
        L.min_g = G;
        L.argmin = k;
    }
    if (G < R(0))
        L.status |= kStNegQ1;

    const R y = fmaf_t(s.GIs, c.gi_scale, z[5]);   // y_k = g(x(t_k)) + v_k

    constexpr bool kFeat = CTRL == kCtrlMlp || (OUT & kOutRecord);
    R f[kMlpIn];
    if (kFeat) {
        if (k == 0) {
#pragma unroll
            for (int q = 0; q < 5; ++q)
                pl.yh[q] = y;
        }
        policy_features<R, CTRL == kCtrlMlp>(pl, s, y, dr, f);
    }

    R u, label = R(0);
    R u_bol = R(0), un = R(0);   // dual-hormone AP: bolus insulin (mU/min), glucagon (ug/min)
    if constexpr (kBase == kCtrlPid) {   // control state (integral, previous y), Sec. III-B form
        // u = u_b + kp e_k + ki sum_{i<k} ts e_i + kd (y_k - y_k-1)/ts with e = y - sp,
        // clamped to [0, umax]; the integral grows only while u is not clamped. Regrouped
        // as pid_b + (kp + kd/ts) y_k - (kd/ts) y_k-1 with pid_b = u_b - kp sp + ki sum ts e_i.
        if (k == 0)
            L.y_prev = y;
        const R u_unc = fmaf_t(cc.kpd, y, fmaf_t(-cc.kd_ts, L.y_prev, L.pid_b));
        u = vclamp(u_unc, R(0), cc.umax);
        if (u == u_unc)   // not clamped (a NaN u_unc is clamped to 0 and never integrates)
            L.pid_b = fmaf_t(cc.kits, y, L.pid_b - cc.kits_sp);
        L.y_prev = y;
    } else if constexpr (kBase == kCtrlMpc) {   // control state (Kalman estimate, input plan)
        u = mpc_step<R>((const R *)a.mpc, a.n, j, ms, mplan, c, lin, R(a.h), R(a.h * a.ag), a.em_per_ctrl, y, dr,
                        R(a.g_target - a.setpoint), a.mpc_iters);
    } else if constexpr (kBase == kCtrlMlp) {
        // control state (CGM history, Kalman estimate, input plan): the network acts unless
        // an input leaves the box it was trained on, or the sensor reads low (y < mlp_safe_g)
        // while the network asks for more than mlp_safe_out u_b; then the MPC solves its QP.
        // The Kalman filter runs on every sample so the MPC is ready to take over. With recording on,
        // the MPC's QP is solved on every sample and its action recorded as the label of
        // the network's inputs (data aggregation along the network's own closed loop).
        const R *M = (const R *)a.mpc;
        {
            R kg[kNx];
#pragma unroll
            for (int q = 0; q < kNx; ++q)
                kg[q] = pl.co.get(kPcKg + q);
            mpc_measure_gain<R>(kg, ms, y);
        }
        // The fixed inputs f8..f11 decided the lane order: every patient of a tile wave has
        // them inside the box (the same comparisons), every other patient is alone on a
        // wave and falls back on every sample. Only the time-varying inputs are tested here.
        bool ood = ps.rest;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            ood |= !(f[q] >= R(ps.lo[q]) && f[q] <= R(ps.hi[q]));
        // (a wave whose patient is outside the box needs no network: its fallback is certain)
        const float o = ps.rest ? 0.0f : policy_forward<R>(ps, f);
        const bool fb = ood || (y < R(a.mlp_safe_g) && o > (float)a.mlp_safe_out);
        // every live lane that needs the MPC's action gets it from a wave-cooperative solve
        R du_mpc = R(0);
        for (uint64_t need = __ballot(live && (fb || (OUT & kOutRecord))); need; need &= need - 1) {
            const int L = __builtin_ctzll(need);
            const R d = coop_qp<R>(a, M, j, live, k, ms, dr, L, ps.lane);
            if (ps.lane == L)
                du_mpc = d;
        }
        R du;
        if (fb) {
            du = du_mpc;
            u = cc.ub + du;
            ++pl.fallbacks;
        } else {
            u = vclamp(cc.ub * R(o), R(0), cc.umax);
            du = u - cc.ub;
        }
        label = cc.ub + du_mpc;
        mpc_predict<R>(ms, c, lin_from<R>(pl.co), du, dr, R(a.h), R(a.h * a.ag), a.em_per_ctrl);
    } else if constexpr (kBase == kCtrlDual) {
        // dual-hormone AP (Sec. IV-C): glucagon mode below glu_enter until y >= glu_exit (a
        // non-finite reading changes nothing). The PID runs on every sample, as above, and is
        // delivered in insulin mode only, with the meal bolus less the insulin on board;
        // glucagon mode gives microboli less the glucagon on board; an exercise onset below
        // ex_bolus_below adds the exercise bolus in either mode.
        xl.glu = xl.glu ? !(y >= R(a.glu_exit)) : (y < R(a.glu_enter));
        if (k == 0)
            L.y_prev = y;
        const R u_unc = fmaf_t(cc.kpd, y, fmaf_t(-cc.kd_ts, L.y_prev, L.pid_b));
        const R u_pid = vclamp(u_unc, R(0), cc.umax);
        if (u_pid == u_unc)
            L.pid_b = fmaf_t(cc.kits, y, L.pid_b - cc.kits_sp);
        L.y_prev = y;
        R n_ug = R(0);
        if (xl.glu) {
            u = R(0);
            n_ug = vmin(R(a.glu_max), vmax(R(0), fmaf_t(R(a.glu_kp), R(a.glu_target) - y, -(xl.x.z1 + xl.x.z2))));
        } else {
            u = u_pid;
            if (a.meal_bolus && dr > R(0)) {
                const R iob = fmaf_t(s.S1s, xl.iob_s1, fmaf_t(s.S2s, xl.iob_s2, -xl.iob0));
                u_bol = vmax(R(0), fmaf_t(dr, xl.bolus_per_rate, -iob)) / R(a.ts_min);
            }
        }
        if (kd == xl.ex_k && y < R(a.ex_bolus_below))
            n_ug += R(a.ex_bolus);
        un = n_ug / R(a.ts_min);
    } else {
        u = cc.u_open;
    }
    if constexpr (ctrl_ext<CTRL>()) {   // delivered doses: basal and bolus insulin, glucagon
        xl.basal += (double)u * cc.ts_d;
        xl.bolus += (double)u_bol * cc.ts_d;
        xl.glucagon += (double)un * cc.ts_d;
        u = u + u_bol;
    }
    if (kFeat) {
#pragma unroll
        for (int q = 4; q > 0; --q)
            pl.yh[q] = pl.yh[q - 1];
        pl.yh[0] = y;
    }
    if ((OUT & kOutRecord) && live) {   // row (k, j): the 12 inputs, then u_k / u_b
        auto row = as_global(a.record) + ((int64_t)k * a.n + j) * (kMlpIn + 1);
#pragma unroll
        for (int q = 0; q < kMlpIn; ++q)
            row[q] = (float)f[q];
        row[kMlpIn] = (float)((CTRL == kCtrlMlp ? label : u) / cc.ub);
    }
    if ((OUT & kOutTraj) && live && j < a.n_traj) {
        a.traj[(0 * (int64_t)a.n_traj + j) * a.K + k] = (double)G;
        a.traj[(1 * (int64_t)a.n_traj + j) * a.K + k] = (double)y;
        a.traj[(2 * (int64_t)a.n_traj + j) * a.K + k] = (double)u;
    }

    const R du = c.u_in * u, dd = c.d_in * dr;
    if constexpr (ctrl_ext<CTRL>()) {   // the extended model: glucagon into the depot, exercise input
        const bool session = xl.ex_k >= 0 && kd >= xl.ex_k && kd < xl.ex_k + a.ex_samples;
        const R dh = session ? xl.c.b_e1 * R(a.ex_hrr) : R(0);
        const R dn = R(a.h) * un;
#pragma unroll
        for (int q = 0; q < 5; ++q)
            em_step_ext<R>(s, xl.x, c, xl.c, du, dd, z[q], dn, dh);
    } else {
#pragma unroll
        for (int q = 0; q < 5; ++q)
            em_step<R>(s, c, du, dd, z[q]);
    }
    L.sum_u += (double)u * cc.ts_d;
}

// The whole horizon of patient j of the population described by a (one lane).
template <typename R, int CTRL, bool NOISY, int OUT>
__device__ __forceinline__ void run_patient(const SimArgs &a, int64_t j, bool live, const PolicyShared &ps)
{
    const uint32_t pid = (uint32_t)(a.patient_base + j);

    double p[15];
#pragma unroll
    for (int q = 0; q < 15; ++q)
        p[q] = a.params[(int64_t)q * a.n + j];
    const double ub_d = a.params[(int64_t)kUb * a.n + j];
    const double istar = a.params[(int64_t)kIstar * a.n + j];

    Lane<R> L{};
    L.status = (uint32_t)a.params[(int64_t)kStatus * a.n + j];
    L.min_g = R(INFINITY);
    L.argmin = -1;

    State<R> s;
    basal_state<R>(p, istar, ub_d, a.g_target, a.h, a.tau, s);
    if (!(ub_d > 0.0)) {   // no basal state exists even for the nominal vector
        const R nan = R(NAN);
        s = State<R>{nan, nan, nan, nan, nan, nan, nan, nan, nan, nan, nan};
    }
    StepConst<R> c;
    step_constants<R>(p, a.h, a.tau, a.ag, c);

    MpcState<R> ms;
    MpcPlan<R> mplan;
    LinStep<R> lin;
    if (CTRL == kCtrlMpc || CTRL == kCtrlMlp) {
        mpc_load_state<R>((const R *)a.mpc, a.n, j, ms);
        lin_step_constants<R>(p, istar, a.h, a.g_target, lin);
    }
    if (CTRL == kCtrlMpc) {
        mpc_load_h<R>((const R *)a.mpc, a.n, j, mplan.h);
#pragma unroll
        for (int i = 0; i < kMpcN; ++i)
            mplan.dU[i] = R(0);
    }
    if (CTRL == kCtrlMlp && live) {   // empty plan, computed "before" sample 0
        R *P = (R *)a.plan;
#pragma unroll
        for (int i = 0; i < kMpcN; ++i)
            P[(int64_t)i * a.n + j] = R(0);
        a.kplan[j] = -1;
    }
    PolicyLane<R, CTRL == kCtrlMlp> pl;
    if constexpr (CTRL == kCtrlMlp) {
        pl.co.p = (R *)ps.pc;
        pl.co.lane = ps.lane;
    }
    if (CTRL == kCtrlMlp || (OUT & kOutRecord)) {
        // f6, f7 from the horizon-mean prediction rows (FP64 here, then the working precision)
        const auto M = as_global((const R *)a.mpc);
        double fb[kNx];
#pragma unroll
        for (int q = 0; q < kNx; ++q)
            fb[q] = (double)M[(int64_t)(kMFbar + q) * a.n + j];
        const double ti = p[kTmaxI], vi = p[kVI] * p[kBW], h = a.h, egp0 = p[kEGP0] * p[kBW];
        const double c_ui = h / (ti * vi), b_i = h / ti;
        // unscaled states: S1 = S1s/(c_ui b_i), S2 = S2s/c_ui, x1 = x1h/h, x2 = x2s h ka2 SID,
        // x3 = 1 - e3/(h EGP0); basal: S1* = S2* = u_b tmaxI, I*, x_j* = S_j I*
        pl.co.set(kPcIns + 0, R(fb[kXS1] / (c_ui * b_i)));
        pl.co.set(kPcIns + 1, R(fb[kXS2] / c_ui));
        pl.co.set(kPcIns + 2, R(fb[kXI]));
        pl.co.set(kPcIns + 3, R(fb[kXx1] / h));
        pl.co.set(kPcIns + 4, R(fb[kXx2] * h * p[kKa2] * p[kSID]));
        pl.co.set(kPcIns + 5, R(-fb[kXx3] / (h * egp0)));
        pl.co.set(kPcIns0, R(fb[kXx3] - (fb[kXS1] + fb[kXS2]) * ub_d * ti - fb[kXI] * istar -
                             (fb[kXx1] * p[kSIT] + fb[kXx2] * p[kSID] + fb[kXx3] * p[kSIE]) * istar));
        pl.co.set(kPcMealD1, R(fb[kXD1] * p[kTmaxG] / h));
        pl.co.set(kPcMealD2, R(fb[kXD2]));
        pl.co.set(kPcWbar, R((double)M[(int64_t)kMwbar * a.n + j]));
        R st[4];
        patient_inputs<R>(a, j, st);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            pl.co.set(kPcSt + q, st[q]);
        pl.fallbacks = 0;
        if constexpr (CTRL == kCtrlMlp) {
#pragma unroll
            for (int q = 0; q < kNx; ++q)
                pl.co.set(kPcKg + q, M[(int64_t)(kMK + q) * a.n + j]);
            pl.co.set(kPcLin + 0, lin.s2s1);
            pl.co.set(kPcLin + 1, lin.is2);
            pl.co.set(kPcLin + 2, lin.x1i);
            pl.co.set(kPcLin + 3, lin.x2i);
            pl.co.set(kPcLin + 4, lin.x3i);
            pl.co.set(kPcLin + 5, lin.hq1);
            pl.co.set(kPcLin + 6, lin.q1x3);
            pl.co.set(kPcLin + 7, lin.q1q1);
            pl.co.set(kPcLin + 8, lin.q2x2);
            pl.co.set(kPcLin + 9, lin.q2q1);
            pl.co.set(kPcLin + 10, lin.q2q2);
            if (!ps.rest)
                policy_fixed_inputs<R>(ps, st);
        }
    }

    CtrlConst<R> cc;   // gains relative to u_b
    // the controller's own basal rate: the patient's, or a mis-set one (basal_scale != 1,
    // PID and open loop only; Sec. IV-E trial B underestimates it by 50 %)
    const double ubc = a.basal_scale * ub_d;
    const double kp = a.kp * ubc, ki = a.ki * ubc, kd_ts = a.kd * ubc / (double)a.ts_min;
    cc.kpd = R(kp + kd_ts);
    cc.kd_ts = R(kd_ts);
    cc.kits = R(ki * a.ts_min);
    cc.kits_sp = R(ki * a.ts_min * a.setpoint);
    L.pid_b = R(ubc - kp * a.setpoint);
    cc.umax = R(a.umax_rel * ubc);
    cc.ub = R(ubc);
    cc.u_open = R(a.u_rel * ubc);
    cc.k_sig = Rng<R>::scaled_const(a.sig_sqh);
    cc.sig_sqh = R(a.sig_sqh);
    cc.sqrt_r = R(a.sqrt_r);
    cc.ts_d = (double)a.ts_min;
    const R bw = R(p[kBW]);   // body weight: the Northern-European protocol's meal sizes are per kg

    ExtLane<R> xl{};
    if constexpr (ctrl_ext<CTRL>()) {
        ext_constants<R>(a.h, a.tau_n, a.e_n, a.tau_e1, a.tau_e2, a.tau_e3, a.alpha_e, a.beta_e, xl.c);
        xl.x = ExtState<R>{R(0), R(0), R(0), R(0), R(0)};   // no glucagon, no exercise: the basal state
        xl.glu = 0;
        xl.ex_k = -1;
        // insulin on board above basal from the scaled depot states (S1 = S1s/(c_ui b_i),
        // S2 = S2s/c_ui, basal S1 = S2 = u_b tmaxI); the bolus per announced intake from
        // the ICR rule (carbs = intake Ts 180.16/1000 g, ICR = icr_rule / TDD g/U,
        // TDD = 2 x 1440 u_b / 1000 U)
        const double ti = p[kTmaxI], vi = p[kVI] * p[kBW];
        const double c_ui = a.h / (ti * vi), b_i = a.h / ti;
        xl.iob_s1 = R(1.0 / (c_ui * b_i));
        xl.iob_s2 = R(1.0 / c_ui);
        xl.iob0 = R(2.0 * ub_d * ti);
        const double tdd = 2.0 * ub_d * 1440.0 / 1000.0;
        xl.bolus_per_rate = R((double)a.ts_min * 180.16 / 1000.0 * tdd / a.icr_rule * 1000.0);
        xl.basal = xl.bolus = xl.glucagon = 0.0;
    }

    for (int32_t day = 0; day < a.n_days; ++day) {
        DayMeals<R> ml = draw_meals<R>(a, pid, day, bw);
        if constexpr (ctrl_ext<CTRL>())
            xl.ex_k = exercise_onset(a, pid, day);
        for (int32_t kk = 0; kk < a.kday; kk += 2) {
            const int32_t k = day * a.kday + kk;
            // normals of the sample pair (k, k+1): blocks (k/2, patient, DIFF, 0..2), normals
            // 0..5 for sample k and 6..11 for sample k+1 (EM normals first, sensor last)
            R z[12];
            if (NOISY) {
                const uint32_t jp = (uint32_t)(k >> 1);
                const U4 b0 = philox4x32_10_lane1(jp, pid, kTagDiff, 0u, a.key0, a.key1);
                const U4 b1 = philox4x32_10_lane1(jp, pid, kTagDiff, 1u, a.key0, a.key1);
                const U4 b2 = philox4x32_10_lane1(jp, pid, kTagDiff, 2u, a.key0, a.key1);
                // pure diffusion pairs come out scaled by sqrt(h) sigma; the two pairs that
                // mix an EM normal with the sensor normal are scaled per normal
                R r0, r1;
                Rng<R>::box_muller_scaled(Rng<R>::uniform(b0.x), Rng<R>::uniform(b0.y), cc.k_sig, z[0], z[1]);
                Rng<R>::box_muller_scaled(Rng<R>::uniform(b0.z), Rng<R>::uniform(b0.w), cc.k_sig, z[2], z[3]);
                Rng<R>::box_muller(Rng<R>::uniform(b1.x), Rng<R>::uniform(b1.y), r0, r1);
                z[4] = cc.sig_sqh * r0;
                z[5] = cc.sqrt_r * r1;
                Rng<R>::box_muller_scaled(Rng<R>::uniform(b1.z), Rng<R>::uniform(b1.w), cc.k_sig, z[6], z[7]);
                Rng<R>::box_muller_scaled(Rng<R>::uniform(b2.x), Rng<R>::uniform(b2.y), cc.k_sig, z[8], z[9]);
                Rng<R>::box_muller(Rng<R>::uniform(b2.z), Rng<R>::uniform(b2.w), r0, r1);
                z[10] = cc.sig_sqh * r0;
                z[11] = cc.sqrt_r * r1;
            } else {
#pragma unroll
                for (int q = 0; q < 12; ++q)
                    z[q] = R(0);
            }
            // held meal inputs of the pair: the queue is touched only when its first meal
            // starts at kk or kk + 1 (one unsigned compare per pair; -1 never matches)
            R dr0 = R(0), dr1 = R(0);
            if ((uint32_t)(ml.k0 - kk) <= 1u) {
                if (ml.k0 == kk)
                    dr0 = pop_front(ml);
                if (ml.k0 == kk + 1)
                    dr1 = pop_front(ml);
            }
            sample_step<R, CTRL, OUT>(a, j, live, k, kk, dr0, z, s, c, cc, L, ms, mplan, lin, pl, ps, xl);
            sample_step<R, CTRL, OUT>(a, j, live, k + 1, kk + 1, dr1, z + 6, s, c, cc, L, ms, mplan, lin, pl, ps,
                                      xl);
        }
        if (!all_finite(s))
            L.status |= kStNonFinite;
        if constexpr (ctrl_ext<CTRL>()) {
            if (!(isfinite(xl.x.z1) && isfinite(xl.x.z2) && isfinite(xl.x.ex1) && isfinite(xl.x.ex2) &&
                  isfinite(xl.x.ex3)))
                L.status |= kStNonFinite;
        }
    }
    if (OUT & kOutPop)
        span_flush(a, ps.span, ps.lane, live);

    if (!live)
        return;
    if (CTRL == kCtrlMlp && a.fallback)
        a.fallback[j] = pl.fallbacks;
    if constexpr (ctrl_ext<CTRL>()) {
        if (a.doses) {
            a.doses[0 * a.out_stride + j] = xl.basal;
            a.doses[1 * a.out_stride + j] = xl.bolus;
            a.doses[2 * a.out_stride + j] = xl.glucagon;
        }
    }
    const int64_t st = a.out_stride;
    const int32_t K = (int32_t)a.K;
    a.sum_g[j] = L.sum_g;
    a.min_g[j] = (double)L.min_g;
    a.sum_u[j] = L.sum_u;
    a.bins[0 * st + j] = K - L.c30;
    a.bins[1 * st + j] = L.c30 - L.c39;
    a.bins[2 * st + j] = L.c39 - L.c100;
    a.bins[3 * st + j] = L.c100 - L.c139;
    a.bins[4 * st + j] = L.c139;
    a.events[0 * st + j] = L.e_hypo;
    a.events[1 * st + j] = L.e_sev;
    a.events[2 * st + j] = L.e_hyper;
    a.argmin_k[j] = L.argmin;
    a.status[j] = L.status;
}

// Waves per SIMD the plain kernels are compiled for: the FP32 open-loop and PID loops
// without per-sample outputs fit in 128 registers without spilling, which lets four waves
// share a SIMD; the FP32 dual-hormone loop fits in 168 (three waves; 186 registers and two
// waves by the compiler's own choice, 8 % slower); the rest keep the compiler's choice.
template <typename R, int CTRL, int OUT>
constexpr int sim_waves_per_simd()
{
    if (sizeof(R) == 4 && OUT == 0)
        return CTRL <= kCtrlPid ? 4 : (CTRL == kCtrlDual ? 3 : 1);
    return 1;
}

// Workgroup size of simulate_kernel: one wave with the population curves on (its 14.4 KB of
// LDS counters per wave then limit occupancy per wave, not per 4-wave group), else 256.
template <int OUT>
constexpr int sim_block()
{
    return (OUT & kOutPop) ? 64 : 256;
}

template <typename R, int CTRL, bool NOISY, int OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sim_waves_per_simd<R, CTRL, OUT>())))
void simulate_kernel(const SimArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr ((OUT & kOutPop) != 0) {
        // the population reduction needs every lane of a wave: lanes past the last patient
        // replay it and write nothing; a wave wholly past it exits
        __shared__ uint32_t hist[sim_block<OUT>() / 64][kPopBins];
        __shared__ uint32_t span[sim_block<OUT>() / 64][kSpanBins * 64];
        if ((j & ~(int64_t)63) >= a.n)
            return;
        const bool live = j < a.n;
        PolicyShared ps{};
        ps.lane = threadIdx.x & 63;
        ps.hist = hist[threadIdx.x >> 6];
        ps.span = span[threadIdx.x >> 6];
        for (int b = 0; b < kSpanBins; ++b)
            ps.span[b * 64 + ps.lane] = 0u;
        pop_hist_clear(ps.hist, threadIdx.x & 63);
        run_patient<R, CTRL, NOISY, OUT>(a, live ? j : a.n - 1, live, ps);
        pop_hist_flush(a, ps.hist, threadIdx.x & 63);
    } else if (j < a.n) {
        run_patient<R, CTRL, NOISY, OUT>(a, j, true, PolicyShared{});
    }
}

// The learned controller: the same per-patient loop, with the network evaluated by each
// wave for its 64 patients on every sample. The weights and biases are staged into LDS
// once per workgroup; each wave owns an input tile, and the hidden activations stay in
// registers. Lanes take patients in the order a.order: each patient whose fixed inputs lie
// outside the box (the MPC acts on every sample, so the network is skipped) alone on a
// wave, then tiles of 64 patients. Every lane of a tile wave takes part in the MFMA chain,
// so the padding lanes of the last tile replay a patient and write nothing.
// Workgroup size: four waves; two for FP64 with the population curves (their LDS).
template <typename R, int OUT> constexpr int policy_block()
{
    return (sizeof(R) == 8 && (OUT & kOutPop)) ? 128 : 256;
}
using PolicyNet = NetImage<PaddedLayout>;
// per wave: the input tile [64][24] BF16, the 64 outputs and the lanes' coefficients
// [kPcRows][64] in the working precision
template <typename R> constexpr int policy_wave_bytes()
{
    return 64 * PaddedLayout::ldi * 2 + 64 * 4 + kPcRows * 64 * (int)sizeof(R);
}
// Workgroups per CU the kernel is compiled for: two (two waves per SIMD, 256 registers
// each) for FP32 without the population curves; one otherwise (FP64 state needs twice the
// registers; the curves' LDS counters leave room for one workgroup).
template <typename R, int OUT> constexpr int policy_blocks_per_cu()
{
    return (sizeof(R) == 4 && !(OUT & kOutPop)) ? 2 : 1;
}

template <typename R, bool NOISY, int OUT>
__global__ __launch_bounds__((policy_block<R, OUT>()), (policy_blocks_per_cu<R, OUT>())) void simulate_policy_kernel(
    const SimArgs a, const int32_t *counts, int32_t nb, uint32_t *queue)
{
    constexpr int kBlock = policy_block<R, OUT>();
    __shared__ __align__(16) unsigned char lds[PolicyNet::bytes + (kBlock / 64) * policy_wave_bytes<R>()];
    stage_net<PaddedLayout>(a.mlp, lds, threadIdx.x, kBlock);
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    unsigned char *wl = lds + PolicyNet::bytes + wave * policy_wave_bytes<R>();
    PolicyShared ps;
    ps.img = lds;
    ps.xs = (uint16_t *)wl;
    ps.o = (float *)(wl + 64 * PaddedLayout::ldi * 2);
    ps.pc = wl + 64 * PaddedLayout::ldi * 2 + 64 * 4;
    ps.mean = (const float *)(lds + PolicyNet::tail + (kOffMean - kOffB1));
    ps.istd = (const float *)(lds + PolicyNet::tail + (kOffIstd - kOffB1));
    ps.lo = (const float *)(lds + PolicyNet::tail + (kOffLo - kOffB1));
    ps.hi = (const float *)(lds + PolicyNet::tail + (kOffHi - kOffB1));
    ps.lane = threadIdx.x & 63;
    ps.hist = nullptr;
    ps.span = nullptr;
    if constexpr ((OUT & kOutPop) != 0) {
        __shared__ uint32_t phist[kBlock / 64][kPopBins];
        __shared__ uint32_t pspan[kBlock / 64][kSpanBins * 64];
        ps.hist = phist[wave];
        ps.span = pspan[wave];
        for (int b = 0; b < kSpanBins; ++b)
            ps.span[b * 64 + ps.lane] = 0u;
        pop_hist_clear(ps.hist, ps.lane);
    }
    // Work items, longest first: each patient outside the box alone on a wave (the MPC acts
    // on every sample, solved cooperatively), then tiles of 64 patients inside the box.
    const int32_t n_in = counts[nb];
    const int32_t n_rest = (int32_t)a.n - n_in;
    const int32_t n_items = n_rest + (n_in + 63) / 64;
    for (;;) {
        int32_t item = 0;
        if (ps.lane == 0)
            item = (int32_t)atomicAdd(queue, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items)
            break;
        int64_t slot;
        bool live;
        if (item < n_rest) {
            slot = (int64_t)n_in + item;
            live = ps.lane == 0;
        } else {
            const int64_t s0 = (int64_t)(item - n_rest) * 64 + ps.lane;
            live = s0 < n_in;
            slot = live ? s0 : (int64_t)n_in - 1;
        }
        ps.rest = item < n_rest;
        run_patient<R, kCtrlMlp, NOISY, OUT>(a, (int64_t)a.order[slot], live, ps);
    }
    if constexpr ((OUT & kOutPop) != 0)
        pop_hist_flush(a, ps.hist, ps.lane);
}

// Lane order of the learned controller: a stable partition of the patients into those whose
// fixed inputs f8..f11 lie inside the network's box and the rest, in three
// launches (per-block counts, one-block scan, scatter). Only the placement of patients on
// lanes depends on it, never a result.
constexpr int kPartBlock = 1024;

template <typename R>
__device__ __forceinline__ bool fixed_inputs_in_box(const SimArgs &a, int64_t j)
{
    const float *lo = (const float *)(a.mlp + kOffLo), *hi = (const float *)(a.mlp + kOffHi);
    R v[4];
    patient_inputs<R>(a, j, v);
    bool in = true;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        in = in && v[q] >= R(lo[8 + q]) && v[q] <= R(hi[8 + q]);
    return in;
}

template <typename R>
__global__ __launch_bounds__(kPartBlock) void policy_count_kernel(const SimArgs a, int32_t *counts)
{
    const int64_t j = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
    const int c = __syncthreads_count(j < a.n && fixed_inputs_in_box<R>(a, j));
    if (threadIdx.x == 0)
        counts[blockIdx.x] = c;
}

// Exclusive scan of counts[0 .. nb) in place; counts[nb] = total.
__global__ __launch_bounds__(kPartBlock) void policy_scan_kernel(int32_t *counts, int32_t nb)
{
    __shared__ int32_t part[kPartBlock];
    int32_t carry = 0;
    for (int32_t base = 0; base < nb; base += kPartBlock) {
        const int32_t i = base + (int32_t)threadIdx.x;
        const int32_t v = i < nb ? counts[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kPartBlock; off <<= 1) {
            const int32_t t = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb)
            counts[i] = carry + part[threadIdx.x] - v;
        carry += part[kPartBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[nb] = carry;
        counts[nb + 1] = 0;   // work-queue head of the simulation launch that follows
    }
}

template <typename R>
__global__ __launch_bounds__(kPartBlock) void policy_scatter_kernel(const SimArgs a, const int32_t *scan,
                                                                    int32_t *order)
{
    __shared__ int32_t wsum[kPartBlock / 64];
    const int64_t j = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
    const bool valid = j < a.n;
    const bool in = valid && fixed_inputs_in_box<R>(a, j);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t m = __ballot(in);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0)
        wsum[w] = __popcll(m);
    __syncthreads();
    int32_t rank_in = __popcll(m & below);
    for (int q = 0; q < w; ++q)
        rank_in += wsum[q];
    if (valid) {
        const int32_t in_before = scan[blockIdx.x];
        const int64_t pos = in ? (int64_t)in_before + rank_in
                               : (int64_t)scan[gridDim.x] + ((int64_t)blockIdx.x * kPartBlock - in_before) +
                                     ((int32_t)threadIdx.x - rank_in);
        order[pos] = (int32_t)j;
    }
}

size_t policy_scratch_bytes(int64_t n, int precision)
{
    const size_t rb = precision == 1 ? sizeof(float) : sizeof(double);
    const int64_t nb = (n + kPartBlock - 1) / kPartBlock;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    // plans, plan times, lane order, per-block counts + total + work-queue head
    return up((size_t)kMpcN * n * rb) + up((size_t)n * 4) + up((size_t)n * 4) + up((size_t)(nb + 2) * 4);
}

void policy_scratch_views(SimArgs &a, void *scratch, int precision)
{
    const size_t rb = precision == 1 ? sizeof(float) : sizeof(double);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = (char *)scratch;
    a.plan = p;
    p += up((size_t)kMpcN * a.n * rb);
    a.kplan = (int32_t *)p;
    p += up((size_t)a.n * 4);
    a.order = (const int32_t *)p;
}

static int32_t *policy_counts(const SimArgs &a)
{
    return (int32_t *)((char *)a.order + (((size_t)a.n * 4 + 255) & ~(size_t)255));
}

// ------------------------------------------------------------ batched arms ----
// Persistent kernel over a queue of work items (arm, first patient of a tile of
// blockDim.x patients), ordered longest horizon first. Thread 0 of a workgroup takes
// the next item with one atomic; the whole workgroup runs that tile for the arm's full
// horizon, then takes the next. Every workgroup exits once the queue is drained. Each
// patient runs exactly the code of simulate_kernel, so results do not depend on the
// batching.
template <typename R, int CTRL, bool NOISY, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sim_waves_per_simd<R, CTRL, 0>())))
void batch_kernel(const SimArgs *__restrict__ arms,
                                                      const BatchItem *__restrict__ items, int32_t n_items,
                                                      uint32_t *__restrict__ counter)
{
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0)
            next = (int32_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int32_t it = next;
        __syncthreads();
        if (it >= n_items)
            return;
        const BatchItem w = items[it];
        const SimArgs &a = arms[w.arm];
        const int64_t j = (int64_t)w.first + threadIdx.x;
        if (j < a.n)
            run_patient<R, CTRL, NOISY, 0>(a, j, true, PolicyShared{});
    }
}

__global__ void zero_counter_kernel(uint32_t *c) { *c = 0u; }

template <typename R, int CTRL, bool NOISY, int BLOCK>
static hipError_t launch_batch_t(const BatchLaunch &b, hipStream_t s)
{
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, b.counter);
    hipLaunchKernelGGL((batch_kernel<R, CTRL, NOISY, BLOCK>), dim3(b.grid), dim3(BLOCK), 0, s, b.arms, b.items,
                       b.n_items, b.counter);
    return hipGetLastError();
}

template <typename R, int CTRL, bool NOISY>
static hipError_t launch_batch_b(const BatchLaunch &b, hipStream_t s)
{
    switch (b.block) {
    case 64: return launch_batch_t<R, CTRL, NOISY, 64>(b, s);
    case 128: return launch_batch_t<R, CTRL, NOISY, 128>(b, s);
    case 256: return launch_batch_t<R, CTRL, NOISY, 256>(b, s);
    case 512: return launch_batch_t<R, CTRL, NOISY, 512>(b, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
static hipError_t launch_batch_r(const BatchLaunch &b, hipStream_t s)
{
    if (b.ctrl == kCtrlPid)
        return b.noisy ? launch_batch_b<R, kCtrlPid, true>(b, s) : launch_batch_b<R, kCtrlPid, false>(b, s);
    return b.noisy ? launch_batch_b<R, kCtrlOpen, true>(b, s) : launch_batch_b<R, kCtrlOpen, false>(b, s);
}

hipError_t launch_batch(const BatchLaunch &b, hipStream_t s)
{
    return b.precision == 1 ? launch_batch_r<float>(b, s) : launch_batch_r<double>(b, s);
}

template <typename R, int CTRL, bool NOISY, int BLOCK>
static int resident_t()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<R, CTRL, NOISY, BLOCK>, BLOCK, 0) !=
        hipSuccess)
        return 0;
    return per_cu;
}

template <typename R, int CTRL, bool NOISY>
static int resident_b(int block)
{
    switch (block) {
    case 64: return resident_t<R, CTRL, NOISY, 64>();
    case 128: return resident_t<R, CTRL, NOISY, 128>();
    case 256: return resident_t<R, CTRL, NOISY, 256>();
    case 512: return resident_t<R, CTRL, NOISY, 512>();
    default: return 0;
    }
}

int batch_blocks_per_cu(int precision, int ctrl, bool noisy, int block)
{
    if (precision == 1) {
        if (ctrl == kCtrlPid)
            return noisy ? resident_b<float, kCtrlPid, true>(block) : resident_b<float, kCtrlPid, false>(block);
        return noisy ? resident_b<float, kCtrlOpen, true>(block) : resident_b<float, kCtrlOpen, false>(block);
    }
    if (ctrl == kCtrlPid)
        return noisy ? resident_b<double, kCtrlPid, true>(block) : resident_b<double, kCtrlPid, false>(block);
    return noisy ? resident_b<double, kCtrlOpen, true>(block) : resident_b<double, kCtrlOpen, false>(block);
}

template <typename R, int CTRL, bool NOISY, int OUT>
static void launch_sim_o(const SimArgs &a, hipStream_t s)
{
    if (CTRL == kCtrlMlp) {
        const unsigned nb = (unsigned)((a.n + kPartBlock - 1) / kPartBlock);
        int32_t *counts = policy_counts(a);
        hipLaunchKernelGGL((policy_count_kernel<R>), dim3(nb), dim3(kPartBlock), 0, s, a, counts);
        hipLaunchKernelGGL(policy_scan_kernel, dim3(1), dim3(kPartBlock), 0, s, counts, (int32_t)nb);
        hipLaunchKernelGGL((policy_scatter_kernel<R>), dim3(nb), dim3(kPartBlock), 0, s, a, (const int32_t *)counts,
                           (int32_t *)a.order);
        // persistent grid: every resident workgroup, but no more waves than there can be items
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        constexpr int PB = policy_block<R, OUT>();
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, simulate_policy_kernel<R, NOISY, OUT>, PB, 0) !=
            hipSuccess)
            per_cu = 1;
        const int64_t need = (a.n + PB / 64 - 1) / (PB / 64);
        const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * std::max(1, per_cu)));
        hipLaunchKernelGGL((simulate_policy_kernel<R, NOISY, OUT>), dim3(blocks), dim3(PB), 0, s, a,
                           (const int32_t *)counts, (int32_t)nb, (uint32_t *)(counts + nb + 1));
    } else {
        constexpr int B = sim_block<OUT>();
        const unsigned blocks = (unsigned)((a.n + B - 1) / B);
        hipLaunchKernelGGL((simulate_kernel<R, CTRL, NOISY, OUT>), dim3(blocks), dim3(B), 0, s, a);
    }
}

template <typename R, int CTRL, bool NOISY>
static void launch_sim_n(const SimArgs &a, hipStream_t s)
{
    const bool traj = a.traj != nullptr && a.n_traj > 0;
    const bool rec = a.record != nullptr;
    if (a.pop_sum) {   // not combined with traj / record (checked by the ABI)
        hipLaunchKernelGGL(popbg_init_kernel, dim3(256), dim3(256), 0, s, a.pop_sum, a.pop_min, a.pop_max, a.pop_hist,
                           a.pop_nonfinite, a.K);
        launch_sim_o<R, CTRL, NOISY, kOutPop>(a, s);
        return;
    }
    if (CTRL == kCtrlMpc || CTRL == kCtrlMlp) {
        if (rec) {
            if (traj)
                launch_sim_o<R, CTRL, NOISY, kOutTraj | kOutRecord>(a, s);
            else
                launch_sim_o<R, CTRL, NOISY, kOutRecord>(a, s);
            return;
        }
    }
    if (traj)
        launch_sim_o<R, CTRL, NOISY, kOutTraj>(a, s);
    else
        launch_sim_o<R, CTRL, NOISY, 0>(a, s);
}

template <typename R, int CTRL>
static hipError_t launch_sim_t(const SimArgs &a, bool noisy, hipStream_t s)
{
    if (noisy)
        launch_sim_n<R, CTRL, true>(a, s);
    else
        launch_sim_n<R, CTRL, false>(a, s);
    return hipGetLastError();
}

// The extended model (glucagon and exercise states): the noise is always drawn (zero noise
// scales give the noise-free run exactly); trajectories optional.
template <typename R, int CTRL>
static hipError_t launch_sim_ext(const SimArgs &a, hipStream_t s)
{
    if (a.traj != nullptr && a.n_traj > 0)
        launch_sim_o<R, CTRL, true, kOutTraj>(a, s);
    else
        launch_sim_o<R, CTRL, true, 0>(a, s);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_sim_r(const SimArgs &a, bool noisy, hipStream_t s)
{
    if (a.ext) {
        switch (a.ctrl) {
        case kCtrlDual: return launch_sim_ext<R, kCtrlDual>(a, s);
        case kCtrlPid: return launch_sim_ext<R, kCtrlPidExt>(a, s);
        default: return launch_sim_ext<R, kCtrlOpenExt>(a, s);
        }
    }
    switch (a.ctrl) {
    case kCtrlPid: return launch_sim_t<R, kCtrlPid>(a, noisy, s);
    case kCtrlMpc: return launch_sim_t<R, kCtrlMpc>(a, noisy, s);
    case kCtrlMlp: return launch_sim_t<R, kCtrlMlp>(a, noisy, s);
    default: return launch_sim_t<R, kCtrlOpen>(a, noisy, s);
    }
}

hipError_t launch_simulate(const SimArgs &a, int precision, hipStream_t s)
{
    const bool noisy = a.sig_sqh != 0.0 || a.sqrt_r != 0.0;
    return precision == 1 ? launch_sim_r<float>(a, noisy, s) : launch_sim_r<double>(a, noisy, s);
}

}  // namespace vct
