// mpc.hpp -- per-patient linear MPC data layout and the online controller step.
//
// The controller has the sampled form of Sec. III-B: its state is the Kalman estimate of
// the deviation from the basal steady state and the planned input sequence; each sample
// it corrects the estimate with the sensor value, solves a box-constrained QP over the
// next N = 24 samples by projected gradient, applies the first input and predicts.
// Setup (linearised model, stationary Kalman gain, prediction matrices, step length) is
// FP64 and done once per patient by mpc_setup_kernel; the online step runs in the
// kernel's working precision.
#pragma once

#include "model.hpp"

namespace vct {

constexpr int kMpcN = 24;   // prediction = control horizon (samples)
constexpr int kNx = 11;

// Row offsets of the per-patient MPC buffer (SoA: row r of patient j at r * n + j).
enum : int {
    kMA = 0,                       // A[11][11], row-major
    kMB = kMA + kNx * kNx,         // B[11]
    kME = kMB + kNx,               // E[11]: response to a held glucose intake
    kMK = kME + kNx,               // Kalman gain for the sensor state GI
    kMGx = kMK + kNx,              // Gamma^T F, [24][11]
    kMgd = kMGx + kMpcN * kNx,     // Gamma^T w (announced intake)
    kMg1 = kMgd + kMpcN,           // Gamma^T 1 (G* - set point)
    kMh = kMg1 + kMpcN,            // Markov parameters h_1..h_24
    kMstep = kMh + kMpcN,          // 1 / (lambda_max(Gamma^T Gamma) + rho/u_b^2)
    kMrho = kMstep + 1,            // rho / u_b^2
    kMgi = kMrho + 1,              // GI at the basal state (= G*)
    kMub = kMgi + 1,
    kMumax = kMub + 1,
    kMFbar = kMumax + 1,           // mean over the horizon of the prediction rows c_G A^(j+1)
    kMwbar = kMFbar + kNx,         // mean over the horizon of the intake response c_G A^j E
    kMRows = kMwbar + 1
};

// Model state order of the linear model (unscaled deviations).
enum : int { kXD1 = 0, kXD2, kXS1, kXS2, kXI, kXx1, kXx2, kXx3, kXQ1, kXQ2, kXGI };

// Estimator and QP constants of one lane (loop-carried).
// Row r of the per-patient SoA buffer for the patient at lane offset j: a uniform row base
// plus a 32-bit lane offset, which maps to the scalar-base form of the global loads, so no
// per-lane 64-bit address has to be kept for each of the ~80 rows read per sample.
template <typename R>
__device__ __forceinline__ R soa(const R *__restrict__ M, int64_t n, uint32_t j, int r)
{
    const auto row = (const __attribute__((address_space(1))) char *)(as_global(M) + (size_t)r * (size_t)n);
    return *(const __attribute__((address_space(1))) R *)(row + j * (uint32_t)sizeof(R));
}

template <typename R> struct MpcState {
    R xh[kNx];      // estimate of x - x_ss (prior)
    R step, rho_p, lo, hi, gi_ss, ub;
};

// The input plan (planned u - u_b) and the Markov parameters of the prediction.
template <typename R> struct MpcPlan {
    R dU[kMpcN];
    R h[kMpcN];
};

template <typename R>
__device__ __forceinline__ void mpc_load_state(const R *__restrict__ M, int64_t n, int64_t j, MpcState<R> &L)
{
#pragma unroll
    for (int i = 0; i < kNx; ++i)
        L.xh[i] = R(0);
    L.step = soa<R>(M, n, (uint32_t)j, kMstep);
    L.rho_p = soa<R>(M, n, (uint32_t)j, kMrho);
    L.gi_ss = soa<R>(M, n, (uint32_t)j, kMgi);
    L.ub = soa<R>(M, n, (uint32_t)j, kMub);
    L.lo = -L.ub;
    L.hi = soa<R>(M, n, (uint32_t)j, kMumax) - L.ub;
}

template <typename R>
__device__ __forceinline__ void mpc_load_h(const R *__restrict__ M, int64_t n, int64_t j, R h[kMpcN])
{
#pragma unroll
    for (int i = 0; i < kMpcN; ++i)
        h[i] = soa<R>(M, n, (uint32_t)j, kMh + i);
}

// The controller sample in parts, so that a learned policy can act while the estimator keeps
// running: measurement update; QP (linear term, projected gradient); time update.
template <typename R>
__device__ __forceinline__ void mpc_measure(const R *__restrict__ M, int64_t n, int64_t j, MpcState<R> &L, R y)
{
    const R innov = (y - L.gi_ss) - L.xh[kXGI];
#pragma unroll
    for (int i = 0; i < kNx; ++i)
        L.xh[i] = fmaf_t(soa<R>(M, n, (uint32_t)j, kMK + i), innov, L.xh[i]);
}

// The same with the Kalman gain held in registers (kg = rows kMK.. of the patient).
template <typename R>
__device__ __forceinline__ void mpc_measure_gain(const R kg[kNx], MpcState<R> &L, R y)
{
    const R innov = (y - L.gi_ss) - L.xh[kXGI];
#pragma unroll
    for (int i = 0; i < kNx; ++i)
        L.xh[i] = fmaf_t(kg[i], innov, L.xh[i]);
}

// g = Gamma^T (F xh + w dhat + (G* - ybar) 1).
template <typename R>
__device__ __forceinline__ void mpc_linear_term(const R *__restrict__ M, int64_t n, int64_t j, const MpcState<R> &L,
                                                R dhat, R gofs, R g[kMpcN])
{
#pragma unroll
    for (int i = 0; i < kMpcN; ++i) {
        R acc = fmaf_t(soa<R>(M, n, (uint32_t)j, kMgd + i), dhat, soa<R>(M, n, (uint32_t)j, kMg1 + i) * gofs);
#pragma unroll
        for (int c = 0; c < kNx; ++c)
            acc = fmaf_t(soa<R>(M, n, (uint32_t)j, kMGx + i * kNx + c), L.xh[c], acc);
        g[i] = acc;
    }
}

// `iters` projected-gradient steps on 1/2 |Gamma dU|^2 + rho'/2 |dU|^2 + g.dU, lo <= dU <= hi,
// from the start dU (overwritten). Gamma is lower-triangular Toeplitz in h.
template <typename R>
__device__ __forceinline__ void mpc_pg(const MpcState<R> &L, const R h[kMpcN], const R g[kMpcN], R dU[kMpcN],
                                       int iters)
{
    for (int it = 0; it < iters; ++it) {
        // r = Gamma dU, r_jj = sum_{d <= jj} h_d dU_(jj-d), d ascending (the order of the
        // wave-cooperative solver, so that both give identical results)
        R r[kMpcN];
#pragma unroll
        for (int jj = 0; jj < kMpcN; ++jj) {
            R acc = R(0);
#pragma unroll
            for (int d = 0; d <= jj; ++d)
                acc = fmaf_t(h[d], dU[jj - d], acc);
            r[jj] = acc;
        }
#pragma unroll
        for (int i = 0; i < kMpcN; ++i) {
            R acc = fmaf_t(L.rho_p, dU[i], g[i]);
#pragma unroll
            for (int jj = i; jj < kMpcN; ++jj)
                acc = fmaf_t(h[jj - i], r[jj], acc);
            dU[i] = vclamp(fmaf_t(-L.step, acc, dU[i]), L.lo, L.hi);
        }
    }
}

// Warm start: the previous plan moved one sample on (its last entry repeated).
template <typename R>
__device__ __forceinline__ void mpc_shift(R dU[kMpcN])
{
#pragma unroll
    for (int i = 0; i + 1 < kMpcN; ++i)
        dU[i] = dU[i + 1];
}

// Time update. The sample-to-sample model is A = M^E, B = h sum_m M^m e_S1, E = h AG sum_m
// M^m e_D1 with M = I + hJ (E Euler steps of the linearised drift), so A xh + B du + E dhat
// is computed as E steps z <- M z + h e_S1 du + h AG e_D1 dhat, without reading A, B, E.
// M shares most entries with the plant's step constants; the others are below.
template <typename R> struct LinStep {
    R s2s1, is2, x1i, x2i, x3i;   // h/tmaxI, h/(tmaxI VI), h ka_j S_j
    R hq1, q1x3, q1q1;            // h Q1*, -h EGP0 [x3* < 1], 1 + h dQ1'/dQ1
    R q2x2, q2q1, q2q2;           // -h Q2*, h x1*, 1 - h (k12 + x2*)
};

// The Jacobian entries of the setup kernel (basal state at G*, same formulas), times h.
template <typename R>
__device__ __forceinline__ void lin_step_constants(const double *p, double I, double h, double g_target, LinStep<R> &L)
{
    const double bw = p[kBW], vi = p[kVI] * bw, vg = p[kVG] * bw, ti = p[kTmaxI], egp0 = p[kEGP0] * bw;
    const double x1 = p[kSIT] * I, x2 = p[kSID] * I, x3 = p[kSIE] * I;
    const double q1 = g_target * vg, q2 = q1 * x1 / (p[kK12] + x2);
    const double G = g_target;
    L.s2s1 = R(h * (1.0 / ti));
    L.is2 = R(h * (1.0 / (ti * vi)));
    L.x1i = R(h * (p[kKa1] * p[kSIT]));
    L.x2i = R(h * (p[kKa2] * p[kSID]));
    L.x3i = R(h * (p[kKa3] * p[kSIE]));
    L.hq1 = R(h * q1);
    L.q1x3 = R(h * (x3 < 1.0 ? -egp0 : 0.0));
    L.q1q1 = R(1.0 + h * (-x1 - (G < 4.5 ? p[kF01] * bw / (4.5 * vg) : 0.0) - (G > 9.0 ? 0.003 : 0.0)));
    L.q2x2 = R(h * -q2);
    L.q2q1 = R(h * x1);
    L.q2q2 = R(1.0 + h * -(p[kK12] + x2));
}

template <typename R>
__device__ __forceinline__ void mpc_predict(MpcState<R> &L, const StepConst<R> &c, const LinStep<R> &m, R du, R dhat,
                                           R h, R hag, int steps)
{
    R z[kNx];
#pragma unroll
    for (int r = 0; r < kNx; ++r)
        z[r] = L.xh[r];
    const R dS1 = h * du, dD1 = hag * dhat;
    for (int e = 0; e < steps; ++e) {
        R n[kNx];
        n[kXD1] = fmaf_t(c.a_g, z[kXD1], dD1);
        n[kXD2] = fmaf_t(c.b_g, z[kXD1], c.a_g * z[kXD2]);
        n[kXS1] = fmaf_t(c.a_i, z[kXS1], dS1);
        n[kXS2] = fmaf_t(m.s2s1, z[kXS1], c.a_i * z[kXS2]);
        n[kXI] = fmaf_t(m.is2, z[kXS2], c.a_e * z[kXI]);
        n[kXx1] = fmaf_t(m.x1i, z[kXI], c.a1 * z[kXx1]);
        n[kXx2] = fmaf_t(m.x2i, z[kXI], c.a2 * z[kXx2]);
        n[kXx3] = fmaf_t(m.x3i, z[kXI], c.a3 * z[kXx3]);
        n[kXQ1] = fmaf_t(c.hk12, z[kXQ2],
                         fmaf_t(m.q1q1, z[kXQ1], fmaf_t(m.q1x3, z[kXx3], fmaf_t(-m.hq1, z[kXx1], c.b_g * z[kXD2]))));
        n[kXQ2] = fmaf_t(m.q2q2, z[kXQ2], fmaf_t(m.q2q1, z[kXQ1], fmaf_t(m.q2x2, z[kXx2], m.hq1 * z[kXx1])));
        n[kXGI] = fmaf_t(c.gi_scale, z[kXQ1], c.a_c * z[kXGI]);
#pragma unroll
        for (int r = 0; r < kNx; ++r)
            z[r] = n[r];
    }
#pragma unroll
    for (int r = 0; r < kNx; ++r)
        L.xh[r] = z[r];
}

// One full MPC sample: y is the sensor value, dhat the announced held intake (mmol/min),
// gofs = G* - set point. Returns u.
template <typename R>
__device__ __forceinline__ R mpc_step(const R *__restrict__ M, int64_t n, int64_t j, MpcState<R> &L, MpcPlan<R> &P,
                                      const StepConst<R> &c, const LinStep<R> &m, R h, R hag, int steps, R y, R dhat,
                                      R gofs, int iters)
{
    mpc_measure<R>(M, n, j, L, y);
    R g[kMpcN];
    mpc_linear_term<R>(M, n, j, L, dhat, gofs, g);
    mpc_shift<R>(P.dU);
    mpc_pg<R>(L, P.h, g, P.dU, iters);
    const R du = P.dU[0];
    mpc_predict<R>(L, c, m, du, dhat, h, hag, steps);
    return L.ub + du;
}

}  // namespace vct
