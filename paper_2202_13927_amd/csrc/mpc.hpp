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
    kMRows = kMumax + 1
};

// Model state order of the linear model (unscaled deviations).
enum : int { kXD1 = 0, kXD2, kXS1, kXS2, kXI, kXx1, kXx2, kXx3, kXQ1, kXQ2, kXGI };

template <typename R> struct MpcLane {
    R xh[kNx];      // estimate of x - x_ss (prior)
    R dU[kMpcN];    // planned u - u_b
    R h[kMpcN];
    R step, rho_p, lo, hi, gi_ss, ub;
};

template <typename R>
__device__ __forceinline__ void mpc_load(const R *__restrict__ M, int64_t n, int64_t j, MpcLane<R> &L)
{
#pragma unroll
    for (int i = 0; i < kNx; ++i)
        L.xh[i] = R(0);
#pragma unroll
    for (int i = 0; i < kMpcN; ++i) {
        L.dU[i] = R(0);
        L.h[i] = M[(int64_t)(kMh + i) * n + j];
    }
    L.step = M[(int64_t)kMstep * n + j];
    L.rho_p = M[(int64_t)kMrho * n + j];
    L.gi_ss = M[(int64_t)kMgi * n + j];
    L.ub = M[(int64_t)kMub * n + j];
    L.lo = -L.ub;
    L.hi = M[(int64_t)kMumax * n + j] - L.ub;
}

// The controller sample split in three parts, so that a learned policy can act while the
// estimator keeps running: measurement update; plan (QP by projected gradient); time update.
template <typename R>
__device__ __forceinline__ void mpc_measure(const R *__restrict__ M, int64_t n, int64_t j, MpcLane<R> &L, R y)
{
    const R innov = (y - L.gi_ss) - L.xh[kXGI];
#pragma unroll
    for (int i = 0; i < kNx; ++i)
        L.xh[i] = fmaf_t(M[(int64_t)(kMK + i) * n + j], innov, L.xh[i]);
}

// Plan: QP linear term g = Gamma^T (F xh + w dhat + (G* - ybar) 1), warm start from the
// shifted previous plan, `iters` projected-gradient steps. Returns u_0 - u_b.
template <typename R>
__device__ __forceinline__ R mpc_plan(const R *__restrict__ M, int64_t n, int64_t j, MpcLane<R> &L, R dhat, R gofs,
                                      int iters)
{
    R g[kMpcN];
#pragma unroll
    for (int i = 0; i < kMpcN; ++i) {
        R acc = fmaf_t(M[(int64_t)(kMgd + i) * n + j], dhat, M[(int64_t)(kMg1 + i) * n + j] * gofs);
#pragma unroll
        for (int c = 0; c < kNx; ++c)
            acc = fmaf_t(M[(int64_t)(kMGx + i * kNx + c) * n + j], L.xh[c], acc);
        g[i] = acc;
    }
#pragma unroll
    for (int i = 0; i + 1 < kMpcN; ++i)
        L.dU[i] = L.dU[i + 1];
    // projected gradient on 1/2 |Gamma dU|^2 + rho'/2 |dU|^2 + g.dU, lo <= dU <= hi
    for (int it = 0; it < iters; ++it) {
        R r[kMpcN];
#pragma unroll
        for (int jj = 0; jj < kMpcN; ++jj) {
            R acc = R(0);
#pragma unroll
            for (int i = 0; i <= jj; ++i)
                acc = fmaf_t(L.h[jj - i], L.dU[i], acc);
            r[jj] = acc;
        }
#pragma unroll
        for (int i = 0; i < kMpcN; ++i) {
            R acc = fmaf_t(L.rho_p, L.dU[i], g[i]);
#pragma unroll
            for (int jj = i; jj < kMpcN; ++jj)
                acc = fmaf_t(L.h[jj - i], r[jj], acc);
            L.dU[i] = vmin(vmax(fmaf_t(-L.step, acc, L.dU[i]), L.lo), L.hi);
        }
    }
    return L.dU[0];
}

// The plan is not solved this sample (another policy acts): only shift it.
template <typename R>
__device__ __forceinline__ void mpc_shift(MpcLane<R> &L)
{
#pragma unroll
    for (int i = 0; i + 1 < kMpcN; ++i)
        L.dU[i] = L.dU[i + 1];
}

// Time update with the applied input deviation du and the announced intake.
template <typename R>
__device__ __forceinline__ void mpc_predict(const R *__restrict__ M, int64_t n, int64_t j, MpcLane<R> &L, R du, R dhat)
{
    R nx[kNx];
#pragma unroll
    for (int r = 0; r < kNx; ++r) {
        R acc = fmaf_t(M[(int64_t)(kMB + r) * n + j], du, M[(int64_t)(kME + r) * n + j] * dhat);
#pragma unroll
        for (int c = 0; c < kNx; ++c)
            acc = fmaf_t(M[(int64_t)(kMA + r * kNx + c) * n + j], L.xh[c], acc);
        nx[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < kNx; ++r)
        L.xh[r] = nx[r];
}

// One full MPC sample: y is the sensor value, dhat the announced held intake (mmol/min),
// gofs = G* - set point. Returns u.
template <typename R>
__device__ __forceinline__ R mpc_step(const R *__restrict__ M, int64_t n, int64_t j, MpcLane<R> &L, R y, R dhat,
                                      R gofs, int iters)
{
    mpc_measure<R>(M, n, j, L, y);
    const R du = mpc_plan<R>(M, n, j, L, dhat, gofs, iters);
    mpc_predict<R>(M, n, j, L, du, dhat);
    return L.ub + du;
}

}  // namespace vct
