// mpc_setup.hip -- FP64 per-patient setup of the linear MPC (one patient per lane).
//
// For each patient: the Jacobian of the drift at the basal state (x_ss, u_b, D = 0),
// discretised the way the plant is integrated (M = I + hJ, A = M^E, B and E the matching
// sums over E Euler steps); the stationary Kalman gain for the sensor state from a fixed
// number of Riccati iterations, Q = 1e-6 I + sigma^2 h E e_Q1 e_Q1^T, R = max(R_cgm, 1e-4);
// the prediction of G = Q1/VG over 24 samples (Markov parameters h, free response F,
// intake response w) condensed into Gamma^T F, Gamma^T w, Gamma^T 1; and the projected-
// gradient step 1/(lambda_max(Gamma^T Gamma) + rho/u_b^2) with lambda from power
// iteration; and the horizon means of the prediction rows and of the intake response.
// mpc_setup_kernel does all of it except the Kalman gain, one patient per lane with the
// matrices in private arrays, and hands A over in FP64. The Riccati iteration, 500 steps of
// two 11x11 products, runs in mpc_riccati_kernel with one patient per 16-lane row: lane r
// holds row r of A and of P, and the rows another lane needs are broadcast inside the row
// with DPP (row_newbcast), so the matrices stay in registers.
#include <utility>

#include "internal.hpp"
#include "mpc.hpp"

namespace vct {

namespace {

constexpr int NX = kNx;

__device__ void mat_mul(const double *X, const double *Y, double *Z)   // Z may alias X or Y
{
    double T[NX * NX];
    for (int r = 0; r < NX; ++r)
        for (int c = 0; c < NX; ++c) {
            double acc = 0.0;
            for (int q = 0; q < NX; ++q)
                acc = fma(X[r * NX + q], Y[q * NX + c], acc);
            T[r * NX + c] = acc;
        }
    for (int i = 0; i < NX * NX; ++i)
        Z[i] = T[i];
}

}  // namespace

template <typename R>
__global__ __launch_bounds__(64) void mpc_setup_kernel(const MpcSetupArgs a, R *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n)
        return;
    const int64_t n = a.n;
    double p[15];
    for (int q = 0; q < 15; ++q)
        p[q] = a.params[(int64_t)q * n + j];
    const double ub = a.params[(int64_t)kUb * n + j];
    const double I = a.params[(int64_t)kIstar * n + j];
    if (!(ub > 0.0)) {   // no basal state: a controller that holds nothing (the plant is NaN anyway)
        for (int r = 0; r < kMRows; ++r)
            out[(int64_t)r * n + j] = R(0);
        for (int i = 0; i < NX * NX; ++i)
            a.a64[(int64_t)i * n + j] = 0.0;
        return;
    }
    const double bw = p[kBW];
    const double egp0 = p[kEGP0] * bw, vi = p[kVI] * bw, vg = p[kVG] * bw;
    const double tg = p[kTmaxG], ti = p[kTmaxI];
    const double h = a.h;
    // basal state (unscaled)
    const double x1 = p[kSIT] * I, x2 = p[kSID] * I, x3 = p[kSIE] * I;
    const double q1 = a.g_target * vg, q2 = q1 * x1 / (p[kK12] + x2);

    // Jacobian at the basal state; G* between 4.5 and 9 is not assumed
    double M[NX * NX];
    for (int i = 0; i < NX * NX; ++i)
        M[i] = 0.0;
    const double G = a.g_target;
    M[kXD1 * NX + kXD1] = -1.0 / tg;
    M[kXD2 * NX + kXD1] = 1.0 / tg;
    M[kXD2 * NX + kXD2] = -1.0 / tg;
    M[kXS1 * NX + kXS1] = -1.0 / ti;
    M[kXS2 * NX + kXS1] = 1.0 / ti;
    M[kXS2 * NX + kXS2] = -1.0 / ti;
    M[kXI * NX + kXS2] = 1.0 / (ti * vi);
    M[kXI * NX + kXI] = -p[kKe];
    M[kXx1 * NX + kXI] = p[kKa1] * p[kSIT];
    M[kXx1 * NX + kXx1] = -p[kKa1];
    M[kXx2 * NX + kXI] = p[kKa2] * p[kSID];
    M[kXx2 * NX + kXx2] = -p[kKa2];
    M[kXx3 * NX + kXI] = p[kKa3] * p[kSIE];
    M[kXx3 * NX + kXx3] = -p[kKa3];
    M[kXQ1 * NX + kXD2] = 1.0 / tg;
    M[kXQ1 * NX + kXx1] = -q1;
    M[kXQ1 * NX + kXx3] = x3 < 1.0 ? -egp0 : 0.0;
    M[kXQ1 * NX + kXQ1] = -x1 - (G < 4.5 ? p[kF01] * bw / (4.5 * vg) : 0.0) - (G > 9.0 ? 0.003 : 0.0);
    M[kXQ1 * NX + kXQ2] = p[kK12];
    M[kXQ2 * NX + kXx1] = q1;
    M[kXQ2 * NX + kXx2] = -q2;
    M[kXQ2 * NX + kXQ1] = x1;
    M[kXQ2 * NX + kXQ2] = -(p[kK12] + x2);
    M[kXGI * NX + kXQ1] = 1.0 / (a.tau * vg);
    M[kXGI * NX + kXGI] = -1.0 / a.tau;
    // M = I + h J
    for (int i = 0; i < NX * NX; ++i)
        M[i] *= h;
    for (int i = 0; i < NX; ++i)
        M[i * NX + i] += 1.0;

    // A = M^E and Bsum/Esum = h * (I + M + ... + M^(E-1)) applied to e_S1 / AG e_D1
    double A[NX * NX], Bv[NX], Ev[NX];
    for (int i = 0; i < NX * NX; ++i)
        A[i] = 0.0;
    for (int i = 0; i < NX; ++i) {
        A[i * NX + i] = 1.0;
        Bv[i] = 0.0;
        Ev[i] = 0.0;
    }
    for (int e = 0; e < a.em_per_ctrl; ++e) {
        for (int r = 0; r < NX; ++r) {
            Bv[r] += h * A[r * NX + kXS1];
            Ev[r] += h * a.ag * A[r * NX + kXD1];
        }
        mat_mul(A, M, A);
    }

    // A for the Kalman gain (mpc_riccati_kernel)
    for (int i = 0; i < NX * NX; ++i)
        a.a64[(int64_t)i * n + j] = A[i];

    // prediction rows c_G A^(j+1); Markov parameters h_(j+1) = c_G A^j B; intake response c_G A^j E
    double row[NX], hm[kMpcN], wm[kMpcN];
    for (int i = 0; i < NX; ++i)
        row[i] = i == kXQ1 ? 1.0 / vg : 0.0;
    double Fm[kMpcN * NX];
    for (int jj = 0; jj < kMpcN; ++jj) {
        double hb = 0.0, we = 0.0;
        for (int i = 0; i < NX; ++i) {
            hb = fma(row[i], Bv[i], hb);
            we = fma(row[i], Ev[i], we);
        }
        hm[jj] = hb;
        wm[jj] = we;
        double nr[NX];
        for (int c = 0; c < NX; ++c) {
            double acc = 0.0;
            for (int q = 0; q < NX; ++q)
                acc = fma(row[q], A[q * NX + c], acc);
            nr[c] = acc;
        }
        for (int c = 0; c < NX; ++c) {
            row[c] = nr[c];
            Fm[jj * NX + c] = nr[c];
        }
    }
    // lambda_max(Gamma^T Gamma): power iteration from the all-ones direction
    double v[kMpcN], t[kMpcN], lam = 0.0;
    for (int i = 0; i < kMpcN; ++i)
        v[i] = 1.0 / sqrt((double)kMpcN);
    for (int it = 0; it < a.power_iters; ++it) {
        for (int jj = 0; jj < kMpcN; ++jj) {
            double acc = 0.0;
            for (int i = 0; i <= jj; ++i)
                acc = fma(hm[jj - i], v[i], acc);
            t[jj] = acc;
        }
        double nrm = 0.0;
        for (int i = 0; i < kMpcN; ++i) {
            double acc = 0.0;
            for (int jj = i; jj < kMpcN; ++jj)
                acc = fma(hm[jj - i], t[jj], acc);
            v[i] = acc;
            nrm = fma(acc, acc, nrm);
        }
        nrm = sqrt(nrm);
        lam = nrm;
        if (nrm > 0.0)
            for (int i = 0; i < kMpcN; ++i)
                v[i] /= nrm;
    }
    const double rho_p = a.rho / (ub * ub);

    // write (Gamma^T F, Gamma^T w, Gamma^T 1 folded here)
    auto W = [&](int row_, double val) { out[(int64_t)row_ * n + j] = R(val); };
    for (int i = 0; i < NX * NX; ++i)
        W(kMA + i, A[i]);
    for (int i = 0; i < NX; ++i) {
        W(kMB + i, Bv[i]);
        W(kME + i, Ev[i]);
    }
    for (int i = 0; i < kMpcN; ++i) {
        double gd = 0.0, g1 = 0.0;
        double gx[NX];
        for (int c = 0; c < NX; ++c)
            gx[c] = 0.0;
        for (int jj = i; jj < kMpcN; ++jj) {
            const double gji = hm[jj - i];
            for (int c = 0; c < NX; ++c)
                gx[c] = fma(gji, Fm[jj * NX + c], gx[c]);
            gd = fma(gji, wm[jj], gd);
            g1 += gji;
        }
        for (int c = 0; c < NX; ++c)
            W(kMGx + i * NX + c, gx[c]);
        W(kMgd + i, gd);
        W(kMg1 + i, g1);
        W(kMh + i, hm[i]);
    }
    W(kMstep, 1.0 / (lam + rho_p));
    W(kMrho, rho_p);
    W(kMgi, a.g_target);
    W(kMub, ub);
    W(kMumax, a.umax_rel * ub);
    // horizon means of the free-response rows and of the intake response: the learned
    // controller's insulin and meal inputs are the mean glucose changes they predict
    for (int c = 0; c < NX; ++c) {
        double acc = 0.0;
        for (int jj = 0; jj < kMpcN; ++jj)
            acc += Fm[jj * NX + c];
        W(kMFbar + c, acc / kMpcN);
    }
    double wacc = 0.0;
    for (int jj = 0; jj < kMpcN; ++jj)
        wacc += wm[jj];
    W(kMwbar, wacc / kMpcN);
}

// Lane Q's value of v, for every lane of its 16-lane row (DPP row_newbcast).
template <int Q>
__device__ __forceinline__ double row_bcast(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x150 + Q, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x150 + Q, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
// out[c] = row Q of the matrix whose rows the lanes 0..10 of this row hold in v
template <int Q>
__device__ __forceinline__ void row_of(const double v[NX], double out[NX])
{
#pragma unroll
    for (int c = 0; c < NX; ++c)
        out[c] = row_bcast<Q>(v[c]);
}

// U += A[r][Q] T[Q][:] (row Q of T broadcast); called for Q = 0, 1, ..., 10 in order
template <int Q>
__device__ __forceinline__ void u_term(const double Ar[NX], const double Tr[NX], double Ur[NX])
{
    double t[NX];
    row_of<Q>(Tr, t);
#pragma unroll
    for (int c = 0; c < NX; ++c)
        Ur[c] = fma(Ar[Q], t[c], Ur[c]);
}
template <int... Q>
__device__ __forceinline__ void u_product(std::integer_sequence<int, Q...>, const double Ar[NX], const double Tr[NX],
                                          double Ur[NX])
{
    (u_term<Q>(Ar, Tr, Ur), ...);
}

// (U A^T)[Q][r]: row Q of U (broadcast) with this lane's row r of A
template <int Q>
__device__ __forceinline__ void p_entry(const double Ur[NX], const double Ar[NX], double Pc[NX])
{
    double u[NX];
    row_of<Q>(Ur, u);
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q)
        acc = fma(u[q], Ar[q], acc);
    Pc[Q] = acc;
}
template <int... Q>
__device__ __forceinline__ void p_column(std::integer_sequence<int, Q...>, const double Ur[NX], const double Ar[NX],
                                         double Pc[NX])
{
    (p_entry<Q>(Ur, Ar, Pc), ...);
}

// Kalman prior covariance P <- A (P - P c c^T P / (c P c^T + R)) A^T + Q with c = e_GI, from
// P0 = Q, a fixed number of steps; gain K = P c / (c P c^T + R). One patient per 16-lane row,
// lane r < 11 holding row r of A and of P (lanes 11..15 and rows past n carry zeros and write
// nothing; every lane takes part in the broadcasts). Per step: T = P - P c c^T P / s (row
// GI broadcast), U = A T (lane r combines the broadcast rows of T along its row of A), and
// P = U A^T + Q computed by columns (lane r combines the broadcast rows of U with its row of
// A, giving column r of P). P is symmetric up to rounding, so column r serves as row r of
// the next step; every product sums its terms in the same order as the plain row-by-row
// products.
template <typename R>
__global__ __launch_bounds__(256) void mpc_riccati_kernel(const MpcSetupArgs a, R *__restrict__ out)
{
    const int64_t n = a.n;
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int r = threadIdx.x & 15;
    const bool in = j < n && r < NX;
    const double ub = j < n ? a.params[(int64_t)kUb * n + j] : 0.0;
    double Ar[NX], Pr[NX];
    const double h = a.h;
    const double Rk = a.cgm_var > 1e-4 ? a.cgm_var : 1e-4;
    const double qq1 = a.sigma_q1 * a.sigma_q1 * h * a.em_per_ctrl;
#pragma unroll
    for (int c = 0; c < NX; ++c) {
        Ar[c] = in ? a.a64[(int64_t)(r * NX + c) * n + j] : 0.0;
        Pr[c] = (in && r == c ? 1e-6 : 0.0) + (in && r == kXQ1 && c == kXQ1 ? qq1 : 0.0);
    }
    for (int it = 0; it < a.riccati_iters; ++it) {
        double g[NX], Tr[NX], Ur[NX];
        row_of<kXGI>(Pr, g);   // row GI of P
        const double s = g[kXGI] + Rk;
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            Tr[c] = Pr[c] - Pr[kXGI] * g[c] / s;
            Ur[c] = 0.0;
        }
        // U = A T, then column r of P = U A^T + Q
        u_product(std::make_integer_sequence<int, NX>{}, Ar, Tr, Ur);
        p_column(std::make_integer_sequence<int, NX>{}, Ur, Ar, Pr);
#pragma unroll
        for (int q = 0; q < NX; ++q)
            Pr[q] = Pr[q] + (in && q == r ? 1e-6 : 0.0) + (in && q == kXQ1 && r == kXQ1 ? qq1 : 0.0);
    }
    // K = P e_GI / (P[GI][GI] + R): column GI of P, which lane GI holds
    if (in && r == kXGI && ub > 0.0) {
        const double sk = Pr[kXGI] + Rk;
#pragma unroll
        for (int i = 0; i < NX; ++i)
            out[(int64_t)(kMK + i) * n + j] = R(Pr[i] / sk);
    }
}

hipError_t launch_mpc_setup(const MpcSetupArgs &a, int precision, void *out, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.n + 63) / 64);
    const unsigned rblocks = (unsigned)((a.n + 15) / 16);
    if (precision == 1) {
        hipLaunchKernelGGL(mpc_setup_kernel<float>, dim3(blocks), dim3(64), 0, s, a, (float *)out);
        hipLaunchKernelGGL(mpc_riccati_kernel<float>, dim3(rblocks), dim3(256), 0, s, a, (float *)out);
    } else {
        hipLaunchKernelGGL(mpc_setup_kernel<double>, dim3(blocks), dim3(64), 0, s, a, (double *)out);
        hipLaunchKernelGGL(mpc_riccati_kernel<double>, dim3(rblocks), dim3(256), 0, s, a, (double *)out);
    }
    return hipGetLastError();
}

}  // namespace vct
