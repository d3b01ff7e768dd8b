// mpc_setup.hip -- FP64 per-patient setup of the linear MPC (one patient per lane).
//
// For each patient: the Jacobian of the drift at the basal state (x_ss, u_b, D = 0),
// discretised the way the plant is integrated (M = I + hJ, A = M^E, B and E the matching
// sums over E Euler steps); the stationary Kalman gain for the sensor state from a fixed
// number of Riccati iterations, Q = 1e-6 I + sigma^2 h E e_Q1 e_Q1^T, R = max(R_cgm, 1e-4);
// the prediction of G = Q1/VG over 24 samples (Markov parameters h, free response F,
// intake response w) condensed into Gamma^T F, Gamma^T w, Gamma^T 1; and the projected-
// gradient step 1/(lambda_max(Gamma^T Gamma) + rho/u_b^2) with lambda from power
// iteration; and the horizon means of the prediction rows and of the intake response. The matrices live in per-lane private arrays: this kernel runs once per trial.
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

    // Kalman: prior covariance P <- A (P - P c c^T P / (c P c^T + R)) A^T + Q with c = e_GI
    const double Rk = a.cgm_var > 1e-4 ? a.cgm_var : 1e-4;
    const double qq1 = a.sigma_q1 * a.sigma_q1 * h * a.em_per_ctrl;
    double P[NX * NX], T[NX * NX];
    for (int i = 0; i < NX * NX; ++i)
        P[i] = 0.0;
    for (int i = 0; i < NX; ++i)
        P[i * NX + i] = 1e-6;
    P[kXQ1 * NX + kXQ1] += qq1;
    for (int it = 0; it < a.riccati_iters; ++it) {
        const double s = P[kXGI * NX + kXGI] + Rk;
        for (int r = 0; r < NX; ++r)
            for (int c = 0; c < NX; ++c)
                T[r * NX + c] = P[r * NX + c] - P[r * NX + kXGI] * P[kXGI * NX + c] / s;
        mat_mul(A, T, T);
        // P = T A^T + Q
        for (int r = 0; r < NX; ++r)
            for (int c = 0; c < NX; ++c) {
                double acc = 0.0;
                for (int q = 0; q < NX; ++q)
                    acc = fma(T[r * NX + q], A[c * NX + q], acc);
                P[r * NX + c] = acc + (r == c ? 1e-6 : 0.0) + (r == kXQ1 && c == kXQ1 ? qq1 : 0.0);
            }
    }
    const double sk = P[kXGI * NX + kXGI] + Rk;

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
        W(kMK + i, P[i * NX + kXGI] / sk);
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

hipError_t launch_mpc_setup(const MpcSetupArgs &a, int precision, void *out, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.n + 63) / 64);
    if (precision == 1)
        hipLaunchKernelGGL(mpc_setup_kernel<float>, dim3(blocks), dim3(64), 0, s, a, (float *)out);
    else
        hipLaunchKernelGGL(mpc_setup_kernel<double>, dim3(blocks), dim3(64), 0, s, a, (double *)out);
    return hipGetLastError();
}

}  // namespace vct
