// model.hpp -- patient model of the simulation kernels (gfx950).
//
// Sec. IV-B of the paper: the Hovorka core model extended with a one-state model of
// the measured glucose. Drift f (Sec. III-A eq. 1), units min, mmol, mU, L:
//   G = Q1/VG,  U_G = D2/tmaxG,  U_I = S2/tmaxI,
//   F01c = F01 min(1, G/4.5),  F_R = 0.003 max(0, G - 9) VG,  EGP = EGP0 max(0, 1 - x3),
//   dD1 = AG D - D1/tmaxG,   dD2 = (D1 - D2)/tmaxG,
//   dS1 = u - S1/tmaxI,      dS2 = (S1 - S2)/tmaxI,     dI = U_I/VI - ke I,
//   dx_j = ka_j (S_j I - x_j), S_1..3 = SIT, SID, SIE,
//   dQ1 = -F01c - x1 Q1 + k12 Q2 - F_R + U_G + EGP,   dQ2 = x1 Q1 - (k12 + x2) Q2,
//   dGI = (G - GI)/tau_CGM,
// with diffusion sigma on Q1 only. One Euler-Maruyama step x <- x + h f(x) + sqrt(h) sigma xi
// is written in "decay" form (x (1 - h a) + h b for the linear states) on rescaled states
// so that most states cost one FMA; all reciprocals are precomputed once per patient, so
// the loop has no divides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vct {

// Pointers read from the argument structs are generic; casting them to the global address
// space lets the compiler emit global (not flat) loads, which do not share the LDS wait
// counter and can take a scalar base.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *as_global(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
// min(max(x, lo), hi) for lo <= hi. In FP32 this is one v_med3_f32: the median of x, lo
// and hi is the clamp when lo <= hi, and a NaN x gives lo in both forms (the instruction
// then returns the smallest of the other two). Every caller has lo <= hi.
__device__ __forceinline__ float vclamp(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double vclamp(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }
__device__ __forceinline__ float fmaf_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaf_t(double a, double b, double c) { return fma(a, b, c); }

// Row order of the FP64 population buffer (SoA [row][patient]).
enum : int {
    kEGP0 = 0, kF01, kK12, kKa1, kKa2, kKa3, kSIT, kSID, kSIE, kKe, kVI, kVG, kTmaxI, kTmaxG, kBW,
    kUb = 15, kIstar = 16, kAttempts = 17, kStatus = 18, kRows = 19
};

enum : uint32_t { kStNonFinite = 1u, kStNegQ1 = 2u, kStResample = 4u };

// Several states are carried pre-multiplied by the coefficient through which they act
// on the next state, so that each linear update is a single FMA:
//   D1s = (h/tmaxG) D1,  S1s = (h/(tmaxI VI)) (h/tmaxI) S1,  S2s = (h/(tmaxI VI)) S2,
//   x1h = h x1,  x2s = x2 / (h ka2 SID),  e3 = h EGP0 (1 - x3),  GIs = GI (tau VG)/h,
// e3 being exactly the factor through which x3 acts on EGP. x2s is scaled so that its own
// update is one FMA (x2s' = (1 - h ka2) x2s + I); where it acts on Q2, the factor
// 1 - h k12 - h x2 = (1 - h k12) - (h^2 ka2 SID) x2s is one FMA per step and is not carried
// as a state (that sum is ~0.93 while h x2 is ~0.004, and FP32 would keep only four digits
// of x2).
// Unscaled values are recovered only where they are observed (G at the samples, GI for
// the sensor).
template <typename R> struct State {
    R D1s, D2, S1s, S2s, I, x1h, x2s, e3, Q1, Q2, GIs;
};

// Per-patient constants of the EM step; everything that multiplies h is prescaled.
template <typename R> struct StepConst {
    R a_g, b_g;        // 1 - h/tmaxG, h/tmaxG
    R a_i;             // 1 - h/tmaxI
    R a_e;             // 1 - h ke
    R a1, hb1;         // 1 - h ka1, h^2 ka1 SIT                     (x1h update)
    R a2, hb2;         // 1 - h ka2, h^2 ka2 SID                     (x2s update; h x2 = hb2 x2s)
    R a3, b3e, c3;     // 1 - h ka3, h EGP0 h ka3 SIE, h EGP0 h ka3 (e3 update)
    R a_12, hk12;      // 1 - h k12, h k12
    R f01h, f01h_q;    // h F01, h F01/(4.5 VG)      (h F01c = min(h F01, Q1 h F01/(4.5 VG)))
    R fr1, fr0;        // 0.003 h, 0.027 h VG        (h F_R = max(0, Q1 fr1 - fr0))
    R a_c;             // 1 - h/tau
    R inv_vg;          // 1/VG, for G at the sampling instants
    R gi_scale;        // h/(tau VG): GI = gi_scale GIs
    R u_in, d_in;      // held inputs -> increments: h^2/(tmaxI^2 VI) per mU/min, h^2 AG/tmaxG per mmol/min
};

// x(t0) = basal steady state at G* (closed form of the quadratic in I; see population kernel).
template <typename R>
__device__ __forceinline__ void basal_state(const double *p, double I, double ub, double g_target, double h,
                                            double tau, State<R> &s)
{
    const double vg = p[kVG] * p[kBW], vi = p[kVI] * p[kBW], ti = p[kTmaxI];
    const double x1 = p[kSIT] * I, x2 = p[kSID] * I, x3 = p[kSIE] * I;
    const double q1 = g_target * vg;
    const double c_ui = h / (ti * vi), b_i = h / ti;
    s.D1s = R(0);
    s.D2 = R(0);
    s.S1s = R(c_ui * b_i * ub * ti);
    s.S2s = R(c_ui * ub * ti);
    s.I = R(I);
    s.x1h = R(h * x1);
    s.x2s = R(I / (h * p[kKa2]));   // x2 / (h ka2 SID) with x2 = SID I
    s.e3 = R(h * p[kEGP0] * p[kBW] * (1.0 - x3));
    s.Q1 = R(q1);
    s.Q2 = R(q1 * x1 / (p[kK12] + x2));
    s.GIs = R(g_target * tau * vg / h);
}

template <typename R>
__device__ __forceinline__ void step_constants(const double *p, double h, double tau, double ag, StepConst<R> &c)
{
    const double bw = p[kBW];
    const double vi = p[kVI] * bw, vg = p[kVG] * bw;
    const double tg = p[kTmaxG], ti = p[kTmaxI];
    c.a_g = R(1.0 - h / tg);
    c.b_g = R(h / tg);
    c.a_i = R(1.0 - h / ti);
    c.a_e = R(1.0 - h * p[kKe]);
    c.a1 = R(1.0 - h * p[kKa1]);
    c.hb1 = R(h * h * p[kKa1] * p[kSIT]);
    c.a2 = R(1.0 - h * p[kKa2]);
    c.hb2 = R(h * h * p[kKa2] * p[kSID]);
    const double egp0h = h * p[kEGP0] * bw;
    c.a3 = R(1.0 - h * p[kKa3]);
    c.b3e = R(egp0h * h * p[kKa3] * p[kSIE]);
    c.c3 = R(egp0h * h * p[kKa3]);
    c.a_12 = R(1.0 - h * p[kK12]);
    c.hk12 = R(h * p[kK12]);
    c.f01h = R(h * p[kF01] * bw);
    c.f01h_q = R(h * p[kF01] * bw / (4.5 * vg));
    c.fr1 = R(0.003 * h);
    c.fr0 = R(0.027 * h * vg);
    c.a_c = R(1.0 - h / tau);
    c.inv_vg = R(1.0 / vg);
    c.gi_scale = R(h / (tau * vg));
    c.u_in = R((h / (ti * vi)) * (h / ti) * h);
    c.d_in = R((h / tg) * h * ag);
}

// One EM step. du = u_in u and dd = d_in D are the held inputs of the sampling interval in
// the scaled coordinates; dq = sqrt(h) sigma xi is this step's increment of Q1. Every
// right-hand side uses the pre-step state.
template <typename R>
__device__ __forceinline__ void em_step(State<R> &s, const StepConst<R> &c, R du, R dd, R dq)
{
    const R t = s.x1h * s.Q1;                                       // h x1 Q1
    // terms that do not depend on Q1 first, so the Q1 chain of each step is short
    R side = fmaf_t(c.hk12, s.Q2, dq);                              // h k12 Q2 + noise
    side = fmaf_t(s.D2, c.b_g, side);                               //   + h U_G
    side = side + vmax(R(0), s.e3);                                 //   + h EGP
    const R hf01c = vmin(c.f01h, s.Q1 * c.f01h_q);                   // h F01c
    const R hfr = vmax(R(0), fmaf_t(s.Q1, c.fr1, -c.fr0));           // h F_R
    const R Q1n = ((fmaf_t(-s.x1h, s.Q1, s.Q1) - hf01c) - hfr) + side;
    const R Q2n = fmaf_t(s.Q2, fmaf_t(-c.hb2, s.x2s, c.a_12), t);
    const R GIn = fmaf_t(s.GIs, c.a_c, s.Q1);
    const R D2n = fmaf_t(s.D2, c.a_g, s.D1s);
    const R D1n = fmaf_t(s.D1s, c.a_g, dd);
    const R S2n = fmaf_t(s.S2s, c.a_i, s.S1s);
    const R S1n = fmaf_t(s.S1s, c.a_i, du);
    const R In = fmaf_t(s.I, c.a_e, s.S2s);
    const R x1n = fmaf_t(s.x1h, c.a1, s.I * c.hb1);
    const R x2n = fmaf_t(s.x2s, c.a2, s.I);
    const R e3n = fmaf_t(s.e3, c.a3, fmaf_t(-c.b3e, s.I, c.c3));
    s.D1s = D1n; s.D2 = D2n; s.S1s = S1n; s.S2s = S2n; s.I = In;
    s.x1h = x1n; s.x2s = x2n; s.e3 = e3n; s.Q1 = Q1n; s.Q2 = Q2n; s.GIs = GIn;
}

// ------------------------------------------------------ model extensions ----
// Sec. IV-B extends the model with a two-state subcutaneous glucagon depot and a three-state
// effect of exercise (parameters shared by all patients):
//   dZ1 = u_N - Z1/tau_n,  dZ2 = (Z1 - Z2)/tau_n           (ug; appearance Z2/tau_n ug/min)
//   EGP = EGP0 max(0, 1 - x3) + e_n Z2/tau_n
//   dE1 = (HRR - E1)/tau_e1, dE2 = (E1 - E2)/tau_e2, dE3 = (E1 - E3)/tau_e3
//   Q1 loses alpha_e E2 Q1 (insulin-independent uptake); x1 and x2 act as x_j (1 + beta_e E3).
// The extension states are carried unscaled; each update is one FMA in decay form.
template <typename R> struct ExtState {
    R z1, z2;          // glucagon depot, ug
    R ex1, ex2, ex3;    // exercise: heart rate, uptake, insulin action
};

template <typename R> struct ExtConst {
    R a_n, b_n;          // 1 - h/tau_n, h/tau_n
    R c_n;               // h e_n / tau_n: Q1 increment per ug in Z2
    R a_e1, b_e1;        // 1 - h/tau_e1, h/tau_e1 (b_e1 multiplies HRR)
    R a_e2, b_e2, a_e3, b_e3;
    R h_alpha;           // h alpha_e
    R beta;              // beta_e
};

template <typename R>
__device__ __forceinline__ void ext_constants(double h, double tau_n, double e_n, double tau_e1, double tau_e2,
                                              double tau_e3, double alpha_e, double beta_e, ExtConst<R> &e)
{
    e.a_n = R(1.0 - h / tau_n);
    e.b_n = R(h / tau_n);
    e.c_n = R(h * e_n / tau_n);
    e.a_e1 = R(1.0 - h / tau_e1);
    e.b_e1 = R(h / tau_e1);
    e.a_e2 = R(1.0 - h / tau_e2);
    e.b_e2 = R(h / tau_e2);
    e.a_e3 = R(1.0 - h / tau_e3);
    e.b_e3 = R(h / tau_e3);
    e.h_alpha = R(h * alpha_e);
    e.beta = R(beta_e);
}

// One EM step of the extended model: em_step's update with the glucagon output, the exercise
// uptake and the raised insulin action in the Q1/Q2 balance, then the extension states.
// dn = h u_N (ug into Z1), dh = (h/tau_e1) HRR.
template <typename R>
__device__ __forceinline__ void em_step_ext(State<R> &s, ExtState<R> &x, const StepConst<R> &c, const ExtConst<R> &e,
                                            R du, R dd, R dq, R dn, R dh)
{
    const R gain = fmaf_t(e.beta, x.ex3, R(1));
    const R x1g = s.x1h * gain;                                     // h x1 (1 + beta E3)
    const R t = x1g * s.Q1;
    R side = fmaf_t(c.hk12, s.Q2, dq);
    side = fmaf_t(s.D2, c.b_g, side);
    side = side + vmax(R(0), s.e3);
    side = fmaf_t(e.c_n, x.z2, side);                               //   + h e_n U_N
    const R hf01c = vmin(c.f01h, s.Q1 * c.f01h_q);
    const R hfr = vmax(R(0), fmaf_t(s.Q1, c.fr1, -c.fr0));
    const R Q1n = ((fmaf_t(-fmaf_t(e.h_alpha, x.ex2, x1g), s.Q1, s.Q1) - hf01c) - hfr) + side;
    const R Q2n = fmaf_t(s.Q2, fmaf_t(-c.hb2, s.x2s * gain, c.a_12), t);
    const R GIn = fmaf_t(s.GIs, c.a_c, s.Q1);
    const R D2n = fmaf_t(s.D2, c.a_g, s.D1s);
    const R D1n = fmaf_t(s.D1s, c.a_g, dd);
    const R S2n = fmaf_t(s.S2s, c.a_i, s.S1s);
    const R S1n = fmaf_t(s.S1s, c.a_i, du);
    const R In = fmaf_t(s.I, c.a_e, s.S2s);
    const R x1n = fmaf_t(s.x1h, c.a1, s.I * c.hb1);
    const R x2n = fmaf_t(s.x2s, c.a2, s.I);
    const R e3n = fmaf_t(s.e3, c.a3, fmaf_t(-c.b3e, s.I, c.c3));
    const R z1n = fmaf_t(x.z1, e.a_n, dn);
    const R z2n = fmaf_t(x.z2, e.a_n, x.z1 * e.b_n);
    const R f1n = fmaf_t(x.ex1, e.a_e1, dh);
    const R f2n = fmaf_t(x.ex2, e.a_e2, x.ex1 * e.b_e2);
    const R f3n = fmaf_t(x.ex3, e.a_e3, x.ex1 * e.b_e3);
    s.D1s = D1n; s.D2 = D2n; s.S1s = S1n; s.S2s = S2n; s.I = In;
    s.x1h = x1n; s.x2s = x2n; s.e3 = e3n; s.Q1 = Q1n; s.Q2 = Q2n; s.GIs = GIn;
    x.z1 = z1n; x.z2 = z2n; x.ex1 = f1n; x.ex2 = f2n; x.ex3 = f3n;
}

}  // namespace vct
