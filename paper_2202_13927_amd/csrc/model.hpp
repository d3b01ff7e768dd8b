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
// is written in "decay" form (x (1 - h a) + h b for the linear states) so that every
// state costs one or two VALU instructions; all reciprocals are precomputed once per
// patient, so the loop has no divides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vct {

__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }

// Row order of the FP64 population buffer (SoA [row][patient]).
enum : int {
    kEGP0 = 0, kF01, kK12, kKa1, kKa2, kKa3, kSIT, kSID, kSIE, kKe, kVI, kVG, kTmaxI, kTmaxG, kBW,
    kUb = 15, kIstar = 16, kAttempts = 17, kStatus = 18, kRows = 19
};

enum : uint32_t { kStNonFinite = 1u, kStNegQ1 = 2u, kStResample = 4u };

template <typename R> struct State {
    R D1, D2, S1, S2, I, x1, x2, x3, Q1, Q2, GI;
};

// Per-patient constants of the EM step (already multiplied by h where they are used so).
template <typename R> struct StepConst {
    R a_g, b_g;        // 1 - h/tmaxG, h/tmaxG
    R a_i, b_i;        // 1 - h/tmaxI, h/tmaxI
    R a_e, c_ui;       // 1 - h ke, h/(tmaxI VI)
    R a1, b1, a2, b2, a3, b3;   // 1 - h ka_j, h ka_j S_j
    R a_12, h_k12;     // 1 - h k12, h k12
    R h;               // step, min
    R inv_vg;          // 1/VG (absolute)
    R f01h, f01h_45;   // h F01, h F01/4.5
    R frh;             // h 0.003 VG
    R egp0h;           // h EGP0
    R a_c, b_c;        // 1 - h/tau, h/tau
};

// x(t0) = basal steady state at G* (closed form of the quadratic in I; see population kernel).
template <typename R>
__device__ __forceinline__ void basal_state(const double *p, double I, double ub, double g_target, State<R> &s)
{
    const double vg = p[kVG] * p[kBW];
    const double x1 = p[kSIT] * I, x2 = p[kSID] * I, x3 = p[kSIE] * I;
    const double q1 = g_target * vg;
    s.D1 = R(0);
    s.D2 = R(0);
    s.S1 = R(ub * p[kTmaxI]);
    s.S2 = R(ub * p[kTmaxI]);
    s.I = R(I);
    s.x1 = R(x1);
    s.x2 = R(x2);
    s.x3 = R(x3);
    s.Q1 = R(q1);
    s.Q2 = R(q1 * x1 / (p[kK12] + x2));
    s.GI = R(g_target);
}

template <typename R>
__device__ __forceinline__ void step_constants(const double *p, double h, double ag, double tau, StepConst<R> &c)
{
    const double bw = p[kBW];
    const double vi = p[kVI] * bw, vg = p[kVG] * bw;
    const double tg = p[kTmaxG], ti = p[kTmaxI];
    c.a_g = R(1.0 - h / tg);
    c.b_g = R(h / tg);
    c.a_i = R(1.0 - h / ti);
    c.b_i = R(h / ti);
    c.a_e = R(1.0 - h * p[kKe]);
    c.c_ui = R(h / (ti * vi));
    c.a1 = R(1.0 - h * p[kKa1]);
    c.b1 = R(h * p[kKa1] * p[kSIT]);
    c.a2 = R(1.0 - h * p[kKa2]);
    c.b2 = R(h * p[kKa2] * p[kSID]);
    c.a3 = R(1.0 - h * p[kKa3]);
    c.b3 = R(h * p[kKa3] * p[kSIE]);
    c.a_12 = R(1.0 - h * p[kK12]);
    c.h_k12 = R(h * p[kK12]);
    c.h = R(h);
    c.inv_vg = R(1.0 / vg);
    c.f01h = R(h * p[kF01] * bw);
    c.f01h_45 = R(h * p[kF01] * bw / 4.5);
    c.frh = R(h * 0.003 * vg);
    c.egp0h = R(h * p[kEGP0] * bw);
    c.a_c = R(1.0 - h / tau);
    c.b_c = R(h / tau);
    (void)ag;
}

// One EM step. hu = h u and hagd = h AG D are the held inputs of the current sampling
// interval; dq = sqrt(h) sigma xi is this step's increment of Q1.
template <typename R>
__device__ __forceinline__ void em_step(State<R> &s, const StepConst<R> &c, R hu, R hagd, R dq)
{
    const R G = s.Q1 * c.inv_vg;
    const R hug = s.D2 * c.b_g;                                     // h U_G
    const R hf01c = vmin(c.f01h, c.f01h_45 * G);                  // h F01c
    const R hfr = vmax(R(0), G - R(9)) * c.frh;                   // h F_R
    const R hegp = vmax(R(0), c.egp0h - c.egp0h * s.x3);          // h EGP
    const R t = s.x1 * s.Q1;                                        // x1 Q1
    const R Q1n = s.Q1 - c.h * t + c.h_k12 * s.Q2 - hf01c - hfr + hug + hegp + dq;
    const R Q2n = s.Q2 * (c.a_12 - c.h * s.x2) + c.h * t;
    const R GIn = s.GI * c.a_c + G * c.b_c;
    const R D2n = s.D2 * c.a_g + s.D1 * c.b_g;
    const R D1n = s.D1 * c.a_g + hagd;
    const R S2n = s.S2 * c.a_i + s.S1 * c.b_i;
    const R S1n = s.S1 * c.a_i + hu;
    const R In = s.I * c.a_e + s.S2 * c.c_ui;
    const R x1n = s.x1 * c.a1 + s.I * c.b1;
    const R x2n = s.x2 * c.a2 + s.I * c.b2;
    const R x3n = s.x3 * c.a3 + s.I * c.b3;
    s.D1 = D1n; s.D2 = D2n; s.S1 = S1n; s.S2 = S2n; s.I = In;
    s.x1 = x1n; s.x2 = x2n; s.x3 = x3n; s.Q1 = Q1n; s.Q2 = Q2n; s.GI = GIn;
}

}  // namespace vct
