/*
 * vct_oracle.c -- plain FP64 CPU oracle for closed-loop virtual clinical trials.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark. It shares no code with the GPU library.
 *
 * The method (paper, Sec. III): closed-loop Monte Carlo over independent virtual
 * patients. Each patient is the SDE of Sec. III-A eq. (1) with piecewise-constant
 * inputs (eq. 2), driven by a sampled controller (Sec. III-B eq. 3); the ranges of
 * Sec. IV-A are accumulated while the simulation runs (Sec. III-C). The patient
 * model is the Hovorka core extended with a one-state CGM model (Sec. IV-B); the
 * model equations, the parameter distribution, the noise levels, the meal
 * protocol and the controller are the project's stated readings of what the paper
 * leaves open, written out below next to the code that uses them.
 *
 * Everything is FP64 and follows the definitions literally: no blocking, no
 * reordering, no fused tricks.
 */
#include "vct_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG ---- */
/* Philox4x32-10, from the description of Salmon et al. (SC'11): a 4-word counter
 * and a 2-word key; each of the 10 rounds multiplies words 0 and 2 by the two
 * round multipliers, splits the 64-bit products into high and low halves, and
 * mixes the high halves with the other two words and the round key; the key is
 * advanced by the two Weyl constants between rounds. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u = (2 m + 1) 2^-24 with m the top 23 bits of x: exactly representable in FP32
 * and FP64, never 0 or 1. */
double orc_uniform(uint32_t x)
{
    uint32_t m = x >> 9;
    return (double)(2u * m + 1u) * (1.0 / 16777216.0);
}

/* Box-Muller (1958): z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = sqrt(-2 ln u0) sin(2 pi u1). */
static void box_muller(double u0, double u1, double *z0, double *z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double r = sqrt(-2.0 * log(u0));
    *z0 = r * cos(two_pi * u1);
    *z1 = r * sin(two_pi * u1);
}

void orc_normals4(const uint32_t ctr[4], const uint32_t key[2], double z[4])
{
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    box_muller(orc_uniform(x[0]), orc_uniform(x[1]), &z[0], &z[1]);
    box_muller(orc_uniform(x[2]), orc_uniform(x[3]), &z[2], &z[3]);
}

/* Stream layout: key = (seed low word, seed high word XOR arm id);
 * counter = (index, patient, tag, sub-index). */
#define TAG_PARAM 0u
#define TAG_MEAL  1u
#define TAG_DIFF  2u

static void make_key(uint64_t seed, uint32_t arm, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32) ^ arm;
}

/* --------------------------------------------------------------- model ---- */
/* Parameter order of a sampled vector. EGP0, F01, VI, VG are per kg of body weight. */
enum { P_EGP0, P_F01, P_K12, P_KA1, P_KA2, P_KA3, P_SIT, P_SID, P_SIE, P_KE, P_VI, P_VG,
       P_TMAXI, P_TMAXG, P_BW };
/* State order. */
enum { X_D1, X_D2, X_S1, X_S2, X_I, X_X1, X_X2, X_X3, X_Q1, X_Q2, X_GI };
enum { XE_Z1, XE_Z2, XE_E1, XE_E2, XE_E3 };

/* Hovorka core (glucose absorption, subcutaneous insulin, insulin action on
 * transport, disposal and endogenous production, two glucose compartments) and
 * the one-state sensor model of the extension in Sec. IV-B:
 *   G = Q1/VG, U_G = D2/tmaxG, U_I = S2/tmaxI,
 *   F01c = F01 min(1, G/4.5), F_R = 0.003 max(0, G - 9) VG,
 *   dD1 = AG D - D1/tmaxG,         dD2 = (D1 - D2)/tmaxG,
 *   dS1 = u - S1/tmaxI,            dS2 = (S1 - S2)/tmaxI,
 *   dI  = U_I/VI - ke I,
 *   dx_j = -ka_j x_j + ka_j S_j I  (S_1,S_2,S_3 = SIT, SID, SIE),
 *   dQ1 = -F01c - x1 Q1 + k12 Q2 - F_R + U_G + EGP0 max(0, 1 - x3),
 *   dQ2 = x1 Q1 - (k12 + x2) Q2,
 *   dGI = (G - GI)/tau.
 * Endogenous production is held at zero once insulin action x3 exceeds 1 (a
 * negative hepatic output has no physical meaning). Units: min, mmol, mU, L;
 * u in mU/min, D (ingested glucose) in mmol/min. */
void orc_rhs(const orc_config *cfg, const double p[ORC_NP], const double x[ORC_NX], double u, double d,
             double dx[ORC_NX])
{
    double bw = p[P_BW];
    double egp0 = p[P_EGP0] * bw, f01 = p[P_F01] * bw;
    double vi = p[P_VI] * bw, vg = p[P_VG] * bw;
    double k12 = p[P_K12], ke = p[P_KE];
    double ka1 = p[P_KA1], ka2 = p[P_KA2], ka3 = p[P_KA3];
    double sit = p[P_SIT], sid = p[P_SID], sie = p[P_SIE];
    double tmaxi = p[P_TMAXI], tmaxg = p[P_TMAXG];

    double G = x[X_Q1] / vg;
    double ug = x[X_D2] / tmaxg;
    double ui = x[X_S2] / tmaxi;
    double f01c = f01 * fmin(1.0, G / 4.5);
    double fr = (G > 9.0) ? 0.003 * (G - 9.0) * vg : 0.0;

    dx[X_D1] = cfg->ag * d - x[X_D1] / tmaxg;
    dx[X_D2] = (x[X_D1] - x[X_D2]) / tmaxg;
    dx[X_S1] = u - x[X_S1] / tmaxi;
    dx[X_S2] = (x[X_S1] - x[X_S2]) / tmaxi;
    dx[X_I]  = ui / vi - ke * x[X_I];
    dx[X_X1] = -ka1 * x[X_X1] + ka1 * sit * x[X_I];
    dx[X_X2] = -ka2 * x[X_X2] + ka2 * sid * x[X_I];
    dx[X_X3] = -ka3 * x[X_X3] + ka3 * sie * x[X_I];
    dx[X_Q1] = -f01c - x[X_X1] * x[X_Q1] + k12 * x[X_Q2] - fr + ug + egp0 * fmax(0.0, 1.0 - x[X_X3]);
    dx[X_Q2] = x[X_X1] * x[X_Q1] - (k12 + x[X_X2]) * x[X_Q2];
    dx[X_GI] = (G - x[X_GI]) / cfg->tau_cgm;
}

/* The model extensions of Sec. IV-B (this project's reading; the paper cites the models
 * without their equations, and their parameters are shared by all patients):
 *  - subcutaneous glucagon, two states with equal time constants tau_n (ug):
 *      dZ1 = u_N - Z1/tau_n,  dZ2 = (Z1 - Z2)/tau_n,  appearance U_N = Z2/tau_n (ug/min),
 *    which adds e_n U_N (mmol/min) to the hepatic glucose output, outside the insulin clip:
 *      EGP = EGP0 max(0, 1 - x3) + e_n U_N;
 *  - exercise, three states driven by the heart-rate reserve fraction HRR in [0, 1]:
 *      dE1 = (HRR - E1)/tau_e1  (heart rate),
 *      dE2 = (E1 - E2)/tau_e2   (insulin-independent glucose uptake, -alpha_e E2 Q1),
 *      dE3 = (E1 - E3)/tau_e3   (insulin action raised: x1 and x2 act as x1 (1 + beta_e E3),
 *                                x2 (1 + beta_e E3) on glucose transport and disposal).
 * With u_N = 0 and HRR = 0 from the basal state the extension states stay 0 and the core
 * model is unchanged. */
void orc_rhs_ext(const orc_config *cfg, const double p[ORC_NP], const double x[ORC_NX], const double xe[ORC_NXE],
                 double u, double un, double d, double hrr, double dx[ORC_NX], double dxe[ORC_NXE])
{
    double bw = p[P_BW];
    double egp0 = p[P_EGP0] * bw, f01 = p[P_F01] * bw;
    double vi = p[P_VI] * bw, vg = p[P_VG] * bw;
    double k12 = p[P_K12], ke = p[P_KE];
    double ka1 = p[P_KA1], ka2 = p[P_KA2], ka3 = p[P_KA3];
    double sit = p[P_SIT], sid = p[P_SID], sie = p[P_SIE];
    double tmaxi = p[P_TMAXI], tmaxg = p[P_TMAXG];

    double G = x[X_Q1] / vg;
    double ug = x[X_D2] / tmaxg;
    double ui = x[X_S2] / tmaxi;
    double f01c = f01 * fmin(1.0, G / 4.5);
    double fr = (G > 9.0) ? 0.003 * (G - 9.0) * vg : 0.0;
    double gain = 1.0 + cfg->beta_e * xe[XE_E3];
    double x1e = x[X_X1] * gain, x2e = x[X_X2] * gain;
    double egp = egp0 * fmax(0.0, 1.0 - x[X_X3]) + cfg->e_n * xe[XE_Z2] / cfg->tau_n;

    dx[X_D1] = cfg->ag * d - x[X_D1] / tmaxg;
    dx[X_D2] = (x[X_D1] - x[X_D2]) / tmaxg;
    dx[X_S1] = u - x[X_S1] / tmaxi;
    dx[X_S2] = (x[X_S1] - x[X_S2]) / tmaxi;
    dx[X_I]  = ui / vi - ke * x[X_I];
    dx[X_X1] = -ka1 * x[X_X1] + ka1 * sit * x[X_I];
    dx[X_X2] = -ka2 * x[X_X2] + ka2 * sid * x[X_I];
    dx[X_X3] = -ka3 * x[X_X3] + ka3 * sie * x[X_I];
    dx[X_Q1] = -f01c - x1e * x[X_Q1] + k12 * x[X_Q2] - fr + ug + egp - cfg->alpha_e * xe[XE_E2] * x[X_Q1];
    dx[X_Q2] = x1e * x[X_Q1] - (k12 + x2e) * x[X_Q2];
    dx[X_GI] = (G - x[X_GI]) / cfg->tau_cgm;
    dxe[XE_Z1] = un - xe[XE_Z1] / cfg->tau_n;
    dxe[XE_Z2] = (xe[XE_Z1] - xe[XE_Z2]) / cfg->tau_n;
    dxe[XE_E1] = (hrr - xe[XE_E1]) / cfg->tau_e1;
    dxe[XE_E2] = (xe[XE_E1] - xe[XE_E2]) / cfg->tau_e2;
    dxe[XE_E3] = (xe[XE_E1] - xe[XE_E3]) / cfg->tau_e3;
}

/* Basal steady state at G* = g_target with D = 0 (and x3* < 1). Setting dQ1 = dQ2 = 0 and
 * substituting the insulin steady state x_j = S_j I gives, after multiplying by
 * (k12 + SID I), a I^2 + b I + c = 0 with
 *   a = SID (SIT Q1* + EGP0 SIE), b = SID (F01c + F_R - EGP0) + EGP0 SIE k12,
 *   c = k12 (F01c + F_R - EGP0),  Q1* = G* VG.
 * With a > 0 there is one positive root iff c < 0. Then u_b = I* ke VI. */
int orc_basal(const orc_config *cfg, const double p[ORC_NP], double *i_star, double *u_b, double x0[ORC_NX])
{
    double bw = p[P_BW];
    double egp0 = p[P_EGP0] * bw, f01 = p[P_F01] * bw;
    double vi = p[P_VI] * bw, vg = p[P_VG] * bw;
    double k12 = p[P_K12];
    double gs = cfg->g_target;
    double q1 = gs * vg;
    double f01c = f01 * fmin(1.0, gs / 4.5);
    double fr = (gs > 9.0) ? 0.003 * (gs - 9.0) * vg : 0.0;
    double a = p[P_SID] * (p[P_SIT] * q1 + egp0 * p[P_SIE]);
    double b = p[P_SID] * (f01c + fr - egp0) + egp0 * p[P_SIE] * k12;
    double c = k12 * (f01c + fr - egp0);
    if (!(c < 0.0) || !(a > 0.0))
        return 0;
    double I = (-b + sqrt(b * b - 4.0 * a * c)) / (2.0 * a);
    double ub = I * p[P_KE] * vi;
    *i_star = I;
    *u_b = ub;
    if (x0) {
        double x1 = p[P_SIT] * I, x2 = p[P_SID] * I, x3 = p[P_SIE] * I;
        x0[X_D1] = 0.0;
        x0[X_D2] = 0.0;
        x0[X_S1] = ub * p[P_TMAXI];
        x0[X_S2] = ub * p[P_TMAXI];
        x0[X_I]  = I;
        x0[X_X1] = x1;
        x0[X_X2] = x2;
        x0[X_X3] = x3;
        x0[X_Q1] = q1;
        x0[X_Q2] = q1 * x1 / (k12 + x2);
        x0[X_GI] = gs;
    }
    return 1;
}

/* Population: independent lognormal draws with median = nominal and the given CV,
 * p_j = nom_j exp(s z_j), s = sqrt(ln(1 + CV^2)); z_j is normal j of the four
 * Philox calls with counter (j/4, patient, PARAM, attempt). An attempt is kept iff
 * the basal steady state exists (and u_b >= 0.4 U/h when that flag is set, the
 * rule of Sec. IV-B); up to 32 attempts, else the nominal vector with a status bit.
 * out = [15 parameters, u_b, I*, attempts, status]. */
#define MAX_ATTEMPTS 32
static void sample_patient(const orc_config *cfg, uint32_t patient, double out[ORC_NPOUT])
{
    uint32_t key[2];
    make_key(cfg->pop_seed, cfg->arm_id, key);
    double s = sqrt(log(1.0 + cfg->cv * cfg->cv));
    double p[ORC_NP], I = 0.0, ub = 0.0;
    int attempt;
    uint32_t status = 0;
    for (attempt = 0; attempt < MAX_ATTEMPTS; ++attempt) {
        double z[16];
        for (uint32_t c = 0; c < 4; ++c) {
            uint32_t ctr[4] = {c, patient, TAG_PARAM, (uint32_t)attempt};
            orc_normals4(ctr, key, &z[4 * c]);
        }
        for (int j = 0; j < ORC_NP; ++j)
            p[j] = cfg->nominal[j] * exp(s * z[j]);
        if (!orc_basal(cfg, p, &I, &ub, NULL))
            continue;
        if ((cfg->pop_flags & ORC_POP_MIN_BASAL) && !(ub >= 400.0 / 60.0))
            continue;
        break;
    }
    if (attempt == MAX_ATTEMPTS) {
        for (int j = 0; j < ORC_NP; ++j)
            p[j] = cfg->nominal[j];
        if (!orc_basal(cfg, p, &I, &ub, NULL)) {
            I = 0.0;
            ub = 0.0;
        }
        status |= ORC_ST_RESAMPLE;
    }
    for (int j = 0; j < ORC_NP; ++j)
        out[j] = p[j];
    out[15] = ub;
    out[16] = I;
    out[17] = (double)(attempt < MAX_ATTEMPTS ? attempt + 1 : MAX_ATTEMPTS);
    out[18] = (double)status;
}

void orc_sample_population(const orc_config *cfg, int64_t first, int64_t count, double *out)
{
    for (int64_t j = 0; j < count; ++j)
        sample_patient(cfg, (uint32_t)(first + j), out + j * ORC_NPOUT);
}

/* ------------------------------------------------------------- protocol ---- */
/* One Philox call per (day, slot) with counter (day, patient, MEAL, slot):
 *   carbs   = max(0, mean + sd z), z the cosine normal of (u0, u1);
 *   jitter  = floor(u2 (2J + 1)) - J, evaluated exactly in integers;
 *   present = u3 < prob.
 * The meal is a glucose intake rate over the control interval that contains the
 * onset minute (inputs are held constant between samples, eq. 2). */
typedef struct { int32_t kd; double rate; double carbs; } meal_t;

static void meal_draw(const orc_config *cfg, uint32_t patient, int32_t day, int m, const uint32_t key[2],
                      int *present, int32_t *kd, double *carbs, int32_t *jit)
{
    uint32_t ctr[4] = {(uint32_t)day, patient, TAG_MEAL, (uint32_t)m};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    double z0, z1;
    box_muller(orc_uniform(x[0]), orc_uniform(x[1]), &z0, &z1);
    double c = cfg->carbs_mean[m] + cfg->carbs_sd[m] * z0;
    *carbs = c < 0.0 ? 0.0 : c;
    uint32_t odd = 2u * (x[2] >> 9) + 1u;
    *jit = (int32_t)(((uint64_t)odd * (uint64_t)(2 * cfg->jitter + 1)) >> 24) - cfg->jitter;
    *present = orc_uniform(x[3]) < cfg->prob[m];
    *kd = (cfg->minute_of_day[m] + *jit) / cfg->ts_min;
}

/* ------------------------------------------- Northern-European protocol ---- */
/* Sec. II-B. A year is four seasons of 13 weeks (winter, spring, summer, autumn; day 0 is
 * the first day of winter). Table I gives how many standard, active and vacation weeks
 * each season has, and how many standard days, active days, movie-night days and
 * late-night days each week type has. The order within a season and within a week is not
 * given: each patient gets a random arrangement, a Fisher-Yates shuffle (the last slot
 * swapped with a uniformly chosen slot at or before it, then the one before, ...) of the
 * list written out in table order, with 24-bit uniforms from Philox blocks (season index,
 * patient, PROTO, 0..2) for the weeks and (week index, patient, PROTO, 4..5) for the days,
 * used in order. Table II gives the meal sizes per kg of body weight. The day's meals
 * (clock times and which meal has which size are this project's reading of the text around
 * the missing figure): breakfast 07:00 small; lunch 12:00 medium; dinner 18:00 large in
 * winter and autumn, medium in spring and summer; one snack, at 10:00 in spring and summer
 * and at 15:00 in winter and autumn; a movie night adds a snack at 21:00 and a late night
 * adds snacks at 21:00 and 22:30. In vacation weeks breakfast, lunch and dinner are one
 * size larger (large stays large). The exercise session of an active day is not an input of
 * this model. Each meal draws Philox block (day, patient, MEAL, q) for its kind q (0
 * breakfast, 1 morning snack, 2 lunch, 3 afternoon snack, 4 dinner, 5, 6 evening snacks):
 * carbs = max(0, size BW (1 + meal_cv z)), z the cosine normal of (u0, u1), and the
 * onset jitter from u2 as for the slot protocol. */
#define TAG_PROTO 8u
static const int nordic_season_weeks[4][3] = {{6, 4, 3}, {6, 6, 1}, {7, 3, 3}, {9, 3, 1}};
static const int nordic_week_days[3][4] = {{4, 1, 1, 1}, {3, 3, 1, 0}, {5, 0, 0, 2}};
enum { SIZE_LARGE, SIZE_MEDIUM, SIZE_SMALL, SIZE_SNACK };
static const double nordic_g_per_kg[4] = {1.29, 0.86, 0.57, 0.29};

static void nordic_words(uint32_t c0, uint32_t patient, uint32_t first_sub, int nblocks, const uint32_t key[2],
                         uint32_t *w)
{
    for (int b = 0; b < nblocks; ++b) {
        uint32_t ctr[4] = {c0, patient, TAG_PROTO, first_sub + (uint32_t)b};
        orc_philox4x32_10(ctr, key, w + 4 * b);
    }
}

static void fisher_yates(int *list, int n, const uint32_t *w)
{
    int used = 0;
    for (int i = n - 1; i >= 1; --i) {
        uint64_t u24 = w[used++] >> 8;
        int j = (int)((u24 * (uint64_t)(i + 1)) >> 24);
        int t = list[i];
        list[i] = list[j];
        list[j] = t;
    }
}

static void nordic_day_types(uint32_t patient, int32_t day, const uint32_t key[2], int *season, int *wtype,
                             int *dtype)
{
    *season = (day / 91) % 4;
    int weeks[13], n = 0;
    for (int t = 0; t < 3; ++t)
        for (int e = 0; e < nordic_season_weeks[*season][t]; ++e)
            weeks[n++] = t;
    uint32_t w[12];
    nordic_words((uint32_t)(day / 91), patient, 0u, 3, key, w);
    fisher_yates(weeks, 13, w);
    *wtype = weeks[(day % 91) / 7];
    int days[7];
    n = 0;
    for (int t = 0; t < 4; ++t)
        for (int e = 0; e < nordic_week_days[*wtype][t]; ++e)
            days[n++] = t;
    uint32_t v[8];
    nordic_words((uint32_t)(day / 7), patient, 4u, 2, key, v);
    fisher_yates(days, 7, v);
    *dtype = days[day % 7];
}

void orc_nordic_day(const orc_config *cfg, uint32_t patient, int32_t day, int32_t *out)
{
    uint32_t key[2];
    make_key(cfg->noise_seed, cfg->arm_id, key);
    int s, wt, dt;
    nordic_day_types(patient, day, key, &s, &wt, &dt);
    out[0] = s;
    out[1] = wt;
    out[2] = dt;
}

static int nordic_meals(const orc_config *cfg, uint32_t patient, int32_t day, double bw, const uint32_t key[2],
                        meal_t meals[ORC_MAX_DAY_MEALS])
{
    int season, wtype, dtype;
    nordic_day_types(patient, day, key, &season, &wtype, &dtype);
    const int winter_autumn = season == 0 || season == 3, vacation = wtype == 2;
    /* kind, minute, size, present */
    const int plan[7][3] = {
        {420, vacation ? SIZE_MEDIUM : SIZE_SMALL, 1},
        {600, SIZE_SNACK, !winter_autumn},
        {720, vacation ? SIZE_LARGE : SIZE_MEDIUM, 1},
        {900, SIZE_SNACK, winter_autumn},
        {1080, (winter_autumn || vacation) ? SIZE_LARGE : SIZE_MEDIUM, 1},
        {1260, SIZE_SNACK, dtype == 2 || dtype == 3},
        {1350, SIZE_SNACK, dtype == 3},
    };
    int n = 0;
    for (int q = 0; q < 7; ++q) {
        if (!plan[q][2])
            continue;
        uint32_t ctr[4] = {(uint32_t)day, patient, TAG_MEAL, (uint32_t)q};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        double z0, z1;
        box_muller(orc_uniform(x[0]), orc_uniform(x[1]), &z0, &z1);
        double c = nordic_g_per_kg[plan[q][1]] * bw * (1.0 + cfg->meal_cv * z0);
        uint32_t odd = 2u * (x[2] >> 9) + 1u;
        int32_t jit = (int32_t)(((uint64_t)odd * (uint64_t)(2 * cfg->jitter + 1)) >> 24) - cfg->jitter;
        meals[n].kd = (plan[q][0] + jit) / cfg->ts_min;
        meals[n].carbs = c < 0.0 ? 0.0 : c;
        meals[n].rate = meals[n].carbs * (1000.0 / 180.16) / (double)cfg->ts_min;
        ++n;
    }
    return n;
}

static int meals_for_day(const orc_config *cfg, uint32_t patient, int32_t day, double bw, const uint32_t key[2],
                         meal_t meals[ORC_MAX_DAY_MEALS])
{
    if (cfg->proto == ORC_PROTO_NORDIC)
        return nordic_meals(cfg, patient, day, bw, key, meals);
    int n = 0;
    for (int m = 0; m < cfg->n_slots; ++m) {
        int present;
        int32_t kd, jit;
        double carbs;
        meal_draw(cfg, patient, day, m, key, &present, &kd, &carbs, &jit);
        if (!present)
            continue;
        meals[n].kd = kd;
        meals[n].carbs = carbs;
        meals[n].rate = carbs * (1000.0 / 180.16) / (double)cfg->ts_min;
        ++n;
    }
    return n;
}

/* The day's meals in time order under either protocol (tests): out[n][3] = (sample index
 * within the day, carbs g, intake mmol/min); returns n. */
int orc_day_meals(const orc_config *cfg, uint32_t patient, int32_t day, double *out)
{
    uint32_t key[2];
    make_key(cfg->noise_seed, cfg->arm_id, key);
    double prm[ORC_NPOUT];
    sample_patient(cfg, patient, prm);
    meal_t meals[ORC_MAX_DAY_MEALS];
    int n = meals_for_day(cfg, patient, day, prm[14], key, meals);
    for (int m = 0; m < n; ++m) {
        out[3 * m + 0] = (double)meals[m].kd;
        out[3 * m + 1] = meals[m].carbs;
        out[3 * m + 2] = meals[m].rate;
    }
    return n;
}

/* Exercise (Sec. II-B: the active day has an exercise session; this project's reading of
 * its time and form): on each active day of the Northern-European protocol one session of
 * exercise_duration minutes at heart-rate reserve fraction exercise_hrr, starting in the
 * sample that contains exercise_minute + jitter, the jitter drawn like a meal's from word 2
 * of Philox block (day, patient, EXER, 0); the input is held over whole sampling intervals:
 * ceil(duration / Ts) samples from the onset. */
#define TAG_EXER 9u
static int32_t exercise_onset(const orc_config *cfg, uint32_t patient, int32_t day, const uint32_t key[2])
{
    if (!cfg->model_ext || !cfg->exercise || cfg->proto != ORC_PROTO_NORDIC)
        return -1;
    int season, wtype, dtype;
    nordic_day_types(patient, day, key, &season, &wtype, &dtype);
    if (dtype != 1)
        return -1;
    uint32_t ctr[4] = {(uint32_t)day, patient, TAG_EXER, 0u};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    uint32_t odd = 2u * (x[2] >> 9) + 1u;
    int32_t jit = (int32_t)(((uint64_t)odd * (uint64_t)(2 * cfg->jitter + 1)) >> 24) - cfg->jitter;
    return (cfg->exercise_minute + jit) / cfg->ts_min;
}

static int32_t exercise_samples(const orc_config *cfg)
{
    return (cfg->exercise_duration + cfg->ts_min - 1) / cfg->ts_min;
}

int32_t orc_day_exercise(const orc_config *cfg, uint32_t patient, int32_t day)
{
    uint32_t key[2];
    make_key(cfg->noise_seed, cfg->arm_id, key);
    return exercise_onset(cfg, patient, day, key);
}

/* Meal draws of one (patient, day), for tests: out [n_slots][4] = (present, sample
 * index within the day, carbs in g, jitter in min); absent slots keep their draw. */
void orc_meals(const orc_config *cfg, uint32_t patient, int32_t day, double *out)
{
    uint32_t key[2];
    make_key(cfg->noise_seed, cfg->arm_id, key);
    for (int m = 0; m < cfg->n_slots; ++m) {
        int present;
        int32_t kd, jit;
        double carbs;
        meal_draw(cfg, patient, day, m, key, &present, &kd, &carbs, &jit);
        out[4 * m + 0] = present ? 1.0 : 0.0;
        out[4 * m + 1] = (double)kd;
        out[4 * m + 2] = carbs;
        out[4 * m + 3] = (double)jit;
    }
}

/* ---------------------------------------------------------- integrators ---- */
/* One Euler-Maruyama step x <- x + h f + sqrt(h) sigma .* xi (drift evaluated at the
 * pre-step state for every component). */
static void em_step(int n, double *x, const double *f, double h, double sqrt_h, const double *sig,
                    const double *xi)
{
    for (int i = 0; i < n; ++i)
        x[i] = x[i] + h * f[i] + sqrt_h * sig[i] * xi[i];
}

static void rk4_step(const orc_config *cfg, const double p[ORC_NP], double x[ORC_NX], double u, double d,
                     double h)
{
    double k1[ORC_NX], k2[ORC_NX], k3[ORC_NX], k4[ORC_NX], t[ORC_NX];
    orc_rhs(cfg, p, x, u, d, k1);
    for (int i = 0; i < ORC_NX; ++i) t[i] = x[i] + 0.5 * h * k1[i];
    orc_rhs(cfg, p, t, u, d, k2);
    for (int i = 0; i < ORC_NX; ++i) t[i] = x[i] + 0.5 * h * k2[i];
    orc_rhs(cfg, p, t, u, d, k3);
    for (int i = 0; i < ORC_NX; ++i) t[i] = x[i] + h * k3[i];
    orc_rhs(cfg, p, t, u, d, k4);
    for (int i = 0; i < ORC_NX; ++i)
        x[i] = x[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* The same on the extended model's 16 states (X = core states, then the extension's). */
static void rhs16(const orc_config *cfg, const double p[ORC_NP], const double X[ORC_NX + ORC_NXE], double u,
                  double un, double d, double hrr, double F[ORC_NX + ORC_NXE])
{
    orc_rhs_ext(cfg, p, X, X + ORC_NX, u, un, d, hrr, F, F + ORC_NX);
}

static void rk4_step_ext(const orc_config *cfg, const double p[ORC_NP], double X[ORC_NX + ORC_NXE], double u,
                         double un, double d, double hrr, double h)
{
    enum { N = ORC_NX + ORC_NXE };
    double k1[N], k2[N], k3[N], k4[N], t[N];
    rhs16(cfg, p, X, u, un, d, hrr, k1);
    for (int i = 0; i < N; ++i) t[i] = X[i] + 0.5 * h * k1[i];
    rhs16(cfg, p, t, u, un, d, hrr, k2);
    for (int i = 0; i < N; ++i) t[i] = X[i] + 0.5 * h * k2[i];
    rhs16(cfg, p, t, u, un, d, hrr, k3);
    for (int i = 0; i < N; ++i) t[i] = X[i] + h * k3[i];
    rhs16(cfg, p, t, u, un, d, hrr, k4);
    for (int i = 0; i < N; ++i)
        X[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

void orc_em_ou(double theta, double s, double x0, double h, int32_t n_steps, int64_t n_paths, uint64_t seed,
               double *x_final)
{
    uint32_t key[2];
    make_key(seed, 0u, key);
    double sqrt_h = sqrt(h);
    for (int64_t path = 0; path < n_paths; ++path) {
        double x = x0;
        for (int32_t n = 0; n < n_steps; ++n) {
            uint32_t ctr[4] = {(uint32_t)n, (uint32_t)path, TAG_DIFF, 0u};
            double z[4];
            orc_normals4(ctr, key, z);
            double f = -theta * x;
            em_step(1, &x, &f, h, sqrt_h, &s, &z[0]);
        }
        x_final[path] = x;
    }
}

/* --------------------------------------------------------------- metrics ---- */
/* Ranges of Sec. IV-A, mmol/L: [0] < 3.0, [1] 3.0-3.9, [2] 3.9-10.0 (both ends in
 * range), [3] 10.0-13.9, [4] > 13.9. The index is the number of edges passed, so a
 * non-finite G lands in [0] (and raises a status bit). Events: a maximal run of at
 * least 3 consecutive samples below 3.9, below 3.0, or above 13.9, counted once
 * when the run reaches 3 samples. "Below an edge" is "not at or above it", so a
 * non-finite G, counted in the lowest range, also continues the runs below 3.9
 * and 3.0; for finite G this is the plain comparison. */
static const double EDGE[4] = {3.0, 3.9, 10.0, 13.9};

typedef struct {
    int32_t bins[5], events[3], run[3];
    double sum_g, min_g, sum_u;
    int32_t argmin_k, n_near;
    uint32_t status;
    double ctrl_margin;
} acc_t;

static void acc_sample(acc_t *a, double G, int32_t k, double guard)
{
    int b = (G >= EDGE[0]) + (G >= EDGE[1]) + (G > EDGE[2]) + (G > EDGE[3]);
    a->bins[b] += 1;
    int cond[3] = {!(G >= 3.9), !(G >= 3.0), G > 13.9};
    for (int e = 0; e < 3; ++e) {
        if (cond[e]) {
            a->run[e] += 1;
            if (a->run[e] == 3)
                a->events[e] += 1;
        } else {
            a->run[e] = 0;
        }
    }
    a->sum_g += G;
    if (G < a->min_g) {
        a->min_g = G;
        a->argmin_k = k;
    }
    for (int e = 0; e < 4; ++e)
        if (fabs(G - EDGE[e]) <= guard * EDGE[e]) {
            a->n_near += 1;
            break;
        }
    if (!isfinite(G))
        a->status |= ORC_ST_NONFINITE;
    else if (G < 0.0)
        a->status |= ORC_ST_NEGATIVE_Q1;
}

/* ------------------------------------------------------------ controller ---- */
/* PID on the CGM value, gains scaled by the controller's basal rate u_b (the patient's
 * basal rate times basal_scale; a mis-set basal rate as in trial B of Sec. IV-E):
 *   e = y_k - ybar, u_unc = u_b + Kp e + Ki I_k + Kd (y_k - y_{k-1})/Ts (y_{-1} = y_0),
 *   u_k = min(max(u_unc, 0), u_max),
 *   I_{k+1} = I_k + e Ts only if 0 <= u_unc <= u_max (conditional integration).
 * This is the kappa/lambda form of Sec. III-B with control state (I_k, y_{k-1}). */
typedef struct { double integ, y_prev; int started; } pid_t_;

static double pid_step(const orc_config *cfg, pid_t_ *c, double y, double ub, double *margin)
{
    double kp = cfg->kp * ub, ki = cfg->ki * ub, kd = cfg->kd * ub;
    double umax = cfg->umax_rel * ub;
    double ts = (double)cfg->ts_min;
    if (!c->started) {
        c->y_prev = y;
        c->started = 1;
    }
    double e = y - cfg->setpoint;
    double u_unc = ub + kp * e + ki * c->integ + kd * (y - c->y_prev) / ts;
    double u = u_unc < 0.0 ? 0.0 : u_unc;
    if (u > umax)
        u = umax;
    if (u_unc >= 0.0 && u_unc <= umax)
        c->integ += e * ts;
    c->y_prev = y;
    double m = fmin(fabs(u_unc), fabs(u_unc - umax)) / ub;
    if (m < *margin)
        *margin = m;
    return u;
}

/* Scripted PID run for tests: u[k] for the measurement sequence y[0..n-1]. */
void orc_pid_run(const orc_config *cfg, double ub, int32_t n, const double *y, double *u, double *integ)
{
    pid_t_ c = {0.0, 0.0, 0};
    double margin = INFINITY;
    for (int32_t k = 0; k < n; ++k) {
        u[k] = pid_step(cfg, &c, y[k], ub, &margin);
        if (integ)
            integ[k] = c.integ;
    }
}

/* ------------------------------------------------- dual-hormone AP ---- */
/* Sec. IV-C names the parts of the paper's AP; their laws are this project's reading.
 * Modes: glucagon mode is entered when y_k < glu_enter and left when y_k >= glu_exit.
 *  - insulin mode: microadjustments of the basal rate by the PID above (the PID runs on
 *    every sample, its integral with its own conditional rule, but its output is delivered
 *    only in this mode), plus a meal bolus at each announced meal (meal_bolus = 1): carbs / ICR with
 *    ICR = icr_rule / TDD (g/U) and TDD = 2 x the daily basal insulin (U/day), less the
 *    insulin on board above basal (subcutaneous depot S1 + S2 minus its basal 2 u_b tmaxI),
 *    never negative, delivered over the meal's interval; no glucagon;
 *  - glucagon mode: no insulin; a glucagon microbolus glu_kp (glu_target - y_k) less the
 *    glucagon on board (depot Z1 + Z2), clamped to [0, glu_max] ug, over the interval;
 *  - in either mode, an exercise onset with y_k < ex_bolus_below adds an ex_bolus ug
 *    glucagon bolus over the interval.
 * The insulin and glucagon on board are those of a controller-side replica of the depots
 * driven by the delivered doses; both subsystems are deterministic, so the replica equals
 * the plant's states and is read from them. Announced carbs: the held intake d (mmol/min)
 * over Ts minutes, 180.16/1000 g per mmol. */
typedef struct { pid_t_ pid; int glu; } dual_t;

static void dual_step(const orc_config *cfg, dual_t *st, double y, double ub, double iob, double gob, double d,
                      int ex_onset, double *u_basal, double *u_bolus, double *un, double *margin)
{
    const double ts = (double)cfg->ts_min;
    if (!st->glu && y < cfg->glu_enter)
        st->glu = 1;
    else if (st->glu && y >= cfg->glu_exit)
        st->glu = 0;
    double n_ug = 0.0;
    const double u_pid = pid_step(cfg, &st->pid, y, ub, margin);
    if (st->glu) {
        *u_basal = 0.0;
        *u_bolus = 0.0;
        n_ug = fmin(cfg->glu_max, fmax(0.0, cfg->glu_kp * (cfg->glu_target - y) - gob));
    } else {
        *u_basal = u_pid;
        double bolus_mu = 0.0;
        if (cfg->meal_bolus && d > 0.0) {
            double carbs = d * ts * 180.16 / 1000.0;
            double tdd = 2.0 * ub * 1440.0 / 1000.0;
            bolus_mu = fmax(0.0, carbs / (cfg->icr_rule / tdd) * 1000.0 - iob);
        }
        *u_bolus = bolus_mu / ts;
    }
    if (ex_onset && y < cfg->ex_bolus_below)
        n_ug += cfg->ex_bolus;
    *un = n_ug / ts;
}

/* Scripted run for tests: insulin and glucagon on board held at iob and gob. */
void orc_dual_run(const orc_config *cfg, double ub, double iob, double gob, int32_t n, const double *y,
                  const double *d, const int32_t *ex, double *u_basal, double *u_bolus, double *un, int32_t *mode)
{
    dual_t st;
    memset(&st, 0, sizeof st);
    double margin = INFINITY;
    for (int32_t k = 0; k < n; ++k) {
        dual_step(cfg, &st, y[k], ub, iob, gob, d[k], ex[k], &u_basal[k], &u_bolus[k], &un[k], &margin);
        mode[k] = st.glu;
    }
}

/* ------------------------------------------------------------------- MPC ---- */
/* Linear MPC in the kappa/lambda form of Sec. III-B: the control state is the Kalman
 * estimate of the state deviation from the basal steady state and the planned input
 * sequence; the control law solves a box-constrained quadratic program over N samples.
 *  - model: the drift linearised at the basal state (x_ss, u_b, D = 0), discretised the
 *    way the plant is integrated: M = I + hJ, A = M^E, B = h (I + M + ... + M^(E-1)) B_c,
 *    E likewise, with E = em_per_ctrl Euler steps per sample;
 *  - estimator: stationary Kalman filter for the sensor state GI, gain from a fixed
 *    number of Riccati iterations with Q = 1e-6 I + sigma^2 h E e_Q1 e_Q1^T and
 *    R = max(R_cgm, 1e-4);
 *  - objective over the predicted true glucose G_(k+1..k+N):
 *      sum_j (G_j - ybar)^2 + rho sum_i ((u_i - u_b)/u_b)^2,  0 <= u_i <= u_max,
 *    the announced intake of the current interval known, later ones taken as zero;
 *  - solver: mpc_iters projected-gradient steps of length 1/(lambda_max(G^T G) + rho/u_b^2),
 *    warm-started from the previous plan shifted by one sample. */
static void matmul(const double *X, const double *Y, double *Z)
{
    double T[ORC_NX * ORC_NX];
    for (int r = 0; r < ORC_NX; ++r)
        for (int c = 0; c < ORC_NX; ++c) {
            double acc = 0.0;
            for (int q = 0; q < ORC_NX; ++q)
                acc += X[r * ORC_NX + q] * Y[q * ORC_NX + c];
            T[r * ORC_NX + c] = acc;
        }
    memcpy(Z, T, sizeof T);
}

void orc_jacobian(const orc_config *cfg, const double p[ORC_NP], const double x[ORC_NX], double J[ORC_NX * ORC_NX],
                  double Bc[ORC_NX], double Ec[ORC_NX])
{
    double bw = p[P_BW];
    double egp0 = p[P_EGP0] * bw, f01 = p[P_F01] * bw;
    double vi = p[P_VI] * bw, vg = p[P_VG] * bw;
    double tg = p[P_TMAXG], ti = p[P_TMAXI];
    memset(J, 0, sizeof(double) * ORC_NX * ORC_NX);
    memset(Bc, 0, sizeof(double) * ORC_NX);
    memset(Ec, 0, sizeof(double) * ORC_NX);
#define JJ(r, c) J[(r) * ORC_NX + (c)]
    JJ(X_D1, X_D1) = -1.0 / tg;
    JJ(X_D2, X_D1) = 1.0 / tg;
    JJ(X_D2, X_D2) = -1.0 / tg;
    JJ(X_S1, X_S1) = -1.0 / ti;
    JJ(X_S2, X_S1) = 1.0 / ti;
    JJ(X_S2, X_S2) = -1.0 / ti;
    JJ(X_I, X_S2) = 1.0 / (ti * vi);
    JJ(X_I, X_I) = -p[P_KE];
    JJ(X_X1, X_I) = p[P_KA1] * p[P_SIT];
    JJ(X_X1, X_X1) = -p[P_KA1];
    JJ(X_X2, X_I) = p[P_KA2] * p[P_SID];
    JJ(X_X2, X_X2) = -p[P_KA2];
    JJ(X_X3, X_I) = p[P_KA3] * p[P_SIE];
    JJ(X_X3, X_X3) = -p[P_KA3];
    double G = x[X_Q1] / vg;
    double df01c = G < 4.5 ? f01 / (4.5 * vg) : 0.0;
    double dfr = G > 9.0 ? 0.003 : 0.0;
    JJ(X_Q1, X_D2) = 1.0 / tg;
    JJ(X_Q1, X_X1) = -x[X_Q1];
    JJ(X_Q1, X_X3) = x[X_X3] < 1.0 ? -egp0 : 0.0;
    JJ(X_Q1, X_Q1) = -x[X_X1] - df01c - dfr;
    JJ(X_Q1, X_Q2) = p[P_K12];
    JJ(X_Q2, X_X1) = x[X_Q1];
    JJ(X_Q2, X_X2) = -x[X_Q2];
    JJ(X_Q2, X_Q1) = x[X_X1];
    JJ(X_Q2, X_Q2) = -(p[P_K12] + x[X_X2]);
    JJ(X_GI, X_Q1) = 1.0 / (cfg->tau_cgm * vg);
    JJ(X_GI, X_GI) = -1.0 / cfg->tau_cgm;
#undef JJ
    Bc[X_S1] = 1.0;
    Ec[X_D1] = cfg->ag;
}

int orc_mpc_setup(const orc_config *cfg, const double prm[ORC_NPOUT], orc_mpc *m)
{
    memset(m, 0, sizeof *m);
    double istar, ub;
    if (!orc_basal(cfg, prm, &istar, &ub, m->xss))
        return 0;
    const int N = cfg->mpc_horizon;
    const int E = cfg->em_per_ctrl;
    const double h = (double)cfg->ts_min / (double)E;
    const double vg = prm[P_VG] * prm[P_BW];
    m->N = N;
    m->ub = ub;
    m->umax = cfg->umax_rel * ub;
    m->gstar = cfg->g_target;

    double J[ORC_NX * ORC_NX], Bc[ORC_NX], Ec[ORC_NX], Mx[ORC_NX * ORC_NX], S[ORC_NX * ORC_NX], Pw[ORC_NX * ORC_NX];
    orc_jacobian(cfg, prm, m->xss, J, Bc, Ec);
    for (int i = 0; i < ORC_NX * ORC_NX; ++i)
        Mx[i] = h * J[i];
    for (int i = 0; i < ORC_NX; ++i)
        Mx[i * ORC_NX + i] += 1.0;
    /* A = M^E, S = I + M + ... + M^(E-1) */
    memset(Pw, 0, sizeof Pw);
    memset(S, 0, sizeof S);
    for (int i = 0; i < ORC_NX; ++i)
        Pw[i * ORC_NX + i] = 1.0;
    for (int e = 0; e < E; ++e) {
        for (int i = 0; i < ORC_NX * ORC_NX; ++i)
            S[i] += Pw[i];
        matmul(Pw, Mx, Pw);
    }
    memcpy(m->A, Pw, sizeof Pw);
    for (int r = 0; r < ORC_NX; ++r) {
        double b = 0.0, d = 0.0;
        for (int c = 0; c < ORC_NX; ++c) {
            b += S[r * ORC_NX + c] * Bc[c];
            d += S[r * ORC_NX + c] * Ec[c];
        }
        m->B[r] = h * b;
        m->E[r] = h * d;
    }

    /* Kalman: prior covariance P <- A (P - P c^T c P / (c P c^T + R)) A^T + Q, c = e_GI */
    double Q[ORC_NX * ORC_NX], P[ORC_NX * ORC_NX], T[ORC_NX * ORC_NX], At[ORC_NX * ORC_NX];
    memset(Q, 0, sizeof Q);
    for (int i = 0; i < ORC_NX; ++i)
        Q[i * ORC_NX + i] = 1e-6;
    Q[X_Q1 * ORC_NX + X_Q1] += cfg->sigma_q1 * cfg->sigma_q1 * h * E;
    const double R = cfg->cgm_var > 1e-4 ? cfg->cgm_var : 1e-4;
    for (int r = 0; r < ORC_NX; ++r)
        for (int c = 0; c < ORC_NX; ++c)
            At[r * ORC_NX + c] = m->A[c * ORC_NX + r];
    memcpy(P, Q, sizeof P);
    for (int it = 0; it < cfg->mpc_riccati_iters; ++it) {
        const double s = P[X_GI * ORC_NX + X_GI] + R;
        for (int r = 0; r < ORC_NX; ++r)
            for (int c = 0; c < ORC_NX; ++c)
                T[r * ORC_NX + c] = P[r * ORC_NX + c] - P[r * ORC_NX + X_GI] * P[X_GI * ORC_NX + c] / s;
        matmul(m->A, T, T);
        matmul(T, At, T);
        double change = 0.0;
        for (int i = 0; i < ORC_NX * ORC_NX; ++i) {
            double v = T[i] + Q[i];
            change = fmax(change, fabs(v - P[i]));
            P[i] = v;
        }
        m->P_change = change;
    }
    memcpy(m->P, P, sizeof P);
    const double s = P[X_GI * ORC_NX + X_GI] + R;
    for (int i = 0; i < ORC_NX; ++i)
        m->K[i] = P[i * ORC_NX + X_GI] / s;

    /* prediction of G = Q1/VG over N samples */
    double row[ORC_NX], nrow[ORC_NX];
    for (int i = 0; i < ORC_NX; ++i)
        row[i] = i == X_Q1 ? 1.0 / vg : 0.0;          /* c_G A^0 */
    for (int j = 0; j < N; ++j) {
        double hb = 0.0, we = 0.0;
        for (int i = 0; i < ORC_NX; ++i) {
            hb += row[i] * m->B[i];
            we += row[i] * m->E[i];
        }
        m->h[j] = hb;                                  /* h_(j+1) = c_G A^j B */
        m->w[j] = we;                                  /* c_G A^j E */
        for (int c = 0; c < ORC_NX; ++c) {
            double acc = 0.0;
            for (int q = 0; q < ORC_NX; ++q)
                acc += row[q] * m->A[q * ORC_NX + c];
            nrow[c] = acc;
        }
        memcpy(row, nrow, sizeof row);
        for (int c = 0; c < ORC_NX; ++c)
            m->F[j * ORC_NX + c] = row[c];             /* c_G A^(j+1) */
    }
    /* Gamma[j][i] = h[j - i] (i <= j); Gamma^T F, Gamma^T w, Gamma^T 1 */
    for (int i = 0; i < N; ++i) {
        double gd = 0.0, g1 = 0.0;
        for (int c = 0; c < ORC_NX; ++c)
            m->Gx[i * ORC_NX + c] = 0.0;
        for (int j = i; j < N; ++j) {
            double gji = m->h[j - i];
            for (int c = 0; c < ORC_NX; ++c)
                m->Gx[i * ORC_NX + c] += gji * m->F[j * ORC_NX + c];
            gd += gji * m->w[j];
            g1 += gji;
        }
        m->gd[i] = gd;
        m->g1[i] = g1;
    }
    /* lambda_max(Gamma^T Gamma) by power iteration from the all-ones vector */
    double v[ORC_NMAX], t[ORC_NMAX], lam = 0.0;
    for (int i = 0; i < N; ++i)
        v[i] = 1.0 / sqrt((double)N);
    for (int it = 0; it < cfg->mpc_power_iters; ++it) {
        for (int j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int i = 0; i <= j; ++i)
                acc += m->h[j - i] * v[i];
            t[j] = acc;
        }
        double nrm = 0.0;
        for (int i = 0; i < N; ++i) {
            double acc = 0.0;
            for (int j = i; j < N; ++j)
                acc += m->h[j - i] * t[j];
            v[i] = acc;
            nrm += acc * acc;
        }
        nrm = sqrt(nrm);
        lam = nrm;
        if (nrm > 0.0)
            for (int i = 0; i < N; ++i)
                v[i] /= nrm;
    }
    m->lambda = lam;
    m->rho_p = cfg->mpc_rho / (ub * ub);
    m->step = 1.0 / (lam + m->rho_p);
    return 1;
}

void orc_mpc_pg(const orc_mpc *m, const double g[], double dU[], int iters)
{
    const int N = m->N;
    const double lo = -m->ub, hi = m->umax - m->ub;
    double r[ORC_NMAX];
    for (int it = 0; it < iters; ++it) {
        for (int j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int i = 0; i <= j; ++i)
                acc += m->h[j - i] * dU[i];
            r[j] = acc;                                /* Gamma dU */
        }
        double nu[ORC_NMAX];
        for (int i = 0; i < N; ++i) {
            double acc = 0.0;
            for (int j = i; j < N; ++j)
                acc += m->h[j - i] * r[j];             /* Gamma^T Gamma dU */
            double grad = acc + m->rho_p * dU[i] + g[i];
            double x = dU[i] - m->step * grad;
            nu[i] = x < lo ? lo : (x > hi ? hi : x);
        }
        memcpy(dU, nu, sizeof(double) * N);
    }
}

typedef struct {
    orc_mpc m;
    double xh[ORC_NX];     /* estimate of x - x_ss (prior before the measurement update) */
    double dU[ORC_NMAX];   /* planned u - u_b */
    double Fbar[ORC_NX];   /* mean over the horizon of the prediction rows F_j */
    double wbar;           /* mean over the horizon of the intake response w_j */
    double hsum, hdelay;   /* sum of the Markov parameters, and their mean delay (samples) */
} mpc_state;

/* The controller sample in three parts: measurement update with the sensor value; the plan
 * (QP linear term, warm start from the shifted previous plan, projected gradient); the
 * time update with the applied input deviation and the announced intake. */
static void mpc_measure(mpc_state *st, double y)
{
    const orc_mpc *m = &st->m;
    double innov = (y - m->xss[X_GI]) - st->xh[X_GI];
    for (int i = 0; i < ORC_NX; ++i)
        st->xh[i] += m->K[i] * innov;
}

static void mpc_shift(mpc_state *st)
{
    for (int i = 0; i + 1 < st->m.N; ++i)
        st->dU[i] = st->dU[i + 1];
}

static double mpc_plan(const orc_config *cfg, mpc_state *st, double dhat)
{
    const orc_mpc *m = &st->m;
    const int N = m->N;
    /* linear term of the QP: Gamma^T (F xh + w dhat + (G* - ybar)) */
    double g[ORC_NMAX];
    for (int i = 0; i < N; ++i) {
        double acc = m->gd[i] * dhat + m->g1[i] * (m->gstar - cfg->setpoint);
        for (int c = 0; c < ORC_NX; ++c)
            acc += m->Gx[i * ORC_NX + c] * st->xh[c];
        g[i] = acc;
    }
    mpc_shift(st);
    orc_mpc_pg(m, g, st->dU, cfg->mpc_iters);
    return st->dU[0];
}

static void mpc_predict(mpc_state *st, double du, double dhat)
{
    const orc_mpc *m = &st->m;
    double nx[ORC_NX];
    for (int r = 0; r < ORC_NX; ++r) {
        double acc = m->B[r] * du + m->E[r] * dhat;
        for (int c = 0; c < ORC_NX; ++c)
            acc += m->A[r * ORC_NX + c] * st->xh[c];
        nx[r] = acc;
    }
    memcpy(st->xh, nx, sizeof nx);
}

static double mpc_step(const orc_config *cfg, mpc_state *st, double y, double dhat)
{
    mpc_measure(st, y);
    const double du = mpc_plan(cfg, st, dhat);
    mpc_predict(st, du, dhat);
    return st->m.ub + du;
}

/* ------------------------------------------------------- learned controller ---- */
double orc_bf16(double x)
{
    if (x == 0.0 || !isfinite(x))
        return x;
    int e;
    frexp(x, &e);                          /* |x| in [2^(e-1), 2^e) */
    const double ulp = ldexp(1.0, e - 8);  /* 8 significant bits */
    return nearbyint(x / ulp) * ulp;       /* x/ulp is exact; ties to even */
}

static double mlp_eval(const orc_mlp *n, const double x[ORC_MLP_IN], double z[ORC_MLP_IN], double h1[ORC_MLP_H],
                       double h2[ORC_MLP_H], double h3[ORC_MLP_H])
{
    for (int f = 0; f < ORC_MLP_IN; ++f)
        z[f] = orc_bf16((x[f] - n->mean[f]) * n->istd[f]);
    for (int u = 0; u < ORC_MLP_H; ++u) {
        double a = n->b1[u];
        for (int f = 0; f < ORC_MLP_IN; ++f)
            a += n->W1[u * ORC_MLP_IN + f] * z[f];
        h1[u] = a > 0.0 ? a : 0.0;
    }
    for (int u = 0; u < ORC_MLP_H; ++u) {
        double a = n->b2[u];
        for (int v = 0; v < ORC_MLP_H; ++v)
            a += n->W2[u * ORC_MLP_H + v] * h1[v];
        h2[u] = a > 0.0 ? a : 0.0;
    }
    for (int u = 0; u < ORC_MLP_H; ++u) {
        double a = n->b3[u];
        for (int v = 0; v < ORC_MLP_H; ++v)
            a += n->W3[u * ORC_MLP_H + v] * h2[v];
        h3[u] = a > 0.0 ? a : 0.0;
    }
    double o = n->b4;
    for (int u = 0; u < ORC_MLP_H; ++u)
        o += n->w4[u] * h3[u];
    return o;
}

void orc_mlp_forward(const orc_mlp *net, const double *x, int64_t n, double *out)
{
    double z[ORC_MLP_IN], h1[ORC_MLP_H], h2[ORC_MLP_H], h3[ORC_MLP_H];
    for (int64_t i = 0; i < n; ++i)
        out[i] = mlp_eval(net, x + i * ORC_MLP_IN, z, h1, h2, h3);
}

/* Backpropagation of L = (1/B) sum (o - t)^2 through the chain of mlp_eval; the derivative
 * of ReLU is taken as 1 where the unit is positive and 0 elsewhere. */
double orc_mlp_loss_grad(const orc_mlp *net, const double *rows, const int64_t *idx, int64_t B, orc_mlp *g)
{
    memset(g, 0, sizeof *g);
    double loss = 0.0;
    for (int64_t i = 0; i < B; ++i) {
        const double *r = rows + idx[i] * (ORC_MLP_IN + 1);
        double z[ORC_MLP_IN], h1[ORC_MLP_H], h2[ORC_MLP_H], h3[ORC_MLP_H];
        const double o = mlp_eval(net, r, z, h1, h2, h3);
        const double e = o - r[ORC_MLP_IN];
        loss += e * e / (double)B;
        const double dout = 2.0 * e / (double)B;
        double d3[ORC_MLP_H], d2[ORC_MLP_H], d1[ORC_MLP_H];
        g->b4 += dout;
        for (int u = 0; u < ORC_MLP_H; ++u) {
            g->w4[u] += dout * h3[u];
            d3[u] = h3[u] > 0.0 ? dout * net->w4[u] : 0.0;
        }
        for (int v = 0; v < ORC_MLP_H; ++v) {
            double a = 0.0;
            for (int u = 0; u < ORC_MLP_H; ++u)
                a += d3[u] * net->W3[u * ORC_MLP_H + v];
            d2[v] = h2[v] > 0.0 ? a : 0.0;
        }
        for (int u = 0; u < ORC_MLP_H; ++u) {
            g->b3[u] += d3[u];
            for (int v = 0; v < ORC_MLP_H; ++v)
                g->W3[u * ORC_MLP_H + v] += d3[u] * h2[v];
        }
        for (int v = 0; v < ORC_MLP_H; ++v) {
            double a = 0.0;
            for (int u = 0; u < ORC_MLP_H; ++u)
                a += d2[u] * net->W2[u * ORC_MLP_H + v];
            d1[v] = h1[v] > 0.0 ? a : 0.0;
        }
        for (int u = 0; u < ORC_MLP_H; ++u) {
            g->b2[u] += d2[u];
            for (int v = 0; v < ORC_MLP_H; ++v)
                g->W2[u * ORC_MLP_H + v] += d2[u] * h1[v];
        }
        for (int u = 0; u < ORC_MLP_H; ++u) {
            g->b1[u] += d1[u];
            for (int f = 0; f < ORC_MLP_IN; ++f)
                g->W1[u * ORC_MLP_IN + f] += d1[u] * z[f];
        }
    }
    return loss;
}

#define TAG_MLP_BATCH 5u
#define TAG_MLP_INIT 6u

void orc_mlp_init(uint64_t seed, orc_mlp *net)
{
    memset(net, 0, sizeof *net);
    uint32_t key[2];
    make_key(seed, 0u, key);
    const int P_W1 = 0, P_W2 = 64 * 16, P_W3 = P_W2 + 64 * 64, P_W4 = P_W3 + 64 * 64, P_B = P_W4 + 16 * 64;
    for (int p = 0; p < P_B; ++p) {
        uint32_t ctr[4] = {(uint32_t)(p / 4), 0u, TAG_MLP_INIT, 0u};
        double z4[4];
        orc_normals4(ctr, key, z4);
        const double z = z4[p % 4];
        if (p < P_W2) {
            const int u = (p - P_W1) / 16, f = (p - P_W1) % 16;
            if (f < ORC_MLP_IN)
                net->W1[u * ORC_MLP_IN + f] = z * sqrt(2.0 / ORC_MLP_IN);
        } else if (p < P_W3) {
            net->W2[p - P_W2] = z * sqrt(2.0 / ORC_MLP_H);
        } else if (p < P_W4) {
            net->W3[p - P_W3] = z * sqrt(2.0 / ORC_MLP_H);
        } else if (p - P_W4 < ORC_MLP_H) {
            net->w4[p - P_W4] = z * sqrt(1.0 / ORC_MLP_H);
        }
    }
    net->b4 = 1.0;
}

void orc_mlp_batch_rows(uint64_t seed, int32_t step, int64_t B, int64_t n_rows, int64_t *idx)
{
    uint32_t key[2];
    make_key(seed, 0u, key);
    for (int64_t i = 0; i < B; ++i) {
        uint32_t ctr[4] = {(uint32_t)step, (uint32_t)i, TAG_MLP_BATCH, 0u}, x[4];
        orc_philox4x32_10(ctr, key, x);
        idx[i] = (int64_t)(((uint64_t)x[0] * (uint64_t)n_rows) >> 32);
    }
}

static int cmp_f64(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

void orc_mlp_stats(const double *rows, int64_t n, double box_q, orc_mlp *net)
{
    double *col = (double *)malloc(sizeof(double) * (size_t)n);
    for (int f = 0; f < ORC_MLP_IN; ++f) {
        double s = 0.0, q = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double x = rows[i * (ORC_MLP_IN + 1) + f];
            col[i] = x;
            s += x;
            q += x * x;
        }
        const double mu = s / (double)n;
        double var = q / (double)n - mu * mu;
        if (var < 0.0)
            var = 0.0;
        double sd = sqrt(var);
        if (sd < 1e-6)
            sd = 1e-6;
        net->mean[f] = mu;
        net->istd[f] = 1.0 / sd;
        qsort(col, (size_t)n, sizeof(double), cmp_f64);
        if (box_q <= 0.0) {
            net->lo[f] = col[0];
            net->hi[f] = col[n - 1];
        } else {   /* nearest rank: the smallest value with at least ceil(q n) values <= it */
            const int64_t r_lo = (int64_t)ceil(box_q * (double)n), r_hi = (int64_t)ceil((1.0 - box_q) * (double)n);
            net->lo[f] = col[(r_lo < 1 ? 1 : r_lo) - 1];
            net->hi[f] = col[(r_hi < 1 ? 1 : r_hi) - 1];
        }
    }
    free(col);
}

void orc_adam(int64_t n, double *w, double *m, double *v, const double *g, double lr, int64_t t)
{
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* Inputs of the learned controller at a sample: the sensor history y_k..y_k-5; the insulin
 * on board, as the mean change of G over the MPC's prediction horizon that the insulin
 * states' deviation from basal still causes, sum over S1, S2, I, x1, x2, x3 of
 * Fbar_s (x_s - x*_s); the announced meals likewise, Fbar_D1 D1 + Fbar_D2 D2 + wbar dhat;
 * and the patient: u_b, the insulin response over the horizon (sum of the Markov parameters
 * h_1..h_N), its mean delay (sum m h_m / sum h_m, samples), BW. Fbar and wbar are the horizon
 * means of the prediction rows and of the intake response. (The insulin and absorption subsystems are deterministic and the
 * meals announced exactly, so a controller-side replica driven by the doses and the
 * announcements has the plant's values.) */
static void mlp_inputs(const mpc_state *st, const double *p, double ub, const double x[ORC_NX], const double yh[6],
                       double dhat, double f[ORC_MLP_IN])
{
    static const int ins[6] = {X_S1, X_S2, X_I, X_X1, X_X2, X_X3};
    for (int i = 0; i < 6; ++i)
        f[i] = yh[i];
    double a = 0.0;
    for (int i = 0; i < 6; ++i)
        a += st->Fbar[ins[i]] * (x[ins[i]] - st->m.xss[ins[i]]);
    f[6] = a;
    f[7] = st->Fbar[X_D1] * x[X_D1] + st->Fbar[X_D2] * x[X_D2] + st->wbar * dhat;
    f[8] = ub;
    f[9] = st->hsum;
    f[10] = st->hdelay;
    f[11] = p[P_BW];
}

/* The network acts unless an input is outside its box or, while the sensor reads low
 * (y_k < mlp_safe_g), its output exceeds mlp_safe_out (e.g. 3.0 mmol/L and 1: not above basal);
 * then the MPC solves its QP. The Kalman filter runs on
 * every sample; when the network acts the MPC's plan is only shifted. With `label` non-NULL
 * (data aggregation along the network's closed loop) the QP is solved on every sample and
 * *label receives the MPC's action, whoever acts. */
static double mlp_step(const orc_config *cfg, mpc_state *st, const double f[ORC_MLP_IN], double y, double dhat,
                       int32_t *fallbacks, double *label)
{
    const orc_mlp *net = cfg->mlp;
    mpc_measure(st, y);
    double z[ORC_MLP_IN], h1[ORC_MLP_H], h2[ORC_MLP_H], h3[ORC_MLP_H];
    const double o = mlp_eval(net, f, z, h1, h2, h3);
    int ood = 0;
    for (int q = 0; q < ORC_MLP_IN; ++q)
        if (!(f[q] >= net->lo[q] && f[q] <= net->hi[q]))
            ood = 1;
    const int fb = ood || (y < cfg->mlp_safe_g && o > cfg->mlp_safe_out);
    double du_mpc = 0.0;
    if (fb || label)
        du_mpc = mpc_plan(cfg, st, dhat);
    else
        mpc_shift(st);
    double u, du;
    if (fb) {
        du = du_mpc;
        u = st->m.ub + du;
        ++*fallbacks;
    } else {
        u = st->m.ub * o;
        u = u < 0.0 ? 0.0 : (u > st->m.umax ? st->m.umax : u);
        du = u - st->m.ub;
    }
    if (label)
        *label = st->m.ub + du_mpc;
    mpc_predict(st, du, dhat);
    return u;
}

/* ------------------------------------------------------------ main loop ---- */
static void simulate_patient(const orc_config *cfg, int64_t j, int64_t count, uint32_t patient,
                             const orc_outputs *out)
{
    double prm[ORC_NPOUT];
    sample_patient(cfg, patient, prm);
    const double *p = prm;
    double ub = prm[15], istar, ub2;
    double x[ORC_NX];
    acc_t a;
    memset(&a, 0, sizeof a);
    a.min_g = INFINITY;
    a.argmin_k = -1;
    a.ctrl_margin = INFINITY;
    a.status = (uint32_t)prm[18];
    if (!orc_basal(cfg, p, &istar, &ub2, x)) {
        for (int i = 0; i < ORC_NX; ++i) x[i] = NAN;
        ub = 0.0;
    }
    for (int i = 0; i < ORC_NX; ++i)
        x[i] += cfg->x0_offset[i];

    uint32_t nkey[2];
    make_key(cfg->noise_seed, cfg->arm_id, nkey);
    const int M = cfg->em_per_ctrl;
    const int32_t ts = cfg->ts_min;
    const int32_t kday = 1440 / ts;
    const int64_t K = (int64_t)cfg->n_days * kday;
    const double h = (double)ts / (double)M;
    const double sqrt_h = sqrt(h);
    const double sqrt_r = sqrt(cfg->cgm_var);
    const int noisy = (cfg->sigma_q1 != 0.0) || (cfg->cgm_var != 0.0);
    double sig[ORC_NX] = {0};
    sig[X_Q1] = cfg->sigma_q1;
    const double vg = p[P_VG] * p[P_BW];
    pid_t_ pid = {0.0, 0.0, 0};
    dual_t dual;
    memset(&dual, 0, sizeof dual);
    double xe[ORC_NXE] = {0};           /* extension states (model_ext): 0 at the basal state */
    double dose_basal = 0.0, dose_bolus = 0.0, dose_glucagon = 0.0;
    const int32_t n_ex = exercise_samples(cfg);
    int is_traj = j < out->n_traj;
    mpc_state *mpc = NULL;
    int32_t fallbacks = 0;
    const int use_inputs = cfg->ctrl_kind == ORC_CTRL_MLP || out->record != NULL;
    double yh[6] = {0};   /* y_k, y_k-1, ..., y_k-5 */
    if (cfg->ctrl_kind == ORC_CTRL_MPC || cfg->ctrl_kind == ORC_CTRL_MLP) {
        mpc = (mpc_state *)calloc(1, sizeof *mpc);
        if (!orc_mpc_setup(cfg, prm, &mpc->m)) {
            free(mpc);
            mpc = NULL;
        } else {
            const int N = mpc->m.N;
            for (int c = 0; c < ORC_NX; ++c) {
                double acc = 0.0;
                for (int jj = 0; jj < N; ++jj)
                    acc += mpc->m.F[jj * ORC_NX + c];
                mpc->Fbar[c] = acc / N;
            }
            double wacc = 0.0;
            for (int jj = 0; jj < N; ++jj)
                wacc += mpc->m.w[jj];
            mpc->wbar = wacc / N;
            double hs = 0.0, hm = 0.0;
            for (int m = 0; m < N; ++m) {
                hs += mpc->m.h[m];
                hm += (double)(m + 1) * mpc->m.h[m];
            }
            mpc->hsum = hs;
            mpc->hdelay = hm / hs;
        }
    }

    for (int32_t day = 0; day < cfg->n_days; ++day) {
        meal_t meals[ORC_MAX_DAY_MEALS];
        int nm = meals_for_day(cfg, patient, day, p[14], nkey, meals);
        const int32_t ex0 = exercise_onset(cfg, patient, day, nkey);
        for (int32_t kd = 0; kd < kday; ++kd) {
            int64_t k = (int64_t)day * kday + kd;
            double G = x[X_Q1] / vg;
            acc_sample(&a, G, (int32_t)k, cfg->guard_rel);

            /* normals of this sample: samples are drawn in pairs (2j, 2j+1); pair j takes
               the blocks with counter (j, patient, DIFF, c), c = 0, 1, ..., numbers their
               normals in order, gives normals 0..M to sample 2j and M+1..2M+1 to sample
               2j+1; within a sample xi_s = normal s (s < M) and v_k = normal M */
            double zall[64] = {0};
            const double *z = zall + (k & 1) * (M + 1);
            if (noisy) {
                int ncall = (2 * (M + 1) + 3) / 4;
                for (int c = 0; c < ncall; ++c) {
                    uint32_t ctr[4] = {(uint32_t)(k >> 1), patient, TAG_DIFF, (uint32_t)c};
                    orc_normals4(ctr, nkey, &zall[4 * c]);
                }
            }
            double y = x[X_GI] + sqrt_r * z[M];

            double d = 0.0;   /* held intake of this interval, also the announcement */
            for (int m = 0; m < nm; ++m)
                if (meals[m].kd == kd)
                    d += meals[m].rate;

            double f[ORC_MLP_IN], label = NAN;
            if (use_inputs) {
                if (k == 0)
                    for (int i = 1; i < 6; ++i) yh[i] = y;
                yh[0] = y;
                if (mpc)
                    mlp_inputs(mpc, p, ub, x, yh, d, f);
                else
                    for (int q = 0; q < ORC_MLP_IN; ++q) f[q] = NAN;
            }

            /* exercise input of this interval (model extensions) */
            const int in_session = ex0 >= 0 && kd >= ex0 && kd < ex0 + n_ex;
            const double hrr = cfg->hrr_const + (in_session ? cfg->exercise_hrr : 0.0);
            double u, un = 0.0, u_bolus = 0.0, u_basal = NAN;
            if (cfg->ctrl_kind == ORC_CTRL_DUAL) {
                const double iob = x[X_S1] + x[X_S2] - 2.0 * ub * p[P_TMAXI];
                const double gob = xe[XE_Z1] + xe[XE_Z2];
                dual_step(cfg, &dual, y, ub, iob, gob, d, kd == ex0, &u_basal, &u_bolus, &un, &a.ctrl_margin);
                u = u_basal + u_bolus;
            } else if (cfg->ctrl_kind == ORC_CTRL_PID)
                u = pid_step(cfg, &pid, y, cfg->basal_scale * ub, &a.ctrl_margin);
            else if (cfg->ctrl_kind == ORC_CTRL_MPC)
                u = mpc ? mpc_step(cfg, mpc, y, d) : NAN;
            else if (cfg->ctrl_kind == ORC_CTRL_MLP)
                u = mpc ? mlp_step(cfg, mpc, f, y, d, &fallbacks, out->record ? &label : NULL) : NAN;
            else {
                u = cfg->u_rel * (cfg->basal_scale * ub);
                un = cfg->un_open;
            }

            if (use_inputs) {
                for (int i = 5; i > 0; --i) yh[i] = yh[i - 1];
                if (out->record) {   /* inputs, then the MPC's action / u_b */
                    double *row = out->record + (k * count + j) * (ORC_MLP_IN + 1);
                    for (int q = 0; q < ORC_MLP_IN; ++q) row[q] = f[q];
                    row[ORC_MLP_IN] = (cfg->ctrl_kind == ORC_CTRL_MLP ? label : u) / ub;
                }
            }

            if (is_traj) {
                if (out->traj_g) out->traj_g[j * K + k] = G;
                if (out->traj_y) out->traj_y[j * K + k] = y;
                if (out->traj_u) out->traj_u[j * K + k] = u;
                if (out->traj_x)
                    for (int i = 0; i < ORC_NX; ++i) out->traj_x[(j * K + k) * ORC_NX + i] = x[i];
                if (out->traj_xe)
                    for (int i = 0; i < ORC_NXE; ++i) out->traj_xe[(j * K + k) * ORC_NXE + i] = xe[i];
            }

            if (cfg->model_ext) {   /* the extended model on its 16 states */
                double X[ORC_NX + ORC_NXE];
                memcpy(X, x, sizeof x);
                memcpy(X + ORC_NX, xe, sizeof xe);
                if (cfg->integrator == ORC_INT_RK4) {
                    double hr = (double)ts / (double)cfg->rk4_sub;
                    for (int s = 0; s < cfg->rk4_sub; ++s)
                        rk4_step_ext(cfg, p, X, u, un, d, hrr, hr);
                } else {
                    double sig16[ORC_NX + ORC_NXE] = {0};
                    sig16[X_Q1] = cfg->sigma_q1;
                    for (int s = 0; s < M; ++s) {
                        double F[ORC_NX + ORC_NXE], xi[ORC_NX + ORC_NXE] = {0};
                        rhs16(cfg, p, X, u, un, d, hrr, F);
                        xi[X_Q1] = z[s];
                        em_step(ORC_NX + ORC_NXE, X, F, h, sqrt_h, sig16, xi);
                    }
                }
                memcpy(x, X, sizeof x);
                memcpy(xe, X + ORC_NX, sizeof xe);
            } else if (cfg->integrator == ORC_INT_RK4) {
                double hr = (double)ts / (double)cfg->rk4_sub;
                for (int s = 0; s < cfg->rk4_sub; ++s)
                    rk4_step(cfg, p, x, u, d, hr);
            } else {
                for (int s = 0; s < M; ++s) {
                    double f[ORC_NX], xi[ORC_NX] = {0};
                    orc_rhs(cfg, p, x, u, d, f);
                    xi[X_Q1] = z[s];
                    em_step(ORC_NX, x, f, h, sqrt_h, sig, xi);
                }
            }
            a.sum_u += u * (double)ts;
            dose_basal += (cfg->ctrl_kind == ORC_CTRL_DUAL ? u_basal : u) * (double)ts;
            dose_bolus += u_bolus * (double)ts;
            dose_glucagon += un * (double)ts;
        }
        for (int i = 0; i < ORC_NX; ++i)
            if (!isfinite(x[i]))
                a.status |= ORC_ST_NONFINITE;
        for (int i = 0; i < ORC_NXE; ++i)
            if (!isfinite(xe[i]))
                a.status |= ORC_ST_NONFINITE;
    }
    if (out->doses) {
        out->doses[j * 3 + 0] = dose_basal;
        out->doses[j * 3 + 1] = dose_bolus;
        out->doses[j * 3 + 2] = dose_glucagon;
    }
    free(mpc);

    for (int b = 0; b < 5; ++b) out->bins[j * 5 + b] = a.bins[b];
    for (int e = 0; e < 3; ++e) out->events[j * 3 + e] = a.events[e];
    out->sum_g[j] = a.sum_g;
    out->min_g[j] = a.min_g;
    out->argmin_k[j] = a.argmin_k;
    out->sum_u[j] = a.sum_u;
    out->status[j] = a.status;
    if (out->fallback) out->fallback[j] = fallbacks;
    if (out->n_near) out->n_near[j] = a.n_near;
    if (out->ctrl_margin) out->ctrl_margin[j] = a.ctrl_margin;
    if (out->params)
        for (int i = 0; i < ORC_NPOUT; ++i) out->params[j * ORC_NPOUT + i] = prm[i];
}

typedef struct {
    const orc_config *cfg;
    const orc_outputs *out;
    int64_t first, count;
    int tid, nthreads;
} job_t;

static void *worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    for (int64_t j = jb->tid; j < jb->count; j += jb->nthreads)
        simulate_patient(jb->cfg, j, jb->count, (uint32_t)(jb->first + j), jb->out);
    return NULL;
}

int orc_simulate(const orc_config *cfg, int64_t first, int64_t count, int n_threads, const orc_outputs *out)
{
    if (cfg->ts_min <= 0 || 1440 % cfg->ts_min != 0 || cfg->em_per_ctrl < 1 || cfg->em_per_ctrl > 31)
        return -1;
    if (cfg->n_slots < 0 || cfg->n_slots > ORC_MAX_SLOTS || cfg->n_days < 0 || count < 0)
        return -1;
    if (cfg->proto != ORC_PROTO_SLOTS && cfg->proto != ORC_PROTO_NORDIC)
        return -1;
    if (!(cfg->basal_scale > 0.0))
        return -1;
    for (int m = 0; m < (cfg->proto == ORC_PROTO_SLOTS ? cfg->n_slots : 0); ++m)
        if (cfg->minute_of_day[m] - cfg->jitter < 0 || cfg->minute_of_day[m] + cfg->jitter >= 1440)
            return -1;
    if (cfg->integrator == ORC_INT_RK4 && (cfg->sigma_q1 != 0.0 || cfg->cgm_var != 0.0 || cfg->rk4_sub < 1))
        return -1;
    if (cfg->ctrl_kind == ORC_CTRL_MLP && !cfg->mlp)
        return -1;
    if (out->record && cfg->ctrl_kind != ORC_CTRL_MPC && cfg->ctrl_kind != ORC_CTRL_MLP)
        return -1;   /* the recorded inputs and labels come from the MPC's model */
    if ((cfg->ctrl_kind == ORC_CTRL_MPC || cfg->ctrl_kind == ORC_CTRL_MLP) &&
        (cfg->mpc_horizon < 1 || cfg->mpc_horizon > ORC_NMAX || cfg->mpc_iters < 0 || cfg->mpc_riccati_iters < 0 ||
         cfg->mpc_power_iters < 1 || !(cfg->mpc_rho > 0.0)))
        return -1;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > 256)
        n_threads = 256;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < n_threads; ++t) {
        jobs[t].cfg = cfg;
        jobs[t].out = out;
        jobs[t].first = first;
        jobs[t].count = count;
        jobs[t].tid = t;
        jobs[t].nthreads = n_threads;
    }
    if (n_threads == 1) {
        worker(&jobs[0]);
        return 0;
    }
    for (int t = 0; t < n_threads; ++t)
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t)
        pthread_join(th[t], NULL);
    return 0;
}

/* ------------------------------------------------------------ reduction ---- */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Population summary. Quantile p (percent) is the nearest rank: the value at
 * position ceil(p n / 100) of the sorted per-patient in-range counts. The worst
 * patient is the lexicographic minimum of (min G, patient index). The same totals,
 * quantiles and means are repeated over the unflagged patients (status == 0). */
void orc_reduce(int64_t n, int64_t k, const int32_t *bins, const int32_t *events, const double *sum_g,
                const double *min_g, const int32_t *argmin_k, const uint32_t *status, orc_summary *s)
{
    memset(s, 0, sizeof *s);
    s->n = n;
    s->k = k;
    s->worst_patient = -1;
    s->worst_min_g = INFINITY;
    double total_g = 0.0, total_g_clean = 0.0;
    int32_t *tir = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *tir_clean = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        for (int b = 0; b < 5; ++b) s->bins[b] += (uint64_t)bins[i * 5 + b];
        for (int e = 0; e < 3; ++e) s->events[e] += (uint64_t)events[i * 3 + e];
        total_g += sum_g[i];
        tir[i] = bins[i * 5 + 2];
        if (min_g[i] < s->worst_min_g) {
            s->worst_min_g = min_g[i];
            s->worst_patient = i;
            s->worst_k = argmin_k[i];
        }
        for (int t = 0; t < 3; ++t)
            if (status[i] & (1u << t)) s->status_count[t] += 1;
        if (status[i] == 0) {
            for (int b = 0; b < 5; ++b) s->bins_clean[b] += (uint64_t)bins[i * 5 + b];
            total_g_clean += sum_g[i];
            tir_clean[s->n_clean++] = bins[i * 5 + 2];
        }
    }
    qsort(tir, (size_t)n, sizeof(int32_t), cmp_i32);
    qsort(tir_clean, (size_t)s->n_clean, sizeof(int32_t), cmp_i32);
    static const int64_t pct[5] = {5, 25, 50, 75, 95};
    const int64_t nc = s->n_clean;
    for (int q = 0; q < 5; ++q) {
        int64_t r = (pct[q] * n + 99) / 100;
        s->q_count[q] = n > 0 ? tir[r - 1] : 0;
        int64_t rc = (pct[q] * nc + 99) / 100;
        s->q_count_clean[q] = nc > 0 ? tir_clean[rc - 1] : 0;
    }
    s->mean_tir = (n > 0 && k > 0) ? (double)s->bins[2] / ((double)n * (double)k) : 0.0;
    s->mean_bg = (n > 0 && k > 0) ? total_g / ((double)n * (double)k) : 0.0;
    s->mean_tir_clean = (nc > 0 && k > 0) ? (double)s->bins_clean[2] / ((double)nc * (double)k) : 0.0;
    s->mean_bg_clean = (nc > 0 && k > 0) ? total_g_clean / ((double)nc * (double)k) : 0.0;
    free(tir);
    free(tir_clean);
}
