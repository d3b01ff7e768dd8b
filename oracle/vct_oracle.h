/*
 * vct_oracle.h -- plain FP64 CPU oracle for closed-loop virtual clinical trials.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. The GPU product path never calls it,
 * shares no source with it, and must fail if its own HIP library is missing.
 *
 * What it computes (paper: "High-performance Uncertainty Quantification in
 * Large-scale Virtual Clinical Trials of Closed-loop Diabetes Treatment"):
 *   - the stochastic patient model in the general SDE form of Sec. III-A, eq. (1):
 *     x(t0)=x0, dx = f dt + sigma dw, z = h(x), y_k = g(x(t_k)) + v_k,
 *     dw ~ N(0, I dt), v_k ~ N(0, R), with inputs held constant between samples (eq. 2);
 *     f is the Hovorka core model extended with a one-state CGM model (Sec. IV-B);
 *   - a discrete-time controller in the kappa/lambda form of Sec. III-B (eq. 3);
 *   - the five glucose ranges of Sec. IV-A accumulated on the fly, one simulation at a
 *     time, as the low-memory scheme of Sec. III-C does;
 *   - closed-loop Monte Carlo over independent patients (Sec. III, III-C).
 * Everything is FP64, written step by step in the order the method defines.
 */
#ifndef VCT_ORACLE_H
#define VCT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NP 15          /* sampled patient parameters                       */
#define ORC_NX 11          /* model states                                     */
#define ORC_NPOUT 19       /* 15 parameters + u_b, I*, attempts, status        */
#define ORC_MAX_SLOTS 4
#define ORC_MAX_DAY_MEALS 8   /* meals of one day, either protocol */
#define ORC_PROTO_SLOTS  0
#define ORC_PROTO_NORDIC 1

/* controller kinds */
#define ORC_CTRL_OPEN 0    /* constant u = u_rel * u_b (test mode)              */
#define ORC_CTRL_PID  1
#define ORC_CTRL_MPC  2
#define ORC_CTRL_MLP  3
#define ORC_CTRL_DUAL 4    /* dual-hormone AP (insulin mode / glucagon mode), model extensions on */

/* states of the model extensions (Sec. IV-B), after the 11 core states */
#define ORC_NXE 5          /* Z1, Z2 (subcutaneous glucagon), E1, E2, E3 (exercise) */

/* integrators */
#define ORC_INT_EM  0      /* Euler-Maruyama with em_per_ctrl substeps          */
#define ORC_INT_RK4 1      /* classical RK4, rk4_sub substeps per sample; noise must be off */

/* status bits per patient */
#define ORC_ST_NONFINITE   1u
#define ORC_ST_NEGATIVE_Q1 2u
#define ORC_ST_RESAMPLE    4u

/* population flag */
#define ORC_POP_MIN_BASAL 1u   /* additionally require u_b >= 0.4 U/h (6.6667 mU/min) */

typedef struct {
    /* (1)+(4) population and parameter values */
    uint64_t pop_seed;
    uint32_t arm_id;
    uint32_t pop_flags;
    double   nominal[ORC_NP];   /* EGP0 F01 k12 ka1 ka2 ka3 SIT SID SIE ke VI VG tmaxI tmaxG BW */
    double   cv;                /* coefficient of variation of the lognormal draws          */
    double   ag;                /* carbohydrate bioavailability (shared by all patients)    */
    double   tau_cgm;           /* sensor lag time constant, min (shared)                    */
    double   g_target;          /* glucose level of the basal steady state, mmol/L          */
    /* (2) protocol: meal slots, one draw per (day, slot) */
    int32_t  n_slots;
    int32_t  minute_of_day[ORC_MAX_SLOTS];
    double   carbs_mean[ORC_MAX_SLOTS];
    double   carbs_sd[ORC_MAX_SLOTS];
    double   prob[ORC_MAX_SLOTS];
    int32_t  jitter;            /* onset jitter uniform on the integers [-jitter, jitter] min */
    int32_t  proto;             /* ORC_PROTO_SLOTS: the slots above; ORC_PROTO_NORDIC: Sec. II-B */
    double   meal_cv;           /* ORC_PROTO_NORDIC: relative SD of each meal's carbohydrate */
    /* (5) controller */
    int32_t  ctrl_kind;
    double   setpoint;          /* mmol/L */
    double   kp, ki, kd;        /* relative to u_b: u_b/(mmol/L), u_b/(mmol/L min), u_b min/(mmol/L) */
    double   umax_rel;          /* u_max = umax_rel * u_b */
    double   u_rel;             /* open-loop mode: u = u_rel * u_b */
    double   basal_scale;       /* the controller's basal rate is basal_scale * u_b (PID, open loop) */
    /* (3) model + simulation settings */
    int32_t  n_days;
    int32_t  em_per_ctrl;       /* EM substeps per control interval */
    int32_t  ts_min;            /* control interval, integer minutes dividing 1440 */
    double   sigma_q1;          /* diffusion on Q1, mmol min^-1/2 */
    double   cgm_var;           /* R, (mmol/L)^2 */
    uint64_t noise_seed;
    int32_t  integrator;        /* ORC_INT_EM / ORC_INT_RK4 */
    int32_t  rk4_sub;
    double   x0_offset[ORC_NX]; /* added to the basal steady state (tests only) */
    double   guard_rel;         /* band used for the near-decision diagnostics */
    /* linear MPC */
    int32_t  mpc_horizon;       /* N (prediction = control horizon), <= ORC_NMAX */
    int32_t  mpc_iters;         /* projected-gradient iterations per sample */
    double   mpc_rho;           /* weight of ((u - u_b)/u_b)^2 */
    int32_t  mpc_riccati_iters; /* fixed Riccati iterations for the stationary Kalman gain */
    int32_t  mpc_power_iters;   /* power iterations for lambda_max(Gamma^T Gamma) */
    /* learned controller (ORC_CTRL_MLP): the network, its input normalisation and box, and
       the safety hand-over: the MPC acts when y_k < mlp_safe_g and out > mlp_safe_out */
    const struct orc_mlp_s *mlp;
    double   mlp_safe_g, mlp_safe_out;
    /* model extensions of Sec. IV-B, parameters shared by all patients (model_ext = 0: the
       core model alone, every other field below unused) */
    int32_t  model_ext;
    double   tau_n;             /* subcutaneous glucagon absorption time constant, min       */
    double   e_n;               /* hepatic glucose output per glucagon appearance, mmol/ug    */
    double   tau_e1, tau_e2, tau_e3;   /* exercise: heart rate, uptake, sensitivity; min      */
    double   alpha_e;           /* insulin-independent uptake at full effect, 1/min           */
    double   beta_e;            /* relative rise of insulin action at full effect             */
    /* exercise sessions on the Northern-European protocol's active days (Sec. II-B) */
    int32_t  exercise;          /* 0/1 */
    int32_t  exercise_minute;   /* clock minute of the onset before its jitter                */
    int32_t  exercise_duration; /* minutes                                                    */
    double   exercise_hrr;      /* heart-rate reserve fraction during a session               */
    double   hrr_const;         /* tests: heart-rate reserve fraction held at every sample    */
    double   un_open;           /* open-loop mode: glucagon infusion, ug/min                  */
    /* dual-hormone AP (ORC_CTRL_DUAL, Sec. IV-C) */
    int32_t  meal_bolus;        /* 0/1: meal bolus calculator in insulin mode                 */
    double   icr_rule;          /* ICR = icr_rule / TDD g/U, TDD = 2 x daily basal insulin     */
    double   glu_enter, glu_exit;   /* glucagon mode when y < glu_enter, insulin mode again at y >= glu_exit */
    double   glu_target, glu_kp, glu_max;   /* microbolus min(glu_max, glu_kp (glu_target - y)) ug */
    double   ex_bolus, ex_bolus_below;      /* ug at an exercise onset when y < ex_bolus_below   */
} orc_config;

/* Learned controller: 12 inputs -> 64 -> 64 -> 64 -> 1, ReLU hidden layers. The inputs are
 * z-scored with (mean, istd) and rounded to BF16 (the network's input format); everything
 * after that is exact FP64 arithmetic on the stored weights. */
#define ORC_MLP_IN 12
#define ORC_MLP_H 64
typedef struct orc_mlp_s {
    double W1[ORC_MLP_H * ORC_MLP_IN], b1[ORC_MLP_H];    /* W1[u][f] at u*12 + f */
    double W2[ORC_MLP_H * ORC_MLP_H], b2[ORC_MLP_H];     /* W2[u][v] at u*64 + v */
    double W3[ORC_MLP_H * ORC_MLP_H], b3[ORC_MLP_H];
    double w4[ORC_MLP_H], b4;
    double mean[ORC_MLP_IN], istd[ORC_MLP_IN];           /* input z-score */
    double lo[ORC_MLP_IN], hi[ORC_MLP_IN];               /* box outside which the MPC acts */
} orc_mlp;

#define ORC_NMAX 48

/* Per-patient linear MPC (Sec. III-B form, control state = Kalman estimate + input plan). */
typedef struct {
    int32_t N;
    double A[ORC_NX * ORC_NX], B[ORC_NX], E[ORC_NX];   /* sample-to-sample linear model */
    double K[ORC_NX];                                   /* stationary Kalman gain (sensor GI) */
    double h[ORC_NMAX];                                 /* Markov parameters c_G A^(m-1) B, m = 1..N */
    double F[ORC_NMAX * ORC_NX];                        /* rows c_G A^(j+1), j = 0..N-1 */
    double w[ORC_NMAX];                                 /* c_G A^j E: response to the announced intake */
    double Gx[ORC_NMAX * ORC_NX], gd[ORC_NMAX], g1[ORC_NMAX];   /* Gamma^T F, Gamma^T w, Gamma^T 1 */
    double lambda, rho_p, step;                         /* lambda_max(Gamma^T Gamma), rho/u_b^2, 1/(lambda+rho_p) */
    double xss[ORC_NX], ub, umax, gstar;
    double P[ORC_NX * ORC_NX];                          /* prior covariance at the last Riccati iteration */
    double P_change;                                    /* max |P_n - P_(n-1)| of the last iteration */
} orc_mpc;

typedef struct {
    int32_t  *bins;        /* [count][5] samples per glucose range          */
    int32_t  *events;      /* [count][3] runs >= 3 samples: <3.9, <3.0, >13.9 */
    double   *sum_g;       /* [count] sum of G over samples, mmol/L          */
    double   *min_g;       /* [count]                                         */
    int32_t  *argmin_k;    /* [count] first sample index of min_g            */
    double   *sum_u;       /* [count] delivered insulin, mU                   */
    uint32_t *status;      /* [count]                                         */
    int32_t  *n_near;      /* [count] samples within guard_rel of a range edge */
    double   *ctrl_margin; /* [count] min |u_unc|/u_b, |u_unc-u_max|/u_b over samples */
    double   *params;      /* [count][ORC_NPOUT] or NULL                      */
    int32_t   n_traj;      /* trajectories for the first n_traj patients      */
    double   *traj_g, *traj_y, *traj_u;   /* [n_traj][K] (any may be NULL)   */
    double   *traj_x;      /* [n_traj][K][ORC_NX] state at each sample or NULL */
    double   *record;      /* [K][count][13] controller inputs, then the MPC's action / u_b
                              (MPC; MLP: the QP is then solved on every sample) or NULL */
    int32_t  *fallback;    /* [count] samples on which the MPC acted for the MLP, or NULL */
    double   *doses;       /* [count][3] basal insulin mU, bolus insulin mU, glucagon ug, or NULL */
    double   *traj_xe;     /* [n_traj][K][ORC_NXE] extension states at each sample, or NULL */
} orc_outputs;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void     orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniform on (0,1): odd multiples of 2^-24 built from the top 23 bits. */
double   orc_uniform(uint32_t x);
/* Four normals of one Philox call, Box-Muller pairs (u0,u1) and (u2,u3). */
void     orc_normals4(const uint32_t ctr[4], const uint32_t key[2], double z[4]);

/* Population: sampled parameters of patients [first, first+count). out: [count][ORC_NPOUT]. */
void     orc_sample_population(const orc_config *cfg, int64_t first, int64_t count, double *out);
/* Basal steady state for one parameter vector (absolute units built inside). Returns 1 if feasible. */
int      orc_basal(const orc_config *cfg, const double p[ORC_NP], double *i_star, double *u_b, double x0[ORC_NX]);
/* Drift f(x, u, D) of the patient model for parameter vector p (per-kg units as sampled). */
void     orc_rhs(const orc_config *cfg, const double p[ORC_NP], const double x[ORC_NX], double u, double d, double dx[ORC_NX]);

/* Test hooks: the meal draws of one (patient, day) -> [n_slots][4] = (present, sample index
   in the day, carbs g, jitter min); a PID run over a scripted measurement sequence. */
void     orc_meals(const orc_config *cfg, uint32_t patient, int32_t day, double *out);
/* Northern-European protocol (Sec. II-B, Tables I and II): out[0..2] = season (0 winter,
 * 1 spring, 2 summer, 3 autumn), week type (0 standard, 1 active, 2 vacation) and day type
 * (0 standard, 1 active, 2 movie night, 3 late night) of a patient's day. */
void     orc_nordic_day(const orc_config *cfg, uint32_t patient, int32_t day, int32_t *out);
/* The meals of one (patient, day) under either protocol, in time order: returns their
 * number n and writes out[n][3] = (sample index within the day, carbs g, intake mmol/min). */
int      orc_day_meals(const orc_config *cfg, uint32_t patient, int32_t day, double *out);
void     orc_pid_run(const orc_config *cfg, double ub, int32_t n, const double *y, double *u, double *integ);

/* Linear MPC. Jacobian of the drift at (x, u, D = 0); B_c = df/du, E_c = df/dD. */
void     orc_jacobian(const orc_config *cfg, const double p[ORC_NP], const double x[ORC_NX], double J[ORC_NX * ORC_NX],
                      double Bc[ORC_NX], double Ec[ORC_NX]);
/* Setup from a sampled parameter row ([ORC_NPOUT]); returns 0 if the basal state does not exist. */
int      orc_mpc_setup(const orc_config *cfg, const double prm[ORC_NPOUT], orc_mpc *m);
/* Projected-gradient iterations on the box QP from the start dU (overwritten). */
void     orc_mpc_pg(const orc_mpc *m, const double g[], double dU[], int iters);

/* Learned controller. Round to the nearest BF16 value (8 significant bits, ties to even). */
double   orc_bf16(double x);
/* Network outputs for n raw input rows x[n][12]. */
void     orc_mlp_forward(const orc_mlp *net, const double *x, int64_t n, double *out);
/* Mean squared error (1/B) sum_i (out(x_idx[i]) - t_idx[i])^2 over rows[.][13] (inputs, then
 * target) and its gradient with respect to W1..b4 (written into grad; grad's normalisation
 * fields are zeroed). Returns the loss. */
double   orc_mlp_loss_grad(const orc_mlp *net, const double *rows, const int64_t *idx, int64_t B, orc_mlp *grad);
/* He-normal initial weights (std sqrt(2/fan_in), output layer sqrt(1/64)), zero biases but
 * b4 = 1. Parameters are numbered in the padded order W1[64][16], W2[64][64], W3[64][64],
 * W4[16][64], b1, b2, b3, b4[16]; number p takes normal p%4 of the block (p/4, 0, 6, 0). */
void     orc_mlp_init(uint64_t seed, orc_mlp *net);
/* Minibatch rows drawn with replacement: floor(x n_rows / 2^32), x = word 0 of (step, i, 5, 0). */
void     orc_mlp_batch_rows(uint64_t seed, int32_t step, int64_t B, int64_t n_rows, int64_t *idx);
/* Input mean, 1/std (population std, floor 1e-6) and box: box_q = 0 -> [min, max], else the
 * nearest-rank box_q and 1 - box_q quantiles. */
void     orc_mlp_stats(const double *rows, int64_t n, double box_q, orc_mlp *net);
/* Adam step t (1-based) with beta 0.9 / 0.999, eps 1e-8 on n parameters. */
void     orc_adam(int64_t n, double *w, double *m, double *v, const double *g, double lr, int64_t t);

/* The extended model (Sec. IV-B, model_ext = 1): the core drift plus subcutaneous glucagon
 * and the effect of exercise; xe = (Z1, Z2, E1, E2, E3), un glucagon ug/min, hrr the
 * heart-rate reserve fraction. */
void     orc_rhs_ext(const orc_config *cfg, const double p[ORC_NP], const double x[ORC_NX],
                     const double xe[ORC_NXE], double u, double un, double d, double hrr, double dx[ORC_NX],
                     double dxe[ORC_NXE]);
/* Sample index within the day of patient's exercise onset on that day, -1 if none. */
int32_t  orc_day_exercise(const orc_config *cfg, uint32_t patient, int32_t day);
/* Scripted dual-hormone AP run for tests: inputs y[k], announced intake d[k] (mmol/min) and
 * exercise onsets ex[k] (0/1), insulin on board above basal iob (mU) and glucagon on board
 * gob (ug) held fixed; outputs basal and bolus insulin rates (mU/min), glucagon rate
 * (ug/min) and the mode (1 = glucagon) after each decision. */
void     orc_dual_run(const orc_config *cfg, double ub, double iob, double gob, int32_t n, const double *y,
                      const double *d, const int32_t *ex, double *u_basal, double *u_bolus, double *un,
                      int32_t *mode);

/* Closed-loop Monte Carlo for patients [first, first+count) on n_threads threads. */
int      orc_simulate(const orc_config *cfg, int64_t first, int64_t count, int n_threads, const orc_outputs *out);

/* Generic Euler-Maruyama on the Ornstein-Uhlenbeck SDE dX = -theta X dt + s dW, X(0)=x0,
   path p draws step n's normal as normal #0 of the block with counter (n, p, 2, 0). Writes X_n. */
void     orc_em_ou(double theta, double s, double x0, double h, int32_t n_steps, int64_t n_paths,
                   uint64_t seed, double *x_final);

/* Population summary: exact integer totals, nearest-rank quantiles of per-patient in-range counts.
   The *_clean fields repeat the totals, quantiles and means over the unflagged patients only
   (status == 0: finite state, Q1 never negative, parameters not the resampling fallback). */
typedef struct {
    int64_t  n, k;
    uint64_t bins[5];
    uint64_t events[3];
    int64_t  q_count[5];          /* 5/25/50/75/95 % nearest rank, in samples */
    double   mean_tir;            /* bins[2] / (n k) */
    double   mean_bg;             /* sum of sum_g / (n k) */
    int64_t  worst_patient;       /* lexicographic min (min_g, patient) */
    double   worst_min_g;
    int32_t  worst_k;
    int64_t  status_count[3];
    int64_t  n_clean;             /* patients with status == 0 */
    uint64_t bins_clean[5];
    int64_t  q_count_clean[5];    /* nearest rank over the n_clean patients (0 if none) */
    double   mean_tir_clean;      /* bins_clean[2] / (n_clean k), 0 if none */
    double   mean_bg_clean;
} orc_summary;
void     orc_reduce(int64_t n, int64_t k, const int32_t *bins, const int32_t *events, const double *sum_g,
                    const double *min_g, const int32_t *argmin_k, const uint32_t *status, orc_summary *s);

#ifdef __cplusplus
}
#endif
#endif
