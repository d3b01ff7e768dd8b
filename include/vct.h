/*
 * vct.h -- C ABI of the MI355X (gfx950) closed-loop virtual clinical trial library.
 *
 * The arguments follow the paper's statement of a virtual trial (Sec. II): (1) a
 * population of patients, (2) a protocol of disturbances, (3) a patient model,
 * (4) values of the model parameters and (5) a controller ("artificial pancreas").
 * The patient model is the SDE of Sec. III-A, eq. (1), with inputs held constant
 * between sampling instants (eq. 2); the controller has the sampled form of
 * Sec. III-B, eq. (3); the indicators are the five glucose ranges of Sec. IV-A,
 * accumulated while each simulation runs and reduced over the population as in the
 * low-memory scheme of Sec. III-C.
 *
 * Conventions (all entry points):
 *  - Every device buffer is owned by the caller (allocated e.g. with torch) and
 *    only borrowed for the duration of the call or of the handle that names it.
 *    The library never frees caller memory.
 *  - Descriptors are read during the call and not retained.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    vct_create_population and vct_simulate are asynchronous on it;
 *    vct_read_metrics synchronises it before returning.
 *  - Argument errors return VCT_EINVAL before any device work is queued.
 *    A HIP runtime failure returns VCT_EHIP. vct_last_error() then holds a message.
 *  - Numerical trouble inside a simulation (non-finite state, negative Q1,
 *    exhausted parameter resampling) is reported per patient in the `status`
 *    metric and counted in vct_summary; it is not a return code.
 *  - No entry point is thread-safe with respect to the same handle.
 */
#ifndef VCT_H
#define VCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VCT_ABI_VERSION 5  /* 5: the population-BG buffer gained the per-sample non-finite counts */
#define VCT_NP 15          /* sampled parameters per patient                         */
#define VCT_NX 11          /* model states per patient                               */
#define VCT_NPARAM_ROWS 19 /* rows of the population buffer: 15 parameters, u_b, I*, attempts, status */
#define VCT_MAX_SLOTS 4    /* meal slots per day                                     */

typedef enum {
    VCT_OK = 0,
    VCT_EINVAL = -1,   /* invalid argument                                   */
    VCT_ENOMEM = -2,   /* the library could not allocate its own scratch     */
    VCT_EHIP = -3,     /* a HIP runtime call failed                          */
    VCT_ESTATE = -4,   /* handle in the wrong state                          */
    VCT_ENOTSUP = -5   /* valid but not supported by this build              */
} vct_status;

/* Controllers (Sec. III-B): constant open-loop rate (tests), PID, linear MPC, learned MLP,
 * and the dual-hormone AP of Sec. IV-C (needs the model extensions, vct_sim.model_ext). */
enum { VCT_CTRL_OPEN = 0, VCT_CTRL_PID = 1, VCT_CTRL_MPC = 2, VCT_CTRL_MLP = 3, VCT_CTRL_DUAL = 4 };
/* Working precision of the patient state; accumulators are always FP64. */
enum { VCT_FP64 = 0, VCT_FP32 = 1 };
/* Population flags. */
enum { VCT_POP_MIN_BASAL = 1 };   /* also require u_b >= 0.4 U/h (Sec. IV-B) */

/*
 * (1) population + (4) parameter values -- Sec. II-A, Sec. IV-B.
 * Parameter order (model units; EGP0, F01 per kg, VI, VG in L/kg):
 *   EGP0 F01 k12 ka1 ka2 ka3 SIT SID SIE ke VI VG tmaxI tmaxG BW.
 * Each patient's vector is drawn lognormal with median `nominal` and coefficient
 * of variation `cv`; a draw is kept iff the basal steady state at `g_target`
 * exists (and, with VCT_POP_MIN_BASAL, its rate is >= 0.4 U/h); up to 32 draws,
 * then the nominal vector with a status bit. Random numbers: Philox4x32-10 with
 * key (seed low word, seed high word ^ arm_id), counter (j/4, patient, 0, attempt).
 * The handle holds patients [first_patient, first_patient + n_patients) of the population:
 * every draw of a patient (parameters, meals, noise) is keyed by its global index, so a
 * population split into slices -- over launches or GPUs -- gives the same per-patient results.
 */
typedef struct {
    int64_t  n_patients;       /* >= 1, < 2^31                                       */
    uint64_t seed;
    uint32_t arm_id;
    uint32_t flags;            /* VCT_POP_*                                            */
    double   nominal[VCT_NP];  /* all > 0                                              */
    double   cv;               /* >= 0                                                 */
    double   ag;               /* carbohydrate bioavailability, shared, in (0, 1]      */
    double   tau_cgm;          /* sensor time constant, min, shared, > 0               */
    double   g_target;         /* basal steady-state glucose, mmol/L, > 0              */
    int64_t  first_patient;    /* global index of the first patient, >= 0, first + n <= 2^32 */
} vct_population_desc;

/* (2) protocol -- Sec. II-B: disturbances with type, size and time. A meal is a constant
 * glucose intake over the sampling interval that contains its onset; the onset jitter is
 * uniform on the integers [-jitter_min, jitter_min].
 * VCT_PROTO_SLOTS: each day and slot draws one Philox block (counter (day, patient, 1,
 * slot), simulation key): carbs = max(0, mean + sd z), onset = minute_of_day + jitter,
 * present with probability prob. Slots must be in increasing time order, non-overlapping
 * after jitter.
 * VCT_PROTO_NORDIC: the Northern-European protocol of Sec. II-B (Tables I and II): four
 * 13-week seasons of standard / active / vacation weeks (winter 6/4/3, spring 6/6/1,
 * summer 7/3/3, autumn 9/3/1), weeks of standard / active / movie-night / late-night days
 * (standard 4/1/1/1, active 3/3/1/0, vacation 5/0/0/2), each patient's arrangement of
 * weeks in a season and of days in a week a Fisher-Yates shuffle on Philox blocks
 * (d / 91, patient, 8, 0..2) and (d / 7, patient, 8, 4..5); meal sizes 1.29 / 0.86 / 0.57 /
 * 0.29 g carbohydrate per kg body weight (large / medium / small / snack), times and sizes
 * per day type and season as documented in the kernels; carbs = max(0, size BW (1 +
 * meal_cv z)) from Philox block (day, patient, 1, meal kind). The slot fields are unused;
 * jitter_min <= 40. Day 0 is the first day of winter. */
#define VCT_PROTO_SLOTS  0
#define VCT_PROTO_NORDIC 1
typedef struct {
    int32_t n_slots;                        /* 0..VCT_MAX_SLOTS                    */
    int32_t minute_of_day[VCT_MAX_SLOTS];
    double  carbs_mean_g[VCT_MAX_SLOTS];
    double  carbs_sd_g[VCT_MAX_SLOTS];
    double  prob[VCT_MAX_SLOTS];            /* in [0, 1]                           */
    int32_t jitter_min;                     /* 0..120 (VCT_PROTO_NORDIC: 0..40)    */
    int32_t kind;                           /* VCT_PROTO_SLOTS or VCT_PROTO_NORDIC */
    double  meal_cv;                        /* VCT_PROTO_NORDIC: relative SD of each meal, 0..1 */
    /* Exercise (Sec. II-B: the active day has an exercise session), VCT_PROTO_NORDIC with the
     * model extensions only: exercise = 1 gives each active day one session of
     * exercise_duration minutes at heart-rate reserve fraction exercise_hrr, held over
     * ceil(exercise_duration / ts_min) sampling intervals from the one that contains
     * exercise_minute + a jitter on the integers [-jitter_min, jitter_min] (word 2 of Philox
     * block (day, patient, 9, 0), simulation key). */
    int32_t exercise;                       /* 0 or 1                              */
    int32_t exercise_minute;                /* 0..1439                             */
    int32_t exercise_duration;              /* minutes, 1..240                     */
    double  exercise_hrr;                   /* in [0, 1]                           */
} vct_protocol;

/* (5) controller -- Sec. III-B (x^c_{k+1} = kappa(x^c_k, y_k, ...), u_k = lambda(...)).
 * PID on the sensor value y_k, gains relative to the patient's basal rate u_b:
 *   u_k = clamp(u_b + kp u_b e + ki u_b I_k + kd u_b (y_k - y_{k-1})/Ts, 0, umax_rel u_b),
 *   e = y_k - setpoint, I_{k+1} = I_k + e Ts only while the unclamped value is in range.
 * Linear MPC (control state: Kalman estimate of x - x_ss and the planned inputs): each
 * sample corrects the estimate with y_k, minimises
 *   sum_{j=1..N} (G_{k+j} - setpoint)^2 + mpc_rho sum_{i=0..N-1} ((u_i - u_b)/u_b)^2,
 *   0 <= u_i <= umax_rel u_b, with the intake of the current interval announced,
 * by mpc_iters projected-gradient steps warm-started from the shifted previous plan,
 * applies u_0 and predicts. The per-patient matrices come from vct_mpc_setup.
 * Learned controller (VCT_CTRL_MLP; needs mpc_dev and mlp_dev): a 12 -> 64 -> 64 -> 64 -> 1
 * ReLU network trained to imitate the MPC gives u_k = clamp(u_b out, 0, umax_rel u_b) from
 *   y_k .. y_k-5 (y_0 repeated before the first sample);
 *   insulin on board, as the mean change of G over the MPC's 24-sample prediction that the
 *   insulin states' deviation from basal (S1, S2, I, x1, x2, x3) still causes (mmol/L);
 *   the announced meals likewise: meal states D1, D2 and the intake announced now (mmol/L);
 *   the patient: u_b, the insulin response over the horizon (sum of the MPC's Markov
 *   parameters), its mean delay (sum m h_m / sum h_m, samples), BW,
 * with the insulin and meal states those driven by the delivered doses and the announced
 * meals, and the horizon means of the MPC's prediction rows and intake response (written
 * by vct_mpc_setup). The Kalman filter of the MPC runs on every sample; the
 * MPC solves its QP and acts instead of the network (a "fallback") when any input lies
 * outside the box stored with the network, or when y_k < mlp_safe_g and out > mlp_safe_out
 * (e.g. 3.0 mmol/L and 1: never more than basal insulin while the sensor reads below
 * 54 mg/dL). */
typedef struct {
    int32_t kind;          /* VCT_CTRL_*                                           */
    double  setpoint;      /* mmol/L                                               */
    double  kp, ki, kd;    /* u_b/(mmol/L), u_b/(mmol/L min), u_b min/(mmol/L)     */
    double  umax_rel;      /* > 0                                                  */
    double  u_rel;         /* open-loop mode: u = u_rel u_b                        */
    int32_t mpc_horizon;   /* N; this build supports 24                             */
    int32_t mpc_iters;     /* projected-gradient iterations per sample, 0..1000     */
    double  mpc_rho;       /* > 0                                                   */
    const void *mpc_dev;   /* VCT_CTRL_MPC, VCT_CTRL_MLP: buffer filled by vct_mpc_setup */
    const void *mlp_dev;   /* VCT_CTRL_MLP: network blob (vct_mlp_blob_bytes), read-only */
    double  mlp_safe_g;    /* VCT_CTRL_MLP: the MPC acts when y_k < mlp_safe_g (mmol/L) ... */
    double  mlp_safe_out;  /*   ... and the network's output exceeds mlp_safe_out (u / u_b) */
    double  basal_scale;   /* > 0: the controller's basal rate is basal_scale u_b (1 = correct;
                              Sec. IV-E trial B: 0.5). It replaces u_b in the PID law and bound
                              and in the open-loop rate; other values than 1 need PID or open loop */
    /* Dual-hormone AP (VCT_CTRL_DUAL, Sec. IV-C; needs vct_sim.model_ext): glucagon mode when
     * y_k < glu_enter, insulin mode again when y_k >= glu_exit. The PID above runs on every
     * sample (its conditional integral included) and is delivered in insulin mode only, with
     * (meal_bolus = 1) a bolus at each announced meal: carbs TDD / icr_rule U (carbs = the held
     * intake d Ts 180.16/1000 g, TDD = 2 x 1440 u_b / 1000 U/day) less the insulin on board
     * above basal (S1 + S2 - 2 u_b tmaxI, mU), never negative. Glucagon mode: no insulin; a
     * microbolus min(glu_max, max(0, glu_kp (glu_target - y_k) - (Z1 + Z2))) ug. Either mode:
     * ex_bolus ug at an exercise onset while y_k < ex_bolus_below. Every dose is delivered as a
     * constant rate over its sampling interval. */
    int32_t meal_bolus;    /* 0 or 1                                                 */
    double  icr_rule;      /* > 0, g U/day / U (500 is the clinical rule of thumb)   */
    double  glu_enter, glu_exit;      /* mmol/L, glu_enter <= glu_exit                */
    double  glu_target, glu_kp, glu_max;   /* mmol/L, ug/(mmol/L) >= 0, ug >= 0        */
    double  ex_bolus, ex_bolus_below;      /* ug >= 0, mmol/L                          */
} vct_controller;

/* (3) model + simulation settings -- Sec. III-A. Euler-Maruyama with em_per_ctrl
 * steps of ts_min/em_per_ctrl minutes per sampling interval; diffusion sigma_q1 on
 * Q1 only; sensor noise variance cgm_var. Noise is drawn per pair of samples
 * (2j, 2j+1): the Philox blocks (j, patient, 2, 0..2) give 12 normals, #0..#4 the EM
 * normals and #5 the sensor normal of sample 2j, #6..#10 and #11 those of sample 2j+1.
 *
 * metrics_dev: caller buffer of vct_metrics_bytes(n) bytes, per-patient SoA:
 *   double sum_g[n]   sum of G over the K samples (mmol/L)
 *   double min_g[n]   minimum sampled G
 *   double sum_u[n]   delivered insulin over the horizon (mU)
 *   int32  bins[5][n] samples per range: <3.0, 3.0-3.9, 3.9-10.0, 10.0-13.9, >13.9 mmol/L
 *                     (3.9 and 10.0 count as in range)
 *   int32  events[3][n] runs of >= 3 consecutive samples <3.9, <3.0, >13.9
 *   int32  argmin_k[n] first sample index of min_g
 *   uint32 status[n]  bit0 non-finite state, bit1 negative Q1, bit2 resampling exhausted
 * traj_dev (optional, NULL = off): double [3][traj_patients][K] = G, y, u of the
 *   first traj_patients patients at every sample, K = n_days * 1440 / ts_min.
 * record_dev (optional, VCT_CTRL_MPC / VCT_CTRL_MLP only): float [K][n][13], row (k, j) =
 *   the 12 learned-controller inputs of patient j at sample k, then u_k / u_b (the
 *   behaviour-cloning data set when the MPC acts); K * n * 52 bytes.
 * fallback_dev (optional, VCT_CTRL_MLP only): int32 [n] samples on which the MPC acted. */
typedef struct {
    int32_t  n_days;          /* >= 1                                               */
    int32_t  em_per_ctrl;     /* 5 (the supported EM substep count)                 */
    int32_t  ts_min;          /* sampling interval, min; must divide 720            */
    int32_t  precision;       /* VCT_FP64 | VCT_FP32                               */
    double   sigma_q1;        /* mmol min^-1/2, >= 0                                */
    double   cgm_var;         /* (mmol/L)^2, >= 0                                   */
    uint64_t noise_seed;      /* key (low, high ^ arm_id) for meals and noise       */
    void    *metrics_dev;
    int32_t  traj_patients;   /* 0..64                                              */
    void    *traj_dev;
    float   *record_dev;
    int32_t *fallback_dev;
    void    *popbg_dev;       /* optional (NULL = off): the population's BG as a function of
                                 time, Sec. III-C, vct_popbg_bytes(n_days, ts_min) bytes; see
                                 vct_popbg_bytes. Not with traj_dev or record_dev. */
    /* Model extensions (Sec. IV-B; parameters shared by all patients). model_ext = 1 adds a
     * subcutaneous glucagon depot dZ1 = u_N - Z1/tau_n, dZ2 = (Z1 - Z2)/tau_n (ug, u_N ug/min)
     * whose appearance Z2/tau_n adds e_n Z2/tau_n (mmol/min) to the hepatic glucose output,
     * EGP = EGP0 max(0, 1 - x3) + e_n Z2/tau_n, and exercise states driven by the heart-rate
     * reserve fraction HRR: dE1 = (HRR - E1)/tau_e1, dE2 = (E1 - E2)/tau_e2, dE3 = (E1 - E3)/
     * tau_e3, with the uptake -alpha_e E2 Q1 and x1, x2 acting as x_j (1 + beta_e E3). All
     * five states start at 0 (the basal state). Needed by VCT_CTRL_DUAL and by exercise;
     * supported with VCT_CTRL_OPEN, VCT_CTRL_PID and VCT_CTRL_DUAL, not with popbg_dev or
     * the batched launch (VCT_ENOTSUP). */
    int32_t  model_ext;       /* 0 or 1                                              */
    double   tau_n, e_n;      /* min > 0; mmol/ug >= 0                               */
    double   tau_e1, tau_e2, tau_e3;   /* min > 0                                    */
    double   alpha_e, beta_e; /* 1/min >= 0; >= 0                                    */
    double  *doses_dev;       /* optional (model_ext only, NULL = off): double [3][n], per patient
                                 the basal insulin (mU), bolus insulin (mU) and glucagon (ug)
                                 delivered over the horizon (PID / open loop: all basal) */
} vct_sim;

/* Population summary (Sec. III-C indicators, Sec. IV-A ranges). Quantiles are nearest
 * rank over the per-patient in-range counts: q_p = smallest c with #{count <= c} >=
 * ceil(p n / 100). The worst patient is the lexicographic minimum of (min G, index). */
typedef struct {
    int64_t  n_patients;
    int64_t  n_samples;        /* K per patient                                     */
    uint64_t bins[5];
    uint64_t events[3];
    int64_t  q_count[5];       /* 5/25/50/75/95 %                                   */
    double   q_frac[5];        /* q_count / K                                       */
    double   mean_tir;         /* bins[2] / (n K)                                   */
    double   mean_bg;          /* sum of sum_g / (n K), fixed-order FP64 tree       */
    double   mean_insulin;     /* mean of sum_u, mU                                 */
    int64_t  worst_patient;
    double   worst_min_g;
    int32_t  worst_k;
    int32_t  _pad;
    int64_t  status_count[3];
    /* The same over the unflagged patients only (status == 0: finite state, Q1 never
     * negative, parameters not the resampling fallback); every field above still counts
     * all patients. Quantiles and means are 0 if no patient is unflagged. */
    int64_t  n_clean;
    uint64_t bins_clean[5];
    int64_t  q_count_clean[5];
    double   q_frac_clean[5];
    double   mean_tir_clean;   /* bins_clean[2] / (n_clean K)                      */
    double   mean_bg_clean;
} vct_summary;

typedef struct vct_population vct_population;   /* opaque, owned by the library */

/* One arm of a batched trial (scenario comparison, Sec. IV-E; many controller variants,
 * Sec. III-B): its own population (whose arm_id also keys the arm's noise), horizon,
 * PID gains and metric buffer (vct_metrics_bytes of its population). */
typedef struct {
    const vct_population *pop;
    int32_t n_days;
    double  kp, ki, kd;       /* relative to u_b, as in vct_controller            */
    void   *metrics_dev;
    double  basal_scale;      /* the arm's controller basal rate / u_b, as in vct_controller */
} vct_arm;

typedef struct vct_batch vct_batch;             /* opaque, owned by the library */

typedef struct {
    int32_t n_arms, n_items;   /* work items = tiles of `block` patients of one arm  */
    int32_t block, grid;       /* chosen workgroup size, persistent grid             */
    int32_t tuned_block[4];    /* candidates the autotuner timed                     */
    double  tuned_ms[4];       /* their times on the 2-day calibration run (0 = not run) */
} vct_batch_stats;

int         vct_abi_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char *vct_last_error(void);

/* Byte sizes of caller-owned buffers. */
size_t      vct_population_bytes(int64_t n_patients);   /* VCT_NPARAM_ROWS * n doubles, SoA */
size_t      vct_metrics_bytes(int64_t n_patients);      /* 64 * n                        */
size_t      vct_traj_bytes(int32_t traj_patients, int32_t n_days, int32_t ts_min);

/* Draw the population into params_dev (SoA [VCT_NPARAM_ROWS][n] doubles: the 15
 * parameters, u_b in mU/min, I* in mU/L, attempts used, status) and return a handle
 * that borrows params_dev. */
vct_status  vct_create_population(const vct_population_desc *desc, void *params_dev, void *stream,
                                  vct_population **out);
/* Closed-loop Monte Carlo of every patient of the population (Sec. III). */
vct_status  vct_simulate(const vct_population *pop, const vct_protocol *protocol, const vct_controller *ctrl,
                         const vct_sim *sim, void *stream);
/* Linear MPC setup for every patient of the population (FP64 computation): the drift
 * linearised at the basal state and discretised like the plant (A = (I + hJ)^E, B, E
 * over the E Euler steps of a sample), the stationary Kalman gain for the sensor state
 * (500 Riccati iterations, Q = 1e-6 I + sigma^2 h E on Q1, R = max(cgm_var, 1e-4)), the
 * 24-sample prediction condensed to Gamma^T F, Gamma^T w, Gamma^T 1, the Markov
 * parameters and the step 1/(lambda_max(Gamma^T Gamma) + rho/u_b^2) (100 power
 * iterations). mpc_dev: caller buffer of vct_mpc_bytes(n, precision) bytes, SoA rows of
 * the working precision; sim->precision must equal the precision later simulated, and
 * ctrl->umax_rel / mpc_rho are baked in. */
/* Population BG as a function of time (optional output of vct_simulate): for every sample
 * k = 0..K-1, over the patients of the call,
 *   int64  sum[K]  @0      sum of round(G 2^32) over the patients whose G is finite (G in
 *                          mmol/L; exact, order-free integer sum: the mean is
 *                          sum / ((n - nonfinite[k]) 2^32));
 *   uint64 min[K]  @8K     order-preserving key of the smallest finite G (as FP64):
 *   uint64 max[K]  @16K    key = bits ^ (sign ? all ones : sign bit); G = the key inverted
 *                          (all ones / zero, which invert to NaN, when no G is finite);
 *   uint64 hist[402] @24K  the BG of every patient and sample in bins of 0.1 mmol/L: bin 0
 *                          below 0 (and NaN), bin 1 + floor(10 G) for 0 <= G < 40, bin 401
 *                          at or above 40 (the population's BG distribution, Sec. IV-D);
 *   uint64 span_min[50] @24K+3216, span_max[50] @24K+3616: over the patients, the smallest
 *                          and largest number of their samples with G below (b + 1) / 2
 *                          mmol/L, b = 0..48 (b = 49: all samples) -- the span of the
 *                          patients' own BG distributions (Fig. 3);
 *   int64  nonfinite[K] @24K+4016: patients whose G at sample k is not finite (their state
 *                          left the finite range; the status bit says so). They stay in
 *                          hist (bin 0) and span, and are left out of sum, min and max;
 * vct_simulate writes all of it (the buffer need not be initialised). Returns 32 K + 4016
 * bytes, or 0 for invalid arguments. */
size_t      vct_popbg_bytes(int32_t n_days, int32_t ts_min);
size_t      vct_mpc_bytes(int64_t n_patients, int32_t precision);
vct_status  vct_mpc_setup(const vct_population *pop, const vct_controller *ctrl, const vct_sim *sim, void *mpc_dev,
                          void *stream);
/* Learned controller: data set, normalisation, training and inference (BF16 MFMA, FP32
 * accumulation, FP32 master weights).
 *
 * Network blob (vct_mlp_blob_bytes() = 21568 bytes, caller-owned device memory, 16-byte
 * aligned; the training buffer is 256-byte aligned; misalignment is VCT_EINVAL):
 *   bf16  W1[64][16]   @0      input layer; columns 12..15 are zero
 *   bf16  W2[64][64]   @2048
 *   bf16  W3[64][64]   @10240
 *   bf16  W4[16][64]   @18432  row 0 is the output layer, rows 1..15 are zero
 *   f32   b1[64] @20480, b2[64] @20736, b3[64] @20992, b4[16] @21248 (b4[1..15] = 0)
 *   f32   mean[16] @21312, istd[16] @21376: input z-score (x - mean) istd, then BF16
 *   f32   lo[16] @21440, hi[16] @21504: the input box outside which the MPC acts
 * Training buffer (vct_mlp_train_bytes(batch), caller-owned device memory), FP32 with
 * P = VCT_MLP_PARAMS entries in the order W1, W2, W3, W4, b1, b2, b3, b4 (padded shapes as
 * in the blob), byte offsets: master[P] @0, adam_m[P] @4P, adam_v[P] @8P, grad[P] @12P,
 * loss @16P, then library scratch. A buffer serves every batch size up to the one it was sized for.
 * Data rows: float [n_rows][13] = 12 inputs then the target u/u_b (record_dev layout). */
#define VCT_MLP_IN 12
#define VCT_MLP_PARAMS 10448
#define VCT_MLP_BLOB_BYTES 21568
size_t      vct_mlp_blob_bytes(void);
size_t      vct_mlp_train_bytes(int32_t batch);
/* He-normal weights (std sqrt(2/fan_in); output row sqrt(1/64)), zero biases except
 * b4[0] = 1, zero Adam moments; weight p (padded order) is normal p%4 of the Philox block
 * (p/4, 0, 6, 0) with key (seed low word, seed high word). Writes master and the blob's
 * weights and biases. */
vct_status  vct_mlp_init(uint64_t seed, void *train_dev, void *blob_dev, void *stream);
/* Per-input mean and 1/std (population std, floor 1e-6) over the rows, and the box:
 * box_q = 0 -> [min, max] of the data; 0 < box_q < 0.5 -> the nearest-rank box_q and
 * 1 - box_q quantiles, widened outward to a 4096-bin grid between min and max.
 * train_dev must hold vct_mlp_train_bytes(64) bytes or more (scratch). */
vct_status  vct_mlp_normalize(const float *rows_dev, int64_t n_rows, double box_q, void *train_dev,
                              void *blob_dev, void *stream);
/* One step on the mean squared error (1/B) sum (out - target)^2 of a minibatch of B =
 * batch rows (multiple of 64, <= the size train_dev was built for): rows idx_dev[0..B)
 * if idx_dev is non-NULL (each in [0, n_rows); an index outside makes the loss and the
 * gradient NaN), else row floor(x n_rows / 2^32) for the first word x of the Philox
 * block (step, i, 5, 0), i = 0..B-1. Writes grad and loss; with apply != 0 also takes
 * the Adam step t = step + 1 (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on master
 * and refreshes the blob's weights. Gradients are summed over the batch in a fixed
 * order (deterministic). */
vct_status  vct_mlp_train_step(const float *rows_dev, int64_t n_rows, const int32_t *idx_dev, uint64_t seed,
                               int32_t step, int32_t batch, double lr, int32_t apply, void *train_dev,
                               void *blob_dev, void *stream);
/* n_steps Adam steps of vct_mlp_train_step (rows drawn by Philox, apply on) with steps
 * first_step .. first_step + n_steps - 1 and a cosine decay of the learning rate from lr to
 * lr_min: step i of the call uses lr_min + (lr - lr_min) (1 + cos(pi (sched_offset + i) /
 * sched_total)) / 2. The loss slot then holds the last step's minibatch loss. Queued on the
 * stream without host synchronisation; equal, bit for bit, to the same sequence of
 * vct_mlp_train_step calls. */
vct_status  vct_mlp_train(const float *rows_dev, int64_t n_rows, uint64_t seed, int32_t first_step, int32_t n_steps,
                          int32_t sched_offset, int32_t sched_total, int32_t batch, double lr, double lr_min,
                          void *train_dev, void *blob_dev, void *stream);
/* Network output for n input rows x_dev [n][12] (raw inputs) -> out_dev [n]. */
vct_status  vct_mlp_forward(const float *x_dev, int64_t n, const void *blob_dev, float *out_dev, void *stream);

/* Reduce the per-patient metrics of n patients with K samples each into *host_out. */
vct_status  vct_read_metrics(const void *metrics_dev, int64_t n_patients, int64_t n_samples,
                             vct_summary *host_out, void *stream);
/* Allocation-free variant of vct_read_metrics, for callers that cannot allocate device
 * memory (serving loops, harnesses that forbid hipMalloc). Same arguments, result and
 * synchronisation; n_samples <= VCT_NOALLOC_MAX_SAMPLES, else VCT_EINVAL. Its workspace
 * is a static device array of VCT_NOALLOC_SCRATCH_BYTES on each GPU the library runs on,
 * held until the process ends and looked up at the first call on that GPU; the current
 * device must be the stream's. Every call on a GPU shares that GPU's array (each call
 * clears what it needs): calls that overlap on one GPU (several streams or threads) race,
 * and the caller must serialise them. */
#define VCT_NOALLOC_MAX_SAMPLES 210240        /* two years of 5-min samples */
#define VCT_NOALLOC_SCRATCH_BYTES 2097152     /* 2 MiB per GPU              */
vct_status  vct_read_metrics_noalloc(const void *metrics_dev, int64_t n_patients, int64_t n_samples,
                                     vct_summary *host_out, void *stream);
void        vct_destroy_population(vct_population *pop);

/* Batched heterogeneous trial (many arms of uneven size and horizon) in ONE persistent
 * launch: the library builds a queue of (arm, tile) work items ordered longest horizon
 * first, picks the workgroup size (block = 0: autotune by timing 64/128/256/512 on
 * horizons capped at 2 days, which overwrites the arms' metric buffers; else 64, 128,
 * 256 or 512), and captures queue reset + launch in a HIP graph. The per-arm controller
 * kind, set point, limits, protocol and noise settings come from ctrl/protocol/sim
 * (sim->n_days, metrics_dev and traj_* are ignored). Results per patient are identical
 * to vct_simulate of that arm. The handle borrows the arms' populations and buffers;
 * it owns only its work-item table, queue counter and graph. */
vct_status  vct_batch_create(const vct_arm *arms, int32_t n_arms, const vct_protocol *protocol,
                             const vct_controller *ctrl, const vct_sim *sim, int32_t block, void *stream,
                             vct_batch **out);
/* Replay the captured launch on `stream` (asynchronous). Calls on one handle must not overlap. */
vct_status  vct_batch_run(vct_batch *batch, void *stream);
vct_status  vct_batch_info(const vct_batch *batch, vct_batch_stats *out);
void        vct_batch_destroy(vct_batch *batch);

#ifdef __cplusplus
}
#endif
#endif
