// internal.hpp -- host-side launch descriptors shared by the ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vct {

struct PopArgs {
    double *params;       // SoA [kRows][n]
    int64_t n;
    int64_t patient_base; // global index of patient 0 (Philox counter word 1)
    uint32_t key0, key1;
    uint32_t flags;
    double nominal[15];
    double s;             // sqrt(ln(1 + cv^2))
    double g_target;
};

enum : int32_t { kProtoSlots = 0, kProtoNordic = 1 };   // VCT_PROTO_SLOTS, VCT_PROTO_NORDIC

struct SimArgs {
    const double *params; // SoA [kRows][n], FP64
    int64_t n;
    int64_t patient_base;
    int32_t n_days, kday; // samples per day
    uint32_t key0, key1;  // simulation key (meals + noise)
    // protocol
    int32_t proto;            // kProtoSlots or kProtoNordic
    double meal_cv;           // NORDIC: relative SD of each meal's carbohydrate
    int32_t n_slots;
    int32_t minute_of_day[4];
    double carbs_mean[4], carbs_sd[4], prob[4];
    uint32_t prob_thresh[4];  // ceil(prob 2^24): presence iff (2m + 1) < thresh
    double rate_per_g;        // mmol/min of glucose per gram held over one interval
    int32_t jitter;
    // shared model constants
    double ag, tau, g_target;
    // controller
    int32_t ctrl;
    double setpoint, kp, ki, kd, umax_rel, u_rel;
    double basal_scale;   // controller's basal rate / patient's (1 except PID / open loop)
    const void *mpc;      // per-patient MPC data (SoA [kMRows][n], working precision) or null
    int32_t mpc_iters;
    const unsigned char *mlp;   // learned-controller blob (VCT_CTRL_MLP) or null
    double mlp_safe_g, mlp_safe_out;   // MPC acts when y < mlp_safe_g and out > mlp_safe_out
    float *record;        // [K][n][13] learned-controller inputs + u/u_b, or null
    int32_t *fallback;    // [n] samples on which the MLP handed over to the MPC, or null
    void *plan;           // learned controller: [kMpcN][n] input plans (working precision)
    int32_t *kplan;       //   [n] sample index at which each plan was computed
    const int32_t *order; //   [n] lane -> patient (patients outside the input box last)
    // integration
    int32_t ts_min, em_per_ctrl;
    double h, sig_sqh, sqrt_r;
    // outputs (SoA views of the metrics buffer)
    double *sum_g, *min_g, *sum_u;
    int32_t *bins, *events, *argmin_k;
    uint32_t *status;
    int64_t out_stride;   // n of the metrics buffer (row stride of bins/events)
    int32_t n_traj;
    double *traj;         // [3][n_traj][K] or null
    int64_t *pop_sum;     // [K] sum of round(G 2^32) over the patients, or null
    uint64_t *pop_min, *pop_max;   // [K] order-preserving keys of min / max G
    uint64_t *pop_hist;   // [402] pooled BG bins of 0.1 mmol/L
    uint64_t *span_min, *span_max;   // [50] min / max over patients of the cumulative 0.5 mmol/L bins
    int64_t *pop_nonfinite;   // [K] patients whose G is not finite (left out of sum, min, max)
    int64_t K;
    // model extensions (Sec. IV-B): subcutaneous glucagon and exercise states
    int32_t ext;          // 1: the extended model
    double tau_n, e_n, tau_e1, tau_e2, tau_e3, alpha_e, beta_e;
    // exercise sessions on the Northern-European protocol's active days (Sec. II-B)
    int32_t exercise, ex_minute, ex_samples;
    double ex_hrr;
    // dual-hormone AP (Sec. IV-C)
    int32_t meal_bolus;
    double icr_rule, glu_enter, glu_exit, glu_target, glu_kp, glu_max, ex_bolus, ex_bolus_below;
    double *doses;        // [3][n] basal insulin (mU), bolus insulin (mU), glucagon (ug), or null
};

// One work item of a batched launch: a tile of consecutive patients of one arm.
struct BatchItem {
    int32_t arm;
    int32_t first;
};

struct BatchLaunch {
    const SimArgs *arms;   // device array, one per arm
    const BatchItem *items;
    int32_t n_items;
    uint32_t *counter;     // device queue head, reset by the launch itself
    int32_t grid, block;
    int precision, ctrl;
    bool noisy;
};

struct MpcSetupArgs {
    const double *params;  // population buffer
    int64_t n;
    double h, ag, tau, g_target;
    int32_t em_per_ctrl;
    double sigma_q1, cgm_var;
    double rho, umax_rel;
    int32_t riccati_iters, power_iters;
    double *a64;           // FP64 scratch [kNx * kNx][n]: A, from the setup kernel to the Riccati kernel
};

struct MlpTrain {            // views into the caller's training buffer + the inference blob
    float *master, *m, *v, *grad, *loss, *loss_partial, *partial;
    unsigned char *blob;
};

// Launchers (kernels.hip). They only enqueue work; they return the launch error.
hipError_t launch_population(const PopArgs &a, hipStream_t s);
hipError_t launch_simulate(const SimArgs &a, int precision, hipStream_t s);
hipError_t launch_batch(const BatchLaunch &b, hipStream_t s);
// Two launches: the per-lane setup (everything but the Kalman gain; writes A in FP64 to
// a.a64), then the Riccati iteration with one 16-lane row per patient (writes the gain).
hipError_t launch_mpc_setup(const MpcSetupArgs &a, int precision, void *out, hipStream_t s);
hipError_t launch_mlp_init(const MlpTrain &t, uint32_t k0, uint32_t k1, hipStream_t s);
size_t mlp_stats_scratch_bytes();
hipError_t launch_mlp_stats(const float *data, int64_t n, double box_q, unsigned char *blob, void *scratch,
                            hipStream_t s);
hipError_t launch_mlp_step(const MlpTrain &t, const float *data, int64_t n_rows, const int32_t *idx, uint32_t k0,
                           uint32_t k1, int32_t step, int32_t batch, float lr, float bc1, float bc2, int apply,
                           hipStream_t s);
hipError_t launch_mlp_forward(const float *x, int64_t n, const unsigned char *blob, float *out, hipStream_t s);
int batch_blocks_per_cu(int precision, int ctrl, bool noisy, int block);
// Learned controller: scratch of launch_simulate (plans, plan times, lane order, partition
// counts) and its layout.
size_t policy_scratch_bytes(int64_t n, int precision);
void policy_scratch_views(SimArgs &a, void *scratch, int precision);

struct ReduceOut {
    uint64_t bins[5];
    uint64_t events[3];
    int64_t q_count[5];
    double sum_g;
    double sum_u;
    double worst_min_g;
    int64_t worst_patient;
    int32_t worst_k;
    int32_t pad;
    int64_t status_count[3];
    int64_t n_clean;            // unflagged patients (status == 0) and their totals
    uint64_t bins_clean[5];
    int64_t q_count_clean[5];
    double sum_g_clean;
};

// Reduce metrics (four launches on s). The workspace (reduce_workspace_bytes, 256-byte
// aligned, no initialisation needed) also holds the result: *dev_out points into it.
size_t reduce_workspace_bytes(int64_t n, int64_t K);
hipError_t launch_reduce(const double *sum_g, const double *min_g, const double *sum_u, const int32_t *bins,
                         const int32_t *events, const int32_t *argmin_k, const uint32_t *status, int64_t n,
                         int64_t K, void *workspace, ReduceOut **dev_out, hipStream_t s);

}  // namespace vct
