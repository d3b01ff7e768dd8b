// abi.hip -- host runtime behind include/vct.h: argument validation, launch planning,
// error mapping and the population handle.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/vct.h"
#include "internal.hpp"
#include "mlp.hpp"
#include "mpc.hpp"

struct vct_population {
    int64_t n;
    int64_t first;
    double *params;
    uint32_t arm_id;
    uint32_t flags;
    double ag, tau, g_target;
};

namespace {

thread_local std::string g_err;

vct_status fail(vct_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

vct_status hip_fail(hipError_t e, const char *what)
{
    return fail(VCT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

void split_key(uint64_t seed, uint32_t arm, uint32_t &k0, uint32_t &k1)
{
    k0 = (uint32_t)(seed & 0xffffffffu);
    k1 = (uint32_t)(seed >> 32) ^ arm;
}

const int64_t kMaxPatients = (int64_t)1 << 31;

// Workspace of vct_read_metrics_noalloc: one static array per GPU, held until the process
// ends. Host code never passes `scratch` itself to a kernel (on the host it names a
// stand-in, not device memory); it uses the device address found once per device.
static __device__ __align__(256) unsigned char scratch[VCT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up at the first call there).
hipError_t scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int vct_abi_version(void) { return VCT_ABI_VERSION; }

const char *vct_last_error(void) { return g_err.c_str(); }

size_t vct_population_bytes(int64_t n) { return n > 0 ? (size_t)n * VCT_NPARAM_ROWS * sizeof(double) : 0; }

size_t vct_metrics_bytes(int64_t n) { return n > 0 ? (size_t)n * 64u : 0; }

size_t vct_popbg_bytes(int32_t n_days, int32_t ts_min)
{
    if (n_days <= 0 || ts_min <= 0 || 1440 % ts_min != 0)
        return 0;
    return ((size_t)4 * (size_t)n_days * (size_t)(1440 / ts_min) + 502) * sizeof(int64_t);
}

size_t vct_traj_bytes(int32_t traj_patients, int32_t n_days, int32_t ts_min)
{
    if (traj_patients <= 0 || n_days <= 0 || ts_min <= 0 || 1440 % ts_min != 0)
        return 0;
    return (size_t)3 * traj_patients * (size_t)n_days * (size_t)(1440 / ts_min) * sizeof(double);
}

vct_status vct_create_population(const vct_population_desc *d, void *params_dev, void *stream,
                                 vct_population **out)
{
    g_err.clear();
    if (!d || !params_dev || !out)
        return fail(VCT_EINVAL, "vct_create_population: null argument");
    if (d->n_patients < 1 || d->n_patients >= kMaxPatients)
        return fail(VCT_EINVAL, "vct_create_population: n_patients %lld out of [1, 2^31)",
                    (long long)d->n_patients);
    for (int q = 0; q < VCT_NP; ++q)
        if (!finite_pos(d->nominal[q]))
            return fail(VCT_EINVAL, "vct_create_population: nominal[%d] must be finite and > 0", q);
    if (!(std::isfinite(d->cv) && d->cv >= 0.0))
        return fail(VCT_EINVAL, "vct_create_population: cv must be finite and >= 0");
    if (!(finite_pos(d->ag) && d->ag <= 1.0) || !finite_pos(d->tau_cgm) || !finite_pos(d->g_target))
        return fail(VCT_EINVAL, "vct_create_population: ag in (0,1], tau_cgm > 0, g_target > 0 required");
    if (d->flags & ~(uint32_t)VCT_POP_MIN_BASAL)
        return fail(VCT_EINVAL, "vct_create_population: unknown flags 0x%x", d->flags);
    if (d->first_patient < 0 || d->first_patient + d->n_patients > ((int64_t)1 << 32))
        return fail(VCT_EINVAL, "vct_create_population: patients [%lld, %lld) outside [0, 2^32)",
                    (long long)d->first_patient, (long long)(d->first_patient + d->n_patients));

    vct::PopArgs a{};
    a.params = (double *)params_dev;
    a.n = d->n_patients;
    a.patient_base = d->first_patient;
    split_key(d->seed, d->arm_id, a.key0, a.key1);
    a.flags = d->flags;
    for (int q = 0; q < VCT_NP; ++q)
        a.nominal[q] = d->nominal[q];
    a.s = std::sqrt(std::log1p(d->cv * d->cv));
    a.g_target = d->g_target;
    hipError_t e = vct::launch_population(a, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "vct_create_population: launch");

    vct_population *p = new (std::nothrow) vct_population;
    if (!p)
        return fail(VCT_ENOMEM, "vct_create_population: out of host memory");
    p->n = d->n_patients;
    p->first = d->first_patient;
    p->params = (double *)params_dev;
    p->arm_id = d->arm_id;
    p->flags = d->flags;
    p->ag = d->ag;
    p->tau = d->tau_cgm;
    p->g_target = d->g_target;
    *out = p;
    return VCT_OK;
}

void vct_destroy_population(vct_population *p) { delete p; }

static_assert(vct::kProtoSlots == VCT_PROTO_SLOTS && vct::kProtoNordic == VCT_PROTO_NORDIC, "protocol kinds");

static vct_status check_protocol(const vct_protocol *pr, int32_t ts)
{
    if (pr->n_slots < 0 || pr->n_slots > VCT_MAX_SLOTS)
        return fail(VCT_EINVAL, "protocol: n_slots %d out of [0, %d]", pr->n_slots, VCT_MAX_SLOTS);
    if (pr->jitter_min < 0 || pr->jitter_min > 120)
        return fail(VCT_EINVAL, "protocol: jitter_min %d out of [0, 120]", pr->jitter_min);
    if (pr->kind == VCT_PROTO_NORDIC) {
        // the closest meals are 90 min apart (21:00, 22:30)
        if (pr->jitter_min > 40 || 2 * pr->jitter_min + ts > 90)
            return fail(VCT_EINVAL, "protocol: jitter_min %d too large for the Northern-European day", pr->jitter_min);
        if (!(pr->meal_cv >= 0.0 && pr->meal_cv <= 1.0))
            return fail(VCT_EINVAL, "protocol: meal_cv outside [0, 1]");
        return VCT_OK;
    }
    if (pr->kind != VCT_PROTO_SLOTS)
        return fail(VCT_EINVAL, "protocol: kind %d unknown", pr->kind);
    for (int m = 0; m < pr->n_slots; ++m) {
        const int lo = pr->minute_of_day[m] - pr->jitter_min, hi = pr->minute_of_day[m] + pr->jitter_min;
        if (lo < 0 || hi >= 1440)
            return fail(VCT_EINVAL, "protocol: slot %d onset range [%d, %d] leaves the day", m, lo, hi);
        if (!(std::isfinite(pr->carbs_mean_g[m]) && std::isfinite(pr->carbs_sd_g[m]) && pr->carbs_sd_g[m] >= 0.0))
            return fail(VCT_EINVAL, "protocol: slot %d carbs distribution invalid", m);
        if (!(pr->prob[m] >= 0.0 && pr->prob[m] <= 1.0))
            return fail(VCT_EINVAL, "protocol: slot %d prob outside [0, 1]", m);
        if (m > 0 && pr->minute_of_day[m] - pr->minute_of_day[m - 1] < 2 * pr->jitter_min + ts)
            return fail(VCT_EINVAL, "protocol: slots %d and %d must be ordered and at least 2*jitter+ts apart",
                        m - 1, m);
    }
    return VCT_OK;
}

// Validates one (population, protocol, controller, settings) tuple and fills the kernel
// arguments; metrics_dev/traj are taken from `sim`.
static vct_status build_sim_args(const vct_population *pop, const vct_protocol *pr, const vct_controller *ctrl,
                                 const vct_sim *sim, bool need_metrics, vct::SimArgs &a)
{
    if (!pop || !pr || !ctrl || !sim)
        return fail(VCT_EINVAL, "null argument");
    if (need_metrics && !sim->metrics_dev)
        return fail(VCT_EINVAL, "metrics_dev is null");
    if (sim->n_days < 1 || sim->n_days > 100000)
        return fail(VCT_EINVAL, "n_days %d out of [1, 100000]", sim->n_days);
    if (sim->ts_min < 1 || 1440 % sim->ts_min != 0)
        return fail(VCT_EINVAL, "ts_min %d must divide 1440", sim->ts_min);
    if ((1440 / sim->ts_min) % 2 != 0)
        return fail(VCT_ENOTSUP, "samples per day must be even (noise is drawn per sample pair)");
    if (sim->em_per_ctrl != 5)
        return fail(VCT_ENOTSUP, "em_per_ctrl %d (only 5 EM steps per sample)", sim->em_per_ctrl);
    if (sim->precision != VCT_FP64 && sim->precision != VCT_FP32)
        return fail(VCT_EINVAL, "precision %d", sim->precision);
    if (!(std::isfinite(sim->sigma_q1) && sim->sigma_q1 >= 0.0 && std::isfinite(sim->cgm_var) &&
          sim->cgm_var >= 0.0))
        return fail(VCT_EINVAL, "sigma_q1 and cgm_var must be finite and >= 0");
    if (sim->traj_patients < 0 || sim->traj_patients > 64 || sim->traj_patients > pop->n ||
        (sim->traj_patients > 0 && !sim->traj_dev))
        return fail(VCT_EINVAL, "traj_patients %d invalid (0..min(64, n), buffer required)", sim->traj_patients);
    if (sim->popbg_dev && (sim->traj_patients > 0 || sim->record_dev))
        return fail(VCT_EINVAL, "popbg_dev cannot be combined with traj_dev or record_dev");
    if (sim->popbg_dev && ((uintptr_t)sim->popbg_dev % 8 != 0))
        return fail(VCT_EINVAL, "popbg_dev must be 8-byte aligned");
    const int64_t K = (int64_t)sim->n_days * (1440 / sim->ts_min);
    if (K >= ((int64_t)1 << 31))
        return fail(VCT_EINVAL, "horizon too long");
    if (ctrl->kind != VCT_CTRL_OPEN && ctrl->kind != VCT_CTRL_PID && ctrl->kind != VCT_CTRL_MPC &&
        ctrl->kind != VCT_CTRL_MLP && ctrl->kind != VCT_CTRL_DUAL)
        return fail(VCT_EINVAL, "controller kind %d", ctrl->kind);
    // model extensions, exercise and the dual-hormone AP
    if (sim->model_ext != 0 && sim->model_ext != 1)
        return fail(VCT_EINVAL, "model_ext %d (0 or 1)", sim->model_ext);
    if (sim->model_ext) {
        if (!(finite_pos(sim->tau_n) && finite_pos(sim->tau_e1) && finite_pos(sim->tau_e2) &&
              finite_pos(sim->tau_e3)))
            return fail(VCT_EINVAL, "model extensions: time constants must be finite and > 0");
        if (!(std::isfinite(sim->e_n) && sim->e_n >= 0.0 && std::isfinite(sim->alpha_e) && sim->alpha_e >= 0.0 &&
              std::isfinite(sim->beta_e) && sim->beta_e >= 0.0))
            return fail(VCT_EINVAL, "model extensions: e_n, alpha_e and beta_e must be finite and >= 0");
        if (ctrl->kind == VCT_CTRL_MPC || ctrl->kind == VCT_CTRL_MLP)
            return fail(VCT_ENOTSUP, "model extensions with the MPC or learned controller");
        if (sim->popbg_dev)
            return fail(VCT_ENOTSUP, "model extensions with popbg_dev");
    }
    if (sim->doses_dev && (!sim->model_ext || (uintptr_t)sim->doses_dev % 8 != 0))
        return fail(VCT_EINVAL, "doses_dev needs model_ext and 8-byte alignment");
    if (ctrl->kind == VCT_CTRL_DUAL) {
        if (!sim->model_ext)
            return fail(VCT_EINVAL, "the dual-hormone AP needs the model extensions (model_ext = 1)");
        if (ctrl->meal_bolus != 0 && ctrl->meal_bolus != 1)
            return fail(VCT_EINVAL, "meal_bolus %d (0 or 1)", ctrl->meal_bolus);
        if (!(finite_pos(ctrl->icr_rule) && std::isfinite(ctrl->glu_enter) && std::isfinite(ctrl->glu_exit) &&
              ctrl->glu_enter <= ctrl->glu_exit && std::isfinite(ctrl->glu_target) && std::isfinite(ctrl->glu_kp) &&
              ctrl->glu_kp >= 0.0 && std::isfinite(ctrl->glu_max) && ctrl->glu_max >= 0.0 &&
              std::isfinite(ctrl->ex_bolus) && ctrl->ex_bolus >= 0.0 && std::isfinite(ctrl->ex_bolus_below)))
            return fail(VCT_EINVAL, "dual-hormone AP settings invalid (icr_rule > 0, glu_enter <= glu_exit, "
                                    "glu_kp, glu_max, ex_bolus >= 0, all finite)");
    }
    if (pr->exercise != 0 && pr->exercise != 1)
        return fail(VCT_EINVAL, "protocol: exercise %d (0 or 1)", pr->exercise);
    if (pr->exercise) {
        if (pr->kind != VCT_PROTO_NORDIC || !sim->model_ext)
            return fail(VCT_EINVAL, "exercise needs the Northern-European protocol and the model extensions");
        if (pr->exercise_minute < 0 || pr->exercise_minute > 1439 || pr->exercise_duration < 1 ||
            pr->exercise_duration > 240 || !(pr->exercise_hrr >= 0.0 && pr->exercise_hrr <= 1.0))
            return fail(VCT_EINVAL, "protocol: exercise minute, duration or intensity out of range");
    }
    const bool uses_mpc = ctrl->kind == VCT_CTRL_MPC || ctrl->kind == VCT_CTRL_MLP;
    if (sim->record_dev && !uses_mpc)
        return fail(VCT_EINVAL, "record_dev needs the MPC or the learned controller");
    if (ctrl->kind == VCT_CTRL_MLP && (!ctrl->mlp_dev || (uintptr_t)ctrl->mlp_dev % 16 != 0))
        return fail(VCT_EINVAL, "learned controller needs mlp_dev (a 16-byte aligned network blob)");
    if (ctrl->kind == VCT_CTRL_MLP && !(std::isfinite(ctrl->mlp_safe_g) && std::isfinite(ctrl->mlp_safe_out)))
        return fail(VCT_EINVAL, "learned controller: mlp_safe_g and mlp_safe_out must be finite");
    if (uses_mpc) {
        if (!ctrl->mpc_dev)
            return fail(VCT_EINVAL, "MPC and learned controllers need mpc_dev (from vct_mpc_setup)");
        if (ctrl->mpc_horizon != vct::kMpcN)
            return fail(VCT_ENOTSUP, "MPC horizon %d (this build: %d)", ctrl->mpc_horizon, vct::kMpcN);
        if (ctrl->mpc_iters < 0 || ctrl->mpc_iters > 1000)
            return fail(VCT_EINVAL, "mpc_iters %d out of [0, 1000]", ctrl->mpc_iters);
    }
    if (!(std::isfinite(ctrl->setpoint) && std::isfinite(ctrl->kp) && std::isfinite(ctrl->ki) &&
          std::isfinite(ctrl->kd) && finite_pos(ctrl->umax_rel) && std::isfinite(ctrl->u_rel) && ctrl->u_rel >= 0))
        return fail(VCT_EINVAL, "controller gains must be finite, umax_rel > 0, u_rel >= 0");
    if (!finite_pos(ctrl->basal_scale))
        return fail(VCT_EINVAL, "basal_scale must be finite and > 0");
    if (ctrl->basal_scale != 1.0 && ctrl->kind != VCT_CTRL_PID && ctrl->kind != VCT_CTRL_OPEN)
        return fail(VCT_ENOTSUP, "basal_scale != 1 needs the PID or open-loop controller");
    vct_status st = check_protocol(pr, sim->ts_min);
    if (st != VCT_OK)
        return st;

    a = vct::SimArgs{};
    a.params = pop->params;
    a.n = pop->n;
    a.patient_base = pop->first;
    a.n_days = sim->n_days;
    a.kday = 1440 / sim->ts_min;
    split_key(sim->noise_seed, pop->arm_id, a.key0, a.key1);
    a.proto = pr->kind;
    a.meal_cv = pr->meal_cv;
    a.n_slots = pr->kind == VCT_PROTO_NORDIC ? 0 : pr->n_slots;
    for (int m = 0; m < VCT_MAX_SLOTS; ++m) {
        a.minute_of_day[m] = pr->minute_of_day[m];
        a.carbs_mean[m] = pr->carbs_mean_g[m];
        a.carbs_sd[m] = pr->carbs_sd_g[m];
        a.prob[m] = pr->prob[m];
        a.prob_thresh[m] = m < pr->n_slots ? (uint32_t)std::ceil(pr->prob[m] * 16777216.0) : 0u;
    }
    a.rate_per_g = (1000.0 / 180.16) / (double)sim->ts_min;
    a.jitter = pr->jitter_min;
    a.ag = pop->ag;
    a.tau = pop->tau;
    a.g_target = pop->g_target;
    a.ctrl = ctrl->kind;
    a.setpoint = ctrl->setpoint;
    a.kp = ctrl->kp;
    a.ki = ctrl->ki;
    a.kd = ctrl->kd;
    a.umax_rel = ctrl->umax_rel;
    a.u_rel = ctrl->u_rel;
    a.basal_scale = ctrl->basal_scale;
    a.mpc = uses_mpc ? ctrl->mpc_dev : nullptr;
    a.mpc_iters = ctrl->mpc_iters;
    a.mlp = ctrl->kind == VCT_CTRL_MLP ? (const unsigned char *)ctrl->mlp_dev : nullptr;
    a.mlp_safe_g = ctrl->mlp_safe_g;
    a.mlp_safe_out = ctrl->mlp_safe_out;
    a.record = sim->record_dev;
    a.fallback = ctrl->kind == VCT_CTRL_MLP ? sim->fallback_dev : nullptr;
    a.ts_min = sim->ts_min;
    a.em_per_ctrl = sim->em_per_ctrl;
    a.h = (double)sim->ts_min / (double)sim->em_per_ctrl;
    a.sig_sqh = std::sqrt(a.h) * sim->sigma_q1;
    a.sqrt_r = std::sqrt(sim->cgm_var);
    char *m = (char *)sim->metrics_dev;
    const int64_t n = pop->n;
    a.sum_g = (double *)(m);
    a.min_g = (double *)(m + 8 * n);
    a.sum_u = (double *)(m + 16 * n);
    a.bins = (int32_t *)(m + 24 * n);
    a.events = (int32_t *)(m + 44 * n);
    a.argmin_k = (int32_t *)(m + 56 * n);
    a.status = (uint32_t *)(m + 60 * n);
    a.out_stride = n;
    a.n_traj = sim->traj_patients;
    a.traj = sim->traj_patients > 0 ? (double *)sim->traj_dev : nullptr;
    a.K = K;
    a.pop_sum = (int64_t *)sim->popbg_dev;
    a.pop_min = sim->popbg_dev ? (uint64_t *)sim->popbg_dev + K : nullptr;
    a.pop_max = sim->popbg_dev ? (uint64_t *)sim->popbg_dev + 2 * K : nullptr;
    a.pop_hist = sim->popbg_dev ? (uint64_t *)sim->popbg_dev + 3 * K : nullptr;
    a.span_min = sim->popbg_dev ? (uint64_t *)sim->popbg_dev + 3 * K + 402 : nullptr;
    a.span_max = sim->popbg_dev ? (uint64_t *)sim->popbg_dev + 3 * K + 452 : nullptr;
    a.pop_nonfinite = sim->popbg_dev ? (int64_t *)sim->popbg_dev + 3 * K + 502 : nullptr;
    a.ext = sim->model_ext;
    a.tau_n = sim->tau_n;
    a.e_n = sim->e_n;
    a.tau_e1 = sim->tau_e1;
    a.tau_e2 = sim->tau_e2;
    a.tau_e3 = sim->tau_e3;
    a.alpha_e = sim->alpha_e;
    a.beta_e = sim->beta_e;
    a.exercise = pr->exercise;
    a.ex_minute = pr->exercise_minute;
    a.ex_samples = (pr->exercise_duration + sim->ts_min - 1) / sim->ts_min;
    a.ex_hrr = pr->exercise_hrr;
    a.meal_bolus = ctrl->meal_bolus;
    a.icr_rule = ctrl->icr_rule;
    a.glu_enter = ctrl->glu_enter;
    a.glu_exit = ctrl->glu_exit;
    a.glu_target = ctrl->glu_target;
    a.glu_kp = ctrl->glu_kp;
    a.glu_max = ctrl->glu_max;
    a.ex_bolus = ctrl->ex_bolus;
    a.ex_bolus_below = ctrl->ex_bolus_below;
    a.doses = (double *)sim->doses_dev;
    return VCT_OK;
}

vct_status vct_simulate(const vct_population *pop, const vct_protocol *pr, const vct_controller *ctrl,
                        const vct_sim *sim, void *stream)
{
    g_err.clear();
    vct::SimArgs a;
    vct_status st = build_sim_args(pop, pr, ctrl, sim, true, a);
    if (st != VCT_OK) {
        g_err = "vct_simulate: " + g_err;
        return st;
    }
    hipStream_t s = (hipStream_t)stream;
    void *scratch = nullptr;
    if (ctrl->kind == VCT_CTRL_MLP) {
        const size_t nb = vct::policy_scratch_bytes(a.n, sim->precision);
        hipError_t e = hipMallocAsync(&scratch, nb, s);
        if (e != hipSuccess)
            return fail(VCT_ENOMEM, "vct_simulate: learned-controller scratch of %zu bytes: %s", nb,
                        hipGetErrorString(e));
        vct::policy_scratch_views(a, scratch, sim->precision);
    }
    hipError_t e = vct::launch_simulate(a, sim->precision, s);
    hipError_t e2 = scratch ? hipFreeAsync(scratch, s) : hipSuccess;
    if (e != hipSuccess)
        return hip_fail(e, "vct_simulate: launch");
    if (e2 != hipSuccess)
        return hip_fail(e2, "vct_simulate: free");
    return VCT_OK;
}

size_t vct_mpc_bytes(int64_t n, int32_t precision)
{
    if (n <= 0 || (precision != VCT_FP64 && precision != VCT_FP32))
        return 0;
    return (size_t)n * vct::kMRows * (precision == VCT_FP32 ? sizeof(float) : sizeof(double));
}

vct_status vct_mpc_setup(const vct_population *pop, const vct_controller *ctrl, const vct_sim *sim, void *mpc_dev,
                         void *stream)
{
    g_err.clear();
    if (!pop || !ctrl || !sim || !mpc_dev)
        return fail(VCT_EINVAL, "vct_mpc_setup: null argument");
    if (ctrl->mpc_horizon != vct::kMpcN)
        return fail(VCT_ENOTSUP, "vct_mpc_setup: horizon %d (this build: %d)", ctrl->mpc_horizon, vct::kMpcN);
    if (!(finite_pos(ctrl->mpc_rho) && finite_pos(ctrl->umax_rel)))
        return fail(VCT_EINVAL, "vct_mpc_setup: mpc_rho and umax_rel must be finite and > 0");
    if (sim->precision != VCT_FP64 && sim->precision != VCT_FP32)
        return fail(VCT_EINVAL, "vct_mpc_setup: precision %d", sim->precision);
    if (sim->ts_min < 1 || 1440 % sim->ts_min != 0 || sim->em_per_ctrl < 1 || sim->em_per_ctrl > 64)
        return fail(VCT_EINVAL, "vct_mpc_setup: ts_min / em_per_ctrl invalid");
    if (!(std::isfinite(sim->sigma_q1) && sim->sigma_q1 >= 0.0 && std::isfinite(sim->cgm_var) && sim->cgm_var >= 0.0))
        return fail(VCT_EINVAL, "vct_mpc_setup: sigma_q1 and cgm_var must be finite and >= 0");
    vct::MpcSetupArgs a{};
    a.params = pop->params;
    a.n = pop->n;
    a.h = (double)sim->ts_min / (double)sim->em_per_ctrl;
    a.ag = pop->ag;
    a.tau = pop->tau;
    a.g_target = pop->g_target;
    a.em_per_ctrl = sim->em_per_ctrl;
    a.sigma_q1 = sim->sigma_q1;
    a.cgm_var = sim->cgm_var;
    a.rho = ctrl->mpc_rho;
    a.umax_rel = ctrl->umax_rel;
    a.riccati_iters = 500;
    a.power_iters = 100;
    // FP64 hand-over of A between the setup kernel and the Riccati kernel (stream-ordered,
    // freed after the launches)
    hipStream_t s = (hipStream_t)stream;
    const size_t a64_bytes = (size_t)vct::kNx * vct::kNx * sizeof(double) * (size_t)pop->n;
    hipError_t e = hipMallocAsync((void **)&a.a64, a64_bytes, s);
    if (e != hipSuccess)
        return fail(VCT_ENOMEM, "vct_mpc_setup: scratch of %zu bytes: %s", a64_bytes, hipGetErrorString(e));
    e = vct::launch_mpc_setup(a, sim->precision, mpc_dev, s);
    const hipError_t e2 = hipFreeAsync(a.a64, s);
    if (e != hipSuccess)
        return hip_fail(e, "vct_mpc_setup: launch");
    if (e2 != hipSuccess)
        return hip_fail(e2, "vct_mpc_setup: free");
    return VCT_OK;
}

// ------------------------------------------------------------ learned controller ----
namespace {

const size_t kParamBytes = (size_t)vct::kMlpParams * sizeof(float);
const size_t kLossOff = 4 * kParamBytes;             // loss slot (256 bytes)
const size_t kLossPartOff = kLossOff + 256;           // 1024 partial losses
const size_t kScratchOff = kLossPartOff + 1024 * sizeof(float);
const int32_t kMaxBatch = 65536;

size_t mlp_scratch_bytes(int32_t batch)
{
    return std::max((size_t)(batch / 64) * kParamBytes, vct::mlp_stats_scratch_bytes());
}

vct::MlpTrain train_views(void *train_dev, void *blob_dev)
{
    char *b = (char *)train_dev;
    vct::MlpTrain t;
    t.master = (float *)b;
    t.m = (float *)(b + kParamBytes);
    t.v = (float *)(b + 2 * kParamBytes);
    t.grad = (float *)(b + 3 * kParamBytes);
    t.loss = (float *)(b + kLossOff);
    t.loss_partial = (float *)(b + kLossPartOff);
    t.partial = (float *)(b + kScratchOff);
    t.blob = (unsigned char *)blob_dev;
    return t;
}

}  // namespace

size_t vct_mlp_blob_bytes(void) { return (size_t)vct::kMlpBlobBytes; }

size_t vct_mlp_train_bytes(int32_t batch)
{
    if (batch < 64 || batch > kMaxBatch || batch % 64 != 0)
        return 0;
    return kScratchOff + mlp_scratch_bytes(batch);
}

vct_status vct_mlp_init(uint64_t seed, void *train_dev, void *blob_dev, void *stream)
{
    g_err.clear();
    if (!train_dev || !blob_dev)
        return fail(VCT_EINVAL, "vct_mlp_init: null buffer");
    if ((uintptr_t)train_dev % 256 != 0 || (uintptr_t)blob_dev % 16 != 0)
        return fail(VCT_EINVAL, "vct_mlp_init: train_dev must be 256-byte and blob_dev 16-byte aligned");
    uint32_t k0, k1;
    split_key(seed, 0u, k0, k1);
    hipError_t e = vct::launch_mlp_init(train_views(train_dev, blob_dev), k0, k1, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "vct_mlp_init: launch");
    return VCT_OK;
}

vct_status vct_mlp_normalize(const float *rows_dev, int64_t n_rows, double box_q, void *train_dev, void *blob_dev,
                             void *stream)
{
    g_err.clear();
    if (!rows_dev || !train_dev || !blob_dev)
        return fail(VCT_EINVAL, "vct_mlp_normalize: null buffer");
    if ((uintptr_t)train_dev % 256 != 0 || (uintptr_t)blob_dev % 16 != 0 || (uintptr_t)rows_dev % 4 != 0)
        return fail(VCT_EINVAL, "vct_mlp_normalize: misaligned buffer");
    if (n_rows < 1 || n_rows >= ((int64_t)1 << 40))
        return fail(VCT_EINVAL, "vct_mlp_normalize: n_rows %lld", (long long)n_rows);
    if (!(box_q >= 0.0 && box_q < 0.5))
        return fail(VCT_EINVAL, "vct_mlp_normalize: box_q must be in [0, 0.5)");
    const vct::MlpTrain t = train_views(train_dev, blob_dev);
    hipError_t e = vct::launch_mlp_stats(rows_dev, n_rows, box_q, (unsigned char *)blob_dev, t.partial,
                                         (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "vct_mlp_normalize: launch");
    return VCT_OK;
}

// Arguments shared by the single-step and multi-step training entry points.
static vct_status check_train_buffers(const char *fn, const float *rows_dev, int64_t n_rows, const int32_t *idx_dev,
                                      int32_t batch, void *train_dev, void *blob_dev)
{
    if (!rows_dev || !train_dev || !blob_dev)
        return fail(VCT_EINVAL, "%s: null buffer", fn);
    if ((uintptr_t)train_dev % 256 != 0 || (uintptr_t)blob_dev % 16 != 0 || (uintptr_t)rows_dev % 4 != 0 ||
        (uintptr_t)idx_dev % 4 != 0)
        return fail(VCT_EINVAL, "%s: misaligned buffer", fn);
    if (n_rows < 1 || n_rows > ((int64_t)1 << 32))
        return fail(VCT_EINVAL, "%s: n_rows %lld out of [1, 2^32]", fn, (long long)n_rows);
    if (batch < 64 || batch > kMaxBatch || batch % 64 != 0)
        return fail(VCT_EINVAL, "%s: batch %d (a multiple of 64 in [64, %d])", fn, batch, kMaxBatch);
    return VCT_OK;
}

vct_status vct_mlp_train_step(const float *rows_dev, int64_t n_rows, const int32_t *idx_dev, uint64_t seed,
                              int32_t step, int32_t batch, double lr, int32_t apply, void *train_dev,
                              void *blob_dev, void *stream)
{
    g_err.clear();
    const vct_status st = check_train_buffers("vct_mlp_train_step", rows_dev, n_rows, idx_dev, batch, train_dev,
                                              blob_dev);
    if (st != VCT_OK)
        return st;
    if (step < 0)
        return fail(VCT_EINVAL, "vct_mlp_train_step: step %d < 0", step);
    if (!(std::isfinite(lr) && lr >= 0.0))
        return fail(VCT_EINVAL, "vct_mlp_train_step: lr must be finite and >= 0");
    uint32_t k0, k1;
    split_key(seed, 0u, k0, k1);
    const double t = (double)step + 1.0;
    const float bc1 = (float)(1.0 - std::pow(0.9, t)), bc2 = (float)(1.0 - std::pow(0.999, t));
    hipError_t e = vct::launch_mlp_step(train_views(train_dev, blob_dev), rows_dev, n_rows, idx_dev, k0, k1, step,
                                        batch, (float)lr, bc1, bc2, apply != 0, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "vct_mlp_train_step: launch");
    return VCT_OK;
}

// Learning rate of step i of a vct_mlp_train call: cosine decay from lr to lr_min over
// sched_total steps.
static double cosine_lr(double lr, double lr_min, int32_t sched_offset, int32_t i, int32_t sched_total)
{
    return lr_min + 0.5 * (lr - lr_min) * (1.0 + std::cos(M_PI * (double)(sched_offset + i) / (double)sched_total));
}

vct_status vct_mlp_train(const float *rows_dev, int64_t n_rows, uint64_t seed, int32_t first_step, int32_t n_steps,
                         int32_t sched_offset, int32_t sched_total, int32_t batch, double lr, double lr_min,
                         void *train_dev, void *blob_dev, void *stream)
{
    g_err.clear();
    if (n_steps < 0 || sched_offset < 0 || sched_total < 1 || first_step < 0 || first_step > INT32_MAX - n_steps)
        return fail(VCT_EINVAL, "vct_mlp_train: steps or schedule out of range");
    if (!(std::isfinite(lr_min) && lr_min >= 0.0 && std::isfinite(lr) && lr >= lr_min))
        return fail(VCT_EINVAL, "vct_mlp_train: need finite 0 <= lr_min <= lr");
    const vct_status st = check_train_buffers("vct_mlp_train", rows_dev, n_rows, nullptr, batch, train_dev, blob_dev);
    if (st != VCT_OK)
        return st;
    for (int32_t i = 0; i < n_steps; ++i) {
        const vct_status s = vct_mlp_train_step(rows_dev, n_rows, nullptr, seed, first_step + i, batch,
                                                cosine_lr(lr, lr_min, sched_offset, i, sched_total), 1, train_dev,
                                                blob_dev, stream);
        if (s != VCT_OK)
            return s;
    }
    return VCT_OK;
}

vct_status vct_mlp_forward(const float *x_dev, int64_t n, const void *blob_dev, float *out_dev, void *stream)
{
    g_err.clear();
    if (!x_dev || !blob_dev || !out_dev)
        return fail(VCT_EINVAL, "vct_mlp_forward: null buffer");
    if ((uintptr_t)blob_dev % 16 != 0 || (uintptr_t)x_dev % 4 != 0 || (uintptr_t)out_dev % 4 != 0)
        return fail(VCT_EINVAL, "vct_mlp_forward: misaligned buffer");
    if (n < 1 || n >= ((int64_t)1 << 37))
        return fail(VCT_EINVAL, "vct_mlp_forward: n %lld", (long long)n);
    hipError_t e = vct::launch_mlp_forward(x_dev, n, (const unsigned char *)blob_dev, out_dev, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "vct_mlp_forward: launch");
    return VCT_OK;
}

// Copies a device-side reduction result into the caller's summary.
static void fill_summary(const vct::ReduceOut &h, int64_t n, int64_t K, vct_summary *out)
{
    std::memset(out, 0, sizeof *out);
    out->n_patients = n;
    out->n_samples = K;
    for (int q = 0; q < 5; ++q) out->bins[q] = h.bins[q];
    for (int q = 0; q < 3; ++q) out->events[q] = h.events[q];
    for (int q = 0; q < 5; ++q) {
        out->q_count[q] = h.q_count[q];
        out->q_frac[q] = (double)h.q_count[q] / (double)K;
    }
    out->mean_tir = (double)h.bins[2] / ((double)n * (double)K);
    out->mean_bg = h.sum_g / ((double)n * (double)K);
    out->mean_insulin = h.sum_u / (double)n;
    out->worst_patient = h.worst_patient;
    out->worst_min_g = h.worst_min_g;
    out->worst_k = h.worst_k;
    for (int q = 0; q < 3; ++q) out->status_count[q] = h.status_count[q];
    const int64_t nc = h.n_clean;
    out->n_clean = nc;
    for (int q = 0; q < 5; ++q) {
        out->bins_clean[q] = h.bins_clean[q];
        out->q_count_clean[q] = h.q_count_clean[q];
        out->q_frac_clean[q] = (double)h.q_count_clean[q] / (double)K;
    }
    out->mean_tir_clean = nc > 0 ? (double)h.bins_clean[2] / ((double)nc * (double)K) : 0.0;
    out->mean_bg_clean = nc > 0 ? h.sum_g_clean / ((double)nc * (double)K) : 0.0;
}

// Launches the reduction into `ws`, copies the result to the host and synchronises.
static hipError_t reduce_to_host(const void *metrics_dev, int64_t n, int64_t K, void *ws, vct::ReduceOut *h,
                                 hipStream_t s)
{
    const char *m = (const char *)metrics_dev;
    vct::ReduceOut *dres = nullptr;
    hipError_t e = vct::launch_reduce((const double *)m, (const double *)(m + 8 * n), (const double *)(m + 16 * n),
                                      (const int32_t *)(m + 24 * n), (const int32_t *)(m + 44 * n),
                                      (const int32_t *)(m + 56 * n), (const uint32_t *)(m + 60 * n), n, K, ws, &dres,
                                      s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, dres, sizeof *h, hipMemcpyDeviceToHost, s);
    return e;
}

vct_status vct_read_metrics(const void *metrics_dev, int64_t n, int64_t K, vct_summary *out, void *stream)
{
    g_err.clear();
    if (!metrics_dev || !out)
        return fail(VCT_EINVAL, "vct_read_metrics: null argument");
    if (n < 1 || n >= kMaxPatients || K < 1 || K >= ((int64_t)1 << 31))
        return fail(VCT_EINVAL, "vct_read_metrics: n %lld or K %lld out of range", (long long)n, (long long)K);
    hipStream_t s = (hipStream_t)stream;
    const size_t ws_bytes = vct::reduce_workspace_bytes(n, K);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, ws_bytes, s);
    if (e != hipSuccess)
        return fail(VCT_ENOMEM, "vct_read_metrics: workspace of %zu bytes: %s", ws_bytes, hipGetErrorString(e));
    vct::ReduceOut h{};
    e = reduce_to_host(metrics_dev, n, K, ws, &h, s);
    hipError_t e2 = hipFreeAsync(ws, s);
    hipError_t e3 = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "vct_read_metrics: reduction");
    if (e2 != hipSuccess)
        return hip_fail(e2, "vct_read_metrics: free");
    if (e3 != hipSuccess)
        return hip_fail(e3, "vct_read_metrics: synchronize");
    fill_summary(h, n, K, out);
    return VCT_OK;
}

vct_status vct_read_metrics_noalloc(const void *metrics_dev, int64_t n, int64_t K, vct_summary *out, void *stream)
{
    g_err.clear();
    if (!metrics_dev || !out)
        return fail(VCT_EINVAL, "vct_read_metrics_noalloc: null argument");
    if (n < 1 || n >= kMaxPatients || K < 1 || K > VCT_NOALLOC_MAX_SAMPLES)
        return fail(VCT_EINVAL, "vct_read_metrics_noalloc: n %lld or K %lld out of range (K <= %d)", (long long)n,
                    (long long)K, VCT_NOALLOC_MAX_SAMPLES);
    const size_t ws_bytes = vct::reduce_workspace_bytes(n, K);
    if (ws_bytes > sizeof scratch)
        return fail(VCT_EINVAL, "vct_read_metrics_noalloc: workspace of %zu bytes exceeds the static %zu", ws_bytes,
                    sizeof scratch);
    void *ws = nullptr;
    hipError_t e = scratch_address(&ws);
    if (e != hipSuccess)
        return hip_fail(e, "vct_read_metrics_noalloc: scratch address");
    hipStream_t s = (hipStream_t)stream;
    vct::ReduceOut h{};
    e = reduce_to_host(metrics_dev, n, K, ws, &h, s);
    hipError_t e2 = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "vct_read_metrics_noalloc: reduction");
    if (e2 != hipSuccess)
        return hip_fail(e2, "vct_read_metrics_noalloc: synchronize");
    fill_summary(h, n, K, out);
    return VCT_OK;
}

// ------------------------------------------------------------- batched arms ----
struct vct_batch {
    int32_t n_arms = 0;
    int precision = 0, ctrl = 0;
    bool noisy = false;
    vct::SimArgs *d_arms = nullptr;
    vct::BatchItem *d_items = nullptr;
    uint32_t *d_counter = nullptr;
    int32_t n_items = 0;
    int32_t block = 0, grid = 0;
    double tuned_ms[4] = {0, 0, 0, 0};
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static const int kBlocks[4] = {64, 128, 256, 512};

// Work items of one block size: tiles of `block` patients, longest horizon first (LPT),
// then arm and patient order.
static std::vector<vct::BatchItem> make_items(const std::vector<vct::SimArgs> &arms, int block)
{
    std::vector<int32_t> order(arms.size());
    for (size_t q = 0; q < arms.size(); ++q)
        order[q] = (int32_t)q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return arms[x].n_days > arms[y].n_days; });
    std::vector<vct::BatchItem> items;
    for (int32_t q : order)
        for (int64_t f = 0; f < arms[q].n; f += block)
            items.push_back(vct::BatchItem{q, (int32_t)f});
    return items;
}

static void free_batch(vct_batch *b)
{
    if (!b)
        return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->cap) hipStreamDestroy(b->cap);
    if (b->d_arms) hipFree(b->d_arms);
    if (b->d_items) hipFree(b->d_items);
    if (b->d_counter) hipFree(b->d_counter);
    delete b;
}

static vct_status upload_items(vct_batch *b, const std::vector<vct::BatchItem> &items)
{
    if (b->d_items) {
        hipFree(b->d_items);
        b->d_items = nullptr;
    }
    hipError_t e = hipMalloc(&b->d_items, items.size() * sizeof(vct::BatchItem));
    if (e != hipSuccess)
        return fail(VCT_ENOMEM, "vct_batch_create: item table: %s", hipGetErrorString(e));
    e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(vct::BatchItem), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return hip_fail(e, "vct_batch_create: item upload");
    b->n_items = (int32_t)items.size();
    return VCT_OK;
}

static vct::BatchLaunch launch_of(const vct_batch *b, const vct::SimArgs *arms)
{
    vct::BatchLaunch L;
    L.arms = arms;
    L.items = b->d_items;
    L.n_items = b->n_items;
    L.counter = b->d_counter;
    L.grid = b->grid;
    L.block = b->block;
    L.precision = b->precision;
    L.ctrl = b->ctrl;
    L.noisy = b->noisy;
    return L;
}

static int grid_for(const vct_batch *b, int block, int n_items)
{
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int per_cu = vct::batch_blocks_per_cu(b->precision, b->ctrl, b->noisy, block);
    const int resident = std::max(1, cus * std::max(1, per_cu));
    return std::min(resident, n_items);
}

vct_status vct_batch_create(const vct_arm *arms, int32_t n_arms, const vct_protocol *pr, const vct_controller *ctrl,
                            const vct_sim *sim, int32_t block, void *stream, vct_batch **out)
{
    g_err.clear();
    if (!arms || !out || n_arms < 1 || n_arms > 65536)
        return fail(VCT_EINVAL, "vct_batch_create: need 1..65536 arms and an output handle");
    if (block != 0 && block != 64 && block != 128 && block != 256 && block != 512)
        return fail(VCT_EINVAL, "vct_batch_create: block %d (0 = autotune, or 64/128/256/512)", block);
    if (!ctrl || !sim || !pr)
        return fail(VCT_EINVAL, "vct_batch_create: null argument");
    if (ctrl->kind != VCT_CTRL_PID && ctrl->kind != VCT_CTRL_OPEN)
        return fail(VCT_ENOTSUP, "vct_batch_create: batched arms run the PID or open-loop controller");
    if (sim->model_ext || sim->doses_dev)
        return fail(VCT_ENOTSUP, "vct_batch_create: batched arms run the core model");
    if (sim->record_dev || sim->fallback_dev || sim->popbg_dev)
        return fail(VCT_EINVAL, "vct_batch_create: record_dev / fallback_dev / popbg_dev are per-population outputs");
    std::vector<vct::SimArgs> hargs(n_arms);
    for (int32_t q = 0; q < n_arms; ++q) {
        if (!arms[q].pop)
            return fail(VCT_EINVAL, "vct_batch_create: arm %d has no population", q);
        vct_sim s = *sim;
        s.n_days = arms[q].n_days;
        s.metrics_dev = arms[q].metrics_dev;
        s.traj_patients = 0;
        s.traj_dev = nullptr;
        vct_controller c = *ctrl;
        c.kp = arms[q].kp;
        c.ki = arms[q].ki;
        c.kd = arms[q].kd;
        c.basal_scale = arms[q].basal_scale;
        vct_status st = build_sim_args(arms[q].pop, pr, &c, &s, true, hargs[q]);
        if (st != VCT_OK) {
            g_err = "vct_batch_create: arm " + std::to_string(q) + ": " + g_err;
            return st;
        }
    }
    vct_batch *b = new (std::nothrow) vct_batch;
    if (!b)
        return fail(VCT_ENOMEM, "vct_batch_create: out of host memory");
    b->n_arms = n_arms;
    b->precision = sim->precision;
    b->ctrl = ctrl->kind;
    b->noisy = sim->sigma_q1 != 0.0 || sim->cgm_var != 0.0;
    hipStream_t us = (hipStream_t)stream;
    hipError_t e = hipMalloc(&b->d_arms, sizeof(vct::SimArgs) * (size_t)n_arms * 2);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_counter, sizeof(uint32_t));
    if (e != hipSuccess) {
        free_batch(b);
        return fail(VCT_ENOMEM, "vct_batch_create: %s", hipGetErrorString(e));
    }
    // second copy of the arm table with horizons capped at 2 days: autotuning runs
    std::vector<vct::SimArgs> cal = hargs;
    for (auto &a : cal) {
        a.n_days = std::min(a.n_days, 2);
        a.K = (int64_t)a.n_days * a.kday;
    }
    vct::SimArgs *d_cal = b->d_arms + n_arms;
    e = hipMemcpy(b->d_arms, hargs.data(), sizeof(vct::SimArgs) * n_arms, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d_cal, cal.data(), sizeof(vct::SimArgs) * n_arms, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "vct_batch_create: arm upload");
    }

    // autotuner: time each block shape on the capped horizons, keep the fastest
    int chosen = block;
    if (chosen == 0) {
        hipEvent_t e0, e1;
        hipEventCreate(&e0);
        hipEventCreate(&e1);
        double best = 1e30;
        for (int t = 0; t < 4; ++t) {
            const int blk = kBlocks[t];
            vct_status st = upload_items(b, make_items(hargs, blk));
            if (st != VCT_OK) {
                free_batch(b);
                return st;
            }
            b->block = blk;
            b->grid = grid_for(b, blk, b->n_items);
            vct::BatchLaunch L = launch_of(b, d_cal);
            float ms = 0.0f, best_t = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                hipEventRecord(e0, us);
                e = vct::launch_batch(L, us);
                hipEventRecord(e1, us);
                if (e == hipSuccess)
                    e = hipEventSynchronize(e1);
                if (e != hipSuccess) {
                    hipEventDestroy(e0);
                    hipEventDestroy(e1);
                    free_batch(b);
                    return hip_fail(e, "vct_batch_create: autotune launch");
                }
                hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0)
                    best_t = std::min(best_t, ms);
            }
            b->tuned_ms[t] = best_t;
            if (best_t < best) {
                best = best_t;
                chosen = blk;
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
    }
    vct_status st = upload_items(b, make_items(hargs, chosen));
    if (st != VCT_OK) {
        free_batch(b);
        return st;
    }
    b->block = chosen;
    b->grid = grid_for(b, chosen, b->n_items);

    // capture counter reset + persistent launch once; vct_batch_run replays it
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t el = vct::launch_batch(launch_of(b, b->d_arms), b->cap);
        e = hipStreamEndCapture(b->cap, &b->graph);
        if (el != hipSuccess)
            e = el;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "vct_batch_create: graph capture");
    }
    *out = b;
    return VCT_OK;
}

vct_status vct_batch_run(vct_batch *b, void *stream)
{
    g_err.clear();
    if (!b || !b->exec)
        return fail(VCT_EINVAL, "vct_batch_run: invalid batch");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "vct_batch_run: graph launch");
    return VCT_OK;
}

vct_status vct_batch_info(const vct_batch *b, vct_batch_stats *out)
{
    g_err.clear();
    if (!b || !out)
        return fail(VCT_EINVAL, "vct_batch_info: null argument");
    out->n_arms = b->n_arms;
    out->n_items = b->n_items;
    out->block = b->block;
    out->grid = b->grid;
    for (int t = 0; t < 4; ++t) {
        out->tuned_block[t] = kBlocks[t];
        out->tuned_ms[t] = b->tuned_ms[t];
    }
    return VCT_OK;
}

void vct_batch_destroy(vct_batch *b) { free_batch(b); }

}  // extern "C"

