"""Thin ctypes binding of the C ABI in include/vct.h (argument marshalling only).

Every step of the trial runs in the HIP library ``libvct.so``; this module only
fills the C structs, passes device pointers (torch tensors are accepted and their
``data_ptr()`` is used) and stream handles, and turns error codes into
exceptions. Importing it does not load the library; the first call does, and it
raises if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvct.so")

VCT_NP, VCT_NX, VCT_NPARAM_ROWS, VCT_MAX_SLOTS = 15, 11, 19, 4
VCT_OK, VCT_EINVAL, VCT_ENOMEM, VCT_EHIP, VCT_ESTATE, VCT_ENOTSUP = 0, -1, -2, -3, -4, -5
VCT_CTRL_OPEN, VCT_CTRL_PID, VCT_CTRL_MPC, VCT_CTRL_MLP, VCT_CTRL_DUAL = 0, 1, 2, 3, 4
VCT_PROTO_SLOTS, VCT_PROTO_NORDIC = 0, 1
VCT_FP64, VCT_FP32 = 0, 1
VCT_POP_MIN_BASAL = 1
VCT_NOALLOC_MAX_SAMPLES, VCT_NOALLOC_SCRATCH_BYTES = 210240, 2097152
VCT_MLP_IN, VCT_MLP_PARAMS, VCT_MLP_BLOB_BYTES = 12, 10448, 21568
# byte offsets inside a learned-controller blob
MLP_BLOB = {"W1": 0, "W2": 2048, "W3": 10240, "W4": 18432, "b1": 20480, "b2": 20736, "b3": 20992, "b4": 21248,
            "mean": 21312, "istd": 21376, "lo": 21440, "hi": 21504}
# FP32 parameter order (padded shapes) of master / Adam moments / gradient
MLP_PARAM_SHAPES = (("W1", (64, 16)), ("W2", (64, 64)), ("W3", (64, 64)), ("W4", (16, 64)), ("b1", (64,)),
                    ("b2", (64,)), ("b3", (64,)), ("b4", (16,)))

# byte offsets of the per-patient metric arrays inside a metrics buffer of n patients
METRIC_LAYOUT = (("sum_g", "f8", 0, 1), ("min_g", "f8", 8, 1), ("sum_u", "f8", 16, 1),
                 ("bins", "i4", 24, 5), ("events", "i4", 44, 3), ("argmin_k", "i4", 56, 1),
                 ("status", "u4", 60, 1))


class vct_population_desc(C.Structure):
    _fields_ = [("n_patients", C.c_int64), ("seed", C.c_uint64), ("arm_id", C.c_uint32), ("flags", C.c_uint32),
                ("nominal", C.c_double * VCT_NP), ("cv", C.c_double), ("ag", C.c_double),
                ("tau_cgm", C.c_double), ("g_target", C.c_double), ("first_patient", C.c_int64)]


class vct_protocol(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("minute_of_day", C.c_int32 * VCT_MAX_SLOTS),
                ("carbs_mean_g", C.c_double * VCT_MAX_SLOTS), ("carbs_sd_g", C.c_double * VCT_MAX_SLOTS),
                ("prob", C.c_double * VCT_MAX_SLOTS), ("jitter_min", C.c_int32), ("kind", C.c_int32),
                ("meal_cv", C.c_double), ("exercise", C.c_int32), ("exercise_minute", C.c_int32),
                ("exercise_duration", C.c_int32), ("exercise_hrr", C.c_double)]


class vct_controller(C.Structure):
    _fields_ = [("kind", C.c_int32), ("setpoint", C.c_double), ("kp", C.c_double), ("ki", C.c_double),
                ("kd", C.c_double), ("umax_rel", C.c_double), ("u_rel", C.c_double), ("mpc_horizon", C.c_int32),
                ("mpc_iters", C.c_int32), ("mpc_rho", C.c_double), ("mpc_dev", C.c_void_p),
                ("mlp_dev", C.c_void_p), ("mlp_safe_g", C.c_double), ("mlp_safe_out", C.c_double),
                ("basal_scale", C.c_double), ("meal_bolus", C.c_int32), ("icr_rule", C.c_double),
                ("glu_enter", C.c_double), ("glu_exit", C.c_double), ("glu_target", C.c_double),
                ("glu_kp", C.c_double), ("glu_max", C.c_double), ("ex_bolus", C.c_double),
                ("ex_bolus_below", C.c_double)]


class vct_sim(C.Structure):
    _fields_ = [("n_days", C.c_int32), ("em_per_ctrl", C.c_int32), ("ts_min", C.c_int32), ("precision", C.c_int32),
                ("sigma_q1", C.c_double), ("cgm_var", C.c_double), ("noise_seed", C.c_uint64),
                ("metrics_dev", C.c_void_p), ("traj_patients", C.c_int32), ("traj_dev", C.c_void_p),
                ("record_dev", C.c_void_p), ("fallback_dev", C.c_void_p), ("popbg_dev", C.c_void_p),
                ("model_ext", C.c_int32), ("tau_n", C.c_double), ("e_n", C.c_double), ("tau_e1", C.c_double),
                ("tau_e2", C.c_double), ("tau_e3", C.c_double), ("alpha_e", C.c_double), ("beta_e", C.c_double),
                ("doses_dev", C.c_void_p)]


class vct_summary(C.Structure):
    _fields_ = [("n_patients", C.c_int64), ("n_samples", C.c_int64), ("bins", C.c_uint64 * 5),
                ("events", C.c_uint64 * 3), ("q_count", C.c_int64 * 5), ("q_frac", C.c_double * 5),
                ("mean_tir", C.c_double), ("mean_bg", C.c_double), ("mean_insulin", C.c_double),
                ("worst_patient", C.c_int64), ("worst_min_g", C.c_double), ("worst_k", C.c_int32),
                ("_pad", C.c_int32), ("status_count", C.c_int64 * 3), ("n_clean", C.c_int64),
                ("bins_clean", C.c_uint64 * 5), ("q_count_clean", C.c_int64 * 5), ("q_frac_clean", C.c_double * 5),
                ("mean_tir_clean", C.c_double), ("mean_bg_clean", C.c_double)]

    def as_dict(self) -> dict:
        return {
            "n_patients": self.n_patients, "n_samples": self.n_samples, "bins": list(self.bins),
            "events": list(self.events), "q_count": list(self.q_count), "q_frac": list(self.q_frac),
            "mean_tir": self.mean_tir, "mean_bg": self.mean_bg, "mean_insulin": self.mean_insulin,
            "worst_patient": self.worst_patient, "worst_min_g": self.worst_min_g, "worst_k": self.worst_k,
            "status_count": list(self.status_count), "n_clean": self.n_clean,
            "bins_clean": list(self.bins_clean), "q_count_clean": list(self.q_count_clean),
            "q_frac_clean": list(self.q_frac_clean), "mean_tir_clean": self.mean_tir_clean,
            "mean_bg_clean": self.mean_bg_clean,
        }


class vct_arm(C.Structure):
    _fields_ = [("pop", C.c_void_p), ("n_days", C.c_int32), ("kp", C.c_double), ("ki", C.c_double),
                ("kd", C.c_double), ("metrics_dev", C.c_void_p), ("basal_scale", C.c_double)]


class vct_batch_stats(C.Structure):
    _fields_ = [("n_arms", C.c_int32), ("n_items", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32),
                ("tuned_block", C.c_int32 * 4), ("tuned_ms", C.c_double * 4)]

    def as_dict(self) -> dict:
        return {"n_arms": self.n_arms, "n_items": self.n_items, "block": self.block, "grid": self.grid,
                "tuned": dict(zip(list(self.tuned_block), list(self.tuned_ms)))}


class VctError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


# every symbol include/vct.h declares
EXPORTS = ("vct_abi_version", "vct_last_error", "vct_population_bytes", "vct_metrics_bytes", "vct_traj_bytes",
           "vct_create_population", "vct_simulate", "vct_read_metrics", "vct_read_metrics_noalloc",
           "vct_destroy_population",
           "vct_batch_create", "vct_batch_run", "vct_batch_info", "vct_batch_destroy", "vct_mpc_bytes",
           "vct_mpc_setup", "vct_mlp_blob_bytes", "vct_mlp_train_bytes", "vct_mlp_init", "vct_mlp_normalize",
           "vct_mlp_train_step", "vct_mlp_train", "vct_mlp_forward", "vct_popbg_bytes")

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.vct_abi_version.restype = C.c_int
        L.vct_last_error.restype = C.c_char_p
        L.vct_population_bytes.argtypes = [C.c_int64]
        L.vct_population_bytes.restype = C.c_size_t
        L.vct_metrics_bytes.argtypes = [C.c_int64]
        L.vct_metrics_bytes.restype = C.c_size_t
        L.vct_traj_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.vct_traj_bytes.restype = C.c_size_t
        L.vct_popbg_bytes.argtypes = [C.c_int32, C.c_int32]
        L.vct_popbg_bytes.restype = C.c_size_t
        L.vct_create_population.argtypes = [C.POINTER(vct_population_desc), C.c_void_p, C.c_void_p,
                                             C.POINTER(C.c_void_p)]
        L.vct_create_population.restype = C.c_int
        L.vct_simulate.argtypes = [C.c_void_p, C.POINTER(vct_protocol), C.POINTER(vct_controller),
                                   C.POINTER(vct_sim), C.c_void_p]
        L.vct_simulate.restype = C.c_int
        L.vct_read_metrics.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(vct_summary), C.c_void_p]
        L.vct_read_metrics.restype = C.c_int
        L.vct_read_metrics_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(vct_summary),
                                               C.c_void_p]
        L.vct_read_metrics_noalloc.restype = C.c_int
        L.vct_destroy_population.argtypes = [C.c_void_p]
        L.vct_destroy_population.restype = None
        L.vct_batch_create.argtypes = [C.POINTER(vct_arm), C.c_int32, C.POINTER(vct_protocol),
                                       C.POINTER(vct_controller), C.POINTER(vct_sim), C.c_int32, C.c_void_p,
                                       C.POINTER(C.c_void_p)]
        L.vct_batch_create.restype = C.c_int
        L.vct_batch_run.argtypes = [C.c_void_p, C.c_void_p]
        L.vct_batch_run.restype = C.c_int
        L.vct_batch_info.argtypes = [C.c_void_p, C.POINTER(vct_batch_stats)]
        L.vct_batch_info.restype = C.c_int
        L.vct_batch_destroy.argtypes = [C.c_void_p]
        L.vct_batch_destroy.restype = None
        L.vct_mpc_bytes.argtypes = [C.c_int64, C.c_int32]
        L.vct_mpc_bytes.restype = C.c_size_t
        L.vct_mpc_setup.argtypes = [C.c_void_p, C.POINTER(vct_controller), C.POINTER(vct_sim), C.c_void_p, C.c_void_p]
        L.vct_mpc_setup.restype = C.c_int
        L.vct_mlp_blob_bytes.argtypes = []
        L.vct_mlp_blob_bytes.restype = C.c_size_t
        L.vct_mlp_train_bytes.argtypes = [C.c_int32]
        L.vct_mlp_train_bytes.restype = C.c_size_t
        L.vct_mlp_init.argtypes = [C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.vct_mlp_init.restype = C.c_int
        L.vct_mlp_normalize.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
        L.vct_mlp_normalize.restype = C.c_int
        L.vct_mlp_train_step.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_uint64, C.c_int32, C.c_int32,
                                         C.c_double, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.vct_mlp_train_step.restype = C.c_int
        L.vct_mlp_train.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
        L.vct_mlp_train.restype = C.c_int
        L.vct_mlp_forward.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.vct_mlp_forward.restype = C.c_int
        _lib = L
    return _lib


def _ptr(x) -> int | None:
    """Device pointer of a torch tensor, or an int address, or None."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x)


def _stream(s) -> int | None:
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    return int(s)


def _check(fn: str, rc: int) -> None:
    if rc != VCT_OK:
        raise VctError(fn, rc, lib().vct_last_error().decode())


# ------------------------------------------------------------------ the ABI
def vct_abi_version() -> int:
    return lib().vct_abi_version()


def vct_last_error() -> str:
    return lib().vct_last_error().decode()


def vct_population_bytes(n: int) -> int:
    return lib().vct_population_bytes(n)


def vct_metrics_bytes(n: int) -> int:
    return lib().vct_metrics_bytes(n)


def vct_traj_bytes(traj_patients: int, n_days: int, ts_min: int) -> int:
    return lib().vct_traj_bytes(traj_patients, n_days, ts_min)


def vct_popbg_bytes(n_days: int, ts_min: int) -> int:
    return lib().vct_popbg_bytes(n_days, ts_min)


def popbg_decode(buf, n: int, K: int) -> dict:
    """Population BG per sample from a vct_popbg_bytes buffer (torch int64): mean, min, max
    in mmol/L over the patients with a finite G, as numpy float64 arrays (NaN where no G is
    finite), and the count of the others (the layout documented in vct.h)."""
    import numpy as np
    full = buf.cpu().numpy()
    a = full[:3 * K].reshape(3, K)
    keys = a[1:].view(np.uint64)
    neg = (keys >> np.uint64(63)) == 0
    bits = np.where(neg, ~keys, keys ^ np.uint64(1 << 63))
    mn, mx = bits.view(np.float64)
    nonfinite = full[3 * K + 502:4 * K + 502].copy()
    n_fin = n - nonfinite
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(n_fin > 0, a[0].astype(np.float64) / (np.maximum(n_fin, 1) * 4294967296.0), np.nan)
    return {"pop_mean": mean, "pop_sum_q32": a[0].copy(), "pop_nonfinite": nonfinite,
            "pop_min": mn.copy(), "pop_max": mx.copy(), "pop_hist": full[3 * K:3 * K + 402].view(np.uint64).copy(),
            "span_min": full[3 * K + 402:3 * K + 452].copy(), "span_max": full[3 * K + 452:3 * K + 502].copy()}


def vct_create_population(desc: vct_population_desc, params_dev, stream=None) -> C.c_void_p:
    h = C.c_void_p()
    _check("vct_create_population",
           lib().vct_create_population(C.byref(desc), _ptr(params_dev), _stream(stream), C.byref(h)))
    return h


def vct_simulate(pop, protocol: vct_protocol, ctrl: vct_controller, sim: vct_sim, stream=None) -> None:
    _check("vct_simulate", lib().vct_simulate(pop, C.byref(protocol), C.byref(ctrl), C.byref(sim), _stream(stream)))


def vct_read_metrics(metrics_dev, n_patients: int, n_samples: int, stream=None) -> vct_summary:
    out = vct_summary()
    _check("vct_read_metrics",
           lib().vct_read_metrics(_ptr(metrics_dev), n_patients, n_samples, C.byref(out), _stream(stream)))
    return out


def vct_read_metrics_noalloc(metrics_dev, n_patients: int, n_samples: int, stream=None) -> vct_summary:
    out = vct_summary()
    _check("vct_read_metrics_noalloc",
           lib().vct_read_metrics_noalloc(_ptr(metrics_dev), n_patients, n_samples, C.byref(out), _stream(stream)))
    return out


def vct_destroy_population(pop) -> None:
    if pop:
        lib().vct_destroy_population(pop)


def vct_mpc_bytes(n: int, precision: int) -> int:
    return lib().vct_mpc_bytes(n, precision)


def vct_mpc_setup(pop, ctrl: vct_controller, sim: vct_sim, mpc_dev, stream=None) -> None:
    _check("vct_mpc_setup", lib().vct_mpc_setup(pop, C.byref(ctrl), C.byref(sim), _ptr(mpc_dev), _stream(stream)))


def vct_mlp_blob_bytes() -> int:
    return lib().vct_mlp_blob_bytes()


def vct_mlp_train_bytes(batch: int) -> int:
    return lib().vct_mlp_train_bytes(batch)


def vct_mlp_init(seed: int, train_dev, blob_dev, stream=None) -> None:
    _check("vct_mlp_init", lib().vct_mlp_init(int(seed), _ptr(train_dev), _ptr(blob_dev), _stream(stream)))


def vct_mlp_normalize(rows_dev, n_rows: int, box_q: float, train_dev, blob_dev, stream=None) -> None:
    _check("vct_mlp_normalize", lib().vct_mlp_normalize(_ptr(rows_dev), int(n_rows), float(box_q),
                                                         _ptr(train_dev), _ptr(blob_dev), _stream(stream)))


def vct_mlp_train_step(rows_dev, n_rows: int, idx_dev, seed: int, step: int, batch: int, lr: float, apply: bool,
                       train_dev, blob_dev, stream=None) -> None:
    _check("vct_mlp_train_step",
           lib().vct_mlp_train_step(_ptr(rows_dev), int(n_rows), _ptr(idx_dev), int(seed), int(step), int(batch),
                                    float(lr), int(bool(apply)), _ptr(train_dev), _ptr(blob_dev), _stream(stream)))


def vct_mlp_train(rows_dev, n_rows: int, seed: int, first_step: int, n_steps: int, sched_offset: int,
                  sched_total: int, batch: int, lr: float, lr_min: float, train_dev, blob_dev, stream=None) -> None:
    _check("vct_mlp_train", lib().vct_mlp_train(_ptr(rows_dev), n_rows, seed, first_step, n_steps, sched_offset,
                                                sched_total, batch, lr, lr_min, _ptr(train_dev), _ptr(blob_dev),
                                                _stream(stream)))


def vct_mlp_forward(x_dev, n: int, blob_dev, out_dev, stream=None) -> None:
    _check("vct_mlp_forward", lib().vct_mlp_forward(_ptr(x_dev), int(n), _ptr(blob_dev), _ptr(out_dev),
                                                     _stream(stream)))


def vct_batch_create(arms, protocol: vct_protocol, ctrl: vct_controller, sim: vct_sim, block: int = 0,
                     stream=None) -> C.c_void_p:
    arr = (vct_arm * len(arms))(*arms)
    h = C.c_void_p()
    _check("vct_batch_create", lib().vct_batch_create(arr, len(arms), C.byref(protocol), C.byref(ctrl),
                                                       C.byref(sim), int(block), _stream(stream), C.byref(h)))
    return h


def vct_batch_run(batch, stream=None) -> None:
    _check("vct_batch_run", lib().vct_batch_run(batch, _stream(stream)))


def vct_batch_info(batch) -> vct_batch_stats:
    out = vct_batch_stats()
    _check("vct_batch_info", lib().vct_batch_info(batch, C.byref(out)))
    return out


def vct_batch_destroy(batch) -> None:
    if batch:
        lib().vct_batch_destroy(batch)


# ------------------------------------------------- marshalling of trial dicts
def population_desc(trial: dict) -> vct_population_desc:
    d = vct_population_desc()
    d.n_patients = int(trial["n_patients"])
    d.seed = int(trial["pop_seed"])
    d.arm_id = int(trial["arm_id"])
    d.flags = int(trial["pop_flags"])
    for i, v in enumerate(trial["nominal"]):
        d.nominal[i] = float(v)
    d.cv, d.ag, d.tau_cgm, d.g_target = (float(trial[k]) for k in ("cv", "ag", "tau_cgm", "g_target"))
    d.first_patient = int(trial.get("first_patient", 0))
    return d


def protocol(trial: dict) -> vct_protocol:
    p = vct_protocol()
    p.n_slots = int(trial["n_slots"])
    for m in range(VCT_MAX_SLOTS):
        p.minute_of_day[m] = int(trial["minute_of_day"][m])
        p.carbs_mean_g[m] = float(trial["carbs_mean"][m])
        p.carbs_sd_g[m] = float(trial["carbs_sd"][m])
        p.prob[m] = float(trial["prob"][m])
    p.jitter_min = int(trial["jitter"])
    p.kind = int(trial.get("proto", VCT_PROTO_SLOTS))
    p.meal_cv = float(trial.get("meal_cv", 0.0))
    p.exercise = int(trial.get("exercise", 0))
    p.exercise_minute = int(trial.get("exercise_minute", 960))
    p.exercise_duration = int(trial.get("exercise_duration", 45))
    p.exercise_hrr = float(trial.get("exercise_hrr", 0.5))
    return p


def controller(trial: dict, mpc_dev=None, mlp_dev=None) -> vct_controller:
    c = vct_controller()
    c.kind = int(trial["ctrl_kind"])
    for k in ("setpoint", "kp", "ki", "kd", "umax_rel", "u_rel", "mpc_rho"):
        setattr(c, k, float(trial[k]))
    c.mpc_horizon, c.mpc_iters = int(trial["mpc_horizon"]), int(trial["mpc_iters"])
    c.mpc_dev = _ptr(mpc_dev)
    c.mlp_dev = _ptr(mlp_dev)
    c.mlp_safe_g = float(trial.get("mlp_safe_g", 3.0))
    c.mlp_safe_out = float(trial.get("mlp_safe_out", 1.0))
    c.basal_scale = float(trial.get("basal_scale", 1.0))
    c.meal_bolus = int(trial.get("meal_bolus", 1))
    for k, v in (("icr_rule", 1000.0), ("glu_enter", 3.5), ("glu_exit", 5.0), ("glu_target", 5.0), ("glu_kp", 5.0),
                 ("glu_max", 10.0), ("ex_bolus", 100.0), ("ex_bolus_below", 7.0)):
        setattr(c, k, float(trial.get(k, v)))
    return c


def sim_settings(trial: dict, metrics_dev, traj_patients: int = 0, traj_dev=None, record_dev=None,
                 fallback_dev=None, popbg_dev=None, doses_dev=None) -> vct_sim:
    s = vct_sim()
    s.n_days, s.em_per_ctrl, s.ts_min = int(trial["n_days"]), int(trial["em_per_ctrl"]), int(trial["ts_min"])
    s.precision = int(trial["precision"])
    s.sigma_q1, s.cgm_var = float(trial["sigma_q1"]), float(trial["cgm_var"])
    s.noise_seed = int(trial["noise_seed"])
    s.metrics_dev = _ptr(metrics_dev)
    s.traj_patients = int(traj_patients)
    s.traj_dev = _ptr(traj_dev)
    s.record_dev = _ptr(record_dev)
    s.fallback_dev = _ptr(fallback_dev)
    s.popbg_dev = _ptr(popbg_dev)
    s.model_ext = int(trial.get("model_ext", 0))
    for k, v in (("tau_n", 20.0), ("e_n", 0.3), ("tau_e1", 5.0), ("tau_e2", 20.0), ("tau_e3", 300.0),
                 ("alpha_e", 0.015), ("beta_e", 1.0)):
        setattr(s, k, float(trial.get(k, v)))
    s.doses_dev = _ptr(doses_dev)
    return s


def arm(pop, n_days: int, kp: float, ki: float, kd: float, metrics_dev, basal_scale: float = 1.0) -> vct_arm:
    a = vct_arm()
    a.pop = pop.value if isinstance(pop, C.c_void_p) else pop
    a.n_days = int(n_days)
    a.kp, a.ki, a.kd = float(kp), float(ki), float(kd)
    a.metrics_dev = _ptr(metrics_dev)
    a.basal_scale = float(basal_scale)
    return a


def metric_views(buf, n: int) -> dict:
    """Per-patient views (torch) into a metrics buffer laid out as documented in vct.h."""
    import torch
    dt = {"f8": torch.float64, "i4": torch.int32, "u4": torch.int32}
    out = {}
    for name, kind, off, rows in METRIC_LAYOUT:
        v = buf[off * n:(off + (8 if kind == "f8" else 4) * rows) * n].view(dt[kind])
        out[name] = v.view(rows, n) if rows > 1 else v
    return out
