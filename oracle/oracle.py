"""ctypes front end of the FP64 CPU oracle (oracle/vct_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark. It takes a trial dict (plain numbers) and returns
numpy arrays; it never touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

NP, NX, NPOUT, MAX_SLOTS = 15, 11, 19, 4
NXE = 5   # extension states: Z1, Z2 (glucagon), E1, E2, E3 (exercise)
INT_EM, INT_RK4 = 0, 1


class OrcConfig(C.Structure):
    _fields_ = [
        ("pop_seed", C.c_uint64), ("arm_id", C.c_uint32), ("pop_flags", C.c_uint32),
        ("nominal", C.c_double * NP), ("cv", C.c_double), ("ag", C.c_double), ("tau_cgm", C.c_double),
        ("g_target", C.c_double),
        ("n_slots", C.c_int32), ("minute_of_day", C.c_int32 * MAX_SLOTS), ("carbs_mean", C.c_double * MAX_SLOTS),
        ("carbs_sd", C.c_double * MAX_SLOTS), ("prob", C.c_double * MAX_SLOTS), ("jitter", C.c_int32),
        ("proto", C.c_int32), ("meal_cv", C.c_double),
        ("ctrl_kind", C.c_int32), ("setpoint", C.c_double), ("kp", C.c_double), ("ki", C.c_double),
        ("kd", C.c_double), ("umax_rel", C.c_double), ("u_rel", C.c_double), ("basal_scale", C.c_double),
        ("n_days", C.c_int32), ("em_per_ctrl", C.c_int32), ("ts_min", C.c_int32), ("sigma_q1", C.c_double),
        ("cgm_var", C.c_double), ("noise_seed", C.c_uint64), ("integrator", C.c_int32), ("rk4_sub", C.c_int32),
        ("x0_offset", C.c_double * NX), ("guard_rel", C.c_double),
        ("mpc_horizon", C.c_int32), ("mpc_iters", C.c_int32), ("mpc_rho", C.c_double),
        ("mpc_riccati_iters", C.c_int32), ("mpc_power_iters", C.c_int32), ("mlp", C.c_void_p),
        ("mlp_safe_g", C.c_double), ("mlp_safe_out", C.c_double),
        ("model_ext", C.c_int32), ("tau_n", C.c_double), ("e_n", C.c_double), ("tau_e1", C.c_double),
        ("tau_e2", C.c_double), ("tau_e3", C.c_double), ("alpha_e", C.c_double), ("beta_e", C.c_double),
        ("exercise", C.c_int32), ("exercise_minute", C.c_int32), ("exercise_duration", C.c_int32),
        ("exercise_hrr", C.c_double), ("hrr_const", C.c_double), ("un_open", C.c_double),
        ("meal_bolus", C.c_int32), ("icr_rule", C.c_double), ("glu_enter", C.c_double), ("glu_exit", C.c_double),
        ("glu_target", C.c_double), ("glu_kp", C.c_double), ("glu_max", C.c_double), ("ex_bolus", C.c_double),
        ("ex_bolus_below", C.c_double),
    ]


MLP_IN, MLP_H = 12, 64
MLP_FIELDS = (("W1", (MLP_H, MLP_IN)), ("b1", (MLP_H,)), ("W2", (MLP_H, MLP_H)), ("b2", (MLP_H,)),
              ("W3", (MLP_H, MLP_H)), ("b3", (MLP_H,)), ("w4", (MLP_H,)), ("b4", ()), ("mean", (MLP_IN,)),
              ("istd", (MLP_IN,)), ("lo", (MLP_IN,)), ("hi", (MLP_IN,)))


class OrcMlp(C.Structure):
    _fields_ = [(name, C.c_double * int(np.prod(shape)) if shape else C.c_double) for name, shape in MLP_FIELDS]


NMAX = 48


class OrcMpc(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("A", C.c_double * (NX * NX)), ("B", C.c_double * NX), ("E", C.c_double * NX),
        ("K", C.c_double * NX), ("h", C.c_double * NMAX), ("F", C.c_double * (NMAX * NX)), ("w", C.c_double * NMAX),
        ("Gx", C.c_double * (NMAX * NX)), ("gd", C.c_double * NMAX), ("g1", C.c_double * NMAX),
        ("lam", C.c_double), ("rho_p", C.c_double), ("step", C.c_double), ("xss", C.c_double * NX),
        ("ub", C.c_double), ("umax", C.c_double), ("gstar", C.c_double), ("P", C.c_double * (NX * NX)),
        ("P_change", C.c_double),
    ]


_P = C.POINTER


class OrcOutputs(C.Structure):
    _fields_ = [
        ("bins", _P(C.c_int32)), ("events", _P(C.c_int32)), ("sum_g", _P(C.c_double)), ("min_g", _P(C.c_double)),
        ("argmin_k", _P(C.c_int32)), ("sum_u", _P(C.c_double)), ("status", _P(C.c_uint32)),
        ("n_near", _P(C.c_int32)), ("ctrl_margin", _P(C.c_double)), ("params", _P(C.c_double)),
        ("n_traj", C.c_int32), ("traj_g", _P(C.c_double)), ("traj_y", _P(C.c_double)), ("traj_u", _P(C.c_double)),
        ("traj_x", _P(C.c_double)), ("record", _P(C.c_double)), ("fallback", _P(C.c_int32)),
        ("doses", _P(C.c_double)), ("traj_xe", _P(C.c_double)),
    ]


class OrcSummary(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("k", C.c_int64), ("bins", C.c_uint64 * 5), ("events", C.c_uint64 * 3),
        ("q_count", C.c_int64 * 5), ("mean_tir", C.c_double), ("mean_bg", C.c_double),
        ("worst_patient", C.c_int64), ("worst_min_g", C.c_double), ("worst_k", C.c_int32),
        ("status_count", C.c_int64 * 3), ("n_clean", C.c_int64), ("bins_clean", C.c_uint64 * 5),
        ("q_count_clean", C.c_int64 * 5), ("mean_tir_clean", C.c_double), ("mean_bg_clean", C.c_double),
    ]


_lib = None


def lib() -> C.CDLL:
    """Load the oracle library, compiling it first only if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_philox4x32_10.argtypes = [_P(C.c_uint32), _P(C.c_uint32), _P(C.c_uint32)]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_normals4.argtypes = [_P(C.c_uint32), _P(C.c_uint32), _P(C.c_double)]
        L.orc_sample_population.argtypes = [_P(OrcConfig), C.c_int64, C.c_int64, _P(C.c_double)]
        L.orc_basal.argtypes = [_P(OrcConfig), _P(C.c_double), _P(C.c_double), _P(C.c_double), _P(C.c_double)]
        L.orc_basal.restype = C.c_int
        L.orc_rhs.argtypes = [_P(OrcConfig), _P(C.c_double), _P(C.c_double), C.c_double, C.c_double,
                              _P(C.c_double)]
        L.orc_simulate.argtypes = [_P(OrcConfig), C.c_int64, C.c_int64, C.c_int, _P(OrcOutputs)]
        L.orc_simulate.restype = C.c_int
        L.orc_rhs_ext.argtypes = [_P(OrcConfig), _P(C.c_double), _P(C.c_double), _P(C.c_double), C.c_double,
                                  C.c_double, C.c_double, C.c_double, _P(C.c_double), _P(C.c_double)]
        L.orc_day_exercise.argtypes = [_P(OrcConfig), C.c_uint32, C.c_int32]
        L.orc_day_exercise.restype = C.c_int32
        L.orc_dual_run.argtypes = [_P(OrcConfig), C.c_double, C.c_double, C.c_double, C.c_int32, _P(C.c_double),
                                   _P(C.c_double),
                                   _P(C.c_int32), _P(C.c_double), _P(C.c_double), _P(C.c_double), _P(C.c_int32)]
        L.orc_em_ou.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int64,
                                C.c_uint64, _P(C.c_double)]
        L.orc_reduce.argtypes = [C.c_int64, C.c_int64, _P(C.c_int32), _P(C.c_int32), _P(C.c_double),
                                 _P(C.c_double), _P(C.c_int32), _P(C.c_uint32), _P(OrcSummary)]
        L.orc_meals.argtypes = [_P(OrcConfig), C.c_uint32, C.c_int32, _P(C.c_double)]
        L.orc_nordic_day.argtypes = [_P(OrcConfig), C.c_uint32, C.c_int32, _P(C.c_int32)]
        L.orc_day_meals.argtypes = [_P(OrcConfig), C.c_uint32, C.c_int32, _P(C.c_double)]
        L.orc_day_meals.restype = C.c_int
        L.orc_jacobian.argtypes = [_P(OrcConfig), _P(C.c_double), _P(C.c_double), _P(C.c_double), _P(C.c_double),
                                   _P(C.c_double)]
        L.orc_mpc_setup.argtypes = [_P(OrcConfig), _P(C.c_double), _P(OrcMpc)]
        L.orc_mpc_setup.restype = C.c_int
        L.orc_mpc_pg.argtypes = [_P(OrcMpc), _P(C.c_double), _P(C.c_double), C.c_int]
        L.orc_pid_run.argtypes = [_P(OrcConfig), C.c_double, C.c_int32, _P(C.c_double), _P(C.c_double),
                                  _P(C.c_double)]
        L.orc_bf16.argtypes = [C.c_double]
        L.orc_bf16.restype = C.c_double
        L.orc_mlp_forward.argtypes = [_P(OrcMlp), _P(C.c_double), C.c_int64, _P(C.c_double)]
        L.orc_mlp_loss_grad.argtypes = [_P(OrcMlp), _P(C.c_double), _P(C.c_int64), C.c_int64, _P(OrcMlp)]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_mlp_init.argtypes = [C.c_uint64, _P(OrcMlp)]
        L.orc_mlp_batch_rows.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int64, _P(C.c_int64)]
        L.orc_mlp_stats.argtypes = [_P(C.c_double), C.c_int64, C.c_double, _P(OrcMlp)]
        L.orc_adam.argtypes = [C.c_int64, _P(C.c_double), _P(C.c_double), _P(C.c_double), _P(C.c_double),
                               C.c_double, C.c_int64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None, ctype):
    if a is None:
        return C.cast(None, _P(ctype))
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_P(ctype))


def config(trial: dict, integrator: int = INT_EM, rk4_sub: int = 64, x0_offset=None,
           guard_rel: float = 1e-4) -> OrcConfig:
    c = OrcConfig()
    c.pop_seed = int(trial["pop_seed"])
    c.arm_id = int(trial["arm_id"])
    c.pop_flags = int(trial["pop_flags"])
    for i, v in enumerate(trial["nominal"]):
        c.nominal[i] = float(v)
    c.cv, c.ag, c.tau_cgm, c.g_target = (float(trial[k]) for k in ("cv", "ag", "tau_cgm", "g_target"))
    c.n_slots = int(trial["n_slots"])
    for m in range(MAX_SLOTS):
        c.minute_of_day[m] = int(trial["minute_of_day"][m])
        c.carbs_mean[m] = float(trial["carbs_mean"][m])
        c.carbs_sd[m] = float(trial["carbs_sd"][m])
        c.prob[m] = float(trial["prob"][m])
    c.jitter = int(trial["jitter"])
    c.proto = int(trial.get("proto", 0))
    c.basal_scale = float(trial.get("basal_scale", 1.0))
    c.meal_cv = float(trial.get("meal_cv", 0.0))
    c.ctrl_kind = int(trial["ctrl_kind"])
    for k in ("setpoint", "kp", "ki", "kd", "umax_rel", "u_rel", "sigma_q1", "cgm_var"):
        setattr(c, k, float(trial[k]))
    c.n_days, c.em_per_ctrl, c.ts_min = int(trial["n_days"]), int(trial["em_per_ctrl"]), int(trial["ts_min"])
    c.noise_seed = int(trial["noise_seed"])
    c.integrator = int(integrator)
    c.rk4_sub = int(rk4_sub)
    if x0_offset is not None:
        for i, v in enumerate(x0_offset):
            c.x0_offset[i] = float(v)
    c.guard_rel = float(guard_rel)
    c.mpc_horizon = int(trial.get("mpc_horizon", 24))
    c.mpc_iters = int(trial.get("mpc_iters", 50))
    c.mpc_rho = float(trial.get("mpc_rho", 1.0))
    c.mpc_riccati_iters = int(trial.get("mpc_riccati_iters", 500))
    c.mpc_power_iters = int(trial.get("mpc_power_iters", 100))
    c.mlp_safe_g = float(trial.get("mlp_safe_g", 3.0))
    c.mlp_safe_out = float(trial.get("mlp_safe_out", 1.0))
    for k in ("model_ext", "exercise", "exercise_minute", "exercise_duration", "meal_bolus"):
        setattr(c, k, int(trial.get(k, 0)))
    for k in ("tau_n", "e_n", "tau_e1", "tau_e2", "tau_e3", "alpha_e", "beta_e", "exercise_hrr", "hrr_const",
              "un_open", "icr_rule", "glu_enter", "glu_exit", "glu_target", "glu_kp", "glu_max", "ex_bolus",
              "ex_bolus_below"):
        setattr(c, k, float(trial.get(k, 0.0)))
    return c


# ---------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def uniform(x: int) -> float:
    return lib().orc_uniform(int(x) & 0xFFFFFFFF)


def normals4(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_double * 4)()
    lib().orc_normals4(c, k, o)
    return np.array(list(o))


def sample_population(trial: dict, first: int | None = None, count: int | None = None) -> np.ndarray:
    if first is None:
        first = int(trial.get("first_patient", 0))
        n = int(trial["n_patients"]) if count is None else int(count)
    else:
        n = int(trial["n_patients"]) - first if count is None else int(count)
    out = np.zeros((n, NPOUT))
    cfg = config(trial)
    lib().orc_sample_population(C.byref(cfg), first, n, _ptr(out, C.c_double))
    return out


def basal(trial: dict, p) -> tuple[bool, float, float, np.ndarray]:
    cfg = config(trial)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    i_star, u_b = C.c_double(), C.c_double()
    x0 = np.zeros(NX)
    ok = lib().orc_basal(C.byref(cfg), _ptr(pa, C.c_double), C.byref(i_star), C.byref(u_b), _ptr(x0, C.c_double))
    return bool(ok), i_star.value, u_b.value, x0


def rhs(trial: dict, p, x, u: float, d: float) -> np.ndarray:
    cfg = config(trial)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64)
    dx = np.zeros(NX)
    lib().orc_rhs(C.byref(cfg), _ptr(pa, C.c_double), _ptr(xa, C.c_double), float(u), float(d),
                  _ptr(dx, C.c_double))
    return dx


def rhs_ext(trial: dict, p, x, xe, u: float, un: float, d: float, hrr: float) -> tuple[np.ndarray, np.ndarray]:
    cfg = config(trial)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64)
    xea = np.ascontiguousarray(xe, dtype=np.float64)
    dx, dxe = np.zeros(NX), np.zeros(NXE)
    lib().orc_rhs_ext(C.byref(cfg), _ptr(pa, C.c_double), _ptr(xa, C.c_double), _ptr(xea, C.c_double), float(u),
                      float(un), float(d), float(hrr), _ptr(dx, C.c_double), _ptr(dxe, C.c_double))
    return dx, dxe


def day_exercise(trial: dict, patient: int, day: int) -> int:
    """Sample index within the day of the patient's exercise onset, -1 if none."""
    return int(lib().orc_day_exercise(C.byref(config(trial)), int(patient), int(day)))


def dual_run(trial: dict, ub: float, y, d, ex, iob: float = 0.0, gob: float = 0.0) -> dict:
    """Scripted dual-hormone AP: basal and bolus insulin (mU/min), glucagon (ug/min), mode;
    insulin and glucagon on board held at iob (mU above basal) and gob (ug)."""
    ya = np.ascontiguousarray(y, dtype=np.float64)
    da = np.ascontiguousarray(d, dtype=np.float64)
    ea = np.ascontiguousarray(ex, dtype=np.int32)
    n = len(ya)
    out = {"u_basal": np.zeros(n), "u_bolus": np.zeros(n), "un": np.zeros(n), "mode": np.zeros(n, np.int32)}
    lib().orc_dual_run(C.byref(config(trial)), float(ub), float(iob), float(gob), n, _ptr(ya, C.c_double),
                       _ptr(da, C.c_double),
                       _ptr(ea, C.c_int32), _ptr(out["u_basal"], C.c_double), _ptr(out["u_bolus"], C.c_double),
                       _ptr(out["un"], C.c_double), _ptr(out["mode"], C.c_int32))
    return out


def em_ou(theta: float, s: float, x0: float, h: float, n_steps: int, n_paths: int, seed: int) -> np.ndarray:
    out = np.zeros(n_paths)
    lib().orc_em_ou(theta, s, x0, h, n_steps, n_paths, seed, _ptr(out, C.c_double))
    return out


def meals(trial: dict, patient: int, day: int) -> np.ndarray:
    out = np.zeros((int(trial["n_slots"]), 4))
    cfg = config(trial)
    lib().orc_meals(C.byref(cfg), int(patient), int(day), _ptr(out, C.c_double))
    return out


def nordic_day(trial: dict, patient: int, day: int) -> tuple[int, int, int]:
    """(season, week type, day type) of a patient's day under the Northern-European protocol."""
    out = np.zeros(3, dtype=np.int32)
    cfg = config(trial)
    lib().orc_nordic_day(C.byref(cfg), int(patient), int(day), _ptr(out, C.c_int32))
    return int(out[0]), int(out[1]), int(out[2])


def day_meals(trial: dict, patient: int, day: int) -> np.ndarray:
    """The day's meals in time order: rows (sample index within the day, carbs g, mmol/min)."""
    out = np.zeros((8, 3))
    cfg = config(trial)
    n = lib().orc_day_meals(C.byref(cfg), int(patient), int(day), _ptr(out, C.c_double))
    return out[:n].copy()


def pid_run(trial: dict, u_b: float, y) -> tuple[np.ndarray, np.ndarray]:
    ya = np.ascontiguousarray(y, dtype=np.float64)
    u = np.zeros_like(ya)
    integ = np.zeros_like(ya)
    cfg = config(trial)
    lib().orc_pid_run(C.byref(cfg), float(u_b), len(ya), _ptr(ya, C.c_double), _ptr(u, C.c_double),
                      _ptr(integ, C.c_double))
    return u, integ


def jacobian(trial: dict, p, x):
    cfg = config(trial)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64)
    J, Bc, Ec = np.zeros(NX * NX), np.zeros(NX), np.zeros(NX)
    lib().orc_jacobian(C.byref(cfg), _ptr(pa, C.c_double), _ptr(xa, C.c_double), _ptr(J, C.c_double),
                       _ptr(Bc, C.c_double), _ptr(Ec, C.c_double))
    return J.reshape(NX, NX), Bc, Ec


def mpc_setup(trial: dict, prm) -> dict:
    """Per-patient MPC matrices from a sampled parameter row (length NPOUT)."""
    cfg = config(trial)
    pa = np.ascontiguousarray(prm, dtype=np.float64)
    m = OrcMpc()
    if not lib().orc_mpc_setup(C.byref(cfg), _ptr(pa, C.c_double), C.byref(m)):
        raise ValueError("no basal state")
    N = m.N
    return {
        "m": m, "N": N, "A": np.array(m.A).reshape(NX, NX), "B": np.array(m.B), "E": np.array(m.E),
        "K": np.array(m.K), "h": np.array(m.h[:N]), "F": np.array(m.F).reshape(NMAX, NX)[:N],
        "w": np.array(m.w[:N]), "Gx": np.array(m.Gx).reshape(NMAX, NX)[:N], "gd": np.array(m.gd[:N]),
        "g1": np.array(m.g1[:N]), "lam": m.lam, "rho_p": m.rho_p, "step": m.step, "xss": np.array(m.xss),
        "ub": m.ub, "umax": m.umax, "P": np.array(m.P).reshape(NX, NX), "P_change": m.P_change,
    }


def mpc_pg(setup: dict, g, dU0, iters: int) -> np.ndarray:
    ga = np.ascontiguousarray(g, dtype=np.float64)
    du = np.ascontiguousarray(dU0, dtype=np.float64).copy()
    lib().orc_mpc_pg(C.byref(setup["m"]), _ptr(ga, C.c_double), _ptr(du, C.c_double), int(iters))
    return du


# --------------------------------------------------------- learned controller
def bf16(x) -> np.ndarray:
    """Nearest BF16 value of each element (ties to even)."""
    a = np.asarray(x, dtype=np.float64)
    f = lib().orc_bf16
    return np.vectorize(f, otypes=[np.float64])(a) if a.size else a.copy()


def mlp_struct(net: dict) -> OrcMlp:
    m = OrcMlp()
    for name, shape in MLP_FIELDS:
        v = np.asarray(net[name], dtype=np.float64)
        assert v.shape == shape, (name, v.shape, shape)
        if shape:
            getattr(m, name)[:] = [float(t) for t in v.ravel()]
        else:
            setattr(m, name, float(v))
    return m


def mlp_dict(m: OrcMlp) -> dict:
    out = {}
    for name, shape in MLP_FIELDS:
        out[name] = np.array(getattr(m, name)).reshape(shape) if shape else float(getattr(m, name))
    return out


def mlp_forward(net: dict, x) -> np.ndarray:
    xa = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_IN)
    out = np.zeros(xa.shape[0])
    m = mlp_struct(net)
    lib().orc_mlp_forward(C.byref(m), _ptr(xa, C.c_double), xa.shape[0], _ptr(out, C.c_double))
    return out


def mlp_loss_grad(net: dict, rows, idx) -> tuple[float, dict]:
    ra = np.ascontiguousarray(rows, dtype=np.float64).reshape(-1, MLP_IN + 1)
    ia = np.ascontiguousarray(idx, dtype=np.int64)
    m, g = mlp_struct(net), OrcMlp()
    loss = lib().orc_mlp_loss_grad(C.byref(m), _ptr(ra, C.c_double), _ptr(ia, C.c_int64), len(ia), C.byref(g))
    return loss, mlp_dict(g)


def mlp_init(seed: int) -> dict:
    m = OrcMlp()
    lib().orc_mlp_init(int(seed), C.byref(m))
    return mlp_dict(m)


def mlp_batch_rows(seed: int, step: int, B: int, n_rows: int) -> np.ndarray:
    idx = np.zeros(int(B), np.int64)
    lib().orc_mlp_batch_rows(int(seed), int(step), int(B), int(n_rows), _ptr(idx, C.c_int64))
    return idx


def mlp_stats(rows, box_q: float) -> dict:
    ra = np.ascontiguousarray(rows, dtype=np.float64).reshape(-1, MLP_IN + 1)
    m = OrcMlp()
    lib().orc_mlp_stats(_ptr(ra, C.c_double), ra.shape[0], float(box_q), C.byref(m))
    d = mlp_dict(m)
    return {k: d[k] for k in ("mean", "istd", "lo", "hi")}


def adam(w, m, v, g, lr: float, t: int):
    """One Adam step on copies; returns (w, m, v)."""
    w, m, v = (np.ascontiguousarray(a, dtype=np.float64).copy() for a in (w, m, v))
    ga = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_adam(w.size, _ptr(w, C.c_double), _ptr(m, C.c_double), _ptr(v, C.c_double), _ptr(ga, C.c_double),
                   float(lr), int(t))
    return w, m, v


# ------------------------------------------------------------------ simulate
def simulate(trial: dict, first: int | None = None, count: int | None = None, threads: int | None = None,
             n_traj: int = 0, record_x: bool = False, integrator: int = INT_EM, rk4_sub: int = 64,
             x0_offset=None, guard_rel: float = 1e-4, mlp: dict | None = None, record: bool = False) -> dict:
    """Run patients [first, first+count) of the trial (default: the trial's own slice);
    returns per-patient arrays."""
    if first is None:
        first = int(trial.get("first_patient", 0))
        n = int(trial["n_patients"]) if count is None else int(count)
    else:
        n = int(trial["n_patients"]) - first if count is None else int(count)
    K = int(trial["n_days"]) * (1440 // int(trial["ts_min"]))
    nt = min(int(n_traj), n)
    r = {
        "bins": np.zeros((n, 5), np.int32), "events": np.zeros((n, 3), np.int32),
        "sum_g": np.zeros(n), "min_g": np.zeros(n), "argmin_k": np.zeros(n, np.int32), "sum_u": np.zeros(n),
        "status": np.zeros(n, np.uint32), "n_near": np.zeros(n, np.int32), "ctrl_margin": np.zeros(n),
        "params": np.zeros((n, NPOUT)),
    }
    if nt:
        r["traj_g"] = np.zeros((nt, K))
        r["traj_y"] = np.zeros((nt, K))
        r["traj_u"] = np.zeros((nt, K))
        if record_x:
            r["traj_x"] = np.zeros((nt, K, NX))
            if int(trial.get("model_ext", 0)):
                r["traj_xe"] = np.zeros((nt, K, NXE))
    o = OrcOutputs()
    o.bins, o.events = _ptr(r["bins"], C.c_int32), _ptr(r["events"], C.c_int32)
    o.sum_g, o.min_g = _ptr(r["sum_g"], C.c_double), _ptr(r["min_g"], C.c_double)
    o.argmin_k, o.sum_u = _ptr(r["argmin_k"], C.c_int32), _ptr(r["sum_u"], C.c_double)
    o.status, o.n_near = _ptr(r["status"], C.c_uint32), _ptr(r["n_near"], C.c_int32)
    o.ctrl_margin, o.params = _ptr(r["ctrl_margin"], C.c_double), _ptr(r["params"], C.c_double)
    o.n_traj = nt
    o.traj_g = _ptr(r.get("traj_g"), C.c_double)
    o.traj_y = _ptr(r.get("traj_y"), C.c_double)
    o.traj_u = _ptr(r.get("traj_u"), C.c_double)
    o.traj_x = _ptr(r.get("traj_x"), C.c_double)
    o.traj_xe = _ptr(r.get("traj_xe"), C.c_double)
    r["doses"] = np.zeros((n, 3))
    o.doses = _ptr(r["doses"], C.c_double)
    if record:
        r["record"] = np.zeros((K, n, MLP_IN + 1))
    r["fallback"] = np.zeros(n, np.int32)
    o.record = _ptr(r.get("record"), C.c_double)
    o.fallback = _ptr(r["fallback"], C.c_int32)
    cfg = config(trial, integrator=integrator, rk4_sub=rk4_sub, x0_offset=x0_offset, guard_rel=guard_rel)
    net = mlp_struct(mlp) if mlp is not None else None
    cfg.mlp = C.cast(C.pointer(net), C.c_void_p) if net is not None else None
    if threads is None:
        threads = os.cpu_count() or 1
    rc = lib().orc_simulate(C.byref(cfg), first, n, int(threads), C.byref(o))
    if rc != 0:
        raise ValueError("oracle rejected the trial description")
    r["K"] = K
    r["threads"] = int(threads)
    return r


def reduce(r: dict) -> dict:
    n = r["bins"].shape[0]
    s = OrcSummary()
    lib().orc_reduce(n, int(r["K"]), _ptr(r["bins"], C.c_int32), _ptr(r["events"], C.c_int32),
                     _ptr(r["sum_g"], C.c_double), _ptr(r["min_g"], C.c_double), _ptr(r["argmin_k"], C.c_int32),
                     _ptr(r["status"], C.c_uint32), C.byref(s))
    return {
        "n": s.n, "k": s.k, "bins": list(s.bins), "events": list(s.events), "q_count": list(s.q_count),
        "mean_tir": s.mean_tir, "mean_bg": s.mean_bg, "worst_patient": s.worst_patient,
        "worst_min_g": s.worst_min_g, "worst_k": s.worst_k, "status_count": list(s.status_count),
        "n_clean": s.n_clean, "bins_clean": list(s.bins_clean), "q_count_clean": list(s.q_count_clean),
        "mean_tir_clean": s.mean_tir_clean, "mean_bg_clean": s.mean_bg_clean,
    }
