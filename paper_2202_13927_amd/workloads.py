"""Seeded synthetic trial descriptions (inputs only, no model arithmetic).

A trial is a flat dict of plain numbers that both the GPU library and the CPU
oracle take as input: population size and seeds, the nominal parameter vector,
the meal protocol, the controller settings and the simulation settings. The five
named workloads mirror the configurations the project is measured on; every
value the paper leaves open is a stated reading (see the model notes in the
repository's design document).

The paper's trial is (1) a population, (2) a protocol, (3) a model, (4)
parameter values and (5) one or more controllers (Sec. II). The fields below are
grouped the same way.
"""
from __future__ import annotations

import copy

# Hovorka core parameters, in the order both implementations use.
# EGP0, F01 (mmol/kg/min) and VI, VG (L/kg) are per kg of body weight.
PARAM_NAMES = ("EGP0", "F01", "k12", "ka1", "ka2", "ka3", "SIT", "SID", "SIE",
               "ke", "VI", "VG", "tmaxI", "tmaxG", "BW")
NOMINAL = (0.0161, 0.0097, 0.066, 0.006, 0.06, 0.03, 51.2e-4, 8.2e-4, 520e-4,
           0.138, 0.12, 0.16, 55.0, 40.0, 70.0)

# State order of the model (documentation for users of trajectory dumps).
STATE_NAMES = ("D1", "D2", "S1", "S2", "I", "x1", "x2", "x3", "Q1", "Q2", "GI")

CTRL_OPEN, CTRL_PID, CTRL_MPC, CTRL_MLP, CTRL_DUAL = 0, 1, 2, 3, 4
PROTO_SLOTS, PROTO_NORDIC = 0, 1
FP64, FP32 = 0, 1

MG_PER_DL_PER_MMOL = 18.0


def base_trial() -> dict:
    """1,000 patients x 7 days, three meals, PID, FP64 -- the small parity case."""
    return {
        # (1) population + (4) parameter values
        "n_patients": 1000,
        "first_patient": 0,    # global index of patient 0 (slices of a larger population)
        "pop_seed": 0,
        "arm_id": 0,
        "pop_flags": 0,
        "nominal": list(NOMINAL),
        "cv": 0.20,
        "ag": 0.8,
        "tau_cgm": 10.0,
        "g_target": 6.0,
        # (2) protocol: 07:00 / 12:00 / 18:00, N(50, 10) g clipped at 0, jitter +-30 min
        "n_slots": 3,
        "minute_of_day": [420, 720, 1080, 1260],
        "carbs_mean": [50.0, 50.0, 50.0, 20.0],
        "carbs_sd": [10.0, 10.0, 10.0, 5.0],
        "prob": [1.0, 1.0, 1.0, 0.0],
        "jitter": 30,
        # protocol kind: PROTO_SLOTS (the slots above) or PROTO_NORDIC (the paper's
        # Northern-European year, meal sizes per kg; meal_cv = relative SD of each meal)
        "proto": PROTO_SLOTS,
        "meal_cv": 0.0,
        # (5) controller: PID on CGM, gains relative to the basal rate
        "ctrl_kind": CTRL_PID,
        "setpoint": 6.0,
        "kp": 0.5,
        "ki": 0.5 / 600.0,
        "kd": 30.0,
        "umax_rel": 3.0,
        "u_rel": 1.0,
        # linear MPC: horizon 24 samples, 50 projected-gradient iterations, input weight
        "mpc_horizon": 24,
        "mpc_iters": 50,
        "mpc_rho": 1.0,
        # learned controller: the MPC takes over while the sensor reads below mlp_safe_g
        # (mmol/L, level-2 hypoglycaemia) and the network asks for more than mlp_safe_out u_b
        "mlp_safe_g": 3.0,
        "mlp_safe_out": 1.0,
        # the controller's basal rate relative to the patient's (Sec. IV-E trial B: 0.5)
        "basal_scale": 1.0,
        # dual-hormone AP (CTRL_DUAL): the PID above in insulin mode plus a meal bolus
        # (ICR = icr_rule / TDD, TDD = twice the daily basal insulin); glucagon mode below
        # glu_enter until glu_exit, microboli min(glu_max, glu_kp (glu_target - y)) ug; a
        # glucagon bolus of ex_bolus ug at an exercise onset while y < ex_bolus_below
        "meal_bolus": 1,
        "icr_rule": 1000.0,
        "glu_enter": 3.5,
        "glu_exit": 5.0,
        "glu_target": 5.0,
        "glu_kp": 5.0,
        "glu_max": 10.0,
        "ex_bolus": 100.0,
        "ex_bolus_below": 7.0,
        # (3) model extensions of Sec. IV-B, parameters shared by all patients; off by default:
        # subcutaneous glucagon (two states, time constant tau_n min, hepatic output e_n
        # mmol per ug appearing) and exercise (three states driven by the heart-rate reserve:
        # time constants tau_e1..3 min, uptake alpha_e 1/min, insulin action gain beta_e)
        "model_ext": 0,
        "tau_n": 20.0,
        "e_n": 0.3,
        "tau_e1": 5.0,
        "tau_e2": 20.0,
        "tau_e3": 300.0,
        "alpha_e": 0.015,
        "beta_e": 1.0,
        # exercise sessions on the Northern-European protocol's active days (model_ext only)
        "exercise": 0,
        "exercise_minute": 960,
        "exercise_duration": 45,
        "exercise_hrr": 0.5,
        # test inputs (model_ext only): heart-rate reserve held at every sample; open-loop glucagon
        "hrr_const": 0.0,
        "un_open": 0.0,
        # (3) model + simulation settings
        "n_days": 7,
        "em_per_ctrl": 5,
        "ts_min": 5,
        "sigma_q1": 1.0,
        "cgm_var": 2.0 / MG_PER_DL_PER_MMOL ** 2,
        "noise_seed": 0,
        "precision": FP64,
    }


def with_(trial: dict, **kw) -> dict:
    t = copy.deepcopy(trial)
    for k, v in kw.items():
        if k not in t:
            raise KeyError(k)
        t[k] = v
    return t


def noise_free(trial: dict) -> dict:
    """The ODE special case (sigma = 0) with a noise-free sensor."""
    return with_(trial, sigma_q1=0.0, cgm_var=0.0)


def c1_fp64_pid() -> dict:
    """1,000 patients x 7 days, FP64 state, seed 0."""
    return base_trial()


def c2_fp32_pid() -> dict:
    """100,000 patients x 28 days, FP32 state / FP64 accumulators, seed 1."""
    return with_(base_trial(), n_patients=100_000, n_days=28, pop_seed=1, noise_seed=1, precision=FP32)


def c3_paper_scale() -> dict:
    """1,000,000 patients x 364 days, plus a 21:00 snack with probability 0.2, N(20, 5) g."""
    return with_(base_trial(), n_patients=1_000_000, n_days=364, pop_seed=2, noise_seed=2, precision=FP32,
                 n_slots=4, prob=[1.0, 1.0, 1.0, 0.2])


def nordic_year(seed: int = 6) -> dict:
    """The paper's Northern-European protocol (Sec. II-B, Tables I-II) for 1,000,000 patients
    x 364 days (one year: four 13-week seasons), PID, FP32: each patient's own arrangement of
    the season's weeks and the week's days, BW-scaled meals with a 10 % relative SD and
    +-30 min onset jitter."""
    return with_(base_trial(), n_patients=1_000_000, n_days=364, pop_seed=seed, noise_seed=seed, precision=FP32,
                 proto=PROTO_NORDIC, meal_cv=0.1)


def dual_hormone_year(seed: int = 7) -> dict:
    """The paper's own kind of trial (Sec. IV): the Northern-European year with an exercise
    session on every active day, the model extended with subcutaneous glucagon and exercise,
    and the dual-hormone AP (insulin mode: PID microadjustments with doubled gains and a
    meal bolus; glucagon mode below 3.5 mmol/L; 100 ug at an exercise onset below 7 mmol/L),
    1,000,000 patients x 364 days, FP32."""
    return with_(nordic_year(seed), model_ext=1, exercise=1, ctrl_kind=CTRL_DUAL, kp=1.0, ki=1.0 / 600.0, kd=60.0)


def c5_mpc(seed: int = 5) -> dict:
    """Learned-controller trial, exact-MPC arm: 1,000,000 patients x 364 days, FP32, linear MPC
    (24-sample horizon, 50 projected-gradient steps), u_max = 3 u_b. The population keeps
    only parameter sets with a basal rate >= 0.4 U/h (the paper's acceptance rule), which
    removes patients whose basal need is near zero."""
    return with_(base_trial(), n_patients=1_000_000, n_days=364, pop_seed=seed, noise_seed=seed, precision=FP32,
                 pop_flags=1, ctrl_kind=CTRL_MPC)


def mlp_training_population(seed: int = 100) -> dict:
    """Separate population whose MPC closed loop produces the training pairs:
    17,500 patients x 2 days = 10.08 M (inputs, action) pairs -- as many pairs as 5,000 x 7 days
    but a wider sample of patients, which the network's patient inputs need."""
    return with_(c5_mpc(seed), n_patients=17_500, n_days=2)


GAIN_MULTIPLIERS = (0.5, 0.75, 1.0, 1.5)
HORIZON_WEEKS = (1, 4, 13, 26, 52)


def c4_arms(seed: int = 4, n_min: int = 1_000, n_max: int = 200_000) -> list[dict]:
    """64 arms: PID gains on the 4x4x4 grid of multipliers of the nominal (Kp, Ki, Kd),
    arm a = 16 i + 4 j + l; population sizes log-uniform in [n_min, n_max]; horizons
    uniform over {1, 4, 13, 26, 52} weeks. Each arm is a trial dict whose arm_id keys its
    population and noise; sizes and horizons come from numpy's seeded generator."""
    import numpy as np
    rng = np.random.default_rng(seed)
    u_size = rng.random(64)
    u_h = rng.integers(0, len(HORIZON_WEEKS), 64)
    base = with_(base_trial(), pop_seed=seed, noise_seed=seed, precision=FP32)
    arms = []
    for a in range(64):
        i, j, l = a // 16, (a // 4) % 4, a % 4
        n = int(round(np.exp(np.log(n_min) + u_size[a] * np.log(n_max / n_min))))
        arms.append(with_(base, arm_id=a, n_patients=n, n_days=7 * HORIZON_WEEKS[int(u_h[a])],
                          kp=base["kp"] * GAIN_MULTIPLIERS[i], ki=base["ki"] * GAIN_MULTIPLIERS[j],
                          kd=base["kd"] * GAIN_MULTIPLIERS[l]))
    return arms


def days_patients(trial: dict) -> int:
    return int(trial["n_patients"]) * int(trial["n_days"])


def samples_per_day(trial: dict) -> int:
    return 1440 // int(trial["ts_min"])


def c5_mlp(seed: int = 5) -> dict:
    """Learned-controller arm of the same trial (same population, meals and noise)."""
    return with_(c5_mpc(seed), ctrl_kind=CTRL_MLP)


# --------------------------------------------------------- learned-controller inputs
# Order of the 12 inputs: y_k .. y_k-5 (mmol/L), insulin on board and announced meals as the
# mean glucose change they still cause over the MPC's horizon (mmol/L), u_b (mU/min), the
# insulin response over the horizon (sum of the MPC's Markov parameters) and its mean delay
# (samples), BW (kg).
POLICY_INPUTS = ("y0", "y1", "y2", "y3", "y4", "y5", "iob", "meal", "ub", "hsum", "hdelay", "BW")


def synthetic_policy_rows(seed: int, n: int):
    """n rows [12 inputs, target] drawn from numpy's seeded generator, with the ranges of
    a closed loop (glucose 2-25 mmol/L, meals on ~20 % of rows, lognormal patients); the
    target is a smooth function of the inputs in [0, 3]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    y0 = np.clip(7.0 + 2.0 * rng.standard_normal(n), 2.0, 25.0)
    slope = 0.15 * rng.standard_normal(n)
    ys = [np.clip(y0 - slope * i, 2.0, 25.0) for i in range(6)]
    iob = 0.8 * rng.standard_normal(n)
    gob = np.where(rng.random(n) < 0.2, rng.uniform(0.0, 6.0, n), 0.0)
    ub = 10.0 * np.exp(0.3 * rng.standard_normal(n))
    hsum = -0.1 * np.exp(0.4 * rng.standard_normal(n))
    hdelay = 18.5 + 0.2 * rng.standard_normal(n)
    bw = 70.0 * np.exp(0.2 * rng.standard_normal(n))
    target = np.clip(1.0 + 0.5 * (y0 - 6.0) + 2.0 * slope + 0.5 * iob + 0.3 * gob, 0.0, 3.0)
    return np.stack(ys + [iob, gob, ub, hsum, hdelay, bw, target], axis=1)


def synthetic_policy_net(seed: int, gain: float = 1.0, spread: float = 0.05) -> dict:
    """A controller network for closed-loop tests: units 0 and 1 of every hidden layer carry
    relu(z0 - a) and relu(a - z0) for the normalised sensor value z0, so the output is
    1 + gain (z0 - a) (a proportional law around 6 mmol/L) plus a small random network on the
    other 62 units (weights from numpy's seeded generator, output weights ~ spread). The
    normalisation is fixed (sensor values around 7 +- 2 mmol/L) and the box covers glucose
    2.5-16 mmol/L, an insulin response down to -0.25 and body weights within a factor 1.5 of
    nominal."""
    import numpy as np
    rng = np.random.default_rng(seed)
    H = 64
    W1 = 0.4 * rng.standard_normal((H, 12))
    W2 = 0.17 * rng.standard_normal((H, H))
    W3 = 0.17 * rng.standard_normal((H, H))
    b1 = 0.1 * rng.standard_normal(H)
    b2 = 0.1 * rng.standard_normal(H)
    b3 = 0.1 * rng.standard_normal(H)
    w4 = spread * rng.standard_normal(H)
    mean = np.array([7.0] * 6 + [0.0, 0.5, 10.0, -0.1, 18.5, 70.0])
    istd = 1.0 / np.array([2.0] * 6 + [1.0, 1.5, 3.0, 0.05, 0.2, 14.0])
    a = (6.0 - 7.0) / 2.0
    for W, b in ((W2, b2), (W3, b3)):
        W[0:2, :] = 0.0
        W[:, 0:2] = 0.0
        W[0, 0] = W[1, 1] = 1.0
        b[0:2] = 0.0
    W1[0:2, :] = 0.0
    W1[0, 0], b1[0] = 1.0, -a
    W1[1, 0], b1[1] = -1.0, a
    w4[0], w4[1] = gain, -gain
    lo = np.array([2.5] * 6 + [-50.0, -1.0, 0.0, -0.25, 10.0, 70.0 / 1.5])
    hi = np.array([16.0] * 6 + [50.0, 1e3, 1e3, 0.0, 30.0, 70.0 * 1.5])
    # stored precision: FP32 normalisation and biases
    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
    return {"W1": W1, "b1": f32(b1), "W2": W2, "b2": f32(b2), "W3": W3, "b3": f32(b3), "w4": w4, "b4": 1.0,
            "mean": f32(mean), "istd": f32(istd), "lo": f32(lo), "hi": f32(hi)}


def constant_policy_net(value: float, always_fallback: bool = False) -> dict:
    """A network whose output is `value` for every input (zero weights, b4 = value); its box
    admits every finite input, or none (lo > hi) with always_fallback."""
    import numpy as np
    z = lambda *s: np.zeros(s)
    inf = 3.0e38
    lo, hi = (np.full(12, 1.0), np.full(12, -1.0)) if always_fallback else (np.full(12, -inf), np.full(12, inf))
    return {"W1": z(64, 12), "b1": z(64), "W2": z(64, 64), "b2": z(64), "W3": z(64, 64), "b3": z(64),
            "w4": z(64), "b4": float(value), "mean": z(12), "istd": np.ones(12), "lo": lo, "hi": hi}
