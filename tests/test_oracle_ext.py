"""Pins of the oracle's model extensions and dual-hormone AP (Sec. II-B exercise on active
days, Sec. IV-B glucagon and exercise sub-models, Sec. IV-C dual-hormone AP).

* with no glucagon and no exercise the extended model is the core model, bit for bit;
* the glucagon depot (two states) and the exercise states (three states) are linear chains:
  held over each sample interval, their exact sample-to-sample map is expm of the
  augmented matrix (scipy), also with the protocol's sessions switching the input on and off;
* constant glucagon infusion and constant exercise drive G to the closed-form equilibrium
  (the core's regimes with the extra hepatic output and the exercise uptake and action);
* the sessions fall exactly on the active days of Table I's arrangements (76 a year), at the
  stated onset with a uniform integer jitter;
* the AP's law on scripted sensor sequences: modes with hysteresis, the meal bolus from the
  ICR rule less insulin on board, microboli less glucagon on board, the exercise bolus, the
  PID running on every sample but delivered only in insulin mode;
* in a closed-loop trial every delivered dose equals the AP's law applied to the recorded
  sensor values and depots (insulin per sample; basal, bolus and glucagon totals).
"""
import numpy as np
import pytest
from scipy.linalg import expm

from paper_2202_13927_amd import workloads as W

IDX = {n: i for i, n in enumerate(W.PARAM_NAMES)}
SX = {n: i for i, n in enumerate(W.STATE_NAMES)}
Z1, Z2, E1, E2, E3 = range(5)


def quiet_ext(**kw):
    return W.noise_free(W.with_(W.base_trial(), n_slots=0, model_ext=1, **kw))


def test_extension_without_inputs_is_the_core_model(orc):
    t = W.with_(W.base_trial(), n_patients=40, n_days=3)
    a = orc.simulate(t, n_traj=4, record_x=True, threads=4)
    b = orc.simulate(W.with_(t, model_ext=1), n_traj=4, record_x=True, threads=4)
    for k in ("bins", "events", "sum_g", "min_g", "sum_u", "status", "traj_x", "traj_u"):
        assert np.array_equal(a[k], b[k]), k
    assert np.all(b["traj_xe"] == 0.0)
    assert np.array_equal(b["doses"][:, 0], b["sum_u"]) and np.all(b["doses"][:, 1:] == 0.0)


def _chain_expm(A, u, ts):
    """Exact map over one interval of x' = A x + b u (b the input column of A's last column)."""
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A[:, :n]
    M[:n, n] = A[:, n]
    return expm(M * ts)


def test_glucagon_depot_matches_matrix_exponential(orc):
    tau = 20.0
    t = quiet_ext(n_patients=2, n_days=1, ctrl_kind=W.CTRL_OPEN, u_rel=1.0, un_open=0.37, tau_n=tau)
    r = orc.simulate(t, n_traj=2, record_x=True, integrator=1, rk4_sub=64, threads=2)
    A = np.array([[-1 / tau, 0.0, 1.0], [1 / tau, -1 / tau, 0.0]])
    Phi = _chain_expm(A, None, t["ts_min"])
    for j in range(2):
        X = r["traj_xe"][j][:, [Z1, Z2]]
        for k in range(X.shape[0] - 1):
            pred = (Phi @ np.concatenate([X[k], [0.37]]))[:2]
            assert np.allclose(pred, X[k + 1], rtol=1e-9, atol=1e-12), k
        # the depot fills towards tau un in each state
        assert X[-1, 0] == pytest.approx(tau * 0.37, rel=1e-3) and X[-1, 1] == pytest.approx(tau * 0.37, rel=2e-2)


def test_exercise_states_match_matrix_exponential_with_sessions(orc):
    """Northern-European protocol with sessions, open loop: the input is the session's HRR on
    the documented samples of active days and 0 elsewhere; E1..E3 follow the exact map."""
    t = W.noise_free(W.with_(W.base_trial(), n_patients=3, n_days=28, proto=W.PROTO_NORDIC, meal_cv=0.1,
                             model_ext=1, exercise=1, ctrl_kind=W.CTRL_OPEN, u_rel=1.0))
    r = orc.simulate(t, n_traj=3, record_x=True, integrator=1, rk4_sub=64, threads=3)
    t1, t2, t3 = t["tau_e1"], t["tau_e2"], t["tau_e3"]
    A = np.array([[-1 / t1, 0, 0, 1 / t1], [1 / t2, -1 / t2, 0, 0], [1 / t3, 0, -1 / t3, 0]])
    Phi = _chain_expm(A, None, t["ts_min"])
    n_ex = -(-t["exercise_duration"] // t["ts_min"])
    sessions = 0
    for j in range(3):
        hrr = np.zeros(r["K"])
        for day in range(t["n_days"]):
            k0 = orc.day_exercise(t, j, day)
            if k0 >= 0:
                sessions += 1
                hrr[day * 288 + k0: day * 288 + k0 + n_ex] = t["exercise_hrr"]
        X = r["traj_xe"][j][:, [E1, E2, E3]]
        for k in range(X.shape[0] - 1):
            pred = (Phi @ np.concatenate([X[k], [hrr[k]]]))[:3]
            assert np.allclose(pred, X[k + 1], rtol=1e-9, atol=1e-12), (j, k)
    assert sessions > 0


def _g_equilibrium_ext(row, t, u, un, hrr):
    """Closed-form steady glucose for constant insulin u, glucagon un and exercise hrr (D = 0):
    the core balance with EGP raised by e_n un, x1, x2 scaled by 1 + beta_e hrr and the extra
    uptake alpha_e hrr Q1."""
    bw = row[IDX["BW"]]
    egp0, f01, vg, vi = row[IDX["EGP0"]] * bw, row[IDX["F01"]] * bw, row[IDX["VG"]] * bw, row[IDX["VI"]] * bw
    I = u / (row[IDX["ke"]] * vi)
    gain = 1.0 + t["beta_e"] * hrr
    x1, x2, x3 = row[IDX["SIT"]] * I * gain, row[IDX["SID"]] * I * gain, row[IDX["SIE"]] * I
    E = egp0 * max(0.0, 1.0 - x3) + t["e_n"] * un
    c = (x1 * x2 / (row[IDX["k12"]] + x2) + t["alpha_e"] * hrr) * vg
    for g in (E / (f01 / 4.5 + c), (E - f01) / c, (E - f01 + 0.027 * vg) / (0.003 * vg + c)):
        lo, hi = (0, 4.5) if g < 4.5 else ((4.5, 9.0) if g <= 9 else (9.0, np.inf))
        if lo <= g <= hi and abs(E - f01 * min(1, g / 4.5) - 0.003 * max(0, g - 9) * vg - c * g) < 1e-9:
            return g
    raise AssertionError("no consistent regime")


@pytest.mark.parametrize("un,hrr", [(0.3, 0.0), (1.5, 0.0), (0.0, 0.3), (0.0, 0.8), (0.6, 0.5)])
def test_equilibrium_under_glucagon_and_exercise(orc, un, hrr):
    t = quiet_ext(n_patients=5, n_days=40, ctrl_kind=W.CTRL_OPEN, u_rel=1.0, un_open=un, hrr_const=hrr)
    r = orc.simulate(t, n_traj=5, integrator=1, rk4_sub=5, threads=5)
    moved = 0
    for j in range(5):
        row = r["params"][j]
        g_eq = _g_equilibrium_ext(row, t, row[15], un, hrr)
        assert r["traj_g"][j, -1] == pytest.approx(g_eq, rel=1e-6)
        moved += abs(g_eq - 6.0) > 0.05
    assert moved == 5                   # every patient leaves the basal level
    if hrr == 0.0:
        assert np.all(r["traj_g"][:, -1] > 6.0)   # glucagon raises glucose
    if un == 0.0:
        assert np.all(r["traj_g"][:, -1] < 6.0)   # exercise lowers it


def test_exercise_sessions_fall_on_active_days(orc):
    t = W.with_(W.base_trial(), n_days=364, proto=W.PROTO_NORDIC, model_ext=1, exercise=1)
    onsets = []
    for j in range(40):
        n_active = 0
        for day in range(364):
            season, wtype, dtype = orc.nordic_day(t, j, day)
            k0 = orc.day_exercise(t, j, day)
            if dtype == 1:
                n_active += 1
                assert k0 >= 0
                onsets.append(k0)
            else:
                assert k0 == -1
        # Table I: winter 6 standard + 4 active weeks, spring 6 + 6, summer 7 + 3, autumn 9 + 3;
        # a standard week has 1 active day, an active week 3, a vacation week none
        assert n_active == (6 + 12) + (6 + 18) + (7 + 9) + (9 + 9) == 76
    onsets = np.array(onsets)
    # onset floor((960 + jitter) / 5) with jitter uniform on the integers [-30, 30]: minutes
    # 930..989 give samples 186..197 (5 minutes each), minute 990 sample 198
    assert onsets.min() == 186 and onsets.max() == 198
    counts = np.bincount(onsets - 186, minlength=13)
    expected = np.array([5] * 12 + [1]) / 61 * len(onsets)
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 35.0                   # 12 degrees of freedom, p ~ 5e-4
    off = W.with_(t, exercise=0)
    assert all(orc.day_exercise(off, 0, d) == -1 for d in range(28))
    slots = W.with_(t, proto=W.PROTO_SLOTS)
    assert all(orc.day_exercise(slots, 0, d) == -1 for d in range(28))


def _dual(**kw):
    return W.with_(W.base_trial(), model_ext=1, ctrl_kind=W.CTRL_DUAL, **kw)


def test_dual_ap_modes_and_doses_scripted(orc):
    t = _dual()
    ub, ts = 12.0, t["ts_min"]
    y = np.array([6.0, 6.0, 5.0, 4.0, 3.6, 3.4, 3.2, 3.9, 4.6, 4.99, 5.0, 5.5, 6.0, 6.5, 7.5])
    d = np.zeros_like(y)
    ex = np.zeros(len(y), np.int32)
    d[1] = 0.8                       # an announced meal in insulin mode
    d[6] = 0.5                       # and one in glucagon mode: no bolus
    ex[2], ex[6], ex[14] = 1, 1, 1   # exercise onsets at y = 5.0 (< 7), 3.2 (< 7), 7.5 (>= 7)
    r = orc.dual_run(t, ub, y, d, ex)
    mode = (np.arange(len(y)) >= 5) & (np.arange(len(y)) <= 9)        # y < 3.5 at k = 5 until y >= 5 at k = 10
    assert np.array_equal(r["mode"].astype(bool), mode)
    assert np.all(r["u_basal"][mode] == 0) and np.all(r["u_bolus"][mode] == 0)
    # the PID runs on every sample: its outputs on the insulin-mode samples are delivered
    pid = orc.pid_run(t, ub, y)[0]
    assert np.array_equal(r["u_basal"][~mode], pid[~mode])
    # meal bolus: carbs / ICR with ICR = icr_rule / TDD, TDD = 2 x daily basal insulin (U)
    carbs = 0.8 * ts * 180.16 / 1000.0
    tdd = 2.0 * ub * 1440.0 / 1000.0
    assert r["u_bolus"][1] == pytest.approx(carbs * tdd / t["icr_rule"] * 1000.0 / ts, rel=1e-14)
    assert np.count_nonzero(r["u_bolus"]) == 1
    # glucagon: microboli in glucagon mode, the exercise bolus below 7 mmol/L in either mode
    micro = np.where(mode, np.clip(t["glu_kp"] * (t["glu_target"] - y), 0, t["glu_max"]), 0.0)
    bolus = np.where((ex == 1) & (y < t["ex_bolus_below"]), t["ex_bolus"], 0.0)
    assert np.allclose(r["un"] * ts, micro + bolus, rtol=1e-14, atol=0)
    assert r["un"][14] == 0.0 and r["un"][2] * ts == t["ex_bolus"]


def test_dual_ap_on_board_reduces_doses(orc):
    t = _dual()
    ub, ts = 12.0, t["ts_min"]
    y = np.array([6.0, 6.0, 3.0, 3.0])
    d = np.array([0.0, 0.8, 0.0, 0.0])
    ex = np.zeros(4, np.int32)
    full = orc.dual_run(t, ub, y, d, ex)
    tdd = 2.0 * ub * 1440.0 / 1000.0
    bolus_mu = 0.8 * ts * 180.16 / 1000.0 * tdd / t["icr_rule"] * 1000.0
    part = orc.dual_run(t, ub, y, d, ex, iob=0.25 * bolus_mu, gob=4.0)
    assert part["u_bolus"][1] * ts == pytest.approx(0.75 * bolus_mu, rel=1e-12)
    micro = min(t["glu_max"], t["glu_kp"] * (t["glu_target"] - 3.0))
    assert full["un"][2] * ts == pytest.approx(micro, rel=1e-14)
    assert part["un"][2] * ts == pytest.approx(max(0.0, micro - 4.0), rel=1e-14)
    none = orc.dual_run(t, ub, y, d, ex, iob=2 * bolus_mu, gob=100.0)
    assert none["u_bolus"][1] == 0.0 and none["un"][2] == 0.0


def test_dual_closed_loop_doses_follow_the_law(orc):
    """Recompute every dose of a noisy dual-hormone trial from its recorded sensor values and
    depots: insulin per sample and the basal, bolus and glucagon totals."""
    t = W.with_(W.dual_hormone_year(), n_patients=24, n_days=14, precision=W.FP64)
    r = orc.simulate(t, n_traj=24, record_x=True, threads=8)
    ts, K = t["ts_min"], r["K"]
    n_ex = -(-t["exercise_duration"] // ts)
    checked_glu = 0
    for j in range(24):
        row = r["params"][j]
        ub = row[15]
        y, u = r["traj_y"][j], r["traj_u"][j]
        X, XE = r["traj_x"][j], r["traj_xe"][j]
        d = np.zeros(K)
        ex = np.zeros(K, np.int32)
        for day in range(t["n_days"]):
            for kd, _, rate in orc.day_meals(t, j, day):
                d[day * 288 + int(kd)] += rate
            k0 = orc.day_exercise(t, j, day)
            if k0 >= 0:
                ex[day * 288 + k0] = 1
                assert n_ex == 9
        # replay the AP sample by sample with the recorded on-board amounts
        iob = X[:, SX["S1"]] + X[:, SX["S2"]] - 2.0 * ub * row[IDX["tmaxI"]]
        gob = XE[:, Z1] + XE[:, Z2]
        ub_sum = bo_sum = gl_sum = 0.0
        glu = False
        pid = orc.pid_run(t, ub, y)[0]
        for k in range(K):
            if not glu and y[k] < t["glu_enter"]:
                glu = True
            elif glu and y[k] >= t["glu_exit"]:
                glu = False
            carbs = d[k] * ts * 180.16 / 1000.0
            tdd = 2.0 * ub * 1440.0 / 1000.0
            bolus = 0.0 if glu or d[k] <= 0 else max(0.0, carbs * tdd / t["icr_rule"] * 1000.0 - iob[k]) / ts
            basal = 0.0 if glu else pid[k]
            n = min(t["glu_max"], max(0.0, t["glu_kp"] * (t["glu_target"] - y[k]) - gob[k])) if glu else 0.0
            if ex[k] and y[k] < t["ex_bolus_below"]:
                n += t["ex_bolus"]
            assert u[k] == pytest.approx(basal + bolus, rel=1e-12, abs=1e-12), (j, k)
            ub_sum += basal * ts
            bo_sum += bolus * ts
            gl_sum += n
            checked_glu += glu
        assert r["doses"][j, 0] == pytest.approx(ub_sum, rel=1e-10)
        assert r["doses"][j, 1] == pytest.approx(bo_sum, rel=1e-10, abs=1e-9)
        assert r["doses"][j, 2] == pytest.approx(gl_sum, rel=1e-10, abs=1e-9)
        assert r["sum_u"][j] == pytest.approx(r["doses"][j, 0] + r["doses"][j, 1], rel=1e-12)
    assert checked_glu > 0 and r["doses"][:, 2].sum() > 0 and r["doses"][:, 1].sum() > 0
