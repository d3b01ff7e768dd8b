"""Pins of the oracle's patient model and integrators (Sec. III-A eq. 1-2, Sec. IV-B).

* the basal steady state (closed form of the quadratic in I) is a zero of f;
* a noise-free, meal-free run at the set point never leaves it;
* constant open-loop insulin drives G to the closed-form equilibrium in each of
  the three regimes of F01c and F_R;
* the linear part (gut, subcutaneous insulin, plasma insulin, insulin action) matches
  the exact solution exp(A t) of that linear ODE (scipy's expm);
* the sensor state relaxes as (1 - h/tau)^n under EM;
* EM converges to a fine RK4 reference with order 1;
* one EM step adds sigma sqrt(h) xi to Q1 and the sensor adds sqrt(R) v, with the
  normals at the documented counters.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from paper_2202_13927_amd import workloads as W

NOM = np.array(W.NOMINAL)
IDX = {n: i for i, n in enumerate(W.PARAM_NAMES)}
SX = {n: i for i, n in enumerate(W.STATE_NAMES)}


def quiet(**kw):
    return W.noise_free(W.with_(W.base_trial(), n_slots=0, **kw))


def test_basal_state_is_equilibrium(orc):
    t = W.base_trial()
    p = orc.sample_population(W.with_(t, n_patients=300))
    for row in p:
        ok, I, ub, x0 = orc.basal(t, row[:15])
        assert ok
        f = orc.rhs(t, row[:15], x0, ub, 0.0)
        scale = np.maximum(np.abs(x0), 1.0)
        assert np.max(np.abs(f) / scale) < 1e-13
        assert x0[SX["Q1"]] / (row[IDX["VG"]] * row[IDX["BW"]]) == pytest.approx(6.0, rel=1e-15)
        assert I == pytest.approx(row[16], rel=0) and ub == pytest.approx(row[15], rel=0)


def test_steady_state_holds_for_a_week(orc):
    t = quiet(n_patients=16, n_days=7)
    r = orc.simulate(t, n_traj=16, record_x=True, threads=4)
    assert np.max(np.abs(r["traj_g"] - 6.0)) < 1e-10
    ub = r["params"][:, 15]
    assert np.max(np.abs(r["traj_u"] - ub[:, None]) / ub[:, None]) < 1e-10
    assert np.all(r["bins"][:, 2] == r["K"])


def _g_equilibrium(row, u):
    """Closed-form steady glucose for constant insulin u (D = 0)."""
    bw = row[IDX["BW"]]
    egp0, f01, vg, vi = row[IDX["EGP0"]] * bw, row[IDX["F01"]] * bw, row[IDX["VG"]] * bw, row[IDX["VI"]] * bw
    I = u / (row[IDX["ke"]] * vi)
    x1, x2, x3 = row[IDX["SIT"]] * I, row[IDX["SID"]] * I, row[IDX["SIE"]] * I
    E = egp0 * max(0.0, 1.0 - x3)
    c = x1 * x2 * vg / (row[IDX["k12"]] + x2)
    for g in (E / (f01 / 4.5 + c), (E - f01) / c, (E - f01 + 0.027 * vg) / (0.003 * vg + c)):
        lo, hi = (0, 4.5) if g < 4.5 else ((4.5, 9.0) if g <= 9 else (9.0, np.inf))
        if lo <= g <= hi and abs(E - f01 * min(1, g / 4.5) - 0.003 * max(0, g - 9) * vg - c * g) < 1e-9:
            return g
    raise AssertionError("no consistent regime")


@pytest.mark.parametrize("u_rel", [0.35, 0.8, 1.6, 3.0])
def test_open_loop_equilibrium_regimes(orc, u_rel):
    t = quiet(n_patients=6, n_days=40, ctrl_kind=W.CTRL_OPEN, u_rel=u_rel)
    r = orc.simulate(t, n_traj=6, integrator=1, rk4_sub=5, threads=6)
    regimes = set()
    for j in range(6):
        row = r["params"][j]
        g_eq = _g_equilibrium(row, u_rel * row[15])
        regimes.add(0 if g_eq < 4.5 else (1 if g_eq <= 9 else 2))
        assert r["traj_g"][j, -1] == pytest.approx(g_eq, rel=1e-6)
    if u_rel == 3.0:
        assert 0 in regimes
    if u_rel == 0.35:
        assert 2 in regimes


def test_linear_subsystem_matches_matrix_exponential(orc):
    """Gut, insulin and insulin-action states are a linear ODE in (x, u, D); with the
    inputs held over each sample interval the exact sample-to-sample map is expm of
    the augmented matrix [[A, B], [0, 0]] * Ts."""
    t = W.noise_free(W.with_(W.base_trial(), n_patients=3, n_days=2, ctrl_kind=W.CTRL_OPEN, u_rel=1.7))
    r = orc.simulate(t, n_traj=3, record_x=True, integrator=1, rk4_sub=64, threads=3)
    lin = [SX[n] for n in ("D1", "D2", "S1", "S2", "I", "x1", "x2", "x3")]
    for j in range(3):
        row = r["params"][j]
        bw = row[IDX["BW"]]
        tg, ti, vi, ke = row[IDX["tmaxG"]], row[IDX["tmaxI"]], row[IDX["VI"]] * bw, row[IDX["ke"]]
        A = np.zeros((10, 10))    # 8 states + 2 inputs (u, D)
        A[0, 0], A[0, 9] = -1 / tg, t["ag"]
        A[1, 0], A[1, 1] = 1 / tg, -1 / tg
        A[2, 2], A[2, 8] = -1 / ti, 1.0
        A[3, 2], A[3, 3] = 1 / ti, -1 / ti
        A[4, 3], A[4, 4] = 1 / (ti * vi), -ke
        for a, (ka, si) in enumerate([("ka1", "SIT"), ("ka2", "SID"), ("ka3", "SIE")]):
            A[5 + a, 5 + a], A[5 + a, 4] = -row[IDX[ka]], row[IDX[ka]] * row[IDX[si]]
        Phi = expm(A * t["ts_min"])
        X = r["traj_x"][j][:, lin]
        u = r["traj_u"][j]
        D = np.zeros_like(u)
        for day in range(t["n_days"]):
            for pres, kd, carbs, _ in orc.meals(t, j, day):
                if pres:
                    D[day * 288 + int(kd)] += carbs * 1000 / 180.16 / t["ts_min"]
        for k in range(X.shape[0] - 1):
            z = np.concatenate([X[k], [u[k], D[k]]])
            pred = (Phi @ z)[:8]
            assert np.allclose(pred, X[k + 1], rtol=1e-9, atol=1e-9 * np.abs(X[k + 1]).max()), k


def test_sensor_lag_relaxation(orc):
    """At the basal state with the sensor offset by delta, G stays at G* and EM gives
    GI_n - G* = delta (1 - h/tau)^n at every EM step n."""
    t = quiet(n_patients=2, n_days=1, ctrl_kind=W.CTRL_OPEN, u_rel=1.0)
    off = np.zeros(11)
    off[SX["GI"]] = 1.5
    r = orc.simulate(t, n_traj=2, record_x=True, x0_offset=off, threads=2)
    n = np.arange(288) * 5
    expect = 6.0 + 1.5 * (1 - 1.0 / 10.0) ** n
    assert np.allclose(r["traj_x"][0][:, SX["GI"]], expect, rtol=1e-13, atol=1e-13)
    assert np.max(np.abs(r["traj_g"] - 6.0)) < 1e-12


def test_gut_mass_balance(orc):
    """Meals in the rhs: d(D1 + D2)/dt = AG D - D2/tmaxG for any state."""
    t = W.base_trial()
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.uniform(0.1, 50, size=11)
        d = rng.uniform(0, 10)
        f = orc.rhs(t, NOM, x, 3.0, d)
        assert f[0] + f[1] == pytest.approx(0.8 * d - x[1] / NOM[IDX["tmaxG"]], rel=1e-12)
        assert f[2] + f[3] == pytest.approx(3.0 - x[3] / NOM[IDX["tmaxI"]], rel=1e-12)


def _em_vs_rk4_error(orc, t, m):
    tm = W.with_(t, em_per_ctrl=m)
    r_em = orc.simulate(tm, n_traj=4, threads=4)
    r_rk = orc.simulate(t, n_traj=4, integrator=1, rk4_sub=64, threads=4)
    return np.max(np.abs(r_em["traj_g"] - r_rk["traj_g"]))


def test_em_first_order_convergence_open_loop(orc):
    t = W.noise_free(W.with_(W.base_trial(), n_patients=4, n_days=2, ctrl_kind=W.CTRL_OPEN, u_rel=1.0))
    e = [_em_vs_rk4_error(orc, t, m) for m in (5, 10, 20)]
    assert 1.7 < e[0] / e[1] < 2.3 and 1.7 < e[1] / e[2] < 2.3, e
    assert e[0] < 0.3   # mmol/L at h = 1 min


def test_em_converges_closed_loop(orc):
    t = W.noise_free(W.with_(W.base_trial(), n_patients=4, n_days=2))
    e = [_em_vs_rk4_error(orc, t, m) for m in (5, 10, 20)]
    assert e[0] > e[1] > e[2]
    assert e[2] < 0.5 * e[0]   # clamp decisions can switch between step sizes


def test_noise_enters_q1_and_sensor(orc):
    """One-minute samples with one EM step each: after the first step Q1 differs from the
    noise-free run by exactly sigma sqrt(h) xi_0; y_0 = G* + sqrt(R) v_0 where xi_0 and v_0
    are normals #0 and #1 of the block with counter (0, patient, DIFF, 0); sample 1 (the
    second of the pair) takes normals #2 and #3, sample 2 block (1, patient, DIFF, 0)."""
    t = W.with_(W.base_trial(), n_patients=4, n_days=1, n_slots=0, ts_min=1, em_per_ctrl=1,
                ctrl_kind=W.CTRL_OPEN, sigma_q1=0.8, cgm_var=0.01, noise_seed=11)
    r = orc.simulate(t, n_traj=4, record_x=True, threads=2)
    r0 = orc.simulate(W.noise_free(t), n_traj=4, record_x=True, threads=2)
    for j in range(4):
        z = orc.normals4((0, j, 2, 0), (11, 0))
        dq = r["traj_x"][j][1, SX["Q1"]] - r0["traj_x"][j][1, SX["Q1"]]
        assert dq == pytest.approx(0.8 * z[0], rel=1e-9)
        assert r["traj_y"][j][0] - 6.0 == pytest.approx(0.1 * z[1], rel=1e-9)
        # samples come in pairs: sample 1 takes normals #2 (xi) and #3 (v) of the same block,
        # and its sensor state is still exactly G* (one EM step of GI from G* = GI)
        assert r["traj_y"][j][1] - 6.0 == pytest.approx(0.1 * z[3], rel=1e-9)
        z2 = orc.normals4((1, j, 2, 0), (11, 0))
        x2 = r["traj_x"][j][2]
        drift = orc.rhs(t, r["params"][j][:15], x2, r["traj_u"][j][2], 0.0)[SX["Q1"]]
        q2 = r["traj_x"][j][3, SX["Q1"]] - x2[SX["Q1"]]
        assert q2 - drift == pytest.approx(0.8 * z2[0], rel=1e-9)
