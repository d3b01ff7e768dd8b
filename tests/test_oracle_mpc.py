"""Pins of the oracle's linear MPC (Sec. III-B controller form; the MPC itself is a reading).

* Jacobian == central finite differences of the drift;
* (A, B, E) == the nonlinear model's one-sample response to small perturbations of the
  state, the input and the meal intake (the linearisation and its discretisation);
* the Kalman prior covariance solves the filter DARE (scipy.linalg.solve_discrete_are);
* prediction: Markov parameters and free response == the impulse response of (A, B, E)
  iterated forward in numpy; lambda == largest eigenvalue of Gamma^T Gamma (numpy);
* projected gradient: monotone objective, converges to the unconstrained minimiser
  (numpy.linalg.solve) when the box is inactive, satisfies the KKT conditions when it is
  active, and matches brute force over all 3^N active sets for N = 4;
* closed loop: at the set point without meals or noise the plan is u = u_b forever;
* online step: on a noisy, meal-bearing run every applied input equals the one that a
  textbook Kalman measurement/time update and an exact bounded least-squares solve of the
  box QP (scipy BVLS) give from the recorded sensor values, announcements and inputs; with
  two projected-gradient steps, the textbook warm start (previous plan moved one sample on)
  reproduces the inputs and the reversed shift does not; from high glucose the loop doses
  above basal and brings glucose down to the set point.
"""
import itertools

import numpy as np
import pytest
from scipy.linalg import solve_discrete_are

from paper_2202_13927_amd import workloads as W

SX = {n: i for i, n in enumerate(W.STATE_NAMES)}
NX = 11


def mpc_trial(**kw):
    kw = {"ctrl_kind": W.CTRL_MPC, "pop_flags": 1, **kw}
    return W.with_(W.base_trial(), **kw)


@pytest.fixture(scope="module")
def pop(orc):
    return orc.sample_population(W.with_(mpc_trial(), n_patients=6))


def test_jacobian_finite_differences(orc, pop):
    t = mpc_trial()
    rng = np.random.default_rng(0)
    for row in pop[:3]:
        _, _, ub, x0 = orc.basal(t, row[:15])
        for x in (x0, x0 * rng.uniform(0.8, 1.2, NX) + 0.1):
            J, Bc, Ec = orc.jacobian(t, row[:15], x)
            for c in range(NX):
                e = max(abs(x[c]), 1e-3) * 1e-6
                xp, xm = x.copy(), x.copy()
                xp[c] += e
                xm[c] -= e
                fd = (orc.rhs(t, row[:15], xp, ub, 0.0) - orc.rhs(t, row[:15], xm, ub, 0.0)) / (2 * e)
                assert np.allclose(J[:, c], fd, rtol=1e-5, atol=1e-9), c
            fu = (orc.rhs(t, row[:15], x, ub + 1e-3, 0.0) - orc.rhs(t, row[:15], x, ub - 1e-3, 0.0)) / 2e-3
            fd_ = (orc.rhs(t, row[:15], x, ub, 1e-3) - orc.rhs(t, row[:15], x, ub, -1e-3)) / 2e-3
            assert np.allclose(Bc, fu, atol=1e-9) and np.allclose(Ec, fd_, atol=1e-9)


def test_discrete_model_is_the_one_sample_response(orc, pop):
    """x(t1) - x_ss of the EM-integrated nonlinear model for small perturbations."""
    t = W.noise_free(mpc_trial(n_patients=1, n_days=1, n_slots=0, ctrl_kind=W.CTRL_OPEN))
    row = pop[0]
    m = orc.mpc_setup(mpc_trial(), row)
    for c in range(NX):
        eps = 1e-5 * max(abs(m["xss"][c]), 1e-2)
        off = np.zeros(NX)
        off[c] = eps
        r = orc.simulate(t, n_traj=1, record_x=True, x0_offset=off, threads=1)
        dx1 = r["traj_x"][0][1] - m["xss"]
        assert np.allclose(dx1, m["A"][:, c] * eps, rtol=1e-3, atol=1e-9 * np.abs(m["A"][:, c]).max() + 1e-14), c
    du = 1e-4
    r = orc.simulate(W.with_(t, u_rel=1.0 + du), n_traj=1, record_x=True, threads=1)
    assert np.allclose(r["traj_x"][0][1] - m["xss"], m["B"] * du * m["ub"], rtol=1e-3, atol=1e-12)
    # a meal held over the first interval: fixed 1 g at minute 0
    tm = W.with_(t, n_slots=1, minute_of_day=[0, 720, 1080, 1260], carbs_mean=[1.0, 0, 0, 0],
                 carbs_sd=[0.0, 0, 0, 0], prob=[1.0, 0, 0, 0], jitter=0)
    r = orc.simulate(tm, n_traj=1, record_x=True, threads=1)
    d = 1.0 * 1000 / 180.16 / 5
    assert np.allclose(r["traj_x"][0][1] - m["xss"], m["E"] * d, rtol=1e-3, atol=1e-12)


def test_kalman_solves_the_dare(orc, pop):
    t = mpc_trial()
    for row in pop:
        m = orc.mpc_setup(t, row)
        A = m["A"]
        c = np.zeros((1, NX))
        c[0, SX["GI"]] = 1.0
        Q = 1e-6 * np.eye(NX)
        Q[SX["Q1"], SX["Q1"]] += t["sigma_q1"] ** 2 * 1.0 * 5
        R = np.array([[max(t["cgm_var"], 1e-4)]])
        P = solve_discrete_are(A.T, c.T, Q, R)
        assert np.allclose(m["P"], P, rtol=1e-7, atol=1e-10)
        assert m["P_change"] < 1e-10
        K = P[:, SX["GI"]] / (P[SX["GI"], SX["GI"]] + R[0, 0])
        assert np.allclose(m["K"], K, rtol=1e-7, atol=1e-12)


def gamma(h):
    N = len(h)
    G = np.zeros((N, N))
    for j in range(N):
        for i in range(j + 1):
            G[j, i] = h[j - i]
    return G


def test_prediction_matrices(orc, pop):
    t = mpc_trial()
    m = orc.mpc_setup(t, pop[1])
    N, A, B, E = m["N"], m["A"], m["B"], m["E"]
    vg = pop[1][W.PARAM_NAMES.index("VG")] * pop[1][W.PARAM_NAMES.index("BW")]
    cg = np.zeros(NX)
    cg[SX["Q1"]] = 1.0 / vg
    # impulse responses iterated forward
    xb, xe = B.copy(), E.copy()
    Fx = np.eye(NX)
    for j in range(N):
        assert m["h"][j] == pytest.approx(cg @ xb, rel=1e-10, abs=1e-18)
        assert m["w"][j] == pytest.approx(cg @ xe, rel=1e-10, abs=1e-18)
        Fx = A @ Fx
        assert np.allclose(m["F"][j], cg @ Fx, rtol=1e-10, atol=1e-16)
        xb, xe = A @ xb, A @ xe
    G = gamma(m["h"])
    assert np.allclose(m["Gx"], G.T @ m["F"], rtol=1e-10, atol=1e-16)
    assert np.allclose(m["gd"], G.T @ m["w"], rtol=1e-10, atol=1e-18)
    assert np.allclose(m["g1"], G.T @ np.ones(N), rtol=1e-10)
    lam = np.linalg.eigvalsh(G.T @ G).max()
    assert m["lam"] == pytest.approx(lam, rel=1e-6)
    assert m["rho_p"] == pytest.approx(1.0 / m["ub"] ** 2) and m["step"] == pytest.approx(1 / (lam + m["rho_p"]), rel=1e-6)


def objective(m, g, U):
    G = gamma(m["h"])
    return 0.5 * U @ (G.T @ G) @ U + 0.5 * m["rho_p"] * U @ U + g @ U


def test_pg_unconstrained_and_monotone(orc, pop):
    m = orc.mpc_setup(mpc_trial(), pop[2])
    N = m["N"]
    G = gamma(m["h"])
    H = G.T @ G + m["rho_p"] * np.eye(N)
    rng = np.random.default_rng(1)
    target = rng.uniform(-0.2, 0.2, N) * m["ub"]          # interior of the box
    g = -H @ target
    U = np.zeros(N)
    prev = objective(m, g, U)
    for _ in range(50):
        U = orc.mpc_pg(m, g, U, 1)
        cur = objective(m, g, U)
        assert cur <= prev + 1e-15
        prev = cur
    U = orc.mpc_pg(m, g, U, 200000)
    assert np.allclose(U, np.linalg.solve(H, -g), rtol=1e-6, atol=1e-9 * m["ub"])


def test_pg_kkt_with_active_box(orc, pop):
    m = orc.mpc_setup(mpc_trial(), pop[3])
    N = m["N"]
    lo, hi = -m["ub"], m["umax"] - m["ub"]
    G = gamma(m["h"])
    H = G.T @ G + m["rho_p"] * np.eye(N)
    g = np.linspace(-3, 3, N) * H.diagonal().max() * m["ub"] * 4
    U = orc.mpc_pg(m, g, np.zeros(N), 200000)
    grad = H @ U + g
    proj = np.clip(U - grad, lo, hi)
    assert np.max(np.abs(U - proj)) < 1e-9 * m["ub"]
    assert np.any(np.isclose(U, lo)) and np.any(np.isclose(U, hi))


def test_pg_matches_brute_force_small_n(orc, pop):
    t = mpc_trial(mpc_horizon=4)
    m = orc.mpc_setup(t, pop[4])
    N = 4
    lo, hi = -m["ub"], m["umax"] - m["ub"]
    G = gamma(m["h"])
    H = G.T @ G + m["rho_p"] * np.eye(N)
    rng = np.random.default_rng(2)
    for _ in range(5):
        g = rng.normal(0, 1, N) * H.diagonal().max() * m["ub"] * 3
        best, bestU = np.inf, None
        for act in itertools.product((0, 1, 2), repeat=N):     # 0 free, 1 at lo, 2 at hi
            fixed = {i: (lo if a == 1 else hi) for i, a in enumerate(act) if a}
            free = [i for i in range(N) if i not in fixed]
            U = np.zeros(N)
            for i, v in fixed.items():
                U[i] = v
            if free:
                rhs = -g[free] - H[np.ix_(free, list(fixed))] @ np.array(list(fixed.values())) if fixed else -g[free]
                U[free] = np.linalg.solve(H[np.ix_(free, free)], rhs)
            if np.all(U >= lo - 1e-12) and np.all(U <= hi + 1e-12):
                val = 0.5 * U @ H @ U + g @ U
                if val < best:
                    best, bestU = val, U
        Upg = orc.mpc_pg(m, g, np.zeros(N), 200000)
        assert np.allclose(Upg, bestU, rtol=1e-6, atol=1e-8 * m["ub"])


def test_closed_loop_at_setpoint(orc):
    t = W.noise_free(mpc_trial(n_patients=4, n_days=2, n_slots=0))
    r = orc.simulate(t, n_traj=4, threads=4)
    ub = r["params"][:4, 15]
    assert np.max(np.abs(r["traj_u"] - ub[:, None]) / ub[:, None]) < 1e-12
    assert np.max(np.abs(r["traj_g"] - 6.0)) < 1e-10


# ------------------------------------------------------------------ online step
# The controller sample written out in textbook form (Sec. III-B: the controller state is the
# estimate and the plan, the action is the plan's first input), independently of the oracle's
# code: measurement update x+ = x- + K (y - x*_GI - x-_GI); prediction matrices rebuilt here
# from (A, B, E) and c_G = e_Q1 / V_G; the box QP over the input deviations solved exactly as
# a bounded least-squares problem (scipy's BVLS); time update x- = A x+ + B (u - u_b) + E d.
# Only (A, B, E, K), pinned by the tests above, are taken from the oracle's setup.

def textbook_prediction(m, prm):
    N = m["N"]
    vg = prm[W.PARAM_NAMES.index("VG")] * prm[W.PARAM_NAMES.index("BW")]
    cg = np.zeros(NX)
    cg[SX["Q1"]] = 1.0 / vg
    F, h, w = np.zeros((N, NX)), np.zeros(N), np.zeros(N)
    Ap = np.eye(NX)
    for j in range(N):               # G_(k+j+1) - G* = F_j x + sum_i h_(j-i) du_i + w_j d
        h[j] = cg @ Ap @ m["B"]
        w[j] = cg @ Ap @ m["E"]
        Ap = m["A"] @ Ap
        F[j] = cg @ Ap
    return F, h, w


def announced(orc, t, patient, K):
    d = np.zeros(K)
    for day in range(int(t["n_days"])):
        for kd, _carbs, rate in orc.day_meals(t, patient, day):
            d[day * 288 + int(kd)] += rate
    return d


def test_online_step_is_the_textbook_filter_and_exact_qp(orc):
    """A noisy, meal-bearing MPC run: every applied input equals u_b plus the first entry of
    the exact solution of the box QP built from the textbook filter's estimate, on samples
    with an active bound as well (the 50 projected-gradient steps converge: the QP's
    condition number is ~1.3 because rho/u_b^2 dominates Gamma^T Gamma)."""
    from scipy.optimize import lsq_linear
    t = W.with_(mpc_trial(), n_patients=3, n_days=2)
    r = orc.simulate(t, n_traj=3, threads=3)
    K = r["K"]
    n_active = 0
    for j in range(3):
        prm = r["params"][j]
        m = orc.mpc_setup(t, prm)
        F, h, w = textbook_prediction(m, prm)
        N, ub, umax = m["N"], m["ub"], m["umax"]
        Gam = gamma(h)
        rho = t["mpc_rho"] / ub ** 2
        A_ls = np.vstack([Gam, np.sqrt(rho) * np.eye(N)])
        d = announced(orc, t, j, K)
        assert np.count_nonzero(d) >= 6
        xh = np.zeros(NX)
        for k in range(K):
            y, u = r["traj_y"][j, k], r["traj_u"][j, k]
            xh = xh + m["K"] * ((y - m["xss"][SX["GI"]]) - xh[SX["GI"]])
            resid = F @ xh + w * d[k] + (t["g_target"] - t["setpoint"])
            sol = lsq_linear(A_ls, -np.concatenate([resid, np.zeros(N)]),
                             bounds=(np.full(N, -ub), np.full(N, umax - ub)), method="bvls", tol=1e-14)
            n_active += int(np.any(sol.active_mask != 0))
            assert abs(ub + sol.x[0] - u) <= 1e-10 * ub, (j, k)
            xh = m["A"] @ xh + m["B"] * (u - ub) + m["E"] * d[k]
    assert n_active > 50


def test_online_step_warm_start_is_the_shifted_plan(orc):
    """With only two projected-gradient steps the warm start decides the action: it is the
    previous plan moved one sample on (its last entry repeated). The reversed shift misses
    by > 1 % of u_b; the textbook loop matches to rounding."""
    t = W.with_(mpc_trial(), n_patients=2, n_days=1, mpc_iters=2)
    r = orc.simulate(t, n_traj=2, threads=2)
    K = r["K"]
    for j in range(2):
        prm = r["params"][j]
        m = orc.mpc_setup(t, prm)
        F, h, w = textbook_prediction(m, prm)
        N, ub, umax = m["N"], m["ub"], m["umax"]
        Gam = gamma(h)
        H = Gam.T @ Gam + t["mpc_rho"] / ub ** 2 * np.eye(N)
        step = 1.0 / np.linalg.eigvalsh(H).max()
        d = announced(orc, t, j, K)
        xh, U, Urev = np.zeros(NX), np.zeros(N), np.zeros(N)
        worst_rev = 0.0
        for k in range(K):
            y, u = r["traj_y"][j, k], r["traj_u"][j, k]
            xh = xh + m["K"] * ((y - m["xss"][SX["GI"]]) - xh[SX["GI"]])
            g = Gam.T @ (F @ xh + w * d[k] + (t["g_target"] - t["setpoint"]))
            U = np.concatenate([U[1:], U[-1:]])
            Urev = np.concatenate([Urev[:1], Urev[:-1]])
            for _ in range(2):
                U = np.clip(U - step * (H @ U + g), -ub, umax - ub)
                Urev = np.clip(Urev - step * (H @ Urev + g), -ub, umax - ub)
            assert abs(ub + U[0] - u) <= 1e-12 * ub, (j, k)
            worst_rev = max(worst_rev, abs(ub + Urev[0] - u) / ub)
            xh = m["A"] @ xh + m["B"] * (u - ub) + m["E"] * d[k]
        assert worst_rev > 1e-2


def test_mpc_brings_high_glucose_down(orc):
    """Sign of the loop: started at G = G_I = 10 mmol/L (basal insulin states), without meals
    or noise, the first inputs are above u_b (at the bound), glucose falls monotonically for
    the first hour, reaches the set point within four hours, stays above 5 mmol/L and settles
    at 6."""
    t = W.noise_free(mpc_trial(n_patients=3, n_days=1, n_slots=0))
    pop = orc.sample_population(t)
    for j in range(3):
        vg = pop[j][W.PARAM_NAMES.index("VG")] * pop[j][W.PARAM_NAMES.index("BW")]
        off = np.zeros(NX)
        off[SX["Q1"]] = 4.0 * vg
        off[SX["GI"]] = 4.0
        r = orc.simulate(W.with_(t, n_patients=1, first_patient=j), n_traj=1, threads=1, x0_offset=off)
        u, g = r["traj_u"][0], r["traj_g"][0]
        ub = r["params"][0, 15]
        assert g[0] == pytest.approx(10.0, rel=1e-12)
        assert np.all(u[:2] > 2.9 * ub)
        assert np.all(np.diff(g[:12]) < 0)
        assert np.min(np.abs(g[:48] - 6.0)) < 0.3
        assert g.min() > 5.0
        assert abs(g[-1] - 6.0) < 1e-2
