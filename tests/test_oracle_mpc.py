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
* closed loop: at the set point without meals or noise the plan is u = u_b forever.
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
