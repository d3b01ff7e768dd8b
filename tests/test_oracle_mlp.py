"""Pins of the oracle's learned controller (network, gradient, Adam, statistics, closed loop).

Each check compares the oracle with something it does not compute itself: BF16 rounding
against torch's conversion and hand-worked ties; the forward pass against a network built
to compute |z| and against the affine map it reduces to when every ReLU is active; the
gradient against central finite differences; Adam against its closed form for a constant
gradient; the statistics against numpy; the closed loop against the open-loop and MPC
controllers it reduces to and against its own trajectory outputs.
"""
import numpy as np
import pytest
import torch

from paper_2202_13927_amd import workloads as W


def test_bf16_rounding(orc):
    # ties go to the even significand; values already on the grid are unchanged
    assert orc.bf16([1.0 + 2 ** -8])[0] == 1.0
    assert orc.bf16([1.0 + 3 * 2 ** -8])[0] == 1.0 + 2 ** -6
    assert orc.bf16([-(1.0 + 3 * 2 ** -8)])[0] == -(1.0 + 2 ** -6)
    assert orc.bf16([1.0 + 2 ** -8 + 2 ** -20])[0] == 1.0 + 2 ** -7
    assert orc.bf16([3.0, 0.0, -0.5])[:].tolist() == [3.0, 0.0, -0.5]
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(4000) * 10.0 ** rng.integers(-6, 6, 4000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(orc.bf16(x.astype(np.float64)), ref)


def _abs_net():
    """A network computing out = |z0| + 0.5 z1 - 1 via ReLU pairs (identity hidden layers)."""
    z = lambda *s: np.zeros(s)
    net = {"W1": z(64, 12), "b1": z(64), "W2": z(64, 64), "b2": z(64), "W3": z(64, 64), "b3": z(64),
           "w4": z(64), "b4": -1.0, "mean": z(12), "istd": np.ones(12), "lo": z(12), "hi": z(12)}
    net["W1"][0, 0], net["W1"][1, 0] = 1.0, -1.0          # relu(z0), relu(-z0)
    net["W1"][2, 1], net["W1"][3, 1] = 1.0, -1.0          # relu(z1), relu(-z1)
    for k in ("W2", "W3"):
        net[k][np.arange(4), np.arange(4)] = 1.0
    net["w4"][:4] = [1.0, 1.0, 0.5, -0.5]
    return net


def test_forward_abs_network(orc):
    net = _abs_net()
    rng = np.random.default_rng(1)
    x = rng.standard_normal((500, 12)) * 3.0
    z0, z1 = orc.bf16(x[:, 0]), orc.bf16(x[:, 1])
    assert np.array_equal(orc.mlp_forward(net, x), np.abs(z0) + 0.5 * z1 - 1.0)
    # the z-score is applied before the rounding
    net["mean"][0], net["istd"][0] = 2.0, 0.25
    z0 = orc.bf16((x[:, 0] - 2.0) * 0.25)
    assert np.allclose(orc.mlp_forward(net, x), np.abs(z0) + 0.5 * z1 - 1.0, rtol=0, atol=1e-15)


def test_forward_all_active_is_affine(orc):
    """Positive weights and inputs keep every ReLU active: the network is the affine map
    w4 (W3 (W2 (W1 z + b1) + b2) + b3) + b4, evaluated here with numpy's matmul."""
    rng = np.random.default_rng(2)
    net = {"W1": rng.random((64, 12)), "b1": rng.random(64), "W2": rng.random((64, 64)) / 8,
           "b2": rng.random(64), "W3": rng.random((64, 64)) / 8, "b3": rng.random(64), "w4": rng.standard_normal(64),
           "b4": 0.3, "mean": np.zeros(12), "istd": np.ones(12), "lo": np.zeros(12), "hi": np.zeros(12)}
    x = rng.random((300, 12)) + 0.1
    z = orc.bf16(x)
    ref = ((z @ net["W1"].T + net["b1"]) @ net["W2"].T + net["b2"]) @ net["W3"].T + net["b3"]
    ref = ref @ net["w4"] + net["b4"]
    assert np.allclose(orc.mlp_forward(net, x), ref, rtol=1e-13, atol=0)


def _random_net(seed):
    """Dense random weights (no unit sits exactly at a ReLU kink, unlike the structured
    proportional-law units of the closed-loop test network)."""
    net = W.synthetic_policy_net(seed)
    rng = np.random.default_rng(seed + 1000)
    for k, s in (("W1", 0.4), ("W2", 0.17), ("W3", 0.17)):
        net[k] = s * rng.standard_normal(net[k].shape)
    for k in ("b1", "b2", "b3"):
        net[k] = 0.1 * rng.standard_normal(64)
    net["w4"] = 0.2 * rng.standard_normal(64)
    return net


def test_gradient_matches_finite_differences(orc):
    net = _random_net(3)
    rows = W.synthetic_policy_rows(3, 200)
    idx = np.arange(0, 200, 3)
    loss, g = orc.mlp_loss_grad(net, rows, idx)
    o = orc.mlp_forward(net, rows[idx, :12])
    assert loss == pytest.approx(np.mean((o - rows[idx, 12]) ** 2), rel=1e-13)
    rng = np.random.default_rng(4)
    eps = 1e-6
    checked = 0
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4"):
        shape = np.shape(net[name])
        picks = [()] if shape == () else [tuple(rng.integers(0, s) for s in shape) for _ in range(12)]
        for p in picks:
            base = np.array(net[name], dtype=np.float64)
            vals = []
            for s in (+1, -1):
                v = base.copy()
                if p == ():
                    v = float(base) + s * eps
                else:
                    v[p] += s * eps
                n2 = dict(net)
                n2[name] = v
                vals.append(orc.mlp_loss_grad(n2, rows, idx)[0])
            fd = (vals[0] - vals[1]) / (2 * eps)
            an = g[name] if p == () else g[name][p]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, p, an, fd)
            checked += 1
    assert checked == 7 * 12 + 1
    for k in ("mean", "istd", "lo", "hi"):
        assert not np.any(g[k])


def test_adam_constant_gradient_closed_form(orc):
    """With a constant gradient g, m_t = g (1 - b1^t) and v_t = g^2 (1 - b2^t), so after bias
    correction every step moves w by lr g / (|g| + eps), whatever t."""
    g = np.array([0.3, -2.0, 1e-3, -5e-5])
    w, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    lr = 0.01
    for t in range(1, 6):
        w0 = w.copy()
        w, m, v = orc.adam(w, m, v, g, lr, t)
        assert np.allclose(w - w0, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        assert np.allclose(m, g * (1 - 0.9 ** t), rtol=1e-12)
        assert np.allclose(v, g * g * (1 - 0.999 ** t), rtol=1e-12)


def test_init_statistics(orc):
    net = orc.mlp_init(11)
    for k, fan in (("W1", 12), ("W2", 64), ("W3", 64)):
        w = net[k].ravel()
        assert abs(w.mean()) < 4 * np.sqrt(2.0 / fan) / np.sqrt(w.size)
        assert w.std() == pytest.approx(np.sqrt(2.0 / fan), rel=0.08)
    assert net["w4"].std() == pytest.approx(np.sqrt(1.0 / 64), rel=0.3)
    assert net["b4"] == 1.0 and not np.any(net["b1"]) and not np.any(net["b2"]) and not np.any(net["b3"])
    assert not np.array_equal(orc.mlp_init(12)["W2"], net["W2"])
    assert np.array_equal(orc.mlp_init(11)["W2"], net["W2"])


def test_batch_rows_uniform(orc):
    idx = orc.mlp_batch_rows(5, 0, 60000, 10)
    assert idx.min() == 0 and idx.max() == 9
    counts = np.bincount(idx, minlength=10)
    chi2 = ((counts - 6000.0) ** 2 / 6000.0).sum()
    assert chi2 < 27.9   # 99.9 % point of chi-square with 9 degrees of freedom
    assert not np.any(orc.mlp_batch_rows(5, 0, 100, 1))
    assert not np.array_equal(orc.mlp_batch_rows(5, 1, 64, 1000), orc.mlp_batch_rows(5, 0, 64, 1000))


def test_stats_match_numpy(orc):
    rows = W.synthetic_policy_rows(6, 5001)
    s = orc.mlp_stats(rows, 0.0)
    x = rows[:, :12]
    assert np.allclose(s["mean"], x.mean(0), rtol=1e-12)
    assert np.allclose(s["istd"], 1.0 / np.maximum(x.std(0), 1e-6), rtol=1e-9)
    assert np.array_equal(s["lo"], x.min(0)) and np.array_equal(s["hi"], x.max(0))
    q = orc.mlp_stats(rows, 0.001)
    assert np.array_equal(q["lo"], np.quantile(x, 0.001, axis=0, method="inverted_cdf"))
    assert np.array_equal(q["hi"], np.quantile(x, 0.999, axis=0, method="inverted_cdf"))


def _small(trial, **kw):
    return W.with_(trial, **{"n_patients": 40, "n_days": 2, "precision": W.FP64, **kw})


def test_constant_network_is_open_loop(orc):
    """out = 1 everywhere and a box admitting everything: u = u_b on every sample, i.e. the
    open-loop controller with u_rel = 1."""
    t = _small(W.c5_mlp())
    a = orc.simulate(t, n_traj=5, threads=4, mlp=W.constant_policy_net(1.0))
    b = orc.simulate(W.with_(t, ctrl_kind=W.CTRL_OPEN, u_rel=1.0), n_traj=5, threads=4)
    for k in ("bins", "events", "sum_g", "min_g", "traj_g", "traj_u"):
        assert np.array_equal(a[k], b[k]), k
    assert not np.any(a["fallback"])


def test_box_excluding_everything_is_mpc(orc):
    """An empty box hands every sample to the MPC: identical to the MPC controller."""
    t = _small(W.c5_mlp())
    a = orc.simulate(t, n_traj=5, threads=4, mlp=W.constant_policy_net(2.0, always_fallback=True))
    b = orc.simulate(W.with_(t, ctrl_kind=W.CTRL_MPC), n_traj=5, threads=4)
    for k in ("bins", "events", "sum_g", "traj_g", "traj_u"):
        assert np.array_equal(a[k], b[k]), k
    assert np.all(a["fallback"] == a["K"])


def test_safety_rule(orc):
    """out = 2 and a box admitting everything: u = 2 u_b except on samples with y < 3.9
    (the safety threshold set for this test), where the MPC acts; the fallback count is the
    number of such samples."""
    t = _small(W.c5_mlp(), n_patients=24, n_days=3, mlp_safe_g=3.9)
    r = orc.simulate(t, n_traj=24, threads=4, mlp=W.constant_policy_net(2.0))
    low = r["traj_y"] < 3.9
    ub = r["params"][:, 15][:, None]
    assert low.sum() > 0
    assert np.array_equal(r["fallback"], low.sum(1))
    assert np.array_equal(r["traj_u"][~low], np.broadcast_to(2.0 * ub, low.shape)[~low])


def test_recorded_rows(orc):
    """The recorded inputs equal the trajectory outputs, the patient's parameters and the
    basal state; the target is u / u_b."""
    t = _small(W.c5_mpc(), n_patients=12)
    r = orc.simulate(t, n_traj=12, threads=4, record=True)
    rec = r["record"]                     # [K][n][13]
    y, u = r["traj_y"].T, r["traj_u"].T   # [K][n]
    prm = r["params"]
    assert np.array_equal(rec[:, :, 0], y)
    for i in range(1, 6):
        assert np.array_equal(rec[i:, :, i], y[:-i])
        assert np.array_equal(rec[:i, :, i], np.broadcast_to(y[0], (i, y.shape[1])))
    assert np.allclose(rec[0, :, 6], 0.0, rtol=0, atol=1e-12)           # basal: no pending insulin effect
    assert np.array_equal(rec[:, :, 8], np.broadcast_to(prm[:, 15], rec.shape[:2]))
    assert np.array_equal(rec[:, :, 11], np.broadcast_to(prm[:, 14], rec.shape[:2]))
    for j in range(12):   # insulin response over the horizon and its mean delay
        h = orc.mpc_setup(t, prm[j])["h"]
        assert np.allclose(rec[:, j, 9], h.sum(), rtol=1e-12)
        assert np.allclose(rec[:, j, 10], (np.arange(1, 25) * h).sum() / h.sum(), rtol=1e-12)
    assert np.allclose(rec[:, :, 12], u / prm[:, 15], rtol=1e-15)
    # meal input: zero before the day's first meal; at the meal sample the announced intake
    # rate times the horizon mean of the intake response (the meal states are still empty)
    first = [orc.meals(t, j, 0) for j in range(12)]
    for j in range(12):
        k0 = int(first[j][0][1])
        assert np.all(rec[:k0, j, 7] == 0.0)
        rate = first[j][0][2] * (1000.0 / 180.16) / t["ts_min"]
        wbar = orc.mpc_setup(t, prm[j])["w"].mean()
        assert rec[k0, j, 7] == pytest.approx(wbar * rate, rel=1e-12)
        assert rec[k0 + 1, j, 7] > 0.0


def test_labels_along_own_loop(orc):
    """Recording with the learned controller labels every sample with the MPC's action; with
    an empty box the MPC acts everywhere, so the rows equal those of the MPC's own loop."""
    t = _small(W.c5_mlp(), n_patients=10)
    a = orc.simulate(t, threads=4, record=True, mlp=W.constant_policy_net(2.0, always_fallback=True))
    b = orc.simulate(W.with_(t, ctrl_kind=W.CTRL_MPC), threads=4, record=True)
    assert np.array_equal(a["record"], b["record"])
    # with a network that acts, the labels still come from the MPC (u/u_b = 2 is never applied
    # below 3.9, and the labels differ from the applied 2)
    c = orc.simulate(t, threads=4, record=True, n_traj=10, mlp=W.constant_policy_net(2.0))
    applied = c["traj_u"].T / c["params"][:, 15]
    assert np.any(np.abs(c["record"][:, :, 12] - applied) > 1e-3)


def test_insulin_and_meal_inputs_are_the_predicted_mean_glucose_change(orc):
    """The learned controller's inputs 6 and 7 on every sample of a noisy, meal-bearing MPC
    run, recomputed from the recorded plant states: the insulin input is the mean over the
    next 24 samples of the glucose deviation that the insulin states' deviation from basal
    causes, and the meal input the same for the gut states plus the intake announced for the
    current interval. Here the horizon is walked sample by sample with the discrete model
    (x_(j+1) = A x_j, the intake entering through E on the first step), not through the
    oracle's horizon means. Insulin above basal lowers glucose and meals raise it."""
    t = W.with_(W.c5_mpc(), n_patients=6, n_days=2, precision=W.FP64)
    r = orc.simulate(t, n_traj=6, threads=4, record=True, record_x=True)
    rec, X, K = r["record"], r["traj_x"], r["K"]
    SX = {n: i for i, n in enumerate(W.STATE_NAMES)}
    ins = [SX[s] for s in ("S1", "S2", "I", "x1", "x2", "x3")]
    gut = [SX["D1"], SX["D2"]]
    for j in range(6):
        prm = r["params"][j]
        m = orc.mpc_setup(t, prm)
        N, A, E = m["N"], m["A"], m["E"]
        vg = prm[W.PARAM_NAMES.index("VG")] * prm[W.PARAM_NAMES.index("BW")]
        d = np.zeros(K)
        for day in range(2):
            for kd, _c, rate in orc.day_meals(t, j, day):
                d[day * 288 + int(kd)] += rate
        # the walk is linear: propagate all samples' start vectors together (columns)
        dx_ins = np.zeros((11, K))
        dx_ins[ins] = (X[j][:, ins] - m["xss"][ins]).T
        dx_gut = np.zeros((11, K))
        dx_gut[gut] = X[j][:, gut].T
        acc_i, acc_g = np.zeros(K), np.zeros(K)
        xi, xg = dx_ins, dx_gut
        for step in range(N):
            xi = A @ xi
            xg = A @ xg + (np.outer(E, d) if step == 0 else 0.0)
            acc_i += xi[SX["Q1"]] / vg
            acc_g += xg[SX["Q1"]] / vg
        iob, meal = acc_i / N, acc_g / N
        scale_i, scale_g = np.abs(iob).max(), np.abs(meal).max()
        assert scale_i > 0.1 and scale_g > 0.1
        assert np.allclose(rec[:, j, 6], iob, rtol=1e-9, atol=1e-12 * scale_i)
        assert np.allclose(rec[:, j, 7], meal, rtol=1e-9, atol=1e-12 * scale_g)
        above = (X[j][:, SX["S1"]] + X[j][:, SX["S2"]]) > 1.5 * (m["xss"][SX["S1"]] + m["xss"][SX["S2"]])
        above &= X[j][:, SX["I"]] > 1.2 * m["xss"][SX["I"]]
        assert above.sum() > 10 and np.all(rec[above, j, 6] < 0)
        assert np.all(rec[d > 0, j, 7] > 0)
