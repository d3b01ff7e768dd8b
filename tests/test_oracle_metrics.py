"""Pins of the oracle's on-the-fly indicators, protocol draws, PID and population reduction.

* streaming per-patient accumulators == brute-force counts over recorded
  trajectories (ranges of Sec. IV-A; runs of >= 3 samples; sum; first minimum);
* meal draws: presence rate, integer jitter uniform on [-J, J], carbs moments,
  and the intervals where the gut state actually receives glucose;
* PID (Sec. III-B form) on scripted measurements: linear integral growth,
  clamping, conditional integration;
* reduction: nearest-rank quantiles == numpy's inverted-CDF percentile, totals,
  and the lexicographic worst case.
"""
import numpy as np
import pytest
from scipy import stats

from paper_2202_13927_amd import workloads as W

EDGES = (3.0, 3.9, 10.0, 13.9)


def brute_force(g):
    bins = np.zeros(5, int)
    bins[0] = np.sum(~(g >= 3.0))     # below the first edge, or not a number
    bins[1] = np.sum((g >= 3.0) & (g < 3.9))
    bins[2] = np.sum((g >= 3.9) & (g <= 10.0))
    bins[3] = np.sum((g > 10.0) & (g <= 13.9))
    bins[4] = np.sum(g > 13.9)
    ev = []
    for cond in (~(g >= 3.9), ~(g >= 3.0), g > 13.9):   # "below" = not at or above
        runs, n = 0, 0
        for c in cond:
            n = n + 1 if c else 0
            runs += n == 3
        ev.append(runs)
    s = 0.0
    for v in g:            # same order as the streaming sum
        s += v
    return bins, np.array(ev), s, g.min(), int(np.argmin(g))


@pytest.mark.parametrize("noisy", [True, False])
def test_accumulators_equal_brute_force(orc, noisy):
    t = W.with_(W.base_trial(), n_patients=8, n_days=2, kp=1.5, kd=60.0)   # aggressive: reaches all ranges
    if not noisy:
        t = W.noise_free(t)
    r = orc.simulate(t, n_traj=8, threads=4)
    seen = set()
    for j in range(8):
        bins, ev, s, mn, am = brute_force(r["traj_g"][j])
        assert np.array_equal(bins, r["bins"][j])
        assert np.array_equal(ev, r["events"][j])
        assert s == r["sum_g"][j]
        assert mn == r["min_g"][j] and am == r["argmin_k"][j]
        seen |= set(np.nonzero(bins)[0])
        assert r["sum_u"][j] == pytest.approx(r["traj_u"][j].sum() * 5.0, rel=1e-12)
    assert seen == {0, 1, 2, 3, 4}


def test_non_finite_glucose_counts_as_lowest(orc):
    """A patient with no basal state (nominal vector infeasible) has a non-finite state from
    the start: every sample falls in the lowest range, the runs below 3.9 and 3.0 never end
    (one event each), and the non-finite and resample status bits are set."""
    t = W.with_(W.c1_fp64_pid(), n_patients=3, n_days=1, cv=1e-9,
                nominal=[W.NOMINAL[0], W.NOMINAL[0] * 1.5, *W.NOMINAL[2:]])
    r = orc.simulate(t, n_traj=3, threads=3)
    K = r["bins"].sum(1)[0]
    assert K == 288
    for j in range(3):
        assert not np.isfinite(r["traj_g"][j]).any()
        assert np.array_equal(r["bins"][j], [K, 0, 0, 0, 0])
        assert np.array_equal(r["events"][j], [1, 1, 0])
        assert r["status"][j] & 1 and r["status"][j] & 4
        bins, ev, *_ = brute_force(r["traj_g"][j])
        assert np.array_equal(bins, r["bins"][j]) and np.array_equal(ev, r["events"][j])


def test_meal_draws(orc):
    t = W.with_(W.base_trial(), n_slots=4, prob=[1.0, 1.0, 1.0, 0.2])
    draws = np.array([orc.meals(t, p, d) for p in range(400) for d in range(10)])   # [n, slot, 4]
    assert np.all(draws[:, :3, 0] == 1.0)
    snack = draws[:, 3, 0].mean()
    assert abs(snack - 0.2) < 5 * np.sqrt(0.2 * 0.8 / len(draws))
    jit = draws[:, :, 3].ravel()
    assert jit.min() == -30 and jit.max() == 30 and np.all(jit == np.round(jit))
    counts = np.bincount((jit + 30).astype(int), minlength=61)
    assert stats.chisquare(counts).pvalue > 1e-4
    carbs = draws[:, :3, 2].ravel()
    assert abs(carbs.mean() - 50) < 5 * 10 / np.sqrt(carbs.size)
    assert abs(carbs.std() - 10) < 5 * 10 / np.sqrt(2 * carbs.size)
    mod = np.array([420, 720, 1080, 1260])
    assert np.array_equal(draws[:, :, 1], (mod[None, :] + draws[:, :, 3]) // 5)


def test_meals_enter_the_gut_in_their_interval(orc):
    t = W.noise_free(W.with_(W.base_trial(), n_patients=3, n_days=3, ctrl_kind=W.CTRL_OPEN))
    r = orc.simulate(t, n_traj=3, record_x=True, threads=3)
    for j in range(3):
        d1 = r["traj_x"][j][:, 0]
        fed = np.nonzero(np.diff(d1) > 0)[0]
        expect = sorted(day * 288 + int(kd) for day in range(3) for pres, kd, c, _ in orc.meals(t, j, day)
                        if pres and c > 0)
        assert list(fed) == expect


def test_pid_scripted(orc):
    t = W.base_trial()     # kp = 0.5, ki = 0.5/600, kd = 30 (relative to u_b), u_max = 3 u_b
    ub = 2.0
    y = np.full(50, 7.0)   # constant error e = +1
    u, integ = orc.pid_run(t, ub, y)
    k = np.arange(50)
    assert np.allclose(integ, 5.0 * (k + 1))
    assert np.allclose(u, ub * (1 + 0.5 + 0.5 / 600 * 5.0 * k))
    # a large error saturates: u == u_max and the integral freezes while saturated
    y = np.concatenate([np.full(5, 6.0), np.full(20, 12.0), np.full(5, 6.0)])
    u, integ = orc.pid_run(t, ub, y)
    assert np.all(u <= 3 * ub) and np.all(u >= 0)
    assert u[5] == 3 * ub
    assert np.all(integ[5:25] == integ[4])
    # falling measurement: derivative term drives u to 0 and clamps
    y = np.array([6.0, 6.0, 2.0, 2.0])
    u, integ = orc.pid_run(t, ub, y)
    assert u[2] == 0.0 and integ[2] == integ[1]


def test_reduce_quantiles_and_totals(orc):
    rng = np.random.default_rng(3)
    for n in (1, 2, 7, 100, 1001):
        K = 2016
        bins = rng.integers(0, 400, size=(n, 5)).astype(np.int32)
        r = {
            "bins": bins, "events": rng.integers(0, 9, size=(n, 3)).astype(np.int32),
            "sum_g": rng.uniform(0, 1e4, n), "min_g": np.round(rng.uniform(1, 5, n), 1),
            "argmin_k": rng.integers(0, K, n).astype(np.int32), "status": rng.integers(0, 8, n).astype(np.uint32),
            "K": K,
        }
        s = orc.reduce(r)
        for q, pct in zip(s["q_count"], (5, 25, 50, 75, 95)):
            assert q == np.percentile(bins[:, 2], pct, method="inverted_cdf")
        assert s["bins"] == list(bins.sum(0))
        assert s["events"] == list(r["events"].sum(0))
        w = np.lexsort((np.arange(n), r["min_g"]))[0]
        assert s["worst_patient"] == w and s["worst_k"] == r["argmin_k"][w]
        assert s["mean_bg"] == pytest.approx(r["sum_g"].sum() / (n * K), rel=1e-12)
        for b in range(3):
            assert s["status_count"][b] == np.sum((r["status"] >> b) & 1)
        # the same summary over the unflagged patients (status == 0) only
        ok = r["status"] == 0
        assert s["n_clean"] == ok.sum()
        assert s["bins_clean"] == list(bins[ok].sum(0))
        if ok.any():
            for q, pct in zip(s["q_count_clean"], (5, 25, 50, 75, 95)):
                assert q == np.percentile(bins[ok, 2], pct, method="inverted_cdf")
            assert s["mean_tir_clean"] == pytest.approx(bins[ok, 2].sum() / (ok.sum() * K), rel=1e-15)
            assert s["mean_bg_clean"] == pytest.approx(r["sum_g"][ok].sum() / (ok.sum() * K), rel=1e-12)
        else:
            assert s["q_count_clean"] == [0] * 5 and s["mean_tir_clean"] == 0.0
