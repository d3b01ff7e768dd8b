"""GPU vs FP64 oracle parity through the C ABI (closed-loop Monte Carlo, Sec. III).

Bars (the tolerances the project states for this path):
* FP64 state (1,000 patients x 7 days): integer metrics exactly equal, sampled-glucose
  trajectories within 1e-4 relative (observed ~1e-12), sums within 1e-9 relative;
* FP32 state, noise-free: counts equal up to samples the oracle flags as lying within
  1e-4 (relative) of a range edge, for every patient whose PID never came within 1e-4
  u_b of a clamp edge (FP32 rounding can switch such a clamp); trajectories within 1e-4
  relative;
* FP32 state, stochastic (same Philox stream): population TIR within 0.1 pp;
* the reduction equals numpy over the per-patient records (exact integers).
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_2202_13927_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_13927_amd import trial as T
    return T


def run_gpu(T, trial, traj=0):
    _say(f"[gpu] n={trial['n_patients']} days={trial['n_days']} prec={trial['precision']} "
         f"sigma={trial['sigma_q1']} R={trial['cgm_var']} ctrl={trial['ctrl_kind']}")
    s, bufs = T.run(trial, traj_patients=traj)
    return s, T.to_host(bufs)


def numpy_summary(r):
    n, K = r["bins"].shape[0], r["K"]
    tir = r["bins"][:, 2]
    q = [int(np.percentile(tir, p, method="inverted_cdf")) for p in (5, 25, 50, 75, 95)]
    mg = np.where(np.isfinite(r["min_g"]), r["min_g"], np.inf)
    w = int(np.lexsort((np.arange(n), mg))[0])
    return {"bins": list(r["bins"].sum(0).astype(np.uint64)), "events": list(r["events"].sum(0)), "q_count": q,
            "worst_patient": w, "worst_k": int(r["argmin_k"][w])}


def test_population_matches_oracle(gpu, orc):
    t = W.with_(W.c1_fp64_pid(), n_patients=3000)
    _, g = run_gpu(gpu, W.with_(t, n_days=1))
    o = orc.sample_population(t)
    assert np.array_equal(g["params"][:, 17:], o[:, 17:])        # attempts, status
    assert np.allclose(g["params"][:, :17], o[:, :17], rtol=1e-13, atol=0)


def test_c1_fp64_exact(gpu, orc):
    t = W.c1_fp64_pid()
    s, g = run_gpu(gpu, t, traj=8)
    o = orc.simulate(t, n_traj=8, threads=THREADS, guard_rel=1e-9)
    assert np.all(o["n_near"] == 0)
    for k in ("bins", "events", "argmin_k", "status"):
        assert np.array_equal(g[k], o[k]), k
    for k in ("sum_g", "min_g", "sum_u"):
        assert np.allclose(g[k], o[k], rtol=1e-9, atol=0), k
    rel = np.abs(g["traj_g"] - o["traj_g"]) / np.abs(o["traj_g"])
    _say("C1 FP64 max rel traj error", rel.max())
    assert rel.max() < 1e-4
    assert np.allclose(g["traj_u"], o["traj_u"], rtol=1e-6, atol=1e-9)
    so = orc.reduce(o)
    assert s["bins"] == so["bins"] and s["events"] == so["events"] and s["q_count"] == so["q_count"]
    assert s["worst_patient"] == so["worst_patient"] and s["worst_k"] == so["worst_k"]
    assert s["mean_bg"] == pytest.approx(so["mean_bg"], rel=1e-12)
    assert s["mean_tir"] == pytest.approx(so["mean_tir"], rel=0)


def _fp32_slice(noisy):
    t = W.with_(W.c2_fp32_pid(), n_patients=4099)      # several blocks and a ragged tail
    return t if noisy else W.noise_free(t)


def test_c2_noise_free_fp32(gpu, orc):
    t = _fp32_slice(False)
    s, g = run_gpu(gpu, t, traj=8)
    o = orc.simulate(t, n_traj=8, threads=THREADS, guard_rel=1e-4)
    d = np.abs(g["bins"].astype(np.int64) - o["bins"]).sum(1)
    near_edge = d <= 2 * o["n_near"]          # each flagged sample can move one count
    near_clamp = o["ctrl_margin"] <= 1e-4     # a PID clamp decision FP32 rounding can switch
    _say("FP32 noise-free: patients with any count difference", int((d > 0).sum()), "of", len(d),
         "| not explained by flagged samples", int((~near_edge).sum()),
         "| of those near a clamp edge", int((~near_edge & near_clamp).sum()))
    assert np.all(near_edge | near_clamp)
    assert np.mean(d == 0) > 0.95
    exact = (o["n_near"] == 0) & ~near_clamp
    assert np.array_equal(g["bins"][exact], o["bins"][exact])
    assert np.array_equal(g["events"][exact], o["events"][exact])
    assert np.allclose(g["sum_g"][~near_clamp], o["sum_g"][~near_clamp], rtol=1e-4)
    tr = ~near_clamp[:8]
    rel = np.abs(g["traj_g"][tr] - o["traj_g"][tr]) / np.abs(o["traj_g"][tr])
    _say("FP32 noise-free max rel traj error", rel.max())
    assert rel.max() < 1e-4
    tir_g = g["bins"][:, 2].sum() / g["bins"].sum()
    tir_o = o["bins"][:, 2].sum() / o["bins"].sum()
    assert abs(tir_g - tir_o) < 1e-3


def test_c2_stochastic_fp32(gpu, orc):
    t = _fp32_slice(True)
    s, g = run_gpu(gpu, t, traj=4)
    o = orc.simulate(t, n_traj=4, threads=THREADS)
    K = o["K"]
    dtir = (g["bins"][:, 2].astype(np.int64) - o["bins"][:, 2]) / K
    _say("FP32 stochastic per-patient |dTIR| max", np.abs(dtir).max(), "mean", np.abs(dtir).mean())
    assert abs(dtir.mean()) < 1e-3                       # population TIR within 0.1 pp
    assert np.mean(np.abs(dtir) <= 1e-3) > 0.95           # most patients within 0.1 pp themselves
    assert np.array_equal(g["status"], o["status"])
    rel = np.abs(g["traj_g"][:, :288] - o["traj_g"][:, :288]) / np.abs(o["traj_g"][:, :288])
    assert rel.max() < 1e-3                                # first day, before any branch can diverge


def test_reduction_matches_numpy(gpu):
    t = W.with_(W.c2_fp32_pid(), n_patients=50_001, n_days=3)
    s, g = run_gpu(gpu, t)
    ref = numpy_summary(g)
    assert [int(v) for v in s["bins"]] == [int(v) for v in ref["bins"]]
    assert [int(v) for v in s["events"]] == [int(v) for v in ref["events"]]
    assert s["q_count"] == ref["q_count"]
    assert s["worst_patient"] == ref["worst_patient"] and s["worst_k"] == ref["worst_k"]
    assert s["mean_bg"] == pytest.approx(g["sum_g"].sum() / (t["n_patients"] * g["K"]), rel=1e-12)
    assert all(sum(s["bins"]) == t["n_patients"] * g["K"] for _ in [0])


def test_deterministic(gpu):
    t = W.with_(W.c2_fp32_pid(), n_patients=20_000, n_days=2)
    _, a = run_gpu(gpu, t)
    _, b = run_gpu(gpu, t)
    for k in ("bins", "events", "sum_g", "min_g", "sum_u", "argmin_k", "status"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("case", ["one_patient", "ragged", "no_meals", "no_jitter", "cv0", "open_loop",
                                  "min_basal", "snack", "infeasible_nominal"])
def test_edge_cases_fp64(gpu, orc, case):
    t = W.with_(W.c1_fp64_pid(), n_patients=300, n_days=2)
    t = {
        "one_patient": lambda: W.with_(t, n_patients=1),
        "ragged": lambda: W.with_(t, n_patients=257),
        "no_meals": lambda: W.with_(t, n_slots=0),
        "no_jitter": lambda: W.with_(t, jitter=0),
        "cv0": lambda: W.with_(t, cv=0.0),
        "open_loop": lambda: W.with_(t, ctrl_kind=W.CTRL_OPEN, u_rel=1.3),
        "min_basal": lambda: W.with_(t, pop_flags=1),
        "snack": lambda: W.with_(t, n_slots=4, prob=[1.0, 1.0, 0.5, 0.2]),
        "infeasible_nominal": lambda: W.with_(t, n_patients=64, cv=1e-9,
                                              nominal=[W.NOMINAL[0], W.NOMINAL[0] * 1.5, *W.NOMINAL[2:]]),
    }[case]()
    s, g = run_gpu(gpu, t)
    o = orc.simulate(t, threads=THREADS, guard_rel=1e-9)
    assert np.array_equal(g["status"], o["status"])
    if case == "infeasible_nominal":   # non-finite from the start: lowest range, endless low runs
        assert np.all(g["status"] & 4) and np.all(g["status"] & 1)
        for k in ("bins", "events"):
            assert np.array_equal(g[k], o[k]), k
        return
    ok = o["n_near"] == 0
    assert ok.mean() > 0.99
    for k in ("bins", "events", "argmin_k"):
        assert np.array_equal(g[k][ok], o[k][ok]), k
    assert np.allclose(g["sum_g"], o["sum_g"], rtol=1e-9)


def test_full_size_c3_sampled(gpu, orc):
    """1,000,000 patients x 364 days in the benchmark's launch configuration; a sample of
    patients spread over the index range is recomputed by the oracle one by one."""
    t = W.c3_paper_scale()
    s, g = run_gpu(gpu, t)
    K = g["K"]
    assert K == 104_832
    assert np.all(g["bins"].sum(1) == K)
    assert s["n_patients"] == 1_000_000 and sum(s["bins"]) == 1_000_000 * K
    idx = np.linspace(0, t["n_patients"] - 1, 24).astype(int)
    dt = []
    for i in idx:
        o = orc.simulate(t, first=int(i), count=1, threads=1)
        assert np.array_equal(g["params"][i, 17:], o["params"][0, 17:])
        assert np.allclose(g["params"][i, :17], o["params"][0, :17], rtol=1e-13)
        dt.append((int(g["bins"][i, 2]) - int(o["bins"][0, 2])) / K)
        assert g["status"][i] == o["status"][0]
    dt = np.array(dt)
    _say("C3 sampled |dTIR| max", np.abs(dt).max())
    assert np.abs(dt).max() < 5e-3
    assert abs(dt.mean()) < 2e-3
    assert 0.3 < s["mean_tir"] < 0.95 and math.isfinite(s["mean_bg"])


def test_population_slices_equal_whole(gpu):
    """A population run as two slices (first_patient 0 and 600) gives, patient by patient,
    exactly the results of the whole run: every draw is keyed by the global patient index."""
    t = W.with_(W.base_trial(), n_patients=1000, n_days=2, precision=W.FP32, pop_seed=3, noise_seed=4)
    _say("[gpu] population slices vs whole, 1000 x 2 d FP32")
    _, b = gpu.run(t)
    whole = gpu.to_host(b)
    parts = []
    for first, n in ((0, 600), (600, 400)):
        _, b = gpu.run(W.with_(t, first_patient=first, n_patients=n))
        parts.append(gpu.to_host(b))
    for k in ("bins", "events", "sum_g", "min_g", "argmin_k", "sum_u", "status", "params"):
        assert np.array_equal(whole[k], np.concatenate([p[k] for p in parts])), k


def test_nordic_fp64_matches_oracle(gpu, orc):
    """The paper's Northern-European protocol over a whole year (all four seasons, vacation
    weeks, movie and late nights), FP64 state: the GPU's counts equal the oracle's on every
    patient with no sample near a range edge, trajectories agree to rounding."""
    t = W.with_(W.c1_fp64_pid(), proto=W.PROTO_NORDIC, meal_cv=0.1, n_patients=130, n_days=364)
    s, g = run_gpu(gpu, t, traj=4)
    o = orc.simulate(t, n_traj=4, threads=THREADS, guard_rel=1e-9)
    assert np.array_equal(g["status"], o["status"])
    ok = o["n_near"] == 0
    assert ok.mean() > 0.95
    for k in ("bins", "events", "argmin_k"):
        assert np.array_equal(g[k][ok], o[k][ok]), k
    assert np.allclose(g["sum_g"], o["sum_g"], rtol=1e-9)
    rel = np.abs(g["traj_g"] - o["traj_g"]) / np.abs(o["traj_g"])
    _say("Nordic FP64 max rel traj error", rel.max())
    assert rel.max() < 1e-4


def test_nordic_fp32_stochastic(gpu, orc):
    """FP32 state on the same Philox stream: population TIR within 0.1 pp of the oracle."""
    t = W.with_(W.nordic_year(), n_patients=2053, n_days=56)
    s, g = run_gpu(gpu, t)
    o = orc.simulate(t, threads=THREADS)
    dtir = (g["bins"][:, 2].astype(np.int64) - o["bins"][:, 2]) / o["K"]
    _say("Nordic FP32 per-patient |dTIR| max", np.abs(dtir).max(), "mean", dtir.mean())
    assert abs(dtir.mean()) < 1e-3
    assert np.mean(np.abs(dtir) <= 1e-3) > 0.95
    assert np.array_equal(g["status"], o["status"])


def test_nordic_full_size_sampled(gpu, orc):
    """The Northern-European year at the benchmark's size and launch (1,000,000 patients x 364
    days, FP32, PID): patients spread over the index range are recomputed by the oracle one by
    one. The same launch with the population BG per sample on gives the same per-patient
    records, counts every sample once in its pooled bins, its mean curve averages to the
    summary's mean BG, and the upper curve of the span ends at K."""
    t = W.nordic_year()
    s, g = run_gpu(gpu, t)
    n, K = t["n_patients"], g["K"]
    assert K == 104_832 and s["n_patients"] == n and sum(s["bins"]) == n * K
    dt = []
    for i in np.linspace(0, n - 1, 16).astype(int):
        o = orc.simulate(t, first=int(i), count=1, threads=1)
        assert g["status"][i] == o["status"][0]
        dt.append((int(g["bins"][i, 2]) - int(o["bins"][0, 2])) / K)
    dt = np.array(dt)
    _say("Nordic full-size sampled |dTIR| max", np.abs(dt).max(), "mean", dt.mean())
    assert np.abs(dt).max() < 5e-3 and abs(dt.mean()) < 2e-3
    _say("[gpu] the same launch with the population BG per sample")
    b = gpu.TrialBuffers(t, popbg=True)
    gpu.run(t, bufs=b)
    p = gpu.to_host(b)
    for k in ("bins", "events", "sum_g", "min_g", "argmin_k", "sum_u", "status"):
        assert np.array_equal(p[k], g[k]), k
    assert int(p["pop_hist"].sum()) == n * K
    assert p["pop_mean"].mean() == pytest.approx(s["mean_bg"], rel=1e-9)
    assert np.all(p["pop_min"] <= p["pop_mean"]) and np.all(p["pop_mean"] <= p["pop_max"])
    assert p["pop_min"].min() == pytest.approx(float(np.nanmin(g["min_g"])), rel=1e-12)
    assert p["span_max"][-1] == K and np.all(np.diff(p["span_min"]) >= 0) and np.all(p["span_min"] <= p["span_max"])


def test_nordic_rejects_bad_settings(gpu):
    """Invalid protocol settings are refused before any device work."""
    from paper_2202_13927_amd import vct
    t = W.with_(W.c1_fp64_pid(), proto=W.PROTO_NORDIC, n_patients=64, n_days=1)
    bufs = gpu.TrialBuffers(t)
    pop = gpu.create_population(t, bufs)
    try:
        for bad in ({"jitter": 41}, {"meal_cv": -0.1}, {"meal_cv": 1.5}, {"proto": 7}):
            with pytest.raises(vct.VctError) as e:
                gpu.simulate(W.with_(t, **bad), pop, bufs)
            assert e.value.code == vct.VCT_EINVAL, bad
        gpu.simulate(W.with_(t, jitter=40, meal_cv=1.0), pop, bufs)    # the limits themselves are valid
    finally:
        vct.vct_destroy_population(pop)


def test_worst_patient_replay(gpu):
    """The worst-case patient of a population run, re-simulated alone from its counters,
    reproduces its record bit for bit; its trajectory reaches min G at argmin_k, and the
    range counts recomputed from the trajectory equal the streamed counts."""
    t = W.with_(W.c2_fp32_pid(), n_patients=3000, n_days=3)
    s, b = gpu.run(t)
    whole = gpu.to_host(b)
    w = s["worst_patient"]
    _say("[gpu] replay of worst patient", w, "min G", s["worst_min_g"])
    r = gpu.replay_patient(t, w)
    for k in ("bins", "events", "sum_g", "min_g", "argmin_k", "sum_u", "status"):
        assert np.array_equal(r[k][0], whole[k][w]), k
    g = r["traj_g"][0]
    assert g.min() == whole["min_g"][w] and int(np.argmin(g)) == whole["argmin_k"][w] == s["worst_k"]
    g32 = g.astype(np.float32)
    edges = [np.float32(3.0), np.float32(3.9), np.float32(10.0), np.float32(13.9)]
    counts = [int((g32 < edges[0]).sum()), int(((g32 >= edges[0]) & (g32 < edges[1])).sum()),
              int(((g32 >= edges[1]) & (g32 <= edges[2])).sum()), int(((g32 > edges[2]) & (g32 <= edges[3])).sum()),
              int((g32 > edges[3]).sum())]
    assert counts == [int(v) for v in whole["bins"][w]]


def test_basal_scale_needs_pid_or_open_loop(gpu):
    """basal_scale != 1 is refused for the MPC (before any device work)."""
    from paper_2202_13927_amd import vct
    t = W.with_(W.c5_mpc(), n_patients=64, n_days=1)
    bufs = gpu.TrialBuffers(t)
    pop = gpu.create_population(t, bufs)
    try:
        gpu.mpc_setup(t, pop, bufs)
        with pytest.raises(vct.VctError) as e:
            gpu.simulate(W.with_(t, basal_scale=0.5), pop, bufs)
        assert e.value.code == vct.VCT_ENOTSUP
        with pytest.raises(vct.VctError) as e:
            gpu.simulate(W.with_(t, ctrl_kind=W.CTRL_PID, basal_scale=0.0), pop, bufs)
        assert e.value.code == vct.VCT_EINVAL
    finally:
        vct.vct_destroy_population(pop)


def _pop_hist(traj_g):
    """Bins of 0.1 mmol/L: 0 below 0, 1 + floor(10 G) for 0 <= G < 40, 401 at or above 40."""
    g = np.asarray(traj_g, np.float64).ravel()
    g = np.where(np.isnan(g), -1.0, g)          # NaN counts in bin 0
    b = np.where(g >= 0.0, 1 + np.floor(np.minimum(g * 10.0, 400.5)).astype(np.int64), 0)
    return np.bincount(b, minlength=402).astype(np.uint64)


def _span(traj_g):
    """Over the patients, min and max of the number of samples with G below (b + 1) / 2
    mmol/L (bin floor(2 G) clamped to 0..49, cumulative)."""
    g = np.asarray(traj_g, np.float64)
    b = np.where(g >= 0.0, np.floor(np.minimum(g * 2.0, 49.5)).astype(np.int64), 0)
    counts = np.stack([(b == q).sum(1) for q in range(50)], axis=1).cumsum(1)
    return counts.min(0), counts.max(0)


def _pop_from_traj(traj_g):
    """Sum of round(G 2^32), min and max per sample over the patients whose G is finite
    (NaN where none is), and the count of the others."""
    g = np.asarray(traj_g, np.float64)
    fin = np.isfinite(g)
    s = np.rint(np.where(fin, g, 0.0) * 4294967296.0).astype(np.int64).sum(0)
    any_fin = fin.any(0)
    mn = np.where(any_fin, np.where(fin, g, np.inf).min(0), np.nan)
    mx = np.where(any_fin, np.where(fin, g, -np.inf).max(0), np.nan)
    return s, mn, mx, (~fin).sum(0)


@pytest.mark.parametrize("case", ["pid45", "pid64", "mpc45", "mlp45"])
def test_population_bg_equals_trajectories(gpu, case):
    """Population BG per sample (Sec. III-C) equals what the patients' own trajectories give:
    the integer sum of round(G 2^32) exactly, min and max exactly, for a full wave and a
    ragged one, in the plain, MPC and learned-controller kernels."""
    import torch
    from paper_2202_13927_amd import policy
    kind, n = case[:3], int(case[3:])
    base = {"pid": W.c2_fp32_pid(), "mpc": W.c5_mpc(), "mlp": W.c5_mlp()}[kind]
    t = W.with_(base, n_patients=n, n_days=2, precision=W.FP32)
    blob = None
    if kind == "mlp":
        pol = policy.Policy(batch=64)
        pol.load(W.synthetic_policy_net(71))
        blob = pol.blob
    _say(f"[gpu] population BG, {case}")
    b1 = gpu.TrialBuffers(t, popbg=True)
    gpu.run(t, bufs=b1, mlp_blob=blob)
    p = gpu.to_host(b1)
    b2 = gpu.TrialBuffers(t, traj_patients=n)
    gpu.run(t, bufs=b2, mlp_blob=blob)
    s, mn, mx, nf = _pop_from_traj(gpu.to_host(b2)["traj_g"])
    assert np.array_equal(p["pop_sum_q32"], s) and np.array_equal(p["pop_nonfinite"], nf) and not nf.any()
    assert np.array_equal(p["pop_min"], mn) and np.array_equal(p["pop_max"], mx)
    assert np.allclose(p["pop_mean"], s / (n * 4294967296.0), rtol=1e-15)
    tg = gpu.to_host(b2)["traj_g"]
    assert np.array_equal(p["pop_hist"], _pop_hist(tg))
    smin, smax = _span(tg)
    assert np.array_equal(p["span_min"], smin) and np.array_equal(p["span_max"], smax)


def test_population_bg_infeasible_fp64(gpu, orc):
    """A population whose every patient has no finite basal state (the infeasible nominal
    case): every G is NaN from the first sample, in the oracle and on the GPU. The
    population curves leave such patients out and count them: the count is n at every
    sample, the sum 0, mean, min and max NaN; the BG distribution holds them in bin 0."""
    t = W.with_(W.c1_fp64_pid(), n_patients=64, n_days=2, cv=1e-9,
                nominal=[W.NOMINAL[0], W.NOMINAL[0] * 1.5, *W.NOMINAL[2:]])
    _say("[gpu] population BG, infeasible population, 64 x 2 d FP64")
    b = gpu.TrialBuffers(t, popbg=True)
    gpu.run(t, bufs=b)
    p = gpu.to_host(b)
    o = orc.simulate(t, n_traj=64, threads=THREADS)
    s, mn, mx, nf = _pop_from_traj(o["traj_g"])
    assert np.all(nf == 64)
    assert np.array_equal(p["pop_nonfinite"], nf) and np.array_equal(p["pop_sum_q32"], s)
    assert np.all(np.isnan(p["pop_mean"])) and np.all(np.isnan(p["pop_min"])) and np.all(np.isnan(p["pop_max"]))
    assert p["pop_hist"][0] == 64 * o["K"] and int(p["pop_hist"].sum()) == 64 * o["K"]
    assert np.array_equal(p["status"], o["status"])


@pytest.mark.parametrize("prec", [W.FP64, W.FP32])
def test_population_bg_mixed_nonfinite(gpu, prec):
    """Patients whose state turns non-finite part-way (their insulin elimination rate k_e
    replaced by NaN after the population is drawn) beside ordinary ones, in a ragged last wave: the
    population curves equal what the trajectories give with those patients left out of the
    sum, min and max at each sample they are not finite, and counted there."""
    from paper_2202_13927_amd import vct
    n = 45                 # trajectories are recorded for at most 64 patients
    t = W.with_(W.c1_fp64_pid(), n_patients=n, n_days=1, precision=prec)
    bad = np.arange(n) % 3 == 0
    runs = []
    for popbg in (True, False):
        b = gpu.TrialBuffers(t, popbg=popbg, traj_patients=0 if popbg else n)
        pop = gpu.create_population(t, b)
        try:
            rows = b.params.view(vct.VCT_NPARAM_ROWS, n)
            rows[9, bad.nonzero()[0].tolist()] = float("nan")    # k_e: the basal state stays finite
            _say(f"[gpu] population BG, mixed non-finite, {n} x 1 d, prec {prec}, popbg {popbg}")
            gpu.simulate(t, pop, b)
        finally:
            vct.vct_destroy_population(pop)
        runs.append(gpu.to_host(b))
    p, tr = runs
    s, mn, mx, nf = _pop_from_traj(tr["traj_g"])
    assert nf.max() == bad.sum() and nf[-1] == bad.sum() and nf.min() < nf.max()   # turns non-finite part-way
    assert np.array_equal(p["pop_nonfinite"], nf) and np.array_equal(p["pop_sum_q32"], s)
    assert np.array_equal(p["pop_min"], mn) and np.array_equal(p["pop_max"], mx)
    assert np.allclose(p["pop_mean"], s / ((n - nf) * 4294967296.0), rtol=1e-15)
    assert np.all(np.isfinite(p["pop_mean"]))
    assert np.array_equal(p["pop_hist"], _pop_hist(tr["traj_g"]))
    assert np.all(p["status"][bad] & 1) and not np.any(p["status"][~bad] & 1)   # the non-finite bit


def test_population_bg_matches_oracle(gpu, orc):
    t = W.with_(W.c1_fp64_pid(), n_patients=3000, n_days=2)
    _say("[gpu] population BG vs oracle, 3000 x 2 d FP64")
    b = gpu.TrialBuffers(t, popbg=True)
    gpu.run(t, bufs=b)
    p = gpu.to_host(b)
    o = orc.simulate(t, n_traj=3000, threads=THREADS)
    s, mn, mx, nf = _pop_from_traj(o["traj_g"])
    assert not nf.any() and not p["pop_nonfinite"].any()
    assert np.allclose(p["pop_mean"], s / (3000 * 4294967296.0), rtol=1e-9)
    assert np.allclose(p["pop_min"], mn, rtol=1e-9) and np.allclose(p["pop_max"], mx, rtol=1e-9)
    assert np.all(p["pop_min"] <= p["pop_mean"]) and np.all(p["pop_mean"] <= p["pop_max"])
    h = _pop_hist(o["traj_g"]).astype(np.int64)
    assert int(p["pop_hist"].sum()) == 3000 * o["K"]
    # a value within rounding of a bin edge may land on either side (every patient starts at
    # G* = 6.0 exactly, an edge): each such value can move one count between two bins
    g10 = np.asarray(o["traj_g"], np.float64).ravel() * 10.0
    near = int((np.abs(g10 - np.rint(g10)) < 1e-8).sum())
    diff = int(np.abs(p["pop_hist"].astype(np.int64) - h).sum())
    _say("   histogram: counts moved", diff, "values near an edge", near)
    assert diff <= 2 * near
    smin, smax = _span(o["traj_g"])
    g2 = np.asarray(o["traj_g"], np.float64) * 2.0
    near2 = int((np.abs(g2 - np.rint(g2)) < 1e-8).sum())
    assert np.abs(p["span_min"] - smin).max() <= near2 and np.abs(p["span_max"] - smax).max() <= near2
    assert p["span_max"][-1] == o["K"] and np.all(np.diff(p["span_min"]) >= 0)
