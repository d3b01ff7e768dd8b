"""Batched heterogeneous arms in one persistent, graph-captured launch.

* every arm's per-patient record is bitwise identical to a single-arm launch of that
  arm (the batching changes scheduling only), for forced and autotuned block sizes;
* graph replays interleaved with other GPU work all give the first replay's result;
* an FP64 batch matches the FP64 oracle exactly (counts), with per-arm PID gains;
* the 64-arm workload (log-uniform sizes 1k-200k, 1-52 week horizons) runs in full and
  a sample of patients per arm agrees with the oracle.
"""
import os
import sys

import numpy as np
import pytest

from paper_2202_13927_amd import workloads as W

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
KEYS = ("bins", "events", "sum_g", "min_g", "sum_u", "argmin_k", "status")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_13927_amd import trial
    return trial


def small_arms(precision=W.FP32):
    base = W.with_(W.c2_fp32_pid(), precision=precision, pop_seed=9, noise_seed=9)
    spec = [(1000, 7, 1.0, 1.0, 1.0), (257, 28, 0.5, 1.5, 0.75), (3000, 2, 1.5, 0.5, 0.5),
            (64, 14, 0.75, 0.75, 1.5), (1, 6, 1.0, 0.5, 1.0), (700, 4, 1.5, 1.5, 1.5)]
    return [W.with_(base, arm_id=a, n_patients=n, n_days=d, kp=base["kp"] * mp, ki=base["ki"] * mi,
                    kd=base["kd"] * md) for a, (n, d, mp, mi, md) in enumerate(spec)]


def single(T, t):
    s, b = T.run(t)
    return T.to_host(b)


@pytest.mark.parametrize("block", [64, 512, 0])
def test_batch_equals_single_arm(T, block):
    arms = small_arms()
    _say(f"[gpu] batch of {len(arms)} arms, block {block}")
    bt = T.Batch(arms, block=block)
    try:
        bt.run()
        info = bt.info()
        _say("batch info", info)
        if block:
            assert info["block"] == block
        else:
            assert info["block"] in (64, 128, 256, 512) and all(v > 0 for v in info["tuned"].values())
        for t, b in zip(arms, bt.bufs):
            g = T.to_host(b)
            r = single(T, t)
            for k in KEYS:
                assert np.array_equal(g[k], r[k]), (t["arm_id"], k)
    finally:
        bt.close()


def test_batch_graph_replays(T):
    import torch
    arms = small_arms()
    bt = T.Batch(arms, block=128)
    try:
        bt.run()
        first = [T.to_host(b) for b in bt.bufs]
        for rep in range(3):
            x = torch.randn(1 << 20, device="cuda")           # eager work between replays
            torch.cuda.synchronize()
            for b in bt.bufs:
                b.metrics.zero_()
            bt.run()
            _ = (x * 2).sum().item()
            for f, b in zip(first, bt.bufs):
                g = T.to_host(b)
                for k in KEYS:
                    assert np.array_equal(g[k], f[k]), (rep, k)
    finally:
        bt.close()


def test_batch_fp64_matches_oracle(T, orc):
    arms = small_arms(precision=W.FP64)[:4]
    bt = T.Batch(arms, block=256)
    try:
        bt.run()
        for t, b in zip(arms, bt.bufs):
            g = T.to_host(b)
            o = orc.simulate(t, threads=THREADS, guard_rel=1e-9)
            ok = o["n_near"] == 0
            assert ok.mean() > 0.99
            for k in ("bins", "events", "argmin_k", "status"):
                assert np.array_equal(g[k][ok], o[k][ok]), (t["arm_id"], k)
            assert np.allclose(g["sum_g"], o["sum_g"], rtol=1e-9)
    finally:
        bt.close()


def test_c4_full_sampled(T, orc):
    arms = W.c4_arms()
    _say(f"[gpu] C4: {len(arms)} arms, {sum(t['n_patients'] for t in arms)} patients")
    bt = T.Batch(arms)
    try:
        bt.run()
        sums = bt.summaries()
        _say("C4 batch info", bt.info())
        dt = []
        for a in range(0, 64, 8):
            t, s, b = arms[a], sums[a], bt.bufs[a]
            assert s["n_patients"] == t["n_patients"] and sum(s["bins"]) == t["n_patients"] * s["n_samples"]
            g = T.to_host(b)
            for i in (0, t["n_patients"] - 1):
                o = orc.simulate(t, first=i, count=1, threads=1)
                assert g["status"][i] == o["status"][0]
                dt.append((int(g["bins"][i, 2]) - int(o["bins"][0, 2])) / s["n_samples"])
        dt = np.array(dt)
        _say("C4 sampled |dTIR| max", np.abs(dt).max())
        assert np.abs(dt).max() < 1e-2 and abs(dt.mean()) < 3e-3
    finally:
        bt.close()


def test_trial_a_vs_b_arms(T, orc):
    """The scenario comparison of Sec. IV-E as two arms of one batched launch: the same
    patients, meals and noise (same population seed and arm id) under the Northern-European
    protocol, trial B with the controller's basal rate at 50 %. Each arm equals its
    single-arm launch bit for bit; FP64 counts equal the oracle's; trial B delivers less
    insulin."""
    base = W.with_(W.c1_fp64_pid(), proto=W.PROTO_NORDIC, meal_cv=0.1, n_patients=200, n_days=14, pop_seed=12,
                   noise_seed=12)
    arms = [base, W.with_(base, basal_scale=0.5)]
    _say("[gpu] trial A vs B in one batched launch, 200 x 14 d FP64")
    bt = T.Batch(arms, block=128)
    try:
        bt.run()
        got = [T.to_host(b) for b in bt.bufs]
    finally:
        bt.close()
    for t, g in zip(arms, got):
        _, b = T.run(t)
        one = T.to_host(b)
        for k in KEYS:
            assert np.array_equal(g[k], one[k]), k
        o = orc.simulate(t, threads=THREADS, guard_rel=1e-9)
        ok = o["n_near"] == 0
        assert ok.mean() > 0.95
        for k in ("bins", "events", "argmin_k"):
            assert np.array_equal(g[k][ok], o[k][ok]), k
        assert np.allclose(g["sum_u"], o["sum_u"], rtol=1e-9)
    assert got[1]["sum_u"].sum() < got[0]["sum_u"].sum()


def test_scenarios_full_size_sampled(T, orc):
    """Trial A vs trial B at the benchmark's size and launch (two arms of 1,000,000 patients x
    364 days, Northern-European protocol, FP32, one autotuned batched launch): sampled patients
    of each arm against the oracle one by one; trial B delivers less insulin to every sampled
    patient and to the population."""
    a = W.nordic_year()
    arms = [a, W.with_(a, basal_scale=0.5)]
    _say("[gpu] trial A vs B at 2 x 1,000,000 x 364 d, one batched launch")
    bt = T.Batch(arms)
    try:
        bt.run()
        sums = bt.summaries()
        got = [T.to_host(b) for b in bt.bufs]
    finally:
        bt.close()
    n = a["n_patients"]
    idx = np.linspace(0, n - 1, 10).astype(int)
    for t, s, g in zip(arms, sums, got):
        K = s["n_samples"]
        assert s["n_patients"] == n and sum(s["bins"]) == n * K
        dt, du = [], []
        for i in idx:
            o = orc.simulate(t, first=int(i), count=1, threads=1)
            assert g["status"][i] == o["status"][0]
            dt.append((int(g["bins"][i, 2]) - int(o["bins"][0, 2])) / K)
            du.append(g["sum_u"][i] / o["sum_u"][0] - 1.0)
        dt, du = np.array(dt), np.array(du)
        _say("scenario arm", t.get("basal_scale", 1.0), "sampled |dTIR| max", np.abs(dt).max(),
             "insulin rel. diff. max", np.abs(du).max())
        assert np.abs(dt).max() < 5e-3 and abs(dt.mean()) < 2e-3
        assert np.abs(du).max() < 2e-2
    assert np.all(got[1]["sum_u"][idx] < got[0]["sum_u"][idx])
    assert sums[1]["mean_insulin"] < sums[0]["mean_insulin"] and sums[1]["mean_tir"] < sums[0]["mean_tir"]
