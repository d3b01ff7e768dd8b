"""The model extensions and the dual-hormone AP on the GPU against the FP64 oracle
(Sec. II-B exercise sessions, Sec. IV-B glucagon and exercise sub-models, Sec. IV-C AP).

Bars: FP64 state -- integer metrics equal, sums and delivered doses within 1e-9 relative,
sampled-glucose trajectories within 1e-9; FP32 state, stochastic -- population TIR within
0.1 pp and the population's doses within 0.5 %; at the benchmark's size (1,000,000 x 364 d,
one launch) sampled patients against the oracle one by one.
"""
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


def _run(T, t, traj=0):
    _say(f"[gpu] extended model n={t['n_patients']} days={t['n_days']} prec={t['precision']} ctrl={t['ctrl_kind']} "
         f"exercise={t['exercise']}")
    s, bufs = T.run(t, traj_patients=traj)
    return s, T.to_host(bufs)


@pytest.mark.parametrize("ctrl", [W.CTRL_DUAL, W.CTRL_PID])
def test_ext_fp64_matches_oracle(gpu, orc, ctrl):
    t = W.with_(W.dual_hormone_year(), n_patients=300, n_days=14, precision=W.FP64, ctrl_kind=ctrl)
    if ctrl == W.CTRL_PID:
        t = W.with_(t, kp=0.5, ki=0.5 / 600, kd=30.0)
    s, g = _run(gpu, t, traj=8)
    o = orc.simulate(t, n_traj=8, threads=THREADS, guard_rel=1e-9)
    assert np.all(o["n_near"] == 0)
    for k in ("bins", "events", "argmin_k", "status"):
        assert np.array_equal(g[k], o[k]), k
    for k in ("sum_g", "min_g", "sum_u"):
        assert np.allclose(g[k], o[k], rtol=1e-9, atol=0), k
    assert np.allclose(g["doses"], o["doses"], rtol=1e-9, atol=1e-9)
    rel = np.abs(g["traj_g"] - o["traj_g"]) / np.abs(o["traj_g"])
    _say("   max rel traj error", rel.max(), "glucagon ug/patient/day", o["doses"][:, 2].mean() / t["n_days"])
    assert rel.max() < 1e-9
    assert np.allclose(g["traj_u"], o["traj_u"], rtol=1e-9, atol=1e-9)
    if ctrl == W.CTRL_DUAL:
        assert o["doses"][:, 1].sum() > 0 and o["doses"][:, 2].sum() > 0   # boluses and glucagon occur
    else:
        assert np.all(g["doses"][:, 1:] == 0.0)
    so = orc.reduce(o)
    assert s["bins"] == so["bins"] and s["q_count"] == so["q_count"]


def test_dual_fp32_stochastic(gpu, orc):
    t = W.with_(W.dual_hormone_year(), n_patients=4099, n_days=14)
    s, g = _run(gpu, t)
    o = orc.simulate(t, threads=THREADS)
    K = o["K"]
    tir_g, tir_o = g["bins"][:, 2].sum() / (t["n_patients"] * K), o["bins"][:, 2].sum() / (t["n_patients"] * K)
    dtir = (g["bins"][:, 2].astype(np.int64) - o["bins"][:, 2]) / K
    dd = g["doses"].sum(0) / o["doses"].sum(0) - 1.0
    _say("   dual FP32: TIR", tir_g, "oracle", tir_o, "| per-patient |dTIR| max", np.abs(dtir).max(),
         "| doses rel diff", dd)
    assert abs(tir_g - tir_o) < 1e-3
    assert np.mean(np.abs(dtir) <= 1e-3) > 0.95
    assert np.all(np.abs(dd) < 5e-3)
    assert np.array_equal(g["status"], o["status"])


def test_dual_full_size_sampled(gpu, orc):
    """The dual-hormone year at the benchmark's size and launch (1,000,000 x 364 d, FP32):
    patients spread over the index range against the oracle one by one."""
    import concurrent.futures as cf
    t = W.dual_hormone_year()
    assert (t["n_patients"], t["n_days"]) == (1_000_000, 364)
    s, g = _run(gpu, t)
    idx = np.linspace(0, t["n_patients"] - 1, 32).astype(int)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(lambda i: orc.simulate(t, first=int(i), count=1, threads=1), idx))
    K = g["K"]
    dt, dg = [], []
    for i, o in zip(idx, res):
        assert g["status"][i] == o["status"][0], i
        dt.append((int(g["bins"][i, 2]) - int(o["bins"][0, 2])) / K)
        dg.append(g["doses"][i] - o["doses"][0])
    dt = np.array(dt)
    _say("   sampled |dTIR| max", np.abs(dt).max(), "mean", dt.mean(), "| population TIR", s["mean_tir"],
         "| glucagon ug/day", g["doses"][:, 2].mean() / 364)
    assert np.abs(dt).max() < 5e-3 and abs(dt.mean()) < 1e-3
    assert s["n_patients"] == t["n_patients"] and sum(s["bins"]) == t["n_patients"] * K


def test_dual_slices_equal_whole(gpu):
    """The dual-hormone AP on the extended model with exercise: one patient alone, a ragged
    slice and the rest give, patient by patient, the whole run's results and doses bit for
    bit (every draw, the arrangement and the sessions keyed by the global patient index)."""
    t = W.with_(W.dual_hormone_year(), n_patients=130, n_days=14)
    _, whole = _run(gpu, t)
    parts = [_run(gpu, W.with_(t, first_patient=f, n_patients=n))[1] for f, n in ((0, 1), (1, 65), (66, 64))]
    for k in ("bins", "events", "sum_g", "min_g", "argmin_k", "sum_u", "status", "doses"):
        assert np.array_equal(whole[k], np.concatenate([p[k] for p in parts])), k


def test_ext_rejects_unsupported_settings(gpu):
    from paper_2202_13927_amd import trial as T, vct
    t = W.with_(W.dual_hormone_year(), n_patients=64, n_days=1)
    bufs = T.TrialBuffers(t)
    pop = T.create_population(t, bufs)
    try:
        cases = [
            (W.with_(t, model_ext=0), vct.VCT_EINVAL),                      # the AP needs the extensions
            (W.with_(t, ctrl_kind=W.CTRL_PID, model_ext=1, proto=W.PROTO_SLOTS), vct.VCT_EINVAL),  # exercise: Nordic
            (W.with_(t, glu_enter=6.0, glu_exit=5.0), vct.VCT_EINVAL),
            (W.with_(t, icr_rule=0.0), vct.VCT_EINVAL),
            (W.with_(t, tau_n=0.0), vct.VCT_EINVAL),
            (W.with_(t, exercise_hrr=1.5), vct.VCT_EINVAL),
        ]
        for bad, code in cases:
            with pytest.raises(vct.VctError) as e:
                T.simulate(bad, pop, bufs)
            assert e.value.code == code, bad
        # the MPC on the extended model is not supported
        tm = W.with_(t, ctrl_kind=W.CTRL_MPC, exercise=0)
        bm = T.TrialBuffers(tm)
        T.mpc_setup(W.with_(tm, model_ext=0), pop, bm)
        with pytest.raises(vct.VctError) as e:
            T.simulate(tm, pop, bm)
        assert e.value.code == vct.VCT_ENOTSUP
        # doses need the extensions
        tc = W.with_(t, model_ext=0, exercise=0, ctrl_kind=W.CTRL_PID)
        sim = vct.sim_settings(tc, bufs.metrics, doses_dev=bufs.doses)
        with pytest.raises(vct.VctError) as e:
            vct.vct_simulate(pop, vct.protocol(tc), vct.controller(tc), sim)
        assert e.value.code == vct.VCT_EINVAL
    finally:
        vct.vct_destroy_population(pop)
