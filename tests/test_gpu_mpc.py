"""GPU linear MPC vs the FP64 oracle.

* setup (FP64): every per-patient matrix equals the oracle's (1e-9 relative);
* FP64 closed loop: counts exactly equal, glucose trajectories within 1e-6 relative;
* FP32 closed loop (the working precision): population TIR within 0.1 pp, the first day's
  insulin trajectory within 1e-3 relative.
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
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_13927_amd import trial
    return trial


def mpc_trial(**kw):
    return W.with_(W.c5_mpc(), **{"n_patients": 300, "n_days": 2, "precision": W.FP64, **kw})


def test_mpc_setup_matches_oracle(T, orc):
    t = mpc_trial()
    _say("[gpu] MPC setup FP64, 300 patients")
    bufs = T.TrialBuffers(t)
    pop = T.create_population(t, bufs)
    T.mpc_setup(t, pop, bufs)
    g = T.mpc_to_host(bufs, W.FP64)
    params = T.to_host(bufs)["params"]
    for j in range(0, 300, 23):
        o = orc.mpc_setup(t, params[j])
        assert np.allclose(g["A"][j], o["A"].ravel(), rtol=1e-9, atol=1e-14)
        for k in ("B", "E", "K", "h", "gd", "g1"):
            assert np.allclose(g[k][j], o[k], rtol=1e-9, atol=1e-15), k
        assert np.allclose(g["Gx"][j], o["Gx"].ravel(), rtol=1e-9, atol=1e-15)
        assert g["step"][j, 0] == pytest.approx(o["step"], rel=1e-9)
        assert g["rho_p"][j, 0] == pytest.approx(o["rho_p"], rel=1e-12)
        assert g["umax"][j, 0] == pytest.approx(o["umax"], rel=1e-12)
        assert np.allclose(g["Fbar"][j], o["F"].mean(0), rtol=1e-9, atol=1e-15)
        assert g["wbar"][j, 0] == pytest.approx(o["w"].mean(), rel=1e-9)


def test_mpc_fp64_closed_loop(T, orc):
    t = mpc_trial()
    _say("[gpu] MPC FP64 closed loop 300 x 2 d")
    s, bufs = T.run(t, traj_patients=8)
    g = T.to_host(bufs)
    o = orc.simulate(t, n_traj=8, threads=THREADS, guard_rel=1e-9)
    ok = o["n_near"] == 0
    assert ok.mean() > 0.99
    for k in ("bins", "events", "argmin_k", "status"):
        assert np.array_equal(g[k][ok], o[k][ok]), k
    rel = np.abs(g["traj_g"] - o["traj_g"]) / np.abs(o["traj_g"])
    _say("MPC FP64 max rel traj error", rel.max())
    assert rel.max() < 1e-6
    assert np.allclose(g["traj_u"], o["traj_u"], rtol=1e-6, atol=1e-9)


def test_mpc_fp32_closed_loop(T, orc):
    t = mpc_trial(n_patients=1029, n_days=3, precision=W.FP32)
    _say("[gpu] MPC FP32 closed loop 1029 x 3 d")
    s, bufs = T.run(t, traj_patients=4)
    g = T.to_host(bufs)
    o = orc.simulate(t, n_traj=4, threads=THREADS)
    K = o["K"]
    dtir = (g["bins"][:, 2].astype(np.int64) - o["bins"][:, 2]) / K
    _say("MPC FP32 |dTIR| max", np.abs(dtir).max(), "mean", dtir.mean())
    assert abs(dtir.mean()) < 1e-3
    assert np.mean(np.abs(dtir) <= 5e-3) > 0.95
    rel = np.abs(g["traj_u"][:, :288] - o["traj_u"][:, :288]) / np.maximum(np.abs(o["traj_u"][:, :288]), 1e-3)
    _say("MPC FP32 first-day max rel u error", rel.max())
    assert rel.max() < 1e-3
