"""Run one trial end to end through the C ABI: torch allocates the device buffers,
the HIP library does every step (population, closed-loop simulation, reduction).
"""
from __future__ import annotations

import torch

from . import vct
from .workloads import samples_per_day


class TrialBuffers:
    """Caller-owned device buffers of one trial (the library only borrows them)."""

    def __init__(self, trial: dict, device="cuda", traj_patients: int = 0, popbg: bool = False):
        n = int(trial["n_patients"])
        self.n = n
        self.K = int(trial["n_days"]) * samples_per_day(trial)
        self.params = torch.empty(vct.vct_population_bytes(n) // 8, dtype=torch.float64, device=device)
        self.metrics = torch.empty(vct.vct_metrics_bytes(n), dtype=torch.uint8, device=device)
        self.traj_patients = int(traj_patients)
        tb = vct.vct_traj_bytes(self.traj_patients, int(trial["n_days"]), int(trial["ts_min"]))
        self.traj = torch.empty(tb // 8, dtype=torch.float64, device=device) if tb else None
        self.mpc = None
        if int(trial["ctrl_kind"]) in (vct.VCT_CTRL_MPC, vct.VCT_CTRL_MLP):
            self.mpc = torch.empty(vct.vct_mpc_bytes(n, int(trial["precision"])), dtype=torch.uint8, device=device)
        self.popbg = None      # optional int64: population BG per sample (sum, min, max keys, counts)
        if popbg:
            self.popbg = torch.empty(vct.vct_popbg_bytes(int(trial["n_days"]), int(trial["ts_min"])) // 8,
                                     dtype=torch.int64, device=device)
        self.doses = None      # optional double [3][n]: basal, bolus insulin (mU), glucagon (ug)
        if int(trial.get("model_ext", 0)):
            self.doses = torch.empty(3 * n, dtype=torch.float64, device=device)
        self.record = None     # optional float [K][n][13] (MPC / learned controller)
        self.fallback = None   # optional int32 [n] (learned controller)
        if int(trial["ctrl_kind"]) == vct.VCT_CTRL_MLP:
            self.fallback = torch.zeros(n, dtype=torch.int32, device=device)


def create_population(trial: dict, bufs: TrialBuffers, stream=None):
    return vct.vct_create_population(vct.population_desc(trial), bufs.params, stream)


def mpc_setup(trial: dict, pop, bufs: TrialBuffers, stream=None) -> None:
    sim = vct.sim_settings(trial, bufs.metrics)
    vct.vct_mpc_setup(pop, vct.controller(trial), sim, bufs.mpc, stream)


def simulate(trial: dict, pop, bufs: TrialBuffers, stream=None, mlp_blob=None) -> None:
    sim = vct.sim_settings(trial, bufs.metrics, bufs.traj_patients, bufs.traj, bufs.record, bufs.fallback,
                           getattr(bufs, "popbg", None), getattr(bufs, "doses", None))
    vct.vct_simulate(pop, vct.protocol(trial), vct.controller(trial, bufs.mpc, mlp_blob), sim, stream)


def read_metrics(bufs: TrialBuffers, stream=None) -> dict:
    return vct.vct_read_metrics(bufs.metrics, bufs.n, bufs.K, stream).as_dict()


def run(trial: dict, device="cuda", traj_patients: int = 0, stream=None, bufs: TrialBuffers | None = None,
        mlp_blob=None):
    """Population -> (MPC setup) -> simulation -> reduction. Returns (summary dict, buffers).
    The learned controller (ctrl_kind MLP) needs mlp_blob, a trained network blob."""
    bufs = bufs or TrialBuffers(trial, device, traj_patients)
    pop = create_population(trial, bufs, stream)
    try:
        if bufs.mpc is not None:
            mpc_setup(trial, pop, bufs, stream)
        simulate(trial, pop, bufs, stream, mlp_blob)
        summary = read_metrics(bufs, stream)
    finally:
        vct.vct_destroy_population(pop)
    return summary, bufs


def replay_patient(trial: dict, patient: int, device="cuda", stream=None, mlp_blob=None) -> dict:
    """Re-simulate patient `patient` (index within the trial) alone, with its trajectory.
    Every random number is keyed by the global patient index, so the replay reproduces the
    patient's run inside the whole population bit for bit (the paper keeps only the worst
    simulations; here any one, e.g. the summary's worst_patient, is rebuilt on demand from
    the counters). Returns the one-patient record of to_host with traj_g, traj_y, traj_u."""
    t = dict(trial)
    t["first_patient"] = int(trial.get("first_patient", 0)) + int(patient)
    t["n_patients"] = 1
    _, bufs = run(t, device, traj_patients=1, stream=stream, mlp_blob=mlp_blob)
    return to_host(bufs)


def to_host(bufs: TrialBuffers) -> dict:
    """Per-patient arrays (numpy) in the oracle's layout, for comparisons."""
    torch.cuda.synchronize()
    m = {k: v.cpu().numpy() for k, v in vct.metric_views(bufs.metrics, bufs.n).items()}
    out = {
        "bins": m["bins"].T.copy(), "events": m["events"].T.copy(), "sum_g": m["sum_g"], "min_g": m["min_g"],
        "argmin_k": m["argmin_k"], "sum_u": m["sum_u"], "status": m["status"].view("uint32"),
        "params": bufs.params.view(vct.VCT_NPARAM_ROWS, bufs.n).cpu().numpy().T.copy(), "K": bufs.K,
    }
    if bufs.traj is not None:
        t = bufs.traj.view(3, bufs.traj_patients, bufs.K).cpu().numpy()
        out["traj_g"], out["traj_y"], out["traj_u"] = t[0], t[1], t[2]
    if bufs.record is not None:
        out["record"] = bufs.record.view(bufs.K, bufs.n, 13).cpu().numpy()
    if bufs.fallback is not None:
        out["fallback"] = bufs.fallback.cpu().numpy()
    if getattr(bufs, "doses", None) is not None:
        out["doses"] = bufs.doses.view(3, bufs.n).cpu().numpy().T.copy()
    if getattr(bufs, "popbg", None) is not None:
        out.update(vct.popbg_decode(bufs.popbg, bufs.n, bufs.K))
    return out


MPC_ROWS = 11 * 11 + 3 * 11 + 24 * 11 + 3 * 24 + 5 + 11 + 1   # layout of csrc/mpc.hpp


def mpc_to_host(bufs: TrialBuffers, precision: int) -> dict:
    """Per-patient MPC data (numpy), rows named as in the oracle."""
    import numpy as np
    torch.cuda.synchronize()
    dt = torch.float32 if precision == vct.VCT_FP32 else torch.float64
    M = bufs.mpc.view(dt).view(MPC_ROWS, bufs.n).cpu().numpy().astype(np.float64)
    o = 0
    out = {}
    for name, rows in (("A", 121), ("B", 11), ("E", 11), ("K", 11), ("Gx", 264), ("gd", 24), ("g1", 24), ("h", 24),
                       ("step", 1), ("rho_p", 1), ("gi", 1), ("ub", 1), ("umax", 1), ("Fbar", 11), ("wbar", 1)):
        out[name] = M[o:o + rows].T
        o += rows
    return out


class Batch:
    """Many arms (each a trial dict sharing protocol, controller kind and noise settings)
    in one persistent, graph-captured launch."""

    def __init__(self, arms: list[dict], device="cuda", block: int = 0, stream=None):
        self.arms = arms
        self.bufs = [TrialBuffers(t, device) for t in arms]
        self.pops = [create_population(t, b, stream) for t, b in zip(arms, self.bufs)]
        c_arms = [vct.arm(p, t["n_days"], t["kp"], t["ki"], t["kd"], b.metrics, t.get("basal_scale", 1.0))
                  for p, t, b in zip(self.pops, arms, self.bufs)]
        t0 = arms[0]
        sim = vct.sim_settings(t0, None)
        self.handle = vct.vct_batch_create(c_arms, vct.protocol(t0), vct.controller(t0), sim, block, stream)
        self.patient_days = sum(int(t["n_patients"]) * int(t["n_days"]) for t in arms)

    def run(self, stream=None) -> None:
        vct.vct_batch_run(self.handle, stream)

    def info(self) -> dict:
        return vct.vct_batch_info(self.handle).as_dict()

    def summaries(self, stream=None) -> list[dict]:
        return [read_metrics(b, stream) for b in self.bufs]

    def close(self) -> None:
        vct.vct_batch_destroy(self.handle)
        self.handle = None
        for p in self.pops:
            vct.vct_destroy_population(p)
        self.pops = []
