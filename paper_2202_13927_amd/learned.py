"""Learned controller trial: imitate the MPC, then compare the two arms on the same patients.

1. Record the MPC closed loop of a separate training population (every sample's 12 inputs
   and the MPC's action u/u_b) inside the simulation kernel.
2. Fit the network by Adam on minibatches drawn from that data set (BF16 MFMA forward and
   backward, FP32 master weights), after z-scoring the inputs and storing the box of the
   training inputs outside which the MPC keeps control.
3. Run the evaluation population twice on common random numbers (same population, meals and
   noise): exact MPC, and the network with MPC fallback; report the change in time in range,
   the per-arm simulation times and the fallback rate.
All steps run in the HIP library; this module sequences them and times them with HIP events.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import policy as PL
from . import trial as T
from . import vct
from . import workloads as W


def _timed(fn, stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    out = fn()
    e1.record(s)
    e1.synchronize()
    return out, e0.elapsed_time(e1) / 1000.0


def _fit(rows: torch.Tensor, epochs: float, batch: int, lr: float, box_q: float, seed: int, log) -> tuple:
    n_rows = rows.shape[0]
    pol = PL.Policy(batch=batch)
    pol.init(seed)
    pol.normalize(rows, box_q)
    steps = int(math.ceil(epochs * n_rows / batch))
    t0 = time.perf_counter()
    pol.step(rows, seed, 0.0, apply=False)
    loss0 = float(pol.loss().item())
    losses = pol.train(rows, steps, seed, lr=lr, log_every=max(1, steps // 10))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # full-data-set loss of the final network, evaluated in chunks by the inference kernel
    se = 0.0
    for a in range(0, n_rows, 1 << 22):
        x = rows[a:a + (1 << 22)]
        out = pol.forward(x[:, :12].contiguous())
        se += float(((out - x[:, 12]) ** 2).double().sum().item())
    rep = {"rows": int(n_rows), "steps": steps, "train_s": train_s, "loss_first_batch": loss0,
           "loss_last_batch": losses[-1][1], "mse_full": se / n_rows}
    log(f"[learned] {n_rows} rows, {steps} steps of {batch} in {train_s:.2f} s: minibatch loss {loss0:.4f} -> "
        f"{losses[-1][1]:.4f}, data-set MSE {rep['mse_full']:.4f}")
    return pol, rep


def train_policy(train_trial: dict, epochs: float = 10.0, batch: int = 4096, lr: float = 1e-3, box_q: float = 0.0,
                 seed: int = 100, aggregate_rounds: int = 0, log=print) -> tuple[PL.Policy, dict]:
    """Steps 1-2, optionally followed by rounds of data aggregation: run the current network
    (with fallback) on the training population under fresh noise, label every sample with the
    MPC's action along that closed loop, append the rows and refit on all rows so far.
    Returns the trained policy and a report (data-set sizes, times, losses)."""
    rows, mpc_summary = PL.record_dataset(train_trial)
    log(f"[learned] MPC data set from {train_trial['n_patients']} x {train_trial['n_days']} d, "
        f"TIR {mpc_summary['mean_tir']:.4f}")
    pol, fit = _fit(rows, epochs, batch, lr, box_q, seed, log)
    rounds = [fit]
    for r in range(1, aggregate_rounds + 1):
        t = W.with_(train_trial, ctrl_kind=W.CTRL_MLP, noise_seed=int(train_trial["noise_seed"]) + 1000 * r)
        bufs = T.TrialBuffers(t)
        new = torch.empty(bufs.K * bufs.n * PL.ROW, dtype=torch.float32, device="cuda")
        bufs.record = new
        summ, _ = T.run(t, bufs=bufs, mlp_blob=pol.blob)
        log(f"[learned] round {r}: network closed loop TIR {summ['mean_tir']:.4f}, fallback "
            f"{float(bufs.fallback.double().sum().item()) / (bufs.n * bufs.K):.4%}")
        rows = torch.cat([rows, new.view(-1, PL.ROW)])
        del bufs, new
        pol, fit = _fit(rows, epochs, batch, lr, box_q, seed + r, log)
        fit["loop_tir"] = summ["mean_tir"]
        rounds.append(fit)
    rep = {"batch": batch, "epochs": epochs, "box_q": box_q, "mpc_train_tir": mpc_summary["mean_tir"],
           "rounds": rounds}
    return pol, rep


def evaluate(pol: PL.Policy, mpc_trial: dict, log=print, arms=("mpc", "mlp")) -> dict:
    """Step 3 on the evaluation population; each arm is one simulation launch, timed with
    HIP events. The MPC setup (both arms need it: the learned arm for its fallback and
    inputs) is timed separately; the reduction is outside the timed region. arms selects
    the arms to run."""
    mlp_trial = W.with_(mpc_trial, ctrl_kind=W.CTRL_MLP)
    out = {}
    for name, t in (("mpc", mpc_trial), ("mlp", mlp_trial)):
        if name not in arms:
            continue
        bufs = T.TrialBuffers(t)
        pop = T.create_population(t, bufs)
        torch.cuda.synchronize()
        _, setup_s = _timed(lambda: T.mpc_setup(t, pop, bufs))
        _, sim_s = _timed(lambda: T.simulate(t, pop, bufs, mlp_blob=pol.blob if name == "mlp" else None))
        summ = T.read_metrics(bufs)
        vct.vct_destroy_population(pop)
        r = {"sim_s": sim_s, "setup_s": setup_s, "tir": summ["mean_tir"], "bins": summ["bins"], "events": summ["events"],
             "mean_bg": summ["mean_bg"], "q_frac": summ["q_frac"], "worst_min_g": summ["worst_min_g"]}
        if name == "mlp":
            fb = bufs.fallback.double().sum().item()
            r["fallback_rate"] = fb / (bufs.n * bufs.K)
            r["patients_always_fallback"] = int((bufs.fallback == bufs.K).sum().item())
        pd = int(t["n_patients"]) * int(t["n_days"])
        r["patient_days_per_s"] = pd / sim_s
        out[name] = r
        log(f"[learned] {name}: {sim_s:.3f} s, TIR {summ['mean_tir']:.4f}" +
            (f", fallback {r['fallback_rate']:.4%}" if name == "mlp" else ""))
        del bufs
        torch.cuda.empty_cache()
    if "mpc" in out and "mlp" in out:
        out["delta_tir_pp"] = 100.0 * (out["mlp"]["tir"] - out["mpc"]["tir"])
        out["speedup"] = out["mpc"]["sim_s"] / out["mlp"]["sim_s"]
    return out
