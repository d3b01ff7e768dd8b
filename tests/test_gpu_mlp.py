"""GPU learned controller vs the FP64 oracle, through the C ABI.

Tolerances. The oracle evaluates the network exactly (FP64) on BF16 inputs and the stored
BF16 weights; the kernels keep the hidden activations and their gradients in BF16 (relative
rounding <= u = 2^-8 per value) with FP32 accumulation. For the forward pass the bound is
the worst case of that rounding carried through the layers (ReLU is 1-Lipschitz):
|e_0| <= u |z|, |e_l| <= |W_l| |e_(l-1)| (1 + u) + u h_l, |d out| <= |w4| |e_3|, plus FP32
accumulation (1e-5 of |w4| . (|W3| (|W2| h1 + h2) + h3)); it is evaluated per sample on the
exact activations. Gradients are compared as vectors per layer. Their error is dominated by
the BF16 rounding of the hidden-layer gradients, and relative to the batch gradient it grows
as the per-row terms cancel (small batches, residuals o - t that are small next to o): at the
training batch sizes (>= 512) the bound is relative L2 error <= 2e-2 and cosine >= 0.999, at
B = 64 it is 6e-2 and 0.998. The same gradients are also checked against a float64 numpy
evaluation that rounds at the kernel's points (inputs, activations and hidden gradients to
BF16), which they must match to 2e-3: that separates the kernel's arithmetic from the
format's error. Everything that does not pass through BF16 activations (the initial
weights, Adam, the input statistics, the recorded inputs) is compared to FP32 rounding or
exactly.
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
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_13927_amd import policy, trial
    return torch, policy, trial


def _dense_net(seed):
    net = W.synthetic_policy_net(seed)
    rng = np.random.default_rng(seed + 1000)
    for k, s in (("W1", 0.4), ("W2", 0.17), ("W3", 0.17)):
        net[k] = s * rng.standard_normal(net[k].shape)
    for k in ("b1", "b2", "b3"):
        net[k] = np.asarray(0.1 * rng.standard_normal(64), np.float32).astype(np.float64)
    net["w4"] = 0.2 * rng.standard_normal(64)
    rows = W.synthetic_policy_rows(seed, 4096)
    x = rows[:, :12]
    net["mean"] = np.asarray(x.mean(0), np.float32).astype(np.float64)
    net["istd"] = np.asarray(1.0 / x.std(0), np.float32).astype(np.float64)
    return net


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _bf16_bound(orc, net, x):
    """Worst-case effect of BF16 activation storage on the output (see module docstring)."""
    u = 2.0 ** -8
    relu = lambda a: np.maximum(a, 0.0)
    z = orc.bf16((x - net["mean"]) * net["istd"])
    h1 = relu(z @ net["W1"].T + net["b1"])
    h2 = relu(h1 @ net["W2"].T + net["b2"])
    h3 = relu(h2 @ net["W3"].T + net["b3"])
    A1, A2, A3, a4 = (np.abs(net[k]) for k in ("W1", "W2", "W3", "w4"))
    e1 = (np.abs(z) * u) @ A1.T * (1 + u) + u * h1
    e2 = e1 @ A2.T * (1 + u) + u * h2
    e3 = e2 @ A3.T * (1 + u) + u * h3
    acc = 1e-5 * (((h1 @ A2.T + h2) @ A3.T + h3) @ a4)
    return e3 @ a4 + acc


def test_forward_matches_oracle(G, orc):
    torch, policy, _ = G
    net = _dense_net(21)
    pol = policy.Policy(batch=64)
    pol.load(net)
    ref_net = policy.unpack_blob(pol.blob)   # the stored (BF16 / FP32) values
    for n in (1, 63, 64, 1000, 4097):
        x = _f32(W.synthetic_policy_rows(22 + n, n)[:, :12])
        _say(f"[gpu] mlp forward n={n}")
        out = pol.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy().astype(np.float64)
        ref = orc.mlp_forward(ref_net, x)
        bound = _bf16_bound(orc, ref_net, x)
        err = np.abs(out - ref)
        scale = np.sqrt(np.mean(ref ** 2))
        _say("   max |d| / bound", (err / bound).max(), "median |d| / rms", np.median(err) / scale)
        assert np.all(err <= bound)


def _grad_groups(g_gpu: dict, g_orc: dict):
    pairs = {"W1": (g_gpu["W1"][:, :12], g_orc["W1"]), "W2": (g_gpu["W2"], g_orc["W2"]),
             "W3": (g_gpu["W3"], g_orc["W3"]), "w4": (g_gpu["W4"][0], g_orc["w4"]), "b1": (g_gpu["b1"], g_orc["b1"]),
             "b2": (g_gpu["b2"], g_orc["b2"]), "b3": (g_gpu["b3"], g_orc["b3"]),
             "b4": (g_gpu["b4"][:1], np.array([g_orc["b4"]]))}
    return pairs


def _bf16_rounded_grad(torch, net, rows, idx):
    """Gradient in float64 with BF16 rounding where the kernel rounds (test reference for the
    kernel's arithmetic, not the oracle)."""
    bf = lambda a: torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    relu = lambda a: np.maximum(a, 0.0)
    r = rows[idx]
    B = len(idx)
    z = bf(_f32(_f32(r[:, :12] - net["mean"]) * net["istd"]))
    h1 = bf(relu(z @ net["W1"].T + net["b1"]))
    h2 = bf(relu(h1 @ net["W2"].T + net["b2"]))
    h3 = bf(relu(h2 @ net["W3"].T + net["b3"]))
    dout = 2.0 * (h3 @ net["w4"] + net["b4"] - r[:, 12]) / B
    d3 = bf(np.where(h3 > 0, dout[:, None] * net["w4"][None], 0.0))
    d2 = bf(np.where(h2 > 0, d3 @ net["W3"], 0.0))
    d1 = bf(np.where(h1 > 0, d2 @ net["W2"], 0.0))
    return {"W1": d1.T @ z, "W2": d2.T @ h1, "W3": d3.T @ h2, "w4": h3.T @ dout, "b1": d1.sum(0),
            "b2": d2.sum(0), "b3": d3.sum(0), "b4": dout.sum()}


def _check_grads(g_gpu, g_orc, g_emul, batch):
    rel_max, cos_min = (2e-2, 0.999) if batch >= 512 else (6e-2, 0.998)
    bad = []
    for name, (a, b) in _grad_groups(g_gpu, g_orc).items():
        a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
        e = np.asarray(g_emul[name], np.float64).ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        rel_e = np.linalg.norm(a - e) / np.linalg.norm(e)
        _say(f"   grad {name}: rel L2 {rel:.2e} cosine {cos:.6f}; vs BF16-rounded reference {rel_e:.2e}")
        if not (rel <= rel_max and cos >= cos_min and rel_e <= 2e-3):
            bad.append(name)
    assert not bad, bad
    # padded entries stay exactly zero
    assert not np.any(g_gpu["W1"][:, 12:]) and not np.any(g_gpu["W4"][1:]) and not np.any(g_gpu["b4"][1:])


@pytest.mark.parametrize("batch", [64, 1024, 65536])
def test_gradient_matches_oracle(G, orc, batch):
    torch, policy, _ = G
    net = _dense_net(31)
    rows = _f32(W.synthetic_policy_rows(32, 3000))
    idx = np.random.default_rng(33).integers(0, 3000, batch).astype(np.int32)
    pol = policy.Policy(batch=batch)
    pol.load(net)
    ref_net = policy.unpack_blob(pol.blob)
    _say(f"[gpu] mlp gradient batch={batch} (index list)")
    d_rows = torch.tensor(rows, dtype=torch.float32, device="cuda")
    d_idx = torch.tensor(idx, device="cuda")
    pol.step(d_rows, seed=0, lr=0.0, idx=d_idx, apply=False)
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in pol.grad().items()}
    loss_ref, g_ref = orc.mlp_loss_grad(ref_net, rows, idx.astype(np.int64))
    loss = float(pol.loss().item())
    _say("   loss", loss, "oracle", loss_ref)
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    _check_grads(g, g_ref, _bf16_rounded_grad(torch, ref_net, rows, idx), batch)


def test_gradient_philox_rows(G, orc):
    torch, policy, _ = G
    net = _dense_net(41)
    n_rows, batch, seed, step = 100_003, 512, 77, 5
    rows = _f32(W.synthetic_policy_rows(42, n_rows))
    pol = policy.Policy(batch=batch)
    pol.load(net)
    pol.step_count = step
    ref_net = policy.unpack_blob(pol.blob)
    _say("[gpu] mlp gradient, rows drawn by Philox")
    pol.step(torch.tensor(rows, dtype=torch.float32, device="cuda"), seed=seed, lr=0.0, apply=False)
    idx = orc.mlp_batch_rows(seed, step, batch, n_rows)
    loss_ref, g_ref = orc.mlp_loss_grad(ref_net, rows, idx)
    assert float(pol.loss().item()) == pytest.approx(loss_ref, rel=1e-2)
    _check_grads({k: v.cpu().numpy().astype(np.float64) for k, v in pol.grad().items()}, g_ref,
                 _bf16_rounded_grad(torch, ref_net, rows, idx), batch)


def test_invalid_index_poisons_loss(G):
    torch, policy, _ = G
    pol = policy.Policy(batch=64)
    pol.load(_dense_net(5))
    rows = torch.tensor(_f32(W.synthetic_policy_rows(6, 100)), dtype=torch.float32, device="cuda")
    idx = torch.arange(64, dtype=torch.int32, device="cuda")
    idx[7] = 100   # one past the end
    pol.step(rows, seed=0, lr=0.0, idx=idx, apply=False)
    assert np.isnan(float(pol.loss().item()))


def test_init_matches_oracle(G, orc):
    torch, policy, _ = G
    pol = policy.Policy(batch=64)
    _say("[gpu] mlp init")
    pol.init(seed=1234)
    torch.cuda.synchronize()
    m = {k: v.cpu().numpy().astype(np.float64) for k, v in policy.params_view(pol.train_buf, "master").items()}
    ref = orc.mlp_init(1234)
    assert np.allclose(m["W1"][:, :12], ref["W1"], rtol=1e-7, atol=0) and not np.any(m["W1"][:, 12:])
    assert np.allclose(m["W2"], ref["W2"], rtol=1e-7, atol=0)
    assert np.allclose(m["W3"], ref["W3"], rtol=1e-7, atol=0)
    assert np.allclose(m["W4"][0], ref["w4"], rtol=1e-7, atol=0) and not np.any(m["W4"][1:])
    assert m["b4"][0] == 1.0 and not np.any(m["b4"][1:]) and not np.any(m["b1"])
    for k in ("adam_m", "adam_v"):
        assert not any(np.any(v.cpu().numpy()) for v in policy.params_view(pol.train_buf, k).values())
    # the blob holds the master weights rounded to BF16
    blob = policy.unpack_blob(pol.blob)
    bf = lambda a: torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(blob["W2"], bf(m["W2"])) and np.array_equal(blob["w4"], bf(m["W4"][0]))
    assert blob["b4"] == 1.0


def test_adam_step_matches_oracle(G, orc):
    torch, policy, _ = G
    net = _dense_net(51)
    rows = _f32(W.synthetic_policy_rows(52, 2000))
    idx = np.random.default_rng(53).integers(0, 2000, 256).astype(np.int32)
    pol = policy.Policy(batch=256)
    pol.load(net)
    ref_net = policy.unpack_blob(pol.blob)
    rng = np.random.default_rng(54)
    master = policy.params_view(pol.train_buf, "master")
    mv = policy.params_view(pol.train_buf, "adam_m")
    vv = policy.params_view(pol.train_buf, "adam_v")
    init = {}
    for name, shape in [(k, tuple(v.shape)) for k, v in master.items()]:
        w = rng.standard_normal(shape) * 0.1
        m = 100.0 * rng.standard_normal(shape)       # moments far above the gradient, so that
        v = 1.0e4 * (rng.random(shape) + 0.5)        # the BF16 gradient error barely matters
        if name == "W1":
            w[:, 12:] = m[:, 12:] = v[:, 12:] = 0.0
        if name == "W4":
            w[1:] = m[1:] = v[1:] = 0.0
        if name == "b4":
            w[1:] = m[1:] = v[1:] = 0.0
        init[name] = (_f32(w), _f32(m), _f32(v))
        master[name].copy_(torch.tensor(init[name][0], dtype=torch.float32))
        mv[name].copy_(torch.tensor(init[name][1], dtype=torch.float32))
        vv[name].copy_(torch.tensor(init[name][2], dtype=torch.float32))
    step, lr = 2, 1e-3
    pol.step_count = step
    _say("[gpu] mlp Adam step t=3")
    pol.step(torch.tensor(rows, dtype=torch.float32, device="cuda"), seed=0, lr=lr,
             idx=torch.tensor(idx, device="cuda"), apply=True)
    torch.cuda.synchronize()
    _, g_ref = orc.mlp_loss_grad(ref_net, rows, idx.astype(np.int64))
    gpu_w = {k: v.cpu().numpy().astype(np.float64) for k, v in master.items()}
    gref = {"W1": np.pad(g_ref["W1"], ((0, 0), (0, 4))), "W2": g_ref["W2"], "W3": g_ref["W3"],
            "W4": np.vstack([g_ref["w4"][None], np.zeros((15, 64))]), "b1": g_ref["b1"], "b2": g_ref["b2"],
            "b3": g_ref["b3"], "b4": np.r_[g_ref["b4"], np.zeros(15)]}
    # bound of the update's sensitivity to the gradient: it enters as lr (1 - b1)/bc1 dg /
    # sqrt(v_hat); dg is allowed to be as large as the group's largest gradient, which with
    # these moments is still ~1e-3 of the update
    t = step + 1
    bc1, bc2 = 1 - 0.9 ** t, 1 - 0.999 ** t
    worst = 0.0
    for name, (w, m, v) in init.items():
        g = gref[name]
        w2, _, v2 = orc.adam(w, m, v, g, lr, t)
        pad = (w == 0) & (m == 0) & (v == 0)
        dg = np.abs(g[~pad]).max()
        bound = lr * (0.1 / bc1) * dg / np.sqrt(np.maximum(v2, 1e-30) / bc2) + 1e-7 * np.abs(w2) + 1e-6 * lr
        step_size = np.abs(w2 - w)[~pad]
        assert np.median(bound[~pad] / step_size) < 0.01   # the check is much tighter than the step
        err = np.abs(gpu_w[name] - w2)
        worst = max(worst, float((err[~pad] / bound[~pad]).max()))
        assert np.all(err[~pad] <= bound[~pad]), name
        assert np.array_equal(gpu_w[name][pad], w[pad])
    _say("   max |dw| / bound", worst)
    blob = policy.unpack_blob(pol.blob)
    bf = lambda a: torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(blob["W3"], bf(gpu_w["W3"]))
    assert np.array_equal(blob["b2"], gpu_w["b2"])


@pytest.mark.parametrize("box_q", [0.0, 0.001])
def test_normalize_matches_oracle(G, orc, box_q):
    torch, policy, _ = G
    rows = _f32(W.synthetic_policy_rows(61, 200_001))
    pol = policy.Policy(batch=64)
    _say(f"[gpu] mlp normalize box_q={box_q}")
    pol.normalize(torch.tensor(rows, dtype=torch.float32, device="cuda"), box_q)
    got = policy.unpack_blob(pol.blob)
    ref = orc.mlp_stats(rows, box_q)
    assert np.allclose(got["mean"], ref["mean"], rtol=1e-6, atol=1e-12)
    assert np.allclose(got["istd"], ref["istd"], rtol=1e-6)
    x = rows[:, :12]
    if box_q == 0.0:
        assert np.array_equal(got["lo"], x.min(0)) and np.array_equal(got["hi"], x.max(0))
    else:   # the GPU machine is the oracle's quantile rounded outward to the 4096-bin grid
        w = (x.max(0) - x.min(0)) / 4096.0
        slack = 1e-6 * np.abs(x).max(0)
        assert np.all(got["lo"] <= ref["lo"] + slack) and np.all(ref["lo"] - got["lo"] <= w + slack)
        assert np.all(got["hi"] >= ref["hi"] - slack) and np.all(got["hi"] - ref["hi"] <= w + slack)


def test_recorded_rows_match_oracle(G, orc):
    torch, policy, trial = G
    t = W.with_(W.c5_mpc(), n_patients=70, n_days=2, precision=W.FP64)
    _say("[gpu] MPC FP64 with recording, 70 x 2 d")
    rows, _ = policy.record_dataset(t)
    K = 2 * 288
    got = rows.view(K, 70, 13).cpu().numpy().astype(np.float64)
    ref = orc.simulate(t, threads=THREADS, record=True)["record"]
    assert np.allclose(got[:, :, :12], _f32(ref[:, :, :12]), rtol=2e-7, atol=1e-12)
    assert np.allclose(got[:, :, 12], ref[:, :, 12], rtol=1e-5, atol=1e-7)


def _mlp_trial(**kw):
    return W.with_(W.c5_mlp(), **{"n_patients": 300, "n_days": 2, "precision": W.FP64, **kw})


def _run_mlp(G, t, net, traj=0):
    torch, policy, trial = G
    pol = policy.Policy(batch=64)
    pol.load(net)
    bufs = trial.TrialBuffers(t, traj_patients=traj)
    s, bufs = trial.run(t, bufs=bufs, mlp_blob=pol.blob)
    return trial.to_host(bufs), policy.unpack_blob(pol.blob)


def test_constant_network_is_open_loop(G):
    torch, policy, trial = G
    t = _mlp_trial(n_patients=130)
    _say("[gpu] learned controller, constant network = open loop")
    g, _ = _run_mlp(G, t, W.constant_policy_net(1.0), traj=4)
    s, b = trial.run(W.with_(t, ctrl_kind=W.CTRL_OPEN, u_rel=1.0), traj_patients=4)
    o = trial.to_host(b)
    for k in ("bins", "events", "sum_g", "min_g", "traj_g", "traj_u"):
        assert np.array_equal(g[k], o[k]), k
    assert not np.any(g["fallback"])


def test_always_fallback_is_mpc(G, orc):
    torch, policy, trial = G
    t = _mlp_trial(n_patients=130)
    _say("[gpu] learned controller, empty box = MPC")
    g, _ = _run_mlp(G, t, W.constant_policy_net(2.0, always_fallback=True), traj=4)
    s, b = trial.run(W.with_(t, ctrl_kind=W.CTRL_MPC), traj_patients=4)
    m = trial.to_host(b)
    for k in ("bins", "events", "sum_g", "traj_g", "traj_u"):
        assert np.array_equal(g[k], m[k]), k
    assert np.all(g["fallback"] == g["K"])


@pytest.mark.parametrize("ctrl", ["mpc", "mlp"])
def test_slices_equal_whole_controllers(G, ctrl):
    """The MPC and the learned controller: one patient alone, a ragged slice and the rest each
    give, patient by patient, the whole run's results bit for bit (a one-lane tile, ragged
    tiles whose padding lanes replay a patient and write nothing, the partition of the
    patients by the box recomputed per slice, the wave-cooperative fallback solve)."""
    torch, policy, trial = G
    t = _mlp_trial(precision=W.FP32, n_patients=130, n_days=2)
    if ctrl == "mpc":
        t = W.with_(t, ctrl_kind=W.CTRL_MPC)
    net = W.synthetic_policy_net(71)

    def run(tt):
        _say(f"[gpu] {ctrl} slice first {tt.get('first_patient', 0)} n {tt['n_patients']}")
        if ctrl == "mlp":
            return _run_mlp(G, tt, net)[0]
        return trial.to_host(trial.run(tt)[1])

    whole = run(t)
    parts = [run(W.with_(t, first_patient=f, n_patients=n)) for f, n in ((0, 1), (1, 65), (66, 64))]
    keys = ("bins", "events", "sum_g", "min_g", "argmin_k", "sum_u", "status")
    if ctrl == "mlp":
        keys += ("fallback",)
        assert whole["fallback"].sum() > 0 and (whole["fallback"] == 0).sum() > 0
    for k in keys:
        assert np.array_equal(whole[k], np.concatenate([p[k] for p in parts])), k


@pytest.mark.parametrize("precision", [W.FP64, W.FP32])
def test_closed_loop_matches_oracle(G, orc, precision):
    """A proportional-law network with a random perturbation and a box that leaves some
    patients and glucose excursions to the MPC."""
    t = _mlp_trial(precision=precision, n_patients=300 if precision == W.FP64 else 1029)
    _say(f"[gpu] learned controller closed loop, precision {precision}, {t['n_patients']} x 2 d")
    g, ref_net = _run_mlp(G, t, W.synthetic_policy_net(71), traj=8)
    o = orc.simulate(t, n_traj=8, threads=THREADS, mlp=ref_net)
    K = g["K"]
    fb_g, fb_o = g["fallback"], o["fallback"]
    _say("   fallback fraction gpu", fb_g.sum() / (K * len(fb_g)), "oracle", fb_o.sum() / (K * len(fb_o)))
    assert fb_o.sum() > 0 and (fb_o == 0).sum() > 0          # both paths are exercised
    always = fb_o == K                                        # patients outside the box
    assert np.array_equal(fb_g == K, always)
    assert abs(int(fb_g.sum()) - int(fb_o.sum())) <= 0.02 * fb_o.sum() + 5
    dtir = (g["bins"][:, 2].astype(np.int64) - o["bins"][:, 2]) / K
    _say("   |dTIR| max", np.abs(dtir).max(), "mean", dtir.mean())
    assert abs(dtir.mean()) < 1e-3
    assert np.mean(np.abs(dtir) <= 1e-2) > 0.97
    # the first sample starts from the same basal state: same decision, u within the
    # forward-pass tolerance
    u0_g, u0_o = g["traj_u"][:, 0], o["traj_u"][:, 0]
    assert np.allclose(u0_g, u0_o, rtol=2e-2)


def test_learned_full_size_sampled(G, orc):
    """The learned controller at the benchmark's evaluation size and launch (1,000,000 patients
    x 28 days, FP32, the persistent queue of out-of-box waves and 64-patient tiles): patients
    spread over the index range against the oracle one by one, with the same network."""
    t = _mlp_trial(precision=W.FP32, n_patients=1_000_000, n_days=28)
    _say("[gpu] learned controller, 1,000,000 x 28 d FP32")
    g, ref_net = _run_mlp(G, t, W.synthetic_policy_net(71))
    K = g["K"]
    assert K == 28 * 288 and len(g["fallback"]) == t["n_patients"]
    import concurrent.futures as cf
    idx = np.linspace(0, t["n_patients"] - 1, 64).astype(int)
    with cf.ThreadPoolExecutor(THREADS) as ex:     # one patient per oracle call, in parallel
        res = list(ex.map(lambda i: orc.simulate(t, first=int(i), count=1, threads=1, mlp=ref_net), idx))
    dt, fb_g, fb_o = [], 0, 0
    for i, o in zip(idx, res):
        assert (g["fallback"][i] == K) == (o["fallback"][0] == K), i     # outside the box: the MPC throughout
        assert g["status"][i] == o["status"][0]
        fb_g += int(g["fallback"][i])
        fb_o += int(o["fallback"][0])
        dt.append((int(g["bins"][i, 2]) - int(o["bins"][0, 2])) / K)
    dt = np.array(dt)
    _say("   sampled |dTIR| max", np.abs(dt).max(), "mean", dt.mean(), "fallbacks gpu", fb_g, "oracle", fb_o)
    # FP32 against FP64 on the same noise: 0.5 pp per patient, 0.1 pp on the sample's mean
    assert np.abs(dt).max() < 5e-3 and abs(dt.mean()) < 1e-3
    assert abs(fb_g - fb_o) <= 0.05 * fb_o + 50


def test_training_reduces_loss_and_is_deterministic(G):
    """Adam on a smooth synthetic target: the minibatch loss falls by 10x; two runs from the
    same initial weights and seed give bitwise equal weights (fixed-order reductions)."""
    torch, policy, _ = G
    rows = torch.tensor(_f32(W.synthetic_policy_rows(81, 200_000)), dtype=torch.float32, device="cuda")
    blobs = []
    for rep in range(2):
        pol = policy.Policy(batch=1024)
        pol.init(seed=3)
        pol.normalize(rows, 0.0)
        pol.step(rows, seed=9, lr=0.0, apply=False)
        l0 = float(pol.loss().item())
        _say(f"[gpu] mlp training run {rep}, 600 steps of 1024")
        log = pol.train(rows, steps=600, seed=9, lr=3e-3, log_every=100)
        _say("   loss", l0, "->", log)
        assert np.mean([l for _, l in log[-2:]]) < 0.1 * l0
        blobs.append(pol.blob.cpu().numpy().copy())
    assert np.array_equal(blobs[0], blobs[1])


@pytest.mark.parametrize("batch,steps", [(512, 120), (4096, 300), (32768, 20)])
def test_multi_step_training_equals_single_steps(G, batch, steps):
    """vct_mlp_train (many steps per call, the cosine schedule computed in the library) gives
    the same weights, Adam moments and loss bit for bit as the same steps one call each, for
    small and large batches (8 to 512 tiles of 64 rows per step)."""
    import math
    torch, policy, _ = G
    rows = torch.tensor(_f32(W.synthetic_policy_rows(82, 50_000)), dtype=torch.float32, device="cuda")
    lr, lr_min = 2e-3, 1e-4
    pols = []
    for multi in (False, True):
        _say(f"[gpu] mlp training batch {batch}, {steps} steps, {'one call' if multi else 'one call per step'}")
        pol = policy.Policy(batch=batch)
        pol.init(seed=5)
        pol.normalize(rows, 0.0)
        if multi:
            pol.train(rows, steps=steps, seed=11, lr=lr, lr_min=lr_min, log_every=37 if steps < 256 else 0)
        else:
            for s in range(steps):
                pol.step(rows, 11, lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * s / steps)))
        pols.append(pol)
    assert pols[0].step_count == pols[1].step_count == steps
    assert torch.equal(pols[0].train_buf, pols[1].train_buf)
    assert torch.equal(pols[0].blob, pols[1].blob)


def test_labels_with_empty_box_equal_mpc_rows(G):
    """Data aggregation: recording with the learned controller labels each sample with the
    MPC's action; with an empty box the closed loop is the MPC's, so the rows equal the MPC
    arm's rows bit for bit."""
    torch, policy, trial = G
    t = _mlp_trial(n_patients=100)
    pol = policy.Policy(batch=64)
    pol.load(W.constant_policy_net(2.0, always_fallback=True))
    bufs = trial.TrialBuffers(t)
    bufs.record = torch.empty(bufs.K * bufs.n * 13, dtype=torch.float32, device="cuda")
    _say("[gpu] learned controller with labels, empty box")
    trial.run(t, bufs=bufs, mlp_blob=pol.blob)
    rows_mpc, _ = policy.record_dataset(W.with_(t, ctrl_kind=W.CTRL_MPC))
    assert torch.equal(bufs.record.view(-1, 13), rows_mpc)


def test_network_in_the_loop_equals_forward(G):
    """The network inside the simulation kernel and vct_mlp_forward run the same code on the
    same staged weights: on every sample of the recorded patients where the network acts,
    the applied insulin is exactly clamp(u_b out, 0, u_max) with out from vct_mlp_forward on
    the recorded inputs; where the MPC acts it is the recorded MPC label. The fallback
    decision (box, safety rule) recomputed from the recorded inputs gives each patient's
    fallback count exactly."""
    torch, policy, trial = G
    t = _mlp_trial(precision=W.FP32, n_patients=130, n_days=1, mlp_safe_g=3.9)
    pol = policy.Policy(batch=64)
    pol.load(W.synthetic_policy_net(71))
    net = policy.unpack_blob(pol.blob)
    bufs = trial.TrialBuffers(t, traj_patients=8)
    bufs.record = torch.empty(bufs.K * bufs.n * 13, dtype=torch.float32, device="cuda")
    _say("[gpu] learned controller: network in the loop vs vct_mlp_forward, 130 x 1 d FP32")
    trial.run(t, bufs=bufs, mlp_blob=pol.blob)
    h = trial.to_host(bufs)
    rec = bufs.record.view(bufs.K, bufs.n, 13)
    f32 = np.float32
    lo, hi = net["lo"].astype(f32), net["hi"].astype(f32)
    acted = 0
    for p in range(8):
        feats = rec[:, p, :12].contiguous()
        out = pol.forward(feats).cpu().numpy()
        f = feats.cpu().numpy()
        ub = f32(h["params"][p, 15])
        umax = f32(t["umax_rel"] * h["params"][p, 15])
        ood = np.any(~((f >= lo) & (f <= hi)), axis=1)
        fb = ood | ((f[:, 0] < f32(t["mlp_safe_g"])) & (out > f32(t["mlp_safe_out"])))
        assert int(fb.sum()) == int(h["fallback"][p])
        u_net = np.minimum(np.maximum(ub * out, f32(0)), umax)
        u = h["traj_u"][p]
        assert np.array_equal(u[~fb], u_net[~fb].astype(np.float64))
        lab = rec[:, p, 12].cpu().numpy().astype(np.float64) * float(ub)
        assert np.allclose(u[fb], lab[fb], rtol=1e-6, atol=0)
        acted += int((~fb).sum())
    assert acted > 0


def test_trained_network_gain(G):
    """End to end, on the GPU only: record the MPC's closed loop on a training population,
    fit the network, then run a separate population three ways on common random numbers.
    The trained network keeps the population TIR within 0.5 pp of the exact MPC while its
    simulation is faster; the same network untrained (the method without learning) is far
    from the MPC."""
    torch, policy, trial = G
    from paper_2202_13927_amd import learned
    train = W.with_(W.mlp_training_population(), n_patients=4000, n_days=2)
    _say("[gpu] learned controller end to end: train on 4000 x 2 d")
    pol, rep = learned.train_policy(train, epochs=8.0, log=_say)
    ev = W.with_(W.c5_mpc(), n_patients=20000, n_days=7, pop_seed=41, noise_seed=41)
    res = learned.evaluate(pol, ev, log=_say)
    untrained = policy.Policy(batch=64)
    untrained.init(seed=100)
    untrained.blob[vct_norm_slice()] = pol.blob[vct_norm_slice()]   # same normalisation and box
    res0 = learned.evaluate(untrained, ev, log=_say)
    _say("   trained dTIR %.3f pp (speedup %.2f), untrained dTIR %.3f pp" %
         (res["delta_tir_pp"], res["speedup"], res0["delta_tir_pp"]))
    assert abs(res["delta_tir_pp"]) <= 0.5
    assert res["mlp"]["sim_s"] < res["mpc"]["sim_s"]
    assert abs(res0["delta_tir_pp"]) > 5 * max(abs(res["delta_tir_pp"]), 0.1)


def vct_norm_slice():
    from paper_2202_13927_amd import vct
    return slice(vct.MLP_BLOB["mean"], vct.VCT_MLP_BLOB_BYTES)
