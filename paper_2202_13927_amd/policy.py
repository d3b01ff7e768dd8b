"""Learned controller through the C ABI: behaviour-cloning data set, training, inference.

Every computation runs in the HIP library (data-set recording inside the MPC
simulation kernel, BF16 MFMA forward/backward, Adam, statistics); this module
allocates the caller-owned device buffers with torch, passes pointers, and packs or
unpacks the documented blob layout.
"""
from __future__ import annotations

import numpy as np
import torch

from . import trial as T
from . import vct

P = vct.VCT_MLP_PARAMS
ROW = vct.VCT_MLP_IN + 1


def _bf16_bits(a) -> np.ndarray:
    t = torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def pack_blob(net: dict) -> np.ndarray:
    """Host bytes of a network in the blob layout of vct.h. `net` holds W1 (64, 12), W2, W3
    (64, 64), w4 (64,), b1..b3 (64,), b4 (scalar) and mean, istd, lo, hi (12,); weights are
    rounded to BF16 (nearest, ties to even), everything else to FP32."""
    out = np.zeros(vct.VCT_MLP_BLOB_BYTES, np.uint8)

    def put(name, arr):
        b = np.ascontiguousarray(arr).view(np.uint8).ravel()
        o = vct.MLP_BLOB[name]
        out[o:o + b.size] = b

    w1 = np.zeros((64, 16))
    w1[:, :12] = net["W1"]
    w4 = np.zeros((16, 64))
    w4[0] = net["w4"]
    put("W1", _bf16_bits(w1))
    put("W2", _bf16_bits(net["W2"]))
    put("W3", _bf16_bits(net["W3"]))
    put("W4", _bf16_bits(w4))
    for k in ("b1", "b2", "b3"):
        put(k, np.asarray(net[k], np.float32))
    b4 = np.zeros(16, np.float32)
    b4[0] = net["b4"]
    put("b4", b4)
    for k in ("mean", "istd", "lo", "hi"):
        v = np.zeros(16, np.float32)
        v[:12] = net[k]
        put(k, v)
    return out


def unpack_blob(blob) -> dict:
    """The network stored in a blob (host or device bytes) as float64 arrays."""
    b = (blob.cpu().numpy() if hasattr(blob, "cpu") else np.asarray(blob)).astype(np.uint8)

    def bf(name, shape):
        o = vct.MLP_BLOB[name]
        n = int(np.prod(shape))
        bits = b[o:o + 2 * n].view(np.uint16).astype(np.uint32) << 16
        return bits.view(np.float32).astype(np.float64).reshape(shape)

    def f32(name, n):
        o = vct.MLP_BLOB[name]
        return b[o:o + 4 * n].view(np.float32).astype(np.float64)

    net = {"W1": bf("W1", (64, 16))[:, :12].copy(), "W2": bf("W2", (64, 64)), "W3": bf("W3", (64, 64)),
           "w4": bf("W4", (16, 64))[0].copy(), "b1": f32("b1", 64), "b2": f32("b2", 64), "b3": f32("b3", 64),
           "b4": float(f32("b4", 1)[0])}
    for k in ("mean", "istd", "lo", "hi"):
        net[k] = f32(k, 12)
    return net


def params_view(train_buf: torch.Tensor, which: str = "master") -> dict:
    """FP32 parameter groups (torch views) of master / adam_m / adam_v / grad."""
    slot = {"master": 0, "adam_m": 1, "adam_v": 2, "grad": 3}[which]
    flat = train_buf[slot * 4 * P:(slot + 1) * 4 * P].view(torch.float32)
    out, o = {}, 0
    for name, shape in vct.MLP_PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].view(*shape)
        o += n
    return out


class Policy:
    """Device buffers of one learned controller: the inference blob and the training state."""

    def __init__(self, batch: int = 4096, device="cuda"):
        self.batch = int(batch)
        self.blob = torch.zeros(vct.vct_mlp_blob_bytes(), dtype=torch.uint8, device=device)
        nb = vct.vct_mlp_train_bytes(self.batch)
        if nb == 0:
            raise ValueError(f"batch {batch} must be a multiple of 64 in [64, 65536]")
        self.train_buf = torch.zeros(nb, dtype=torch.uint8, device=device)
        self.step_count = 0

    def init(self, seed: int, stream=None) -> None:
        vct.vct_mlp_init(seed, self.train_buf, self.blob, stream)
        self.step_count = 0

    def normalize(self, rows: torch.Tensor, box_q: float = 0.0, stream=None) -> None:
        vct.vct_mlp_normalize(rows, rows.numel() // ROW, box_q, self.train_buf, self.blob, stream)

    def step(self, rows: torch.Tensor, seed: int, lr: float, idx: torch.Tensor | None = None,
             batch: int | None = None, apply: bool = True, stream=None) -> None:
        b = self.batch if batch is None else int(batch)
        vct.vct_mlp_train_step(rows, rows.numel() // ROW, idx, seed, self.step_count, b, lr, apply,
                               self.train_buf, self.blob, stream)
        if apply:
            self.step_count += 1

    def loss(self) -> torch.Tensor:
        return self.train_buf[16 * P:16 * P + 4].view(torch.float32)

    def grad(self) -> dict:
        return params_view(self.train_buf, "grad")

    def train(self, rows: torch.Tensor, steps: int, seed: int, lr: float = 1e-3, lr_min: float = 0.0,
              log_every: int = 0, stream=None) -> list[tuple[int, float]]:
        """Adam with a cosine learning-rate decay from lr to lr_min over `steps` minibatches
        drawn with replacement. Returns (step, loss) at every log_every steps."""
        log = []
        marks = sorted({s for s in range(0, steps, log_every)} | {steps - 1}) if log_every else [steps - 1]
        done = 0
        for m in marks:   # the library runs the steps up to each logged one in one call
            vct.vct_mlp_train(rows, rows.numel() // ROW, seed, self.step_count, m + 1 - done, done, max(1, steps),
                              self.batch, lr, lr_min, self.train_buf, self.blob, stream)
            self.step_count += m + 1 - done
            done = m + 1
            if log_every:
                log.append((m, float(self.loss().item())))
        return log

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        n = x.numel() // vct.VCT_MLP_IN
        out = torch.empty(n, dtype=torch.float32, device=x.device)
        vct.vct_mlp_forward(x, n, self.blob, out, stream)
        return out

    def load(self, net: dict) -> None:
        """Put a host-side network (see pack_blob) into the blob."""
        self.blob.copy_(torch.from_numpy(pack_blob(net)))


def record_dataset(trial: dict, device="cuda", stream=None) -> tuple[torch.Tensor, dict]:
    """Run the MPC arm of `trial` with recording on: returns the (K n, 13) FP32 rows (inputs,
    then u/u_b) and the trial summary."""
    if int(trial["ctrl_kind"]) != vct.VCT_CTRL_MPC:
        raise ValueError("the behaviour-cloning data set is recorded from the MPC")
    bufs = T.TrialBuffers(trial, device)
    rows = torch.empty(bufs.K * bufs.n * ROW, dtype=torch.float32, device=device)
    bufs.record = rows
    summary, _ = T.run(trial, device, bufs=bufs, stream=stream)
    return rows.view(-1, ROW), summary
