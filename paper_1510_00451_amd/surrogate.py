"""Surrogate driver: model packing, a labelled dataset from the plain path,
the training loop and ensemble inference with plain-solve fallback.

Every numeric step (features, network, loss, gradients, Adam, gate, fallback
solves) runs in libshmm.so; this module only allocates buffers, draws the
seeded initial weights and the batch order, and sequences calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import abi

PARAM_FLOATS = abi.SURR_MODEL_BYTES // 4
LAYERS = [(abi.SURR_IN, abi.SURR_WIDTH), (abi.SURR_WIDTH, abi.SURR_WIDTH),
          (abi.SURR_WIDTH, abi.SURR_WIDTH), (abi.SURR_WIDTH, abi.SURR_OUT)]


def pack_params(W: Sequence[np.ndarray], b: Sequence[np.ndarray], mu, sigma) -> np.ndarray:
    """Host image (float32 words) of one model block: params | mu | sigma | bf16 (filled on device)."""
    out = np.zeros(PARAM_FLOATS, np.float32)
    off = 0
    for Wl, bl in zip(W, b):
        out[off:off + Wl.size] = np.asarray(Wl, np.float32).reshape(-1)
        off += Wl.size
        out[off:off + bl.size] = np.asarray(bl, np.float32)
        off += bl.size
    assert off == abi.SURR_PARAMS
    base = abi.SURR_PARAMS_PADDED
    out[base:base + abi.SURR_IN] = np.asarray(mu, np.float32)
    out[base + 64:base + 64 + abi.SURR_IN] = np.asarray(sigma, np.float32)
    return out


def unpack_params(block: np.ndarray):
    W, b = [], []
    off = 0
    for fi, fo in LAYERS:
        W.append(block[off:off + fi * fo].reshape(fo, fi).astype(np.float64))
        off += fi * fo
        b.append(block[off:off + fo].astype(np.float64))
        off += fo
    base = abi.SURR_PARAMS_PADDED
    return W, b, block[base:base + abi.SURR_IN].astype(np.float64), \
        block[base + 64:base + 64 + abi.SURR_IN].astype(np.float64)


def init_params(seed: int):
    """He-uniform initial weights from a seeded generator (zero biases, small last layer)."""
    rng = np.random.default_rng(seed)
    W, b = [], []
    for fi, fo in LAYERS:
        lim = math.sqrt(6.0 / fi)
        W.append(rng.uniform(-lim, lim, (fo, fi)))
        b.append(np.zeros(fo))
    W[-1] *= 0.1
    return W, b


class Ensemble:
    """E models in one device buffer plus their Adam state."""

    def __init__(self, ctx: abi.Context, E: int, mu, sigma, seed0: int = 0):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.E = E
        host = np.concatenate([pack_params(*init_params(seed0 + e), mu, sigma) for e in range(E)])
        self.buf = torch.from_numpy(host).to("cuda")
        self.adam = torch.zeros(E, 2 * abi.SURR_PARAMS_PADDED, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(E, dtype=torch.float64, device="cuda")
        self.step = 0
        s = torch.cuda.current_stream().cuda_stream
        for e in range(E):
            ctx.shmm_surrogate_refresh(self.model_ptr(e), s)

    def model_ptr(self, e: int) -> int:
        return self.buf.data_ptr() + e * abi.SURR_MODEL_BYTES

    def member_host(self, e: int) -> np.ndarray:
        return self.buf[e * (PARAM_FLOATS):(e + 1) * PARAM_FLOATS].cpu().numpy()


@dataclass
class Dataset:
    x: "object"        # torch float32 [S][33] on device
    Kb: "object"       # torch float64 [S][3]
    K: "object"        # torch float64 [S][3]


def train(ens: Ensemble, data: Dataset, steps: int, batch: int, lr0: float = 1e-3, seed: int = 0,
          log=None) -> List[float]:
    """Adam with a cosine learning-rate schedule; each member draws its own batch order."""
    torch = ens.torch
    S = data.x.shape[0]
    rng = np.random.default_rng(seed)
    s = torch.cuda.current_stream().cuda_stream
    xb = torch.empty(batch, abi.SURR_IN, dtype=torch.float32, device="cuda")
    kb = torch.empty(batch, 3, dtype=torch.float64, device="cuda")
    kt = torch.empty(batch, 3, dtype=torch.float64, device="cuda")
    history = []
    for it in range(steps):
        lr = 0.5 * lr0 * (1.0 + math.cos(math.pi * it / steps))
        for e in range(ens.E):
            idx = torch.from_numpy(rng.integers(0, S, batch)).to("cuda")
            torch.index_select(data.x, 0, idx, out=xb)
            torch.index_select(data.Kb, 0, idx, out=kb)
            torch.index_select(data.K, 0, idx, out=kt)
            ens.ctx.shmm_surrogate_train_step(ens.model_ptr(e), ens.adam[e].data_ptr(), xb.data_ptr(),
                                              kb.data_ptr(), kt.data_ptr(), batch, lr, it + 1,
                                              ens.loss[e:e + 1].data_ptr(), 0, s)
        if log is not None and (it % max(1, steps // 10) == 0 or it == steps - 1):
            l = ens.loss.cpu().numpy()
            history.append(float(l.mean()))
            log(f"surrogate step {it}: loss {l}")
    return history


def infer(ens: Ensemble, x, Kb, lo, hi, tau: float):
    """(K_mean [B][3], flags [B] uint8, spread [B]) on the device."""
    torch = ens.torch
    B = x.shape[0]
    K = torch.empty(B, 3, dtype=torch.float64, device="cuda")
    flags = torch.empty(B, dtype=torch.uint8, device="cuda")
    spread = torch.empty(B, dtype=torch.float64, device="cuda")
    ens.ctx.shmm_surrogate_infer(ens.buf.data_ptr(), ens.E, x.data_ptr(), Kb.data_ptr(), B, lo.data_ptr(),
                                 hi.data_ptr(), tau, K.data_ptr(), flags.data_ptr(), spread.data_ptr(), 0,
                                 torch.cuda.current_stream().cuda_stream)
    return K, flags, spread
