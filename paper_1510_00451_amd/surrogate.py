"""Surrogate driver: model packing, a labelled dataset from the plain path,
the training loop and ensemble inference with plain-solve fallback.

Every numeric step (features, network, loss, gradients, Adam, gate, fallback
solves) runs in libshmm.so; this module only allocates buffers, draws the
seeded initial weights and the batch order, and sequences calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import abi


def _torch():
    import torch
    return torch

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
    """He-uniform initial weights from a seeded generator: zero hidden biases, a
    small last layer whose biases start the enhancement K - K_b near
    e^-4 sqrt(det K_b) I."""
    rng = np.random.default_rng(seed)
    W, b = [], []
    for fi, fo in LAYERS:
        lim = math.sqrt(6.0 / fi)
        W.append(rng.uniform(-lim, lim, (fo, fi)))
        b.append(np.zeros(fo))
    W[-1] *= 0.1
    b[-1][0] = b[-1][2] = -2.0
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
        self.loss = torch.zeros(E, 2, dtype=torch.float64, device="cuda")   # loss, gradient norm
        self.step = 0
        s = torch.cuda.current_stream().cuda_stream
        for e in range(E):
            ctx.shmm_surrogate_refresh(self.model_ptr(e), s)

    def model_ptr(self, e: int) -> int:
        return self.buf.data_ptr() + e * abi.SURR_MODEL_BYTES

    def member_losses(self, data: "Dataset") -> np.ndarray:
        """Mean relative squared Frobenius error of every member on `data`."""
        torch = self.torch
        B = data.x.shape[0]
        K = torch.empty(B, 3, dtype=torch.float64, device="cuda")
        flags = torch.empty(B, dtype=torch.uint8, device="cuda")
        Km = torch.empty(self.E, B, 3, dtype=torch.float64, device="cuda")
        hi = torch.full((abi.SURR_IN,), math.inf, dtype=torch.float32, device="cuda")
        lo = -hi
        self.ctx.shmm_surrogate_infer(self.buf.data_ptr(), self.E, data.x.data_ptr(), data.Kb.data_ptr(), B,
                                      lo.data_ptr(), hi.data_ptr(), math.inf, math.inf, K.data_ptr(),
                                      flags.data_ptr(), 0, Km.data_ptr(), torch.cuda.current_stream().cuda_stream)
        Kt = data.K.cpu().numpy()
        return np.array([float(np.mean(relative_frobenius(m, Kt) ** 2)) for m in Km.cpu().numpy()])

    def prune(self, data: "Dataset", factor: float = 3.0) -> np.ndarray:
        """Drop members whose loss on `data` exceeds `factor` times the best
        member's (a member that failed to train would otherwise dominate the
        ensemble spread).  Returns the losses of all members before pruning."""
        losses = self.member_losses(data)
        keep = [e for e in range(self.E) if losses[e] <= factor * losses.min()]
        if len(keep) < self.E:
            words = abi.SURR_MODEL_BYTES // 4
            self.buf = self.torch.cat([self.buf[e * words:(e + 1) * words] for e in keep]).contiguous()
            self.adam = self.adam[keep].contiguous()
            self.loss = self.loss[keep].contiguous()
            self.E = len(keep)
        return losses

    def member_host(self, e: int) -> np.ndarray:
        return self.buf[e * (PARAM_FLOATS):(e + 1) * PARAM_FLOATS].cpu().numpy()


@dataclass
class Dataset:
    x: "object"        # torch float32 [S][35] on device
    Kb: "object"       # torch float64 [S][3]
    K: "object"        # torch float64 [S][3]

    def rescaled(self, ctx: abi.Context, log10_c):
        """The same local problems with velocity and diffusivity scaled by
        c = 10^log10_c (one factor per sample, host array [S]), computed by
        shmm_surrogate_rescale: the corrector is unchanged, so K and K_b scale
        by c, the 32 band features (squared Peclet numbers) are unchanged and
        feature 32 shifts by ln c."""
        torch = _torch()
        S = self.x.shape[0]
        lc = torch.from_numpy(np.ascontiguousarray(log10_c, np.float64)).to(self.K.device)
        out = Dataset(torch.empty_like(self.x), torch.empty_like(self.Kb), torch.empty_like(self.K))
        ctx.shmm_surrogate_rescale(self.x.data_ptr(), self.Kb.data_ptr(), self.K.data_ptr(), lc.data_ptr(), S,
                                   out.x.data_ptr(), out.Kb.data_ptr(), out.K.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        return out

    @staticmethod
    def concat(parts):
        torch = _torch()
        return Dataset(torch.cat([p.x for p in parts]), torch.cat([p.Kb for p in parts]),
                       torch.cat([p.K for p in parts]))


def train(ens: Ensemble, data: Dataset, steps: int, batch: int, lr0: float = 1e-3, seed: int = 0,
          log=None, clip: float = 0.0) -> List[float]:
    """Adam with a linear warm-up over the first 5% of the steps, then a cosine
    decay, on gradients clipped to global norm `clip` (0: no clipping); each
    member draws its own batch order."""
    torch = ens.torch
    S = data.x.shape[0]
    rng = np.random.default_rng(seed)
    s = torch.cuda.current_stream().cuda_stream
    xb = torch.empty(batch, abi.SURR_IN, dtype=torch.float32, device="cuda")
    kb = torch.empty(batch, 3, dtype=torch.float64, device="cuda")
    kt = torch.empty(batch, 3, dtype=torch.float64, device="cuda")
    history = []
    chunk = 64
    for it in range(steps):
        warm = max(1, steps // 20)
        lr = lr0 * (it + 1) / warm if it < warm else \
            0.5 * lr0 * (1.0 + math.cos(math.pi * (it - warm) / max(1, steps - warm)))
        if it % chunk == 0:     # batch indices of the next steps, one upload
            draws = torch.from_numpy(rng.integers(0, S, (min(chunk, steps - it), ens.E, batch))).to("cuda")
        for e in range(ens.E):
            idx = draws[it % chunk, e]
            torch.index_select(data.x, 0, idx, out=xb)
            torch.index_select(data.Kb, 0, idx, out=kb)
            torch.index_select(data.K, 0, idx, out=kt)
            ens.ctx.shmm_surrogate_train_step(ens.model_ptr(e), ens.adam[e].data_ptr(), xb.data_ptr(),
                                              kb.data_ptr(), kt.data_ptr(), batch, lr, clip, it + 1,
                                              ens.loss[e].data_ptr(), 0, s)
        if log is not None and (it % max(1, steps // 10) == 0 or it == steps - 1):
            l = ens.loss.cpu().numpy()
            history.append(float(l[:, 0].mean()))
            log(f"surrogate step {it}: loss {l[:, 0]} gradient norm {l[:, 1]}")
    return history


def infer(ens: Ensemble, x, Kb, lo, hi, tau: float, emax: float = math.inf):
    """(K_mean [B][3], flags [B] uint8, spread [B]) on the device (tau and emax
    may be infinite to gate on the feature range alone)."""
    torch = ens.torch
    B = x.shape[0]
    K = torch.empty(B, 3, dtype=torch.float64, device="cuda")
    flags = torch.empty(B, dtype=torch.uint8, device="cuda")
    spread = torch.empty(B, dtype=torch.float64, device="cuda")
    ens.ctx.shmm_surrogate_infer(ens.buf.data_ptr(), ens.E, x.data_ptr(), Kb.data_ptr(), B, lo.data_ptr(),
                                 hi.data_ptr(), tau, emax, K.data_ptr(), flags.data_ptr(), spread.data_ptr(), 0,
                                 torch.cuda.current_stream().cuda_stream)
    return K, flags, spread


class IsotropicPhase:
    """One phase of a batch of flows (default: the finest level of each), every
    patch on the isotropic base kappa I of its flow: the setting in which the
    surrogate replaces the local solve.

    The constructor only allocates.  ``prepare()`` runs the band filter of the
    phase and plans its steps; then either ``plain()`` (the local solves of
    every patch: labels, or the plain form) or ``surrogate(...)`` (features,
    ensemble inference, plain-solve fallback of the flagged patches) gives
    K [count][3] on the device.  Patches whose diagonal band holds no
    coefficient are inactive: their result is the base exactly and neither form
    spends solver steps on them.
    """

    def __init__(self, problems, phase: int = 0, device: int = 0):
        from .hierarchy import Hierarchy
        torch = _torch()
        self.torch = torch
        H = Hierarchy(problems, device)
        self.H = H
        self.first = int(H.phase[phase])
        self.count = int(H.phase[phase + 1] - H.phase[phase])
        sl = slice(self.first, self.first + self.count)
        kap = np.array([H.problems[i].kappa for i in H.table["instance"][sl]])
        H.host_K[sl] = np.stack([kap, np.zeros_like(kap), kap], 1)
        H.K_base[sl] = torch.from_numpy(H.host_K[sl]).to(H.device)
        self.n = H.table["n"][sl].copy()
        self.x = torch.zeros(self.count, abi.SURR_IN, dtype=torch.float32, device=H.device)
        self.K = torch.zeros(H.nd, 3, dtype=torch.float64, device=H.device)
        self.flags = torch.zeros(self.count, dtype=torch.uint8, device=H.device)
        self.spread = torch.zeros(self.count, dtype=torch.float64, device=H.device)
        self.nsteps = None

    def prepare(self) -> None:
        """Band filter of the phase and its step plan (synchronises: the plan is host work)."""
        H = self.H
        H.status[self.first:self.first + self.count].zero_()
        H.ctx.shmm_band_filter(self.first, self.count, 0, H.vx.data_ptr(), H.vy.data_ptr(), H.f1.data_ptr(),
                               H.f2.data_ptr(), H.lines.data_ptr(), H.stream())
        H.ctx.shmm_plan_steps(self.first, self.count, H.host_K)
        table = H.ctx.shmm_ctx_table()[0]
        self.nsteps = table["nsteps"][self.first:self.first + self.count].copy()
        self.active = self.nsteps > 0
        self.point_steps = int(np.sum(self.n.astype(np.int64) ** 2 * self.nsteps))

    def features(self) -> None:
        """Features of every patch of the phase (runs of equal n, one call each)."""
        H = self.H
        s = H.stream()
        i = 0
        while i < self.count:
            j = i
            while j < self.count and self.n[j] == self.n[i]:
                j += 1
            H.ctx.shmm_patch_features(self.first + i, j - i, H.vx.data_ptr(), H.vy.data_ptr(),
                                      H.K_base.data_ptr(), self.x[i:].data_ptr(), s)
            i = j

    def K_base(self):
        return self.H.K_base[self.first:self.first + self.count]

    def plain(self, adaptive: bool = False):
        """Plain local solves and estimator of every patch; returns K [count][3]
        (device).  `adaptive`: quasi-stationary stop instead of the full plan
        (synchronises after every chunk; the plan is cut to the steps taken)."""
        H = self.H
        s = H.stream()
        a, b = H.cell_range(self.first, self.count)
        H.w.view(2, H.cells)[:, a:b].zero_()
        if adaptive:
            H.ctx.shmm_local_solve_adaptive(self.first, self.count, H.vx.data_ptr(), H.vy.data_ptr(),
                                            H.f1.data_ptr(), H.f2.data_ptr(), H.K_base.data_ptr(), H.w.data_ptr(),
                                            H.adaptive_chunks, H.adaptive_tol, H.status.data_ptr(), s)
        else:
            H.ctx.shmm_local_solve_batch(self.first, self.count, H.vx.data_ptr(), H.vy.data_ptr(),
                                         H.f1.data_ptr(), H.f2.data_ptr(), H.K_base.data_ptr(), H.w.data_ptr(),
                                         0, 2 ** 31 - 1, H.status.data_ptr(), s)
        H.ctx.shmm_effective_diffusivity(self.first, self.count, H.f1.data_ptr(), H.f2.data_ptr(),
                                         H.w.data_ptr(), H.K_base.data_ptr(), H.K_solve.data_ptr(), 0, 0,
                                         H.status.data_ptr(), s)
        return H.K_solve[self.first:self.first + self.count]

    def surrogate(self, ens: "Ensemble", lo, hi, tau: float, emax: float = math.inf, adaptive: bool = False):
        """Surrogate-with-fallback form: features, ensemble estimate and gate,
        plain solves of the flagged patches (with the quasi-stationary stop
        when `adaptive`); returns K [count][3] (device).  Synchronises (the
        fallback reads the flags)."""
        H = self.H
        s = H.stream()
        self.features()
        sl = self.K[self.first:self.first + self.count]
        H.ctx.shmm_surrogate_infer(ens.buf.data_ptr(), ens.E, self.x.data_ptr(), self.K_base().data_ptr(),
                                   self.count, lo.data_ptr(), hi.data_ptr(), tau, emax, sl.data_ptr(),
                                   self.flags.data_ptr(), self.spread.data_ptr(), 0, s)
        H.ctx.shmm_fallback_solve(self.first, self.count, self.flags.data_ptr(), H.vx.data_ptr(),
                                  H.vy.data_ptr(), H.f1.data_ptr(), H.f2.data_ptr(), H.K_base.data_ptr(),
                                  H.w.data_ptr(), self.K.data_ptr(), H.adaptive_chunks if adaptive else 0,
                                  H.adaptive_tol, H.status.data_ptr(), s)
        return sl

    def close(self):
        self.H.close()


def relative_frobenius(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """|A - B|_F / |B|_F of symmetric 2x2 tensors stored as {K11, K12, K22}."""
    d = A - B
    return np.sqrt((d[:, 0] ** 2 + 2 * d[:, 1] ** 2 + d[:, 2] ** 2) /
                   (B[:, 0] ** 2 + 2 * B[:, 1] ** 2 + B[:, 2] ** 2))


def labelled_set(problem_batches, log=None, adaptive: bool = False) -> Dataset:
    """Features and plain-path labels of the finest-level patches of each batch
    of flows (isotropic base kappa I), active patches only (`adaptive`: the
    solves stop at the quasi-stationary test)."""
    torch = _torch()
    xs, kbs, ks = [], [], []
    for i, probs in enumerate(problem_batches):
        ph = IsotropicPhase(probs)
        ph.prepare()
        ph.features()
        K = ph.plain(adaptive)
        act = torch.from_numpy(np.flatnonzero(ph.active)).to(ph.x.device)
        xs.append(ph.x.index_select(0, act))
        kbs.append(ph.K_base().index_select(0, act))
        ks.append(K.index_select(0, act))
        torch.cuda.synchronize()
        ph.close()
        if log is not None:
            log(f"labels: batch {i}, {sum(len(x) for x in xs)} patches")
    return Dataset(torch.cat(xs), torch.cat(kbs), torch.cat(ks))


def chained_set(problem_batches, log=None, adaptive: bool = True) -> Dataset:
    """Features and plain-path labels of every level's patches of whole
    hierarchy passes (Algorithm 3 bases: the finest level's from the
    off-diagonal chain above it, the coarser levels' from K_star - K_off +
    K_in; anisotropic in general), one pass per batch of flows, the local
    solves stopped at the quasi-stationary test when `adaptive`.  Patches with
    an empty diagonal band (their result is the base) are left out."""
    from .hierarchy import Hierarchy
    torch = _torch()
    xs, kbs, ks = [], [], []
    for i, probs in enumerate(problem_batches):
        H = Hierarchy(probs)
        H.run(adaptive=adaptive)
        x = torch.zeros(H.nd, abi.SURR_IN, dtype=torch.float32, device=H.device)
        t = H.ctx.shmm_ctx_table()[0]
        n = t["n"]
        d = 0
        while d < H.nd:                    # runs of one patch size
            e = d
            while e < H.nd and n[e] == n[d]:
                e += 1
            H.ctx.shmm_patch_features(d, e - d, H.vx.data_ptr(), H.vy.data_ptr(), H.K_base.data_ptr(),
                                      x[d].data_ptr(), H.stream())
            d = e
        act = torch.from_numpy(np.flatnonzero(t["nsteps"] > 0)).to(H.device)
        xs.append(x.index_select(0, act))
        kbs.append(H.K_base.index_select(0, act))
        ks.append(H.K_solve.index_select(0, act))
        torch.cuda.synchronize()
        H.close()
        if log is not None:
            log(f"chained labels: batch {i}, {sum(len(v) for v in xs)} patches")
    return Dataset(torch.cat(xs), torch.cat(kbs), torch.cat(ks))


def split(data: Dataset, frac: float, seed: int):
    """(held-out, rest) by a seeded permutation."""
    torch = _torch()
    S = data.x.shape[0]
    perm = torch.from_numpy(np.random.default_rng(seed).permutation(S)).to(data.x.device)
    k = int(S * frac)
    pick = lambda idx: Dataset(data.x[idx], data.Kb[idx], data.K[idx])
    return pick(perm[:k]), pick(perm[k:])


def feature_stats(ctx: abi.Context, x):
    """(mean, std, min, max) of every feature column of x [S][35] (device),
    FP64 host arrays, from shmm_feature_stats."""
    torch = _torch()
    st = torch.empty(4, abi.SURR_IN, dtype=torch.float64, device=x.device)
    ctx.shmm_feature_stats(x.data_ptr(), x.shape[0], st.data_ptr(), torch.cuda.current_stream().cuda_stream)
    h = st.cpu().numpy()
    return h[0], h[1], h[2], h[3]


def gate_range(ctx: abi.Context, data: Dataset, margin: float = 0.1):
    """Per-feature training range widened by `margin` of its width (device
    float32, the gate's bounds; the range itself from shmm_feature_stats)."""
    torch = _torch()
    _, _, lo, hi = feature_stats(ctx, data.x)
    w = hi - lo
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(data.x.device)
    return dev(lo - margin * w), dev(hi + margin * w)


def gate_inputs(ens: Ensemble, data: Dataset, lo, hi):
    """Per labelled patch (host arrays): the relative Frobenius error of the
    ensemble mean against the label, the predicted enhancement
    |K_hat - K_b|_F / |K_b|_F, the ensemble spread, and whether every feature
    lies inside the gate's range."""
    K, flags, spread = infer(ens, data.x, data.Kb, lo, hi, math.inf, math.inf)
    Kn, Kt, Kb = K.cpu().numpy(), data.K.cpu().numpy(), data.Kb.cpu().numpy()
    return (relative_frobenius(Kn, Kt), relative_frobenius(Kn, Kb), spread.cpu().numpy(),
            ~flags.cpu().numpy().astype(bool))


def calibrate_gate(ens: Ensemble, held: Dataset, lo, hi, target: float = 0.01, quantile: float = 0.99,
                   taus=(5e-4, 1e-3, 1.5e-3, 2e-3, 2.5e-3, 3e-3, 4e-3, 5e-3, 6e-3, 7.5e-3, 1e-2, 1.5e-2,
                         2e-2, 3e-2),
                   emaxes=(0.01, 0.02, 0.03, 0.05, 0.07, 0.1, 0.15, 0.2, 0.5, 1.0, 2.0, 5.0, math.inf)):
    """Spread threshold tau and enhancement limit emax of the gate: the pair
    that accepts the most held-out patches while the `quantile` of their
    relative Frobenius error stays within `target`.  Ties go to the larger
    thresholds.  Returns (tau, emax, accepted fraction); when no pair keeps
    the quantile within `target`, (-1, -1, 0): thresholds that flag every
    patch, so the plain path answers everywhere."""
    err, enh, spread, inside = gate_inputs(ens, held, lo, hi)
    best = (-1.0, -1.0, -1.0)
    for tau in taus:
        for emax in emaxes:
            acc = inside & (spread <= tau) & (enh <= emax)
            if not acc.any() or np.quantile(err[acc], quantile) > target:
                continue
            frac = float(acc.mean())
            if frac >= best[2]:
                best = (tau, emax, frac)
    return best if best[2] >= 0 else (-1.0, -1.0, 0.0)
