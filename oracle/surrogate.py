"""FP64 oracle of the learned surrogate of the local solve.  TEST INFRASTRUCTURE
ONLY (see the package docstring).

The paper has no surrogate; these definitions are this project's readings:

* Features of a patch (35): band energies of the patch velocity spectrum in 4
  channels x 8 radial bins.  With the patch samples treated as periodic and
  the DFT normalised so that sum_k |vx^(k)|^2 = mean(vx^2), the channels of a
  mode k are |vx^|^2, |vy^|^2, |vx^ + vy^|^2 / 2 and |vx^ - vy^|^2 / 2 (the
  last two carry the cross spectrum, which decides the sign of K12).  Bin b
  holds the patch-relative integer wavenumbers k with q = |k| in [2^b, 2^(b+1)),
  b = 0..7 (octaves of q from 1 to 256: every mode of a patch of up to 256^2
  but the mean).  Each mode enters its bin weighted by (L / 2 pi)^2 / q^2, L
  the patch side: E_cb = sum over the bin of channel_c(k) / |k_phys|^2, with
  k_phys = 2 pi k / L.  At small Peclet number the local solve gives, to first
  order, K11 - K_b11 = sum_b E_0b / kappa, K22 - K_b22 = sum_b E_1b / kappa and
  K12 - K_b12 = sum_b (E_2b - E_3b) / (2 kappa) for an isotropic base kappa I
  (exactly, for a shear flow), so these energies carry that limit whatever the
  width of the bins; the bins resolve where in the spectrum the energy sits,
  which the higher orders need.  feature_{8c+b} = log((E_cb + 1e-8 E_tot +
  1e-30) / det K_b), E_tot the sum of channels 0 and 1 over the bins (the floor
  sits far above the rounding noise of an FP32 transform, about 1e-12 E_tot,
  so empty bins read the same in FP32 and FP64).  Dividing by det K_b makes
  these 32 features squared Peclet numbers: for an isotropic base the local
  problem is invariant under scaling velocity and diffusivity together (K
  scales with them), so K / kappa depends on them alone.  Feature 32 is log sqrt(det K_b).  Features 33 and
  34 carry the anisotropy of the base: the (1,1) and (1,2) entries of the
  traceless part of the matrix logarithm log K_b (zero for an isotropic base,
  unchanged when the base is scaled, turning with twice the angle of its
  principal axes), so that a base from a coarser level's chain (Algorithm 3)
  can be given to the network.  The directional channels give the network
  the anisotropy of K that radial energies alone cannot.
* Gate: a patch falls back to the plain solve when a feature leaves the
  training range, when the ensemble disagrees (spread > tau), or when the
  predicted enhancement is beyond emax (the regime where the network was not
  shown accurate).
* Network: 35 -> 256 -> 256 -> 256 -> 3 with exact (erf) GELU; inputs are
  standardised with stored means and scales.  Head: L = [[e^o1, 0], [o2, e^o3]],
  K = K_b + sqrt(det K_b) L L^T: the enhancement K - K_b is positive
  semi-definite (the local solve only adds diffusivity), and its logarithmic
  parametrisation keeps small enhancements at the same relative precision as
  large ones.
* Loss: mean over the batch of |K_hat - K|_F^2 / |K|_F^2 (Frobenius norm of the
  full 2x2 tensor).
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master weights.
* Precision emulation: `bf16=True` rounds the network's inputs, weights and
  hidden activations to bfloat16 (round to nearest even) exactly where the
  GPU kernels feed its matrix cores, so both sides decide the same roundings.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

N_BINS = 32
N_IN = 35
WIDTH = 256
N_OUT = 3
LAYERS = [(N_IN, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, N_OUT)]


# ---------------------------------------------------------------- features

N_CHANNELS = 4
N_RADIAL = 8


def bin_of(k1: int, k2: int) -> int:
    """Octave bin of the integer wavenumber (k1, k2): b with 2^b <= |k| < 2^(b+1),
    i.e. 4^b <= k1^2 + k2^2 < 4^(b+1); -1 for the mean and for |k| >= 256."""
    q2 = k1 * k1 + k2 * k2
    return (q2.bit_length() - 1) // 2 if 1 <= q2 < 4 ** N_RADIAL else -1


def channel_energies(vx: np.ndarray, vy: np.ndarray, n: int, N: int) -> np.ndarray:
    """E[c][b]: channel c over |k_phys|^2, summed over octave bin b (see the
    module docstring)."""
    vx = np.asarray(vx, np.float64).reshape(n, n)
    vy = np.asarray(vy, np.float64).reshape(n, n)
    X = np.fft.fft2(vx) / float(n * n)
    Y = np.fft.fft2(vy) / float(n * n)
    s = (n / N) ** 2                                  # (L / 2 pi)^2 with L = n 2 pi / N
    chans = [np.abs(X) ** 2, np.abs(Y) ** 2, np.abs(X + Y) ** 2 / 2, np.abs(X - Y) ** 2 / 2]
    k = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    E = np.zeros((N_CHANNELS, N_RADIAL))
    for j in range(n):               # row: k2 = k[j]
        for i in range(n):           # column: k1 = k[i]
            b = bin_of(int(k[i]), int(k[j]))
            if b < 0:
                continue
            q2 = float(k[i] * k[i] + k[j] * k[j])
            for c in range(N_CHANNELS):
                E[c, b] += chans[c][j, i] * s / q2
    return E


def log_base_anisotropy(K_base) -> Tuple[float, float]:
    """(T11, T12) of T = log K_b - (1/2) tr(log K_b) I, the traceless part of
    the matrix logarithm of the base (its eigen-decomposition by LAPACK)."""
    K11, K12, K22 = [float(v) for v in K_base]
    lam, vec = np.linalg.eigh(np.array([[K11, K12], [K12, K22]]))
    L = vec @ np.diag(np.log(lam)) @ vec.T
    T = L - 0.5 * np.trace(L) * np.eye(2)
    return float(T[0, 0]), float(0.5 * (T[0, 1] + T[1, 0]))


def patch_features(vx: np.ndarray, vy: np.ndarray, n: int, N: int, K_base) -> np.ndarray:
    """35 features of one n x n patch (velocities [y][x]) with spacing 2 pi / N."""
    E = channel_energies(vx, vy, n, N)
    floor = 1e-8 * float(np.sum(E[0]) + np.sum(E[1])) + 1e-30
    K11, K12, K22 = [float(v) for v in K_base]
    logdet = math.log(K11 * K22 - K12 * K12)
    out = np.zeros(N_IN)
    for c in range(N_CHANNELS):
        for b in range(N_RADIAL):
            out[N_RADIAL * c + b] = math.log(E[c, b] + floor) - logdet
    out[N_BINS] = 0.5 * logdet
    out[N_BINS + 1], out[N_BINS + 2] = log_base_anisotropy(K_base)
    return out


# ---------------------------------------------------------------- bf16

def bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- network

def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _erf(z):
    from scipy.special import erf
    return erf(z)


@dataclass
class Net:
    """Weights W_l of shape (out, in) and biases b_l; input standardisation."""
    W: List[np.ndarray]
    b: List[np.ndarray]
    mu: np.ndarray = field(default_factory=lambda: np.zeros(N_IN))
    sigma: np.ndarray = field(default_factory=lambda: np.ones(N_IN))

    def copy(self) -> "Net":
        return Net([w.copy() for w in self.W], [v.copy() for v in self.b], self.mu.copy(), self.sigma.copy())


INIT_LOG_ENHANCEMENT = -2.0     # initial o1 = o3: K - K_b starts near e^-4 sqrt(det K_b) I


def init_net(seed: int) -> Net:
    """He-uniform weights from a seeded generator (an input, not method arithmetic)."""
    rng = np.random.default_rng(seed)
    W, b = [], []
    for fi, fo in LAYERS:
        lim = math.sqrt(6.0 / fi)
        W.append(rng.uniform(-lim, lim, (fo, fi)))
        b.append(np.zeros(fo))
    W[-1] *= 0.1
    b[-1][0] = b[-1][2] = INIT_LOG_ENHANCEMENT
    return Net(W, b)


def forward(net: Net, x: np.ndarray, bf16_mode: bool = False):
    """Forward pass; returns (outputs o [B][3], cache for the backward)."""
    x = (np.asarray(x, np.float64) - net.mu) / net.sigma
    rnd = bf16 if bf16_mode else (lambda a: np.asarray(a, np.float64))
    acts = [rnd(x)]
    pre = []
    h = acts[0]
    for l in range(4):
        z = h @ rnd(net.W[l]).T + net.b[l]
        pre.append(z)
        if l < 3:
            h = rnd(gelu(z))
            acts.append(h)
        else:
            h = z
    return h, (acts, pre)


def head(o: np.ndarray, K_base: np.ndarray) -> np.ndarray:
    """Cholesky head: K = K_b + sqrt(det K_b) L L^T, L = [[e^o1, 0], [o2, e^o3]]; returns [B][3]."""
    o = np.atleast_2d(o)
    Kb = np.atleast_2d(K_base)
    s = np.sqrt(Kb[:, 0] * Kb[:, 2] - Kb[:, 1] ** 2)
    l11, l21, l22 = np.exp(o[:, 0]), o[:, 1], np.exp(o[:, 2])
    return Kb + np.stack([s * l11 * l11, s * l11 * l21, s * (l21 * l21 + l22 * l22)], 1)


def loss_and_grad_o(o: np.ndarray, K_base: np.ndarray, K_true: np.ndarray):
    """Mean relative Frobenius loss and its gradient with respect to the outputs."""
    o = np.atleast_2d(o)
    Kb = np.atleast_2d(K_base)
    Kt = np.atleast_2d(K_true)
    B = o.shape[0]
    s = np.sqrt(Kb[:, 0] * Kb[:, 2] - Kb[:, 1] ** 2)
    l11, l21, l22 = np.exp(o[:, 0]), o[:, 1], np.exp(o[:, 2])
    Kh = head(o, Kb)
    d = Kh - Kt
    nrm = Kt[:, 0] ** 2 + 2 * Kt[:, 1] ** 2 + Kt[:, 2] ** 2
    loss = float(np.mean((d[:, 0] ** 2 + 2 * d[:, 1] ** 2 + d[:, 2] ** 2) / nrm))
    # dloss/dK_hat components (the off-diagonal appears twice in the norm)
    g = np.stack([2 * d[:, 0], 4 * d[:, 1], 2 * d[:, 2]], 1) / nrm[:, None] / B
    # K11 = Kb11 + s l11^2, K12 = Kb12 + s l11 l21, K22 = Kb22 + s (l21^2 + l22^2)
    go = np.zeros_like(o)
    go[:, 0] = (g[:, 0] * 2 * s * l11 * l11 + g[:, 1] * s * l11 * l21)     # dl11/do1 = l11
    go[:, 1] = g[:, 1] * s * l11 + g[:, 2] * 2 * s * l21
    go[:, 2] = g[:, 2] * 2 * s * l22 * l22
    return loss, go


def backward(net: Net, cache, go: np.ndarray, bf16_mode: bool = False):
    """Gradients of the weights and biases for the output gradient go."""
    acts, pre = cache
    rnd = bf16 if bf16_mode else (lambda a: np.asarray(a, np.float64))
    gW = [None] * 4
    gb = [None] * 4
    dz = go
    for l in range(3, -1, -1):
        dzr = rnd(dz)                       # matrix-core operand
        gW[l] = dzr.T @ acts[l]
        gb[l] = dz.sum(axis=0)
        if l > 0:
            dh = dzr @ rnd(net.W[l])
            dz = dh * gelu_grad(pre[l - 1])
    return gW, gb


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: Optional[List[np.ndarray]] = None
    v: Optional[List[np.ndarray]] = None

    def step(self, params: List[np.ndarray], grads: List[np.ndarray], lr: Optional[float] = None,
             clip: Optional[float] = None):
        """One Adam update with bias correction (Kingma & Ba), in place, on the
        gradients scaled to global norm at most `clip` when given."""
        if clip is not None and clip > 0:
            norm = math.sqrt(sum(float(np.sum(g * g)) for g in grads))
            if norm > clip:
                grads = [g * (clip / norm) for g in grads]
        if self.m is None:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros_like(p) for p in params]
        self.t += 1
        a = self.lr if lr is None else lr
        c1 = 1.0 - self.beta1 ** self.t
        c2 = 1.0 - self.beta2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.beta1
            m += (1.0 - self.beta1) * g
            v *= self.beta2
            v += (1.0 - self.beta2) * g * g
            p -= a * (m / c1) / (np.sqrt(v / c2) + self.eps)


# ---------------------------------------------------------------- gate

def ensemble_gate(K_members: np.ndarray, features: np.ndarray, lo: np.ndarray, hi: np.ndarray,
                  tau: float, K_base: Optional[np.ndarray] = None, emax: float = math.inf):
    """Mean prediction and fallback flag of an ensemble.

    K_members [E][B][3].  Flag a patch when any feature lies outside [lo, hi]
    (the training range), when the largest member deviation from the mean,
    in Frobenius norm relative to the mean, exceeds tau, or when the predicted
    enhancement |K_mean - K_base| / |K_base| (Frobenius) exceeds emax."""
    Km = K_members.mean(axis=0)
    d = K_members - Km[None]
    fro = lambda a: np.sqrt(a[..., 0] ** 2 + 2 * a[..., 1] ** 2 + a[..., 2] ** 2)
    spread = fro(d).max(axis=0) / fro(Km)
    out = np.any((features < lo) | (features > hi), axis=1)
    flag = (spread > tau) | out
    if K_base is not None:
        Kb = np.atleast_2d(K_base)
        flag |= ~(fro(Km - Kb) / fro(Kb) <= emax)
    return Km, flag, spread
