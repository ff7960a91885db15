"""FP64 CPU oracle of the SHMM hot path.  TEST INFRASTRUCTURE ONLY (see package doc).

Section / equation names refer to Lee & Engquist, "Multiscale numerical
methods for passive advection-diffusion in incompressible turbulent flow
fields" (arXiv:1510.00451).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shmm_oracle.c")
_SO = os.path.join(_HERE, "_shmm_oracle.so")

DIAG, OFF12, OFF21 = 0, 1, 2

# ---------------------------------------------------------------------------
# native loops (plain C, FP64)
# ---------------------------------------------------------------------------

def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (no contraction into FMAs)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.orc_synth_points.argtypes = [P, ctypes.c_int, P, i64, i64, P, P, P]
        lib.orc_line_energy.argtypes = [P, ctypes.c_int, P, i64, i64, ctypes.c_int, ctypes.c_int, P]
        lib.orc_rhs.argtypes = [ctypes.c_int, f64, P, P, P, P, P, P, P, P, P]
        lib.orc_local_solve_batch.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, i64, P, ctypes.c_int]
        lib.orc_macro.argtypes = [ctypes.c_int, f64, P, P, P, ctypes.c_int, f64, i64, P]
        lib.orc_macro_dirichlet_x.argtypes = [ctypes.c_int, f64, f64, f64, P, P, P, ctypes.c_int, f64, i64, P]
        lib.orc_diffusion.argtypes = [ctypes.c_int, f64, P, P, P]
        lib.orc_operator.argtypes = [ctypes.c_int, f64, P, P, P, P, P, P]
        for name in ("orc_synth_points", "orc_line_energy", "orc_rhs", "orc_local_solve_batch",
                     "orc_macro", "orc_macro_dirichlet_x", "orc_diffusion", "orc_operator"):
            getattr(lib, name).restype = None
        _lib_handle = lib
    return _lib_handle


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# Band split (Section 3.1 and its recursion; equations for psi_2, psi_11,
# psi_12, psi_21)
# ---------------------------------------------------------------------------

def band_split(kmax: int, thresh: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Literal recursive decomposition of the spectrum (Section 3.1).

    At step l the remaining spectrum (initially everything but k = 0) is split
    with edge a = thresh[l]: psi_2 keeps the modes with |k1| > a and |k2| > a;
    the rest, psi_1, becomes psi_11 (both |k_i| <= a, the level's diagonal
    band), psi_12 (|k1| <= a < |k2|) and psi_21 (|k2| <= a < |k1|).  The same
    split is then repeated on psi_2 with the next edge (the paper repeats with
    alpha^2 when psi_2 holds wavenumbers above alpha^2).  What remains after the
    last edge is the diagonal band of the finest level.

    Returns (level, part), int8 arrays of shape (2kmax+1, 2kmax+1) indexed
    [k2 + kmax, k1 + kmax]; level is 0-based (-1 for k = 0), part is
    DIAG / OFF12 / OFF21.
    """
    span = 2 * kmax + 1
    k1 = np.arange(-kmax, kmax + 1)[None, :].repeat(span, 0)
    k2 = np.arange(-kmax, kmax + 1)[:, None].repeat(span, 1)
    a1, a2 = np.abs(k1), np.abs(k2)
    level = np.full((span, span), -1, np.int8)
    part = np.full((span, span), -1, np.int8)
    remaining = ~((k1 == 0) & (k2 == 0))
    for l, a in enumerate(thresh):
        psi2 = remaining & (a1 > a) & (a2 > a)
        psi1 = remaining & ~psi2
        for p, sel in ((DIAG, psi1 & (a1 <= a) & (a2 <= a)),
                       (OFF12, psi1 & (a1 <= a) & (a2 > a)),
                       (OFF21, psi1 & (a1 > a) & (a2 <= a))):
            level[sel] = l
            part[sel] = p
        remaining = psi2
    level[remaining] = len(thresh)
    part[remaining] = DIAG
    return level, part


def band_mask(level: np.ndarray, part: np.ndarray, lev: int, prt: int) -> np.ndarray:
    return ((level == lev) & (part == prt)).astype(np.int8)


# ---------------------------------------------------------------------------
# Bookkeeping: the hierarchy of local domains (Section 3, Figure 1: domains of
# every level centred at the macro points X_ij, each level shrinking side and
# spacing by the same factor so every level costs the same)
# ---------------------------------------------------------------------------

@dataclass
class Domain:
    instance: int
    level: int
    cx: int
    cy: int
    n: int
    N: int          # level grid: spacing h = 2 pi / N
    I0: int         # node origin, in level-grid units, reduced mod N
    J0: int
    parent: int     # coarser domain whose lattice cell holds this centre (-1 at level 0)
    offset: int     # first cell in the packed [domain][y][x] arrays
    line_offset: int  # first entry in the packed per-domain 2n line energies
    h: float


class BookkeepingError(ValueError):
    pass


def _origin(N: int, n: int, M: int, c: int) -> int:
    # centre 2 pi (c + 1/2)/M minus half the side pi n / N, in units of h = 2 pi / N
    num = N * (2 * c + 1) - n * M
    if num % (2 * M) != 0:
        raise BookkeepingError("patch origin is not a grid point")
    return (num // (2 * M)) % N


def domain_table(probs) -> List[Domain]:
    """Domains of every instance, stored phase by phase.

    The bottom-up pass of Algorithm 3 visits the finest level of every instance
    first, so domains are ordered by phase p = (L_i - 1) - level, then instance,
    then cy, then cx.  Each phase, and each (instance, level) group, is then a
    contiguous range.
    """
    if not isinstance(probs, (list, tuple)):
        probs = [probs]
    for p in probs:
        L = len(p.n_cells)
        if not (len(p.n_global) == L and len(p.lattice) == L and len(p.thresh) == L - 1):
            raise BookkeepingError("level arrays disagree in length")
        if not p.kappa > 0:
            raise BookkeepingError("kappa must be positive")
        for a, b in zip(p.thresh[:-1], p.thresh[1:]):
            if not b > a:
                raise BookkeepingError("band edges must increase")
        for l in range(L):
            n, N, M = p.n_cells[l], p.n_global[l], p.lattice[l]
            if n < 4 or (n & (n - 1)) != 0 or n > N:
                raise BookkeepingError("n must be a power of two with 4 <= n <= N")
            if M < 1 or (l > 0 and M % p.lattice[l - 1] != 0):
                raise BookkeepingError("each lattice must refine the coarser one")
    max_L = max(len(p.n_cells) for p in probs)
    out: List[Domain] = []
    first: Dict[Tuple[int, int], int] = {}
    off = 0
    loff = 0
    for phase in range(max_L):
        for inst, p in enumerate(probs):
            L = len(p.n_cells)
            l = L - 1 - phase
            if l < 0:
                continue
            n, N, M = p.n_cells[l], p.n_global[l], p.lattice[l]
            first[(inst, l)] = len(out)
            for cy in range(M):
                for cx in range(M):
                    out.append(Domain(inst, l, cx, cy, n, N, _origin(N, n, M, cx),
                                      _origin(N, n, M, cy), -1, off, loff, 2.0 * math.pi / N))
                    off += n * n
                    loff += 2 * n
    for d in out:
        if d.level > 0:
            p = probs[d.instance]
            M, Mp = p.lattice[d.level], p.lattice[d.level - 1]
            px = ((2 * d.cx + 1) * Mp) // (2 * M)
            py = ((2 * d.cy + 1) * Mp) // (2 * M)
            d.parent = first[(d.instance, d.level - 1)] + py * Mp + px
    return out


def advection_bound(vx: np.ndarray, vy: np.ndarray) -> float:
    """max over cells of (|vx_W| + |vx_E| + |vy_S| + |vy_N|) / 2.

    The centred flux-form advection operator with discretely divergence-free
    face velocities is skew-symmetric with zero diagonal, so by Gershgorin its
    spectral radius is at most this value divided by h."""
    s = (np.abs(vx) + np.abs(np.roll(vx, -1, axis=1)) + np.abs(vy) + np.abs(np.roll(vy, -1, axis=0)))
    return float(np.max(s)) * 0.5


def plan_steps(n: int, h: float, K: Sequence[float], vmax: float, dt_frac: float,
               delta: float) -> Tuple[float, int]:
    """Step size and step count of one local solve (HMM step 2, Section 2.2).

    The paper evolves to a quasi-stationary state without fixing the time.
    Reading used here: stop at T with exp(-lambda T) = delta, where lambda is a
    lower bound of the decay rate of the discrete periodic problem (the
    advection is skew and the diffusion dominates lambda_min(K) times the
    5-point Laplacian, whose smallest nonzero eigenvalue is 4 sin^2(pi/n)/h^2).
    The RK4 step is dt_frac times 1/(rho_D/2.785 + rho_A/2.828), where 2.785 and
    2.828 bound RK4's real and imaginary stability intervals,
    rho_D = (4 K11 + 4 K22 + 2|K12|)/h^2 bounds the 9-point diffusion and
    rho_A = vmax/h (see advection_bound) the skew advection operator.
    Every operation is spelled out so the result is reproducible bit for bit.
    """
    K11, K12, K22 = float(K[0]), float(K[1]), float(K[2])
    rho_d = (4.0 * K11 + 4.0 * K22 + 2.0 * abs(K12)) / (h * h)
    rho_a = vmax / h
    dt_lim = 1.0 / (rho_d / 2.785 + rho_a / 2.828)
    lam = 0.5 * (K11 + K22) - math.sqrt(0.25 * (K11 - K22) * (K11 - K22) + K12 * K12)
    if not lam > 0.0:
        raise BookkeepingError("base diffusivity is not positive definite")
    s = math.sin(math.pi / n)
    decay = lam * 4.0 * s * s / (h * h)
    T = math.log(1.0 / delta) / decay
    nsteps = int(math.ceil(T / (dt_frac * dt_lim)))
    if nsteps < 1:
        nsteps = 1
    dt = T / nsteps
    return dt, nsteps


# ---------------------------------------------------------------------------
# Patch fields
# ---------------------------------------------------------------------------

def synth_points(psi_hat: np.ndarray, kmax: int, mask: np.ndarray, N: int,
                 I: np.ndarray, J: np.ndarray) -> np.ndarray:
    """Band field psi_band(2 pi I/N, 2 pi J/N) by direct Fourier sums (Section 3.1)."""
    ph = _c(np.asarray(psi_hat, np.complex128).view(np.float64).reshape(-1), np.float64)
    m = _c(mask, np.int8)
    I = _c(I, np.int64).reshape(-1)
    J = _c(J, np.int64).reshape(-1)
    out = np.empty(I.size, np.float64)
    _lib().orc_synth_points(_p(ph), int(kmax), _p(m), int(N), int(I.size), _p(I), _p(J), _p(out))
    return out


def synth_patch(psi_hat, kmax, mask, N, I0, J0, n) -> np.ndarray:
    """psi_band at the n x n nodes (x0 + i h, y0 + j h) of one patch, as [j][i]."""
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return synth_points(psi_hat, kmax, mask, N, I0 + ii, J0 + jj).reshape(n, n)


def staggered(psi: np.ndarray, h: float):
    """Face velocities and cell forcings from node values of psi.

    v = (-d psi/d x2, d psi/d x1) (Section 2.1), differenced along each face:
    vx on x-faces, vy on y-faces, so the discrete divergence of every cell
    vanishes identically.  f_j is the cell average of the face component j,
    which is what the centred advection operator gives when applied to the
    linear reconstruction x_j (HMM step 1 with R U = e_j . x).
    """
    vx = -(np.roll(psi, -1, axis=0) - psi) / h
    vy = (np.roll(psi, -1, axis=1) - psi) / h
    f1 = 0.5 * (vx + np.roll(vx, -1, axis=1))
    f2 = 0.5 * (vy + np.roll(vy, -1, axis=0))
    return vx, vy, f1, f2


def taper_weights(n: int, taper: int) -> np.ndarray:
    """Node weights of the patch taper along one axis: 0 at node 0, rising as
    sin^2 over `taper` nodes to 1, 1 in the middle, and falling back
    symmetrically (w(n - i) = w(i)), so that the tapered stream function
    vanishes at the patch seam and its periodic extension is smooth.  taper 0
    leaves every weight 1."""
    i = np.arange(n)
    w = np.ones(n)
    if taper > 0:
        e = np.minimum(i, n - i).astype(np.float64)
        w = np.where(e < taper, np.sin(0.5 * np.pi * e / taper) ** 2, 1.0)
    return w


def windowed_staggered(psi: np.ndarray, h: float, taper: int):
    """The staggered fields of the tapered stream function W psi (windowed
    patches, aimed at the non-periodicity of a component on its patch that
    the continuous-spectrum example of Section 4 lists among the error
    sources): W = w(x) w(y) from taper_weights, then the differences of
    staggered(), so the discrete divergence still vanishes identically."""
    w = taper_weights(psi.shape[0], taper)
    return staggered(psi * np.outer(w, w), h)


def divergence(vx, vy, h):
    return (np.roll(vx, -1, axis=1) - vx) / h + (np.roll(vy, -1, axis=0) - vy) / h


def operator(vx, vy, K, f, u, h) -> np.ndarray:
    """div(v u + K grad u) + f on one periodic patch (constant K)."""
    n = u.shape[0]
    out = np.empty_like(u, dtype=np.float64)
    _lib().orc_operator(n, float(h), _p(None if vx is None else _c(vx, np.float64)),
                        _p(None if vy is None else _c(vy, np.float64)),
                        _p(_c(K, np.float64)), _p(None if f is None else _c(f, np.float64)),
                        _p(_c(u, np.float64)), _p(out))
    return out


def diffusion(K, u, h) -> np.ndarray:
    n = u.shape[0]
    out = np.empty_like(u, dtype=np.float64)
    _lib().orc_diffusion(n, float(h), _p(_c(K, np.float64)), _p(_c(u, np.float64)), _p(out))
    return out


# ---------------------------------------------------------------------------
# Local solves and the estimator (HMM steps 1-3, Section 2.2; K formula after
# eq:homo; cell problem eq:cell)
# ---------------------------------------------------------------------------

def local_solve_batch(n: Sequence[int], h: Sequence[float], vx, vy, f1, f2,
                      Kb: np.ndarray, dt: Sequence[float], nsteps: Sequence[int],
                      w0: Optional[np.ndarray] = None, frame: bool = False) -> np.ndarray:
    """Classic RK4 on both correctors of every domain; returns w [2][cells].

    vx, vy, f1, f2 are packed 1-D float64 arrays (domain after domain, [y][x]).
    frame: the zero-frame (non-periodic) local problem, the last row and
    column of every patch held at zero.
    """
    nn = _c(n, np.int32)
    off = np.zeros(len(nn), np.int64)
    off[1:] = np.cumsum(nn.astype(np.int64) ** 2)[:-1]
    total = int(np.sum(nn.astype(np.int64) ** 2))
    w = np.zeros(2 * total, np.float64) if w0 is None else _c(w0, np.float64).reshape(-1).copy()
    _lib().orc_local_solve_batch(len(nn), _p(nn), _p(off), _p(_c(h, np.float64)),
                                 _p(_c(vx, np.float64)), _p(_c(vy, np.float64)),
                                 _p(_c(f1, np.float64)), _p(_c(f2, np.float64)),
                                 _p(_c(Kb, np.float64).reshape(-1)), _p(_c(dt, np.float64)),
                                 _p(_c(nsteps, np.int64)), total, _p(w), 1 if frame else 0)
    return w.reshape(2, total)


def local_solve_adaptive(n: int, h: float, vx, vy, f1, f2, Kb, dt: float, nsteps: int, delta: float,
                         chunks: int = 32) -> Tuple[np.ndarray, int]:
    """HMM step 2 of Section 2.2 run to the quasi-stationary state of one
    domain: chunks of C = ceil(nsteps / chunks) RK4 steps, stopping after the
    first chunk at which the change dw_j of each corrector over the chunk
    bounds the remaining error of K below delta times its largest entry.

    The steady corrector chi attracts w in the mean square at least at the
    Poincare rate mu of the step plan, so over a chunk the error shrinks by
    rho = exp(-mu C dt) or more, rms(w - chi) <= rho / (1 - rho) rms(dw), and
    each entry <f_i w_j> of K - K_b is within rms(f_i) rms(w_j - chi_j) of its
    limit (Cauchy-Schwarz).  Returns (w [2][n n], steps taken); the plan's
    nsteps caps the count."""
    f1 = _c(f1, np.float64).reshape(-1)
    f2 = _c(f2, np.float64).reshape(-1)
    Kb = _c(Kb, np.float64).reshape(3)
    C = max(1, -(-int(nsteps) // int(chunks)))
    lam = 0.5 * (Kb[0] + Kb[2]) - math.sqrt(0.25 * (Kb[0] - Kb[2]) ** 2 + Kb[1] ** 2)
    mu = lam * 4.0 * math.sin(math.pi / n) ** 2 / (h * h)
    rho = math.exp(-mu * C * dt)
    frms = max(math.sqrt(np.mean(f1 * f1)), math.sqrt(np.mean(f2 * f2)))
    w = np.zeros((2, n * n))
    done = 0
    while done < nsteps:
        c = min(C, nsteps - done)
        prev = w
        w = local_solve_batch([n], [h], vx, vy, f1, f2, Kb[None, :], [dt], [c], w0=prev)
        done += c
        if done >= nsteps:
            break
        dw = max(math.sqrt(np.mean((w[0] - prev[0]) ** 2)), math.sqrt(np.mean((w[1] - prev[1]) ** 2)))
        scale = float(np.max(np.abs(estimate(f1, f2, w[0], w[1], Kb))))
        if rho < 1.0 and frms * dw * rho / (1.0 - rho) <= delta * scale:
            break
    return w, done


def estimate(f1, f2, w1, w2, Kb) -> np.ndarray:
    """K = K_b + sym(<f_i w_j>) (the paper's K = kappa I + (1/2) int (v x chi + chi x v)
    with chi the corrector, here the time-integrated w)."""
    p11 = float(np.mean(f1 * w1))
    p12 = float(np.mean(f1 * w2))
    p21 = float(np.mean(f2 * w1))
    p22 = float(np.mean(f2 * w2))
    return np.array([Kb[0] + p11, Kb[1] + 0.5 * (p12 + p21), Kb[2] + p22])


def estimate_window(f1, f2, w1, w2, Kb, inner: int) -> np.ndarray:
    """The flux-form estimate averaged over the centred inner x inner cells of
    an n x n patch only (oversampled patches: the local problem is posed on a
    patch larger than the region it describes, so that the seam of the
    periodically treated patch lies away from the averaging window; aimed at
    the non-periodicity that the continuous-spectrum example of Section 4
    lists among the error sources).  inner = 0, or inner >= n, is the whole
    patch."""
    n = f1.shape[0]
    m = inner if 0 < inner < n else n
    a = (n - m) // 2
    win = (slice(a, a + m), slice(a, a + m))
    return estimate(f1[win], f2[win], w1[win], w2[win], Kb)


def estimate_energy(w1, w2, Kb, h) -> np.ndarray:
    """Energy form K_b + sym(-<w_i, D w_j>); equals the flux form at steady state."""
    d1 = diffusion(Kb, w1, h)
    d2 = diffusion(Kb, w2, h)
    e11 = -float(np.mean(w1 * d1))
    e12 = -0.5 * (float(np.mean(w1 * d2)) + float(np.mean(w2 * d1)))
    e22 = -float(np.mean(w2 * d2))
    return np.array([Kb[0] + e11, Kb[1] + e12, Kb[2] + e22])


def cell_problem_dense(vx, vy, f1, f2, Kb, h) -> np.ndarray:
    """Steady discrete cell problem solved directly (dense LU; tiny n only).

    Solves L chi_j = -f_j with mean(chi_j) = 0, L = div(v . + K_b grad .),
    which is the discrete eq:cell (read with the Laplacian).  Returns K.
    """
    n = vx.shape[0]
    m = n * n
    A = np.zeros((m + 1, m + 1))
    e = np.zeros((n, n))
    for c in range(m):
        e.reshape(-1)[:] = 0.0
        e.reshape(-1)[c] = 1.0
        A[:m, c] = operator(vx, vy, Kb, None, e, h).reshape(-1)
    A[:m, m] = 1.0
    A[m, :m] = 1.0
    chis = []
    for f in (f1, f2):
        rhs = np.zeros(m + 1)
        rhs[:m] = -f.reshape(-1)
        chis.append(np.linalg.solve(A, rhs)[:m].reshape(n, n))
    return estimate(f1, f2, chis[0], chis[1], Kb)


# ---------------------------------------------------------------------------
# Off-diagonal closed form (Algorithm 1 with eq:shearhomoY / eq:shearhomoX)
# ---------------------------------------------------------------------------

def line_energies(psi_hat, kmax, mask, N, I0, n, direction) -> np.ndarray:
    """Full-period mean of the band field squared along n lines (Parseval).

    direction 0: lines x1 = 2 pi (I0 + i + 1/2)/N (for psi_12);
    direction 1: lines x2 = 2 pi (I0 + j + 1/2)/N (for psi_21).
    """
    ph = _c(np.asarray(psi_hat, np.complex128).view(np.float64).reshape(-1), np.float64)
    out = np.empty(n, np.float64)
    _lib().orc_line_energy(_p(ph), int(kmax), _p(_c(mask, np.int8)), int(N), int(I0), int(n),
                           int(direction), _p(out))
    return out


def offdiag_closed_form(K: Sequence[float], s: np.ndarray, direction: int) -> np.ndarray:
    """Algorithm 1: shear formula on each line, then the harmonic mean across lines.

    direction 0 (psi_12, high wavenumbers in x2): K*_11(x1) = K11 + s(x1)/K22
    (eq:shearhomoY with the base's K11, K22), then K11 <- (mean 1/K*_11)^-1.
    direction 1 (psi_21): K*_22(x2) = K22 + t(x2)/K11 (eq:shearhomoX), harmonic
    mean over the rows.  K12 passes through.
    """
    K11, K12, K22 = float(K[0]), float(K[1]), float(K[2])
    n = len(s)
    if direction == 0:
        acc = 0.0
        for v in s:
            acc += 1.0 / (K11 + float(v) / K22)
        return np.array([n / acc, K12, K22])
    acc = 0.0
    for v in s:
        acc += 1.0 / (K22 + float(v) / K11)
    return np.array([K11, K12, n / acc])


def sum_offdiag(K_in, s12, s21) -> np.ndarray:
    """Algorithm 2: K[psi12 + psi21, K_in] = K[psi12, K_in] + K[psi21, K_in] - K_in."""
    K_in = np.asarray(K_in, np.float64)
    return offdiag_closed_form(K_in, s12, 0) + offdiag_closed_form(K_in, s21, 1) - K_in


def lambda_min(K) -> float:
    """Smallest eigenvalue of the symmetric 2 x 2 tensor {K11, K12, K22}
    (LAPACK's symmetric eigensolver)."""
    K = np.asarray(K, np.float64)
    return float(np.linalg.eigvalsh(np.array([[K[0], K[1]], [K[1], K[2]]]))[0])


def spd_floor(K_net, K_in) -> Tuple[np.ndarray, bool]:
    """Base of a coarse local solve when Algorithm 3's difference is not SPD.

    Step 3 of Algorithm 3 forms K_net = K_star - K_off + K_in as the base of
    the next local solve, which must be a diffusivity.  At the steady state
    K_star dominates K_off (every local solve only adds a positive
    semi-definite enhancement to its base), so K_net dominates K_in.  Reading
    used where rounding or an unfinished solve breaks this: when the smallest
    eigenvalue of K_net falls below that of K_in (or is not a number), the
    eigenvalues of K_net are raised to at least lambda_min(K_in), its
    eigenvectors kept, and the domain is flagged.  Returns (K, clamped);
    K_net is returned unchanged when no clamp is needed.
    """
    K_net = np.asarray(K_net, np.float64)
    floor = lambda_min(K_in)
    if np.all(np.isfinite(K_net)) and lambda_min(K_net) >= floor:
        return K_net.copy(), False
    if not np.all(np.isfinite(K_net)):
        return np.array([floor, 0.0, floor]), True
    lam, vec = np.linalg.eigh(np.array([[K_net[0], K_net[1]], [K_net[1], K_net[2]]]))
    lam = np.maximum(lam, floor)
    M = vec @ np.diag(lam) @ vec.T
    return np.array([M[0, 0], 0.5 * (M[0, 1] + M[1, 0]), M[1, 1]]), True


# ---------------------------------------------------------------------------
# Whole hierarchy (Algorithm 3, extended to L levels)
# ---------------------------------------------------------------------------

@dataclass
class HierarchyResult:
    domains: List[Domain]
    K_in: np.ndarray      # [nd][3] base from above (kappa I at level 0)
    K_off: np.ndarray     # [nd][3] Algorithm 2 result (levels < L-1)
    K_base: np.ndarray    # [nd][3] base of the local solve (K_net, or K_in at the finest level)
    K_solve: np.ndarray   # [nd][3] local solve estimate
    R: np.ndarray         # [nd][3] level result handed to the coarser level
    dt: np.ndarray
    nsteps: np.ndarray
    lines: np.ndarray     # packed [sum 2n] line energies (off12 columns then off21 rows)
    w: Optional[Dict[int, np.ndarray]] = None
    clamped: Optional[List[int]] = None   # domains whose K_net was raised by spd_floor

    def K_total(self) -> np.ndarray:
        return np.array([self.R[i] for i, d in enumerate(self.domains) if d.level == 0])


def macro_diffusivity(res: HierarchyResult, i: int) -> np.ndarray:
    """Diffusivity for a macro grid that resolves domain i's own diagonal band
    as its advecting velocity (eq:homo with v_M, HMM step 4): the level's
    result without that band's local solve, i.e. Algorithm 2's closed form on
    the level's base, S12(K_base) + S21(K_base) - K_base."""
    d = res.domains[i]
    s12 = res.lines[d.line_offset:d.line_offset + d.n]
    s21 = res.lines[d.line_offset + d.n:d.line_offset + 2 * d.n]
    return sum_offdiag(res.K_base[i], s12, s21)


def level_fields(p, level_arr, part_arr, d: Domain, taper: int = 0):
    """Diagonal-band psi, face velocities and forcings of one domain (with
    taper > 0, of the tapered stream function of a windowed patch)."""
    mask = band_mask(level_arr, part_arr, d.level, DIAG)
    psi = synth_patch(p.psi_hat, p.kmax, mask, d.N, d.I0, d.J0, d.n)
    return (psi,) + (windowed_staggered(psi, d.h, taper) if taper > 0 else staggered(psi, d.h))


def run_hierarchy(probs, keep_w: bool = False, steps_override: Optional[int] = None, inner: int = 0,
                  taper: int = 0, frame: bool = False,
                  roots: Optional[Sequence[int]] = None) -> HierarchyResult:
    """K[psi, kappa I; Omega_1] at every centre by Algorithm 3 generalised to L levels.

    R(l, K_in) = LS(diag_l, K_in)                                   l = finest
    R(l, K_in) = LS(diag_l, K_net) + S12(K_net) + S21(K_net) - 2 K_net   otherwise,
        with K_off = S12(K_in) + S21(K_in) - K_in       (Algorithm 2),
             K_star = R(l+1, K_off) at the same centre  (Algorithm 3, step 2),
             K_net = K_star - K_off + K_in              (Algorithm 3, step 3),
    and the final line read with the additive rule of Algorithm 2
    (K[psi11 + psi12 + psi21, K_net] = sum of the three effects minus twice the
    repeated base).  K_in = kappa I at the coarsest level.  When a lattice is
    finer than its parent's, K_star is the mean of the children's results.

    Patch options (all levels): inner > 0 averages each estimate over the
    centred inner x inner window (oversampled patches), taper > 0 tapers each
    patch's stream function (windowed patches), frame holds the correctors at
    zero on each patch's last row and column (zero-frame local problems).

    roots (optional): indices of level-0 domains; only these and the domains
    below them (their children, the children's children, ...) are computed,
    which is all that the level results of these centres depend on.  The
    entries of every other domain are left zero (nsteps 0).

    A base K_net whose smallest eigenvalue falls below that of K_in is raised
    to it (spd_floor); `clamped` lists the domains where that happened.
    """
    if not isinstance(probs, (list, tuple)):
        probs = [probs]
    doms = domain_table(probs)
    nd = len(doms)
    keep = np.ones(nd, bool)
    if roots is not None:
        keep[:] = False
        for r in roots:
            if doms[r].level != 0:
                raise ValueError("roots must be level-0 domains")
            keep[r] = True
        for i in sorted(range(nd), key=lambda i: doms[i].level):
            if doms[i].level > 0 and keep[doms[i].parent]:
                keep[i] = True
    splits = [band_split(p.kmax, p.thresh) for p in probs]
    K_in = np.zeros((nd, 3))
    K_off = np.zeros((nd, 3))
    K_base = np.zeros((nd, 3))
    K_solve = np.zeros((nd, 3))
    R = np.zeros((nd, 3))
    dt = np.zeros(nd)
    nsteps = np.zeros(nd, np.int64)
    lines = np.zeros(sum(2 * d.n for d in doms))
    empty_band: Dict[Tuple[int, int], bool] = {}
    for i, d in enumerate(doms):
        if not keep[i]:
            continue
        p = probs[d.instance]
        lv, pt = splits[d.instance]
        lines[d.line_offset:d.line_offset + d.n] = line_energies(
            p.psi_hat, p.kmax, band_mask(lv, pt, d.level, OFF12), d.N, d.I0, d.n, 0)
        lines[d.line_offset + d.n:d.line_offset + 2 * d.n] = line_energies(
            p.psi_hat, p.kmax, band_mask(lv, pt, d.level, OFF21), d.N, d.J0, d.n, 1)
        key = (d.instance, d.level)
        if key not in empty_band:
            dm = band_mask(lv, pt, d.level, DIAG)
            empty_band[key] = not np.any((dm != 0) & (p.psi_hat != 0))

    def s12(i):
        d = doms[i]
        return lines[d.line_offset:d.line_offset + d.n]

    def s21(i):
        d = doms[i]
        return lines[d.line_offset + d.n:d.line_offset + 2 * d.n]

    L_of = [len(p.n_cells) for p in probs]
    # top-down: Algorithm 2 at every level above the finest, K_in from the parent
    order = sorted(range(nd), key=lambda i: doms[i].level)
    for i in order:
        d = doms[i]
        if not keep[i]:
            continue
        if d.level == 0:
            K_in[i] = [probs[d.instance].kappa, 0.0, probs[d.instance].kappa]
        else:
            K_in[i] = K_off[d.parent]
        if d.level < L_of[d.instance] - 1:
            K_off[i] = sum_offdiag(K_in[i], s12(i), s21(i))

    children: Dict[int, List[int]] = {}
    for i, d in enumerate(doms):
        if d.parent >= 0:
            children.setdefault(d.parent, []).append(i)

    wkeep = {} if keep_w else None
    maxL = max(L_of)
    clamped: List[int] = []
    for lev in range(maxL - 1, -1, -1):
        idx = [i for i, d in enumerate(doms) if d.level == lev and keep[i]]
        if not idx:
            continue
        # fields of this level (one batch)
        fields = [level_fields(probs[doms[i].instance], *splits[doms[i].instance], doms[i], taper) for i in idx]
        # bases of this level
        for t, i in enumerate(idx):
            d = doms[i]
            if lev == L_of[d.instance] - 1:
                K_base[i] = K_in[i]
            else:
                ch = children[i]
                K_star = np.mean(np.array([R[c] for c in ch]), axis=0) if len(ch) > 1 else R[ch[0]].copy()
                K_base[i], low = spd_floor(K_star - K_off[i] + K_in[i], K_in[i])
                if low:
                    clamped.append(i)
            p = probs[d.instance]
            key = (d.instance, lev)
            vmax = advection_bound(fields[t][1], fields[t][2])
            dt[i], nsteps[i] = plan_steps(d.n, d.h, K_base[i], vmax, p.dt_frac, p.delta)
            if empty_band[(d.instance, lev)]:
                # zero forcing: the corrector stays zero, nothing is integrated
                dt[i], nsteps[i] = 0.0, 0
        vx = np.concatenate([f[1].reshape(-1) for f in fields])
        vy = np.concatenate([f[2].reshape(-1) for f in fields])
        f1 = np.concatenate([f[3].reshape(-1) for f in fields])
        f2 = np.concatenate([f[4].reshape(-1) for f in fields])
        ns = nsteps[idx] if steps_override is None else np.full(len(idx), steps_override, np.int64)
        w = local_solve_batch([doms[i].n for i in idx], [doms[i].h for i in idx], vx, vy, f1, f2,
                              K_base[idx], dt[idx], ns, frame=frame)
        o = 0
        for t, i in enumerate(idx):
            d = doms[i]
            m = d.n * d.n
            w1 = w[0, o:o + m].reshape(d.n, d.n)
            w2 = w[1, o:o + m].reshape(d.n, d.n)
            K_solve[i] = estimate_window(fields[t][3], fields[t][4], w1, w2, K_base[i], inner)
            if wkeep is not None:
                wkeep[i] = np.stack([w1, w2])
            if lev == L_of[d.instance] - 1:
                R[i] = K_solve[i]
            else:
                Kn = K_base[i]
                R[i] = (K_solve[i] + offdiag_closed_form(Kn, s12(i), 0)
                        + offdiag_closed_form(Kn, s21(i), 1) - 2.0 * Kn)
            o += m
    return HierarchyResult(doms, K_in, K_off, K_base, K_solve, R, dt, nsteps, lines, wkeep, clamped)


# ---------------------------------------------------------------------------
# Macro solver (HMM step 4 on the homogenized equation eq:homo)
# ---------------------------------------------------------------------------

def macro_plan(N: int, K_cells: np.ndarray, Vb: float, dt_frac: float, T: float) -> Tuple[float, int]:
    """RK4 step for the macro grid: dt_frac of the stability bound, ending at T."""
    h = 2.0 * math.pi / N
    Kc = np.asarray(K_cells, np.float64).reshape(-1, 3)
    worst = 0.0
    for r in range(Kc.shape[0]):
        v = 4.0 * Kc[r, 0] + 4.0 * Kc[r, 2] + 2.0 * abs(Kc[r, 1])
        if v > worst:
            worst = v
    rho_d = worst / (h * h)
    rho_a = Vb / h
    dt_lim = 1.0 / (rho_d / 2.785 + rho_a / 2.828)
    nsteps = int(math.ceil(T / (dt_frac * dt_lim)))
    if nsteps < 1:
        nsteps = 1
    return T / nsteps, nsteps


def macro_run(N: int, vx: Optional[np.ndarray], vy: Optional[np.ndarray], K: np.ndarray,
              u0: np.ndarray, dt: float, nsteps: int,
              dirichlet_x: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """u_t = div(v_M u + K grad u) on the N x N grid of [0, 2 pi]^2, RK4 (FP64):
    periodic, or with u = dirichlet_x[0] on x = 0 and dirichlet_x[1] on
    x = 2 pi and periodic in y (the boundary conditions of Section 4)."""
    K = _c(K, np.float64).reshape(-1)
    is_field = 1 if K.size > 3 else 0
    u = _c(u0, np.float64).copy()
    vxp = _p(None if vx is None else _c(vx, np.float64))
    vyp = _p(None if vy is None else _c(vy, np.float64))
    if dirichlet_x is None:
        _lib().orc_macro(int(N), 2.0 * math.pi / N, vxp, vyp, _p(K), is_field, float(dt), int(nsteps), _p(u))
    else:
        _lib().orc_macro_dirichlet_x(int(N), 2.0 * math.pi / N, float(dirichlet_x[0]), float(dirichlet_x[1]),
                                     vxp, vyp, _p(K), is_field, float(dt), int(nsteps), _p(u))
    return u


def interpolate_centres(Kc: np.ndarray, M: int, N: int) -> np.ndarray:
    """Bilinear periodic interpolation of lattice values (centres 2 pi (i+1/2)/M)
    to the N x N cell centres, component by component (a reading: the paper
    does not say how the macro solver receives the centre values)."""
    Kc = np.asarray(Kc, np.float64).reshape(M, M, 3)
    out = np.zeros((N, N, 3))
    for j in range(N):
        y = (j + 0.5) / N * M - 0.5
        j0 = math.floor(y)
        ty = y - j0
        for i in range(N):
            x = (i + 0.5) / N * M - 0.5
            i0 = math.floor(x)
            tx = x - i0
            a = Kc[j0 % M, i0 % M]
            b = Kc[j0 % M, (i0 + 1) % M]
            c = Kc[(j0 + 1) % M, i0 % M]
            e = Kc[(j0 + 1) % M, (i0 + 1) % M]
            out[j, i] = (1 - ty) * ((1 - tx) * a + tx * b) + ty * ((1 - tx) * c + tx * e)
    return out
