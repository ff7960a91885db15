"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module only *describes* problems: stream-function spectra, the level
geometry a user would choose, and the initial macro field.  It performs none
of the method's arithmetic (no band split, no synthesis, no time stepping, no
bookkeeping of domains), so the oracle and the HIP path can both consume it
without sharing any code that computes a result.

Conventions
-----------
* Periodic domain [0, 2*pi]^2; psi(x) = sum_k psi_hat(k) exp(i k.x) (the
  stream function of the paper's model problem, Section 2.1).
* ``psi_hat`` is a complex128 array of shape (2*kmax+1, 2*kmax+1) indexed
  ``[k2 + kmax, k1 + kmax]`` (x wavenumber fastest).  It is Hermitian
  (psi_hat(-k) = conj psi_hat(k)) so psi is real, and psi_hat(0) = 0.
* Random numbers come from splitmix64 (Steele, Lea & Flood 2014; the
  constants are the published ones of Vigna's reference version), used as a
  counter-based generator: value = splitmix64(seed * 2^32 + counter).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One output of splitmix64 for state ``x`` (the state is advanced first)."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def uniform01(seed: int, counter: int) -> float:
    """Counter-based uniform double in [0, 1) with 53 random bits."""
    return (splitmix64(((seed & 0xFFFFFFFF) << 32) | (counter & 0xFFFFFFFF)) >> 11) * (1.0 / (1 << 53))


@dataclass
class Problem:
    """One flow instance and the level geometry chosen for it.

    Level l (0-based here, 1-based in the paper) uses local patches of
    ``n_cells[l]`` x ``n_cells[l]`` cells whose spacing is 2*pi/``n_global[l]``
    (so the patch side is 2*pi*n/N), centred on a ``lattice[l]`` x
    ``lattice[l]`` lattice of macro points X_ij = 2*pi*(i+1/2)/M.  ``thresh``
    holds the band edges a_1 < ... < a_{L-1} (the paper's alpha, alpha^2, ...).
    """
    kappa: float
    kmax: int
    psi_hat: np.ndarray
    thresh: List[int]
    n_cells: List[int]
    n_global: List[int]
    lattice: List[int]
    dt_frac: float = 0.5
    delta: float = 1e-6
    name: str = ""

    @property
    def n_levels(self) -> int:
        return len(self.n_cells)

    def psi_hat_interleaved(self) -> np.ndarray:
        """psi_hat as contiguous float64 (re, im) pairs, the layout of the C boundary."""
        return np.ascontiguousarray(self.psi_hat.astype(np.complex128)).view(np.float64).reshape(-1)


def _empty_spectrum(kmax: int) -> np.ndarray:
    return np.zeros((2 * kmax + 1, 2 * kmax + 1), dtype=np.complex128)


def add_cellular(ph: np.ndarray, kmax: int, k1: int, k2: int, amp: float,
                 phi1: float = 0.0, phi2: float = 0.0) -> None:
    """Add amp * sin(k1 x + phi1) * sin(k2 y + phi2) to the spectrum ``ph``."""
    # sin a sin b = -(1/4) [e^{i(a+b)} - e^{i(a-b)} - e^{-i(a-b)} + e^{-i(a+b)}]
    terms = [((k1, k2), -0.25 * amp * np.exp(1j * (phi1 + phi2))),
             ((k1, -k2), 0.25 * amp * np.exp(1j * (phi1 - phi2))),
             ((-k1, k2), 0.25 * amp * np.exp(-1j * (phi1 - phi2))),
             ((-k1, -k2), -0.25 * amp * np.exp(-1j * (phi1 + phi2)))]
    for (a, b), c in terms:
        ph[b + kmax, a + kmax] += c


def add_cos_x(ph: np.ndarray, kmax: int, k: int, amp: float) -> None:
    """Add amp * cos(k x) (a shear stream function, velocity (0, -amp k sin kx))."""
    ph[kmax, k + kmax] += 0.5 * amp
    ph[kmax, -k + kmax] += 0.5 * amp


def add_cos_y(ph: np.ndarray, kmax: int, k: int, amp: float) -> None:
    """Add amp * cos(k y) (a shear stream function, velocity (amp k sin ky, 0))."""
    ph[k + kmax, kmax] += 0.5 * amp
    ph[-k + kmax, kmax] += 0.5 * amp


def random_power_spectrum(seed: int, radius: int, p: float, amp: float = 1.0) -> np.ndarray:
    """psi_hat(k) = amp * |k|^p * exp(i theta_k) for 1 <= |k| <= radius, 0 elsewhere.

    theta_k is uniform on [0, 2*pi) and drawn on the half plane
    (k2 > 0, or k2 == 0 and k1 > 0); the other half is the Hermitian mirror.
    The counter of mode k is (k2 + radius) * (2*radius + 1) + (k1 + radius).
    """
    kmax = radius
    ph = _empty_spectrum(kmax)
    r2 = radius * radius
    span = 2 * radius + 1
    for k2 in range(0, radius + 1):
        for k1 in range(-radius, radius + 1):
            if k2 == 0 and k1 <= 0:
                continue
            m2 = k1 * k1 + k2 * k2
            if m2 == 0 or m2 > r2:
                continue
            theta = 2.0 * math.pi * uniform01(seed, (k2 + radius) * span + (k1 + radius))
            c = amp * (m2 ** (0.5 * p)) * complex(math.cos(theta), math.sin(theta))
            ph[k2 + kmax, k1 + kmax] = c
            ph[-k2 + kmax, -k1 + kmax] = c.conjugate()
    return ph


def random_power_spectrum_fast(seed: int, radius: int, p: float, amp: float = 1.0) -> np.ndarray:
    """Vectorised equivalent of :func:`random_power_spectrum` (bit-identical output)."""
    kmax = radius
    span = 2 * radius + 1
    k1 = np.arange(-radius, radius + 1, dtype=np.int64)[None, :]
    k2 = np.arange(0, radius + 1, dtype=np.int64)[:, None]
    m2 = k1 * k1 + k2 * k2
    keep = (m2 >= 1) & (m2 <= radius * radius) & ~((k2 == 0) & (k1 <= 0))
    ctr = ((k2 + radius) * span + (k1 + radius)).astype(np.uint64)
    x = (np.uint64(seed & 0xFFFFFFFF) << np.uint64(32)) | ctr
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    theta = 2.0 * math.pi * u
    mag = amp * np.where(keep, np.power(np.maximum(m2, 1).astype(np.float64), 0.5 * p), 0.0)
    half = mag * (np.cos(theta) + 1j * np.sin(theta))
    ph = _empty_spectrum(kmax)
    ph[kmax:, :] = np.where(keep, half, 0.0)
    # Hermitian completion of the lower half plane (and k2 == 0, k1 < 0)
    upper = ph[kmax:, :].copy()
    ph[:kmax + 1, :] += np.where(keep, np.conj(upper), 0.0)[::-1, ::-1]
    ph[kmax, kmax] = 0.0
    return ph


# --------------------------------------------------------------------------
# Workloads.  Level geometry: patch side 2*pi/4^(l-1) at level l unless a
# workload says otherwise, so n_global = n * 4^(l-1).
# --------------------------------------------------------------------------

def config_two_level_cellular() -> Problem:
    """psi = sin x sin y + 0.25 sin 8x sin 8y, kappa = 0.05, a_1 = 4.

    Level 1 is one 64^2 patch covering the whole periodic domain (the coarse
    grid); level 2 has 16 patches of 32^2 cells with side pi/2.
    """
    kmax = 8
    ph = _empty_spectrum(kmax)
    add_cellular(ph, kmax, 1, 1, 1.0)
    add_cellular(ph, kmax, 8, 8, 0.25)
    return Problem(kappa=0.05, kmax=kmax, psi_hat=ph, thresh=[4], n_cells=[64, 32],
                   n_global=[64, 128], lattice=[1, 4], dt_frac=0.5, delta=1e-6,
                   name="cellular-2level-64")


def macro_initial_gaussian(N: int) -> np.ndarray:
    """u0 = exp(-((x-pi)^2 + (y-pi)^2)/0.5) at the cell centres of an N x N grid, [y][x]."""
    x = (np.arange(N) + 0.5) * (2.0 * math.pi / N)
    X, Y = np.meshgrid(x, x, indexing="xy")
    return np.exp(-((X - math.pi) ** 2 + (Y - math.pi) ** 2) / 0.5)


def config_four_level_cellular(seed: int = 0, n: int = 128, lattice: int = 8) -> Problem:
    """psi = sum_{k in 1,4,16,64} k^(-4/3) sin(kx+p1_k) sin(ky+p2_k), kappa = 1e-2.

    Band edges (2, 8, 32) put each cellular mode alone on its own level; 4
    levels of lattice^2 patches with n^2 cells and side 2*pi/4^(l-1).
    """
    ks = [1, 4, 16, 64]
    kmax = 64
    ph = _empty_spectrum(kmax)
    for j, k in enumerate(ks):
        p1 = 2.0 * math.pi * uniform01(seed, 2 * j)
        p2 = 2.0 * math.pi * uniform01(seed, 2 * j + 1)
        add_cellular(ph, kmax, k, k, k ** (-4.0 / 3.0), p1, p2)
    L = 4
    return Problem(kappa=1e-2, kmax=kmax, psi_hat=ph, thresh=[2, 8, 32],
                   n_cells=[n] * L, n_global=[n * 4 ** l for l in range(L)],
                   lattice=[lattice] * L, dt_frac=0.5, delta=1e-6,
                   name=f"cellular-4level-{lattice * lattice}x{n}")


def config_shear(k: int = 16, V: float = 1.0, kappa: float = 1e-2, n: int = 128,
                 levels: int = 1, thresh: Optional[Sequence[int]] = None) -> Problem:
    """Shear flow v = (0, V sin kx): psi = -(V/k) cos kx.

    Homogenization gives K_yy = kappa + V^2 / (2 kappa k^2) (eq:shearhomoX).
    With levels = 1 the whole field is one local solve; with more levels the
    mode is an off-diagonal component and goes through the closed form.
    """
    kmax = k
    ph = _empty_spectrum(kmax)
    add_cos_x(ph, kmax, k, -V / k)
    if thresh is None:
        thresh = [max(1, k // 2) * 4 ** l for l in range(levels - 1)]
    return Problem(kappa=kappa, kmax=kmax, psi_hat=ph, thresh=list(thresh),
                   n_cells=[n] * levels, n_global=[n * 4 ** l for l in range(levels)],
                   lattice=[1] * levels, dt_frac=0.5, delta=1e-6, name=f"shear-k{k}")


def config_paper_cellular(test: int, scale: float = 1.0, n: int = 128, levels: int = 2,
                          divide: int = 1) -> Problem:
    """The cellular examples of Section 4 (Tests 2 and 3) on [0, 2 pi]^2.

    The paper's [0,1]^2 with kappa = 1 maps to [0, 2 pi]^2 by x' = 2 pi x,
    t' = 4 pi^2 t with the same stream function in x' and kappa = 1, so
    phi_c(a x1, b x2) becomes sin(a x') sin(b y'):
      test 2: psi = (1/3) (phi_c(5, 5) + phi_c(25, 25));
      test 3: psi = (1/5) (phi_c(5, 5) + phi_c(5, 45) + phi_c(45, 5) + phi_c(50, 50)),
    times `scale`.  `divide` divides every wavenumber (5 -> the same
    homogenized K at a fifth of the resolution: the cell problem of a
    periodic flow does not depend on the number of periods in the domain).
    levels = 2: decomposition factor alpha = 5 (band edge 5 / divide), both
    levels on one whole-domain patch of n^2 cells (the fine modes are periodic
    on no smaller power-of-two patch); levels = 1: one band, the direct cell
    problem of the full flow."""
    if test == 2:
        modes = [(5, 5, 1.0 / 3.0), (25, 25, 1.0 / 3.0)]
    elif test == 3:
        modes = [(5, 5, 0.2), (5, 45, 0.2), (45, 5, 0.2), (50, 50, 0.2)]
    else:
        raise ValueError("test must be 2 or 3")
    if any(a % divide or b % divide for a, b, _ in modes):
        raise ValueError("divide must divide every wavenumber")
    modes = [(a // divide, b // divide, amp * scale) for a, b, amp in modes]
    kmax = max(max(a, b) for a, b, _ in modes)
    ph = _empty_spectrum(kmax)
    for a, b, amp in modes:
        add_cellular(ph, kmax, a, b, amp)
    thresh = [5 // divide] if levels == 2 else []
    return Problem(kappa=1.0, kmax=kmax, psi_hat=ph, thresh=thresh, n_cells=[n] * levels,
                   n_global=[n] * levels, lattice=[1] * levels, dt_frac=0.5, delta=1e-6,
                   name=f"paper-test{test}-x{scale:.3g}-div{divide}-L{levels}")


def paper_step_initial(N: int) -> np.ndarray:
    """The step data of Section 4 at the N x N cell centres of [0, 2 pi]^2:
    1 where x <= pi, else 0."""
    xc = (np.arange(N) + 0.5) * (2.0 * np.pi / N)
    return np.tile((xc <= np.pi).astype(np.float64), (N, 1))


def config_continuous(seed: int = 0, radius: int = 512, p: float = -7.0 / 3.0,
                      kappa: float = 1e-3, n: int = 128, lattice: int = 16,
                      levels: int = 5) -> Problem:
    """Random-phase psi_hat ~ |k|^p for 1 <= |k| <= radius; band edges 4^l."""
    ph = random_power_spectrum_fast(seed, radius, p)
    return Problem(kappa=kappa, kmax=radius, psi_hat=ph,
                   thresh=[4 ** l for l in range(1, levels)],
                   n_cells=[n] * levels, n_global=[n * 4 ** l for l in range(levels)],
                   lattice=[lattice] * levels, dt_frac=0.5, delta=1e-6,
                   name=f"continuous-{levels}level-{lattice * lattice}x{n}")


def config_band_pass(seed: int, k_lo: int, k_hi: int, kappa: float, n: int, lattice: int,
                     n_global: int, amp: float = 1.0) -> Problem:
    """One level of a random-phase flow with |psi_k| = amp |k|^-2 on the annulus
    k_lo <= |k| <= k_hi only (a scale-separated field with no mode coarser
    than the annulus): lattice^2 patches of n^2 cells at spacing 2 pi /
    n_global.  With n * lattice = n_global the patches tile the domain; with
    n = n_global and lattice 1 the single patch is the whole periodic domain
    (the direct cell problem of the flow)."""
    ph = random_power_spectrum_fast(seed, k_hi, -2.0, amp)
    k = np.arange(-k_hi, k_hi + 1)
    ph[(k[:, None] ** 2 + k[None, :] ** 2) < k_lo * k_lo] = 0.0
    return Problem(kappa=kappa, kmax=k_hi, psi_hat=ph, thresh=[], n_cells=[n], n_global=[n_global],
                   lattice=[lattice], dt_frac=0.5, delta=1e-6, name=f"band-pass-{k_lo}-{k_hi}-{n}")


def config_batched_instance(seed: int, n: Optional[int] = None, lattice: int = 4) -> Problem:
    """One instance of the uneven batch: draws kappa, L, slope, n, then phases.

    ``n`` and ``lattice`` override the drawn patch size and the 4 x 4 lattice
    (the draws themselves are unchanged), e.g. for surrogate training data at a
    fixed resolution with more patches per flow."""
    u = [uniform01(seed, 0x7F000000 + i) for i in range(4)]
    kappa = 10.0 ** (-3.0 + 2.0 * u[0])
    L = 2 + min(3, int(u[1] * 4))
    s = -3.0 + (3.0 - 5.0 / 3.0) * u[2]
    p = (s - 3.0) / 2.0
    n_drawn = [32, 64, 128, 256][min(3, int(u[3] * 4))]
    n = n_drawn if n is None else n
    radius = 2 * 4 ** (L - 1)
    ph = random_power_spectrum_fast(seed, radius, p)
    return Problem(kappa=kappa, kmax=radius, psi_hat=ph,
                   thresh=[4 ** l for l in range(1, L)], n_cells=[n] * L,
                   n_global=[n * 4 ** l for l in range(L)], lattice=[lattice] * L,
                   dt_frac=0.5, delta=1e-6, name=f"batched-{seed}")
