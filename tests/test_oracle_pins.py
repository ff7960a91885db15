"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself: the
paper's worked examples, closed forms, exact discrete identities, a direct
steady solve, an independent formulation, or a textbook Fourier symbol.
"""
import math
import os

import numpy as np
import pytest

import flowgen
import oracle
from oracle import DIAG, OFF12, OFF21

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- band split

def _closed_rule(kmax, thresh):
    """Independent formulation: level from min(|k1|,|k2|), part from max."""
    L = len(thresh) + 1
    edges = [-1] + list(thresh) + [10 ** 9]
    span = 2 * kmax + 1
    lev = np.full((span, span), -1, np.int8)
    part = np.full((span, span), -1, np.int8)
    for b in range(span):
        for a in range(span):
            k1, k2 = a - kmax, b - kmax
            if k1 == 0 and k2 == 0:
                continue
            m, M = min(abs(k1), abs(k2)), max(abs(k1), abs(k2))
            l = next(l for l in range(L) if edges[l] < m <= edges[l + 1])
            lev[b, a] = l
            if l == L - 1 or M <= edges[l + 1]:
                part[b, a] = DIAG
            elif abs(k1) <= edges[l + 1]:
                part[b, a] = OFF12
            else:
                part[b, a] = OFF21
    return lev, part


@pytest.mark.parametrize("kmax,thresh", [(12, [2]), (20, [1, 4, 9]), (40, [3, 10, 25]), (64, [2, 8, 32])])
def test_band_split_matches_min_max_rule(kmax, thresh):
    lv, pt = oracle.band_split(kmax, thresh)
    lv2, pt2 = _closed_rule(kmax, thresh)
    assert np.array_equal(lv, lv2) and np.array_equal(pt, pt2)


def test_band_split_worked_examples():
    names = {"diag": DIAG, "off12": OFF12, "off21": OFF21}
    lv, pt = oracle.band_split(60, [5])
    n = 0
    for line in open(os.path.join(GOLDEN, "band_split_examples.txt")):
        line = line.split("#")[0].split()
        if not line:
            continue
        k1, k2, level, part = int(line[0]), int(line[1]), int(line[2]), names[line[3]]
        for s1 in (1, -1):
            for s2 in (1, -1):
                assert lv[s2 * k2 + 60, s1 * k1 + 60] == level
                assert pt[s2 * k2 + 60, s1 * k1 + 60] == part
        n += 1
    assert n == 6


def test_band_split_partitions_spectrum():
    lv, pt = oracle.band_split(30, [3, 9])
    assert (lv >= 0).sum() == 61 * 61 - 1
    # the finest level only holds diagonal modes
    assert np.all(pt[lv == 2] == DIAG)


# ---------------------------------------------------------------- synthesis

def test_synthesis_matches_analytic_cellular():
    kmax = 16
    ph = np.zeros((2 * kmax + 1,) * 2, complex)
    flowgen.add_cellular(ph, kmax, 3, 3, 0.7, 0.4, 1.1)
    flowgen.add_cellular(ph, kmax, 16, 16, 0.2, 2.0, 0.3)
    flowgen.add_cos_x(ph, kmax, 5, 0.3)
    N, n, I0, J0 = 96, 24, 17, 70
    mask = np.ones_like(ph.real, np.int8)
    psi = oracle.synth_patch(ph, kmax, mask, N, I0, J0, n)
    i = np.arange(n)
    X, Y = np.meshgrid(2 * np.pi * (I0 + i) / N, 2 * np.pi * (J0 + i) / N, indexing="xy")
    exact = (0.7 * np.sin(3 * X + 0.4) * np.sin(3 * Y + 1.1)
             + 0.2 * np.sin(16 * X + 2.0) * np.sin(16 * Y + 0.3) + 0.3 * np.cos(5 * X))
    assert np.max(np.abs(psi - exact)) < 1e-13


def test_random_spectrum_fast_matches_loop():
    a = flowgen.random_power_spectrum(7, 12, -7.0 / 3.0)
    b = flowgen.random_power_spectrum_fast(7, 12, -7.0 / 3.0)
    assert np.allclose(a, b, rtol=0, atol=1e-15 * np.abs(a).max())   # libm vs numpy last bits
    assert np.array_equal(b, np.conj(b[::-1, ::-1]))   # Hermitian -> real psi
    assert b[12, 12] == 0


# ---------------------------------------------------------------- velocity

def test_discrete_divergence_and_forcing_vanish():
    p = flowgen.config_continuous(seed=3, radius=20, kappa=1e-2, n=32, lattice=2, levels=2)
    lv, pt = oracle.band_split(p.kmax, p.thresh)
    mask = (lv >= 0).astype(np.int8)
    psi = oracle.synth_patch(p.psi_hat, p.kmax, mask, 64, 5, 9, 32)
    h = 2 * np.pi / 64
    vx, vy, f1, f2 = oracle.staggered(psi, h)
    vmax = max(np.abs(vx).max(), np.abs(vy).max())
    assert np.abs(oracle.divergence(vx, vy, h)).max() <= 1e-13 * vmax / h
    assert abs(f1.sum()) <= 1e-12 * np.abs(f1).sum() and abs(f2.sum()) <= 1e-12 * np.abs(f2).sum()


def test_operator_second_order_consistency():
    """div(v u + K grad u) on a smooth field converges to v.grad u + K:grad grad u
    at second order (pins the advection sign, v = (-d2 psi, d1 psi), and the
    cross-derivative term)."""
    K = np.array([0.3, 0.11, 0.2])
    errs = []
    for n in (32, 64):
        h = 2 * np.pi / n
        xn = np.arange(n) * h                      # nodes
        xc = (np.arange(n) + 0.5) * h              # centres
        Xn, Yn = np.meshgrid(xn, xn, indexing="xy")
        psi = np.sin(Xn + 0.2) * np.cos(2 * Yn) + 0.5 * np.cos(Xn - Yn)
        vx, vy, _, _ = oracle.staggered(psi, h)
        X, Y = np.meshgrid(xc, xc, indexing="xy")
        u = np.sin(X + 0.3) * np.cos(2 * Y) + 0.2 * np.sin(2 * X - Y)
        ux = np.cos(X + 0.3) * np.cos(2 * Y) + 0.4 * np.cos(2 * X - Y)
        uy = -2 * np.sin(X + 0.3) * np.sin(2 * Y) - 0.2 * np.cos(2 * X - Y)
        uxx = -np.sin(X + 0.3) * np.cos(2 * Y) - 0.8 * np.sin(2 * X - Y)
        uyy = -4 * np.sin(X + 0.3) * np.cos(2 * Y) - 0.2 * np.sin(2 * X - Y)
        uxy = -2 * np.cos(X + 0.3) * np.sin(2 * Y) + 0.4 * np.sin(2 * X - Y)
        psx = np.cos(X + 0.2) * np.cos(2 * Y) - 0.5 * np.sin(X - Y)
        psy = -2 * np.sin(X + 0.2) * np.sin(2 * Y) + 0.5 * np.sin(X - Y)
        exact = (-psy) * ux + psx * uy + K[0] * uxx + 2 * K[1] * uxy + K[2] * uyy
        got = oracle.operator(vx, vy, K, None, u, h)
        errs.append(np.abs(got - exact).max())
    rate = math.log2(errs[0] / errs[1])
    assert errs[1] < 2e-2 and 1.8 < rate < 2.3, (errs, rate)


# ---------------------------------------------------------------- local solve

def _shear_patch(n, amp, k, kappa_b, delta=1e-10):
    """psi = amp cos(k x) on one whole-domain patch; returns the oracle's K and the
    discrete closed form K22_b + mean((psi - mean psi)^2)/K11_b."""
    h = 2 * np.pi / n
    x = np.arange(n) * h
    psi = np.tile(amp * np.cos(k * x), (n, 1))
    vx, vy, f1, f2 = oracle.staggered(psi, h)
    Kb = np.asarray(kappa_b, float)
    Vb = 2 * abs(0.5 * amp) * k
    dt, ns = oracle.plan_steps(n, h, Kb, Vb, 0.5, delta)
    w = oracle.local_solve_batch([n], [h], vx.ravel(), vy.ravel(), f1.ravel(), f2.ravel(),
                                 Kb[None, :], [dt], [ns])
    K = oracle.estimate(f1, f2, w[0].reshape(n, n), w[1].reshape(n, n), Kb)
    pt = psi[0] - psi[0].mean()
    return K, Kb[2] + np.mean(pt * pt) / Kb[0], (vx, vy, f1, f2, w, h, Kb)


@pytest.mark.parametrize("Kb", [[0.1, 0.0, 0.1], [0.07, 0.02, 0.13]])
def test_local_solve_discrete_taylor_identity(Kb):
    """eq:shearhomoX holds exactly for the staggered scheme:
    K22 = K22_b + mean(psi~^2)/K11_b, K11 and K12 unchanged."""
    K, K22, _ = _shear_patch(32, 0.4, 3, Kb)
    assert abs(K[2] - K22) <= 1e-9 * K22
    assert abs(K[0] - Kb[0]) <= 1e-12 and abs(K[1] - Kb[1]) <= 1e-12


def test_taylor_dispersion_shear_value():
    """v = (0, sin 16 x), kappa = 1e-2: K_yy = kappa + V^2/(2 kappa k^2) = 0.2053125.
    On a 64-cell grid the node samples of cos^2 average to exactly 1/2."""
    K, K22, _ = _shear_patch(64, -1.0 / 16, 16, [1e-2, 0.0, 1e-2])
    assert abs(K22 - 0.2053125) < 1e-15
    assert abs(K[2] - 0.2053125) <= 1e-9 * 0.2053125
    # and through the closed-form path (off-diagonal component of a 2-level split)
    p = flowgen.config_shear(k=16, V=1.0, kappa=1e-2, n=32, levels=2, thresh=[8])
    r = oracle.run_hierarchy(p)
    assert abs(r.K_total()[0][2] - 0.2053125) <= 1e-14
    assert abs(r.K_total()[0][0] - 0.01) <= 1e-16


def test_proposition1_orthogonal_shears_iterate():
    """Prop. 1: K[psi1 + psi2, kappa] = K[psi1, K[psi2, kappa]] for L2-orthogonal
    same-direction shears (exact for the discrete scheme too)."""
    n = 32
    h = 2 * np.pi / n
    x = np.arange(n) * h
    p1 = np.tile(0.3 * np.cos(2 * x), (n, 1))
    p2 = np.tile(0.2 * np.sin(5 * x), (n, 1))

    def solve(psi, Kb, Vb):
        vx, vy, f1, f2 = oracle.staggered(psi, h)
        dt, ns = oracle.plan_steps(n, h, Kb, Vb, 0.5, 1e-11)
        w = oracle.local_solve_batch([n], [h], vx.ravel(), vy.ravel(), f1.ravel(), f2.ravel(),
                                     np.asarray(Kb)[None, :], [dt], [ns])
        return oracle.estimate(f1, f2, w[0].reshape(n, n), w[1].reshape(n, n), Kb)

    kap = np.array([0.1, 0.0, 0.1])
    direct = solve(p1 + p2, kap, 0.3 * 2 + 0.2 * 5)
    inner = solve(p2, kap, 0.2 * 5)
    iterated = solve(p1, inner, 0.3 * 2)
    assert np.allclose(direct, iterated, rtol=1e-9, atol=1e-12)


def _generic_patch(n, seed=1, amp=0.6):
    p = flowgen.config_continuous(seed=seed, radius=3, p=-1.0, kappa=0.1, n=n, lattice=1, levels=1)
    lv, pt = oracle.band_split(p.kmax, p.thresh)
    psi = oracle.synth_patch(amp * p.psi_hat, p.kmax, (lv >= 0).astype(np.int8), n, 0, 0, n)
    h = 2 * np.pi / n
    return psi, h, oracle.advection_bound(*oracle.staggered(psi, h)[:2])


def _rk4_K(psi, h, Kb, Vb, delta):
    n = psi.shape[0]
    vx, vy, f1, f2 = oracle.staggered(psi, h)
    dt, ns = oracle.plan_steps(n, h, Kb, Vb, 0.5, delta)
    w = oracle.local_solve_batch([n], [h], vx.ravel(), vy.ravel(), f1.ravel(), f2.ravel(),
                                 np.asarray(Kb)[None, :], [dt], [ns])
    return (vx, vy, f1, f2), w.reshape(2, n, n)


def test_time_integration_reaches_dense_steady_cell_problem():
    """RK4 to the quasi-stationary state matches a direct (dense LU) solve of the
    discrete cell problem eq:cell."""
    psi, h, Vb = _generic_patch(8)
    Kb = np.array([0.12, 0.03, 0.09])
    (vx, vy, f1, f2), w = _rk4_K(psi, h, Kb, Vb, 1e-12)
    K_rk = oracle.estimate(f1, f2, w[0], w[1], Kb)
    K_lu = oracle.cell_problem_dense(vx, vy, f1, f2, Kb, h)
    assert np.allclose(K_rk, K_lu, rtol=1e-10, atol=1e-13)
    assert np.min(np.linalg.eigvalsh([[K_rk[0] - Kb[0], K_rk[1] - Kb[1]],
                                      [K_rk[1] - Kb[1], K_rk[2] - Kb[2]]])) > -1e-14


def test_energy_form_equals_flux_form_and_mass_conserved():
    psi, h, Vb = _generic_patch(16)
    Kb = np.array([0.1, -0.02, 0.15])
    (vx, vy, f1, f2), w = _rk4_K(psi, h, Kb, Vb, 1e-11)
    Kf = oracle.estimate(f1, f2, w[0], w[1], Kb)
    Ke = oracle.estimate_energy(w[0], w[1], Kb, h)
    assert np.allclose(Kf, Ke, rtol=1e-9, atol=1e-12)
    for j in range(2):
        assert abs(w[j].sum()) <= 1e-13 * np.abs(w[j]).sum()


def test_reversed_flow_and_transpose_symmetries():
    psi, h, Vb = _generic_patch(16, seed=4)
    Kb = np.array([0.1, 0.0, 0.1])
    f = lambda ps: oracle.estimate(*_rk4_K(ps, h, Kb, Vb, 1e-9)[0][2:], *_rk4_K(ps, h, Kb, Vb, 1e-9)[1], Kb)
    K = f(psi)
    Kneg = f(-psi)
    Kt = f(np.ascontiguousarray(psi.T))
    assert np.allclose(K, Kneg, rtol=1e-12, atol=1e-15)
    assert np.allclose([K[2], K[1], K[0]], Kt, rtol=1e-11, atol=1e-14)


def test_small_peclet_cellular_asymptotics():
    """For psi = A sin x sin y and Pe = A/kappa -> 0, K/kappa -> 1 + Pe^2/8
    (perturbation solution of eq:cell); asymptotic pin only."""
    n = 32
    h = 2 * np.pi / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    A, kap = 0.05, 1.0
    psi = A * np.sin(X) * np.sin(Y)
    Kb = np.array([kap, 0.0, kap])
    (vx, vy, f1, f2), w = _rk4_K(psi, h, Kb, 2 * A, 1e-10)
    K = oracle.estimate(f1, f2, w[0], w[1], Kb)
    enh = K[0] / kap - 1
    assert abs(enh - A * A / 8) <= 0.02 * A * A / 8
    assert abs(K[0] - K[2]) < 1e-14


# ---------------------------------------------------------------- closed forms

def test_line_energies_are_line_means_of_band_squared():
    """Parseval line energies equal the brute-force mean of psi_12^2 along x2."""
    p = flowgen.config_continuous(seed=5, radius=24, kappa=1e-2, n=16, lattice=1, levels=2)
    p.thresh = [4]
    lv, pt = oracle.band_split(p.kmax, p.thresh)
    m12 = oracle.band_mask(lv, pt, 0, OFF12)
    m21 = oracle.band_mask(lv, pt, 0, OFF21)
    N, I0, n = 64, 7, 6
    s = oracle.line_energies(p.psi_hat, p.kmax, m12, N, I0, n, 0)
    t = oracle.line_energies(p.psi_hat, p.kmax, m21, N, I0, n, 1)
    G = 2 * N  # the lines sit at half-integer indices of the level grid: use the doubled grid
    J = np.arange(G)
    for i in range(n):
        I = np.full(G, 2 * (I0 + i) + 1)
        vals = oracle.synth_points(p.psi_hat, p.kmax, m12, G, I, J)
        assert abs(np.mean(vals ** 2) - s[i]) <= 1e-12 * s[i]
        vals = oracle.synth_points(p.psi_hat, p.kmax, m21, G, J, I)
        assert abs(np.mean(vals ** 2) - t[i]) <= 1e-12 * t[i]


def test_offdiag_closed_form_equals_local_solve_for_pure_shear():
    """Algorithm 1 on a pure x2-shear (no x1 dependence) is eq:shearhomoY, which the
    time-integrated local solve reproduces exactly on the grid."""
    n = 32
    amp, k = 0.25, 3
    h = 2 * np.pi / n
    y = np.arange(n) * h
    psi = np.tile((amp * np.cos(k * y))[:, None], (1, n))
    Kb = np.array([0.08, 0.01, 0.12])
    (vx, vy, f1, f2), w = _rk4_K(psi, h, Kb, amp * k, 1e-11)
    K_ls = oracle.estimate(f1, f2, w[0], w[1], Kb)
    s = np.full(n, np.mean((psi[:, 0] - psi[:, 0].mean()) ** 2))
    K_cf = oracle.offdiag_closed_form(Kb, s, 0)
    assert np.allclose(K_ls, K_cf, rtol=1e-9, atol=1e-13)


def test_offdiag_layered_harmonic_mean_matches_resolved_solve():
    """A slowly modulated fine shear psi = A cos(x) cos(q y), q >> 1, behaves as a
    layered medium: the resolved local solve approaches the harmonic mean of the
    line-wise shear formula (Algorithm 1).  Scale-separation check (1%)."""
    n, q = 64, 16
    h = 2 * np.pi / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    A = 0.05
    psi = A * (1.0 + 0.5 * np.cos(X)) * np.cos(q * Y)
    Kb = np.array([0.05, 0.0, 0.05])
    (vx, vy, f1, f2), w = _rk4_K(psi, h, Kb, A * 1.5 * (q + 1), 1e-7)
    K_ls = oracle.estimate(f1, f2, w[0], w[1], Kb)
    xc = (np.arange(n) + 0.5) * h
    s = (A * (1.0 + 0.5 * np.cos(xc))) ** 2 / 2
    K_cf = oracle.offdiag_closed_form(Kb, s, 0)
    assert abs(K_ls[0] - K_cf[0]) <= 0.01 * K_cf[0]


def _by_level(r, lev):
    (i,) = [i for i, d in enumerate(r.domains) if d.level == lev]
    return i


def test_empty_bands_reduce_chain_to_single_level():
    """A two-level hierarchy whose second level is empty reproduces the one-level
    direct solve (no off-diagonals -> K_off = K_in, empty LS -> K_b)."""
    base = flowgen.config_continuous(seed=2, radius=3, p=-1.0, kappa=0.1, n=16, lattice=1, levels=1)
    base.psi_hat *= 0.5
    base.delta = 1e-8
    r1 = oracle.run_hierarchy(base)
    two = flowgen.Problem(kappa=0.1, kmax=3, psi_hat=base.psi_hat, thresh=[5], n_cells=[16, 16],
                          n_global=[16, 64], lattice=[1, 1], delta=1e-8)
    r2 = oracle.run_hierarchy(two)
    top, fine = _by_level(r2, 0), _by_level(r2, 1)
    assert np.allclose(r2.K_off[top], [0.1, 0.0, 0.1], rtol=0, atol=1e-16)
    assert np.array_equal(r2.K_solve[fine], r2.K_base[fine])
    assert np.allclose(r1.K_total(), r2.K_total(), rtol=1e-14, atol=1e-16)


def test_algorithm3_two_level_hand_case():
    """Algorithm 3 with hand-computable pieces: a fine-level pure shear in x2
    (psi_22 along y only would be off-diagonal, so use an x-shear on level 2 that
    the local solve turns into eq:shearhomoX exactly) and an off-diagonal x2-shear
    on level 1.  Every intermediate has a closed form."""
    kap = 0.1
    kmax = 12
    ph = np.zeros((2 * kmax + 1,) * 2, complex)
    flowgen.add_cos_y(ph, kmax, 6, 0.2)            # (0, 6): level 0, off12 for a_1 = 3
    flowgen.add_cellular(ph, kmax, 8, 8, 0.16)     # (8, 8): level 1 diag
    p = flowgen.Problem(kappa=kap, kmax=kmax, psi_hat=ph, thresh=[3], n_cells=[16, 16],
                        n_global=[16, 32], lattice=[1, 1], delta=1e-11)
    r = oracle.run_hierarchy(p)
    top, fine = _by_level(r, 0), _by_level(r, 1)
    # Algorithm 2: off12 shear amplitude 0.2 -> line energy 0.02 on every line
    Koff = np.array([kap + 0.02 / kap, 0.0, kap])
    assert np.allclose(r.K_off[top], Koff, rtol=1e-13)
    assert np.allclose(r.K_base[fine], Koff, rtol=1e-13)          # K_in of the fine level
    Kstar = r.R[fine]
    Knet = Kstar - Koff + np.array([kap, 0, kap])
    assert np.allclose(r.K_base[top], Knet, rtol=1e-13)
    # level 0 has an empty diagonal band: LS = K_net, so
    # R = K_net + S12(K_net) + S21(K_net) - 2 K_net = S12(K_net) with S21 = K_net
    expect = np.array([Knet[0] + 0.02 / Knet[2], Knet[1], Knet[2]])
    assert np.allclose(r.K_total()[0], expect, rtol=1e-13)


def _rot(theta, a, b):
    """R(theta) diag(a, b) R(theta)^T as {K11, K12, K22}, written out by hand."""
    c, s = math.cos(theta), math.sin(theta)
    return np.array([a * c * c + b * s * s, (a - b) * c * s, a * s * s + b * c * c])


def test_spd_floor_leaves_a_dominating_base_alone():
    """Algorithm 3, step 3: at the steady state K_net dominates K_in, and the
    base is then K_star - K_off + K_in exactly as formed."""
    K_in = np.array([0.02, 0.005, 0.03])
    K_net = K_in + _rot(0.3, 0.4, 0.001)        # K_in plus a PSD enhancement
    out, low = oracle.spd_floor(K_net, K_in)
    assert not low and np.array_equal(out, K_net)


@pytest.mark.parametrize("theta", [0.0, 0.4, -1.1, math.pi / 2])
def test_spd_floor_raises_the_low_eigenvalue_and_keeps_the_axes(theta):
    """A K_net whose low eigenvalue lies below lambda_min(K_in): the eigenvalue
    is raised to lambda_min(K_in) on the same eigenvector, the other one kept
    (closed form R diag(a, floor) R^T).  K_in is anisotropic with a cross
    term, so taking its larger eigenvalue, or its diagonal, fails."""
    K_in = _rot(0.7, 0.05, 0.01)                # lambda_min = 0.01, lambda_max = 0.05
    floor = 0.01
    out, low = oracle.spd_floor(_rot(theta, 0.3, -0.02), K_in)
    assert low
    np.testing.assert_allclose(out, _rot(theta, 0.3, floor), rtol=0, atol=1e-15)
    out, low = oracle.spd_floor(_rot(theta, 0.3, 0.004), K_in)     # positive but below the floor
    assert low
    np.testing.assert_allclose(out, _rot(theta, 0.3, floor), rtol=0, atol=1e-15)


def test_spd_floor_both_low_or_not_a_number_gives_the_floor():
    K_in = np.array([0.02, 0.0, 0.03])
    out, low = oracle.spd_floor(_rot(0.2, -0.1, -0.3), K_in)
    assert low
    np.testing.assert_allclose(out, [0.02, 0.0, 0.02], rtol=0, atol=1e-16)
    out, low = oracle.spd_floor(np.array([np.nan, 0.0, 1.0]), K_in)
    assert low and np.array_equal(out, [0.02, 0.0, 0.02])


def test_roots_compute_exactly_the_selected_chains():
    """The sampled-centre run (roots) gives the same numbers, bit for bit, as
    the whole hierarchy on the chains it selects, and nothing elsewhere."""
    p = flowgen.config_continuous(seed=4, radius=24, n=8, lattice=2, levels=3)
    full = oracle.run_hierarchy(p)
    lev0 = [i for i, d in enumerate(full.domains) if d.level == 0]
    part = oracle.run_hierarchy(p, roots=[lev0[1], lev0[2]])
    sel = {lev0[1], lev0[2]}
    for i, d in enumerate(full.domains):
        j, top = i, d
        while top.level > 0:
            j = top.parent
            top = full.domains[j]
        if j in sel:
            for name in ("K_in", "K_base", "K_solve", "R"):
                assert np.array_equal(getattr(part, name)[i], getattr(full, name)[i]), (name, i)
            assert part.nsteps[i] == full.nsteps[i]
        else:
            assert np.all(part.R[i] == 0.0) and part.nsteps[i] == 0
    assert full.clamped == [] and part.clamped == []


# ---------------------------------------------------------------- macro

def test_coarse_base_does_not_depend_on_how_its_children_are_numbered():
    """A level-1 lattice of 2 x 2 centres under one level-0 centre whose own
    bands are empty: the coarse base, hence K_total, is built from the four
    children's results.  Translating the flow by one child spacing (pi in x)
    permutes the children, so K_total must not change although the
    children's results differ."""
    kmax, kap = 6, 0.05
    ph = np.zeros((2 * kmax + 1, 2 * kmax + 1), complex)
    flowgen.add_cellular(ph, kmax, 4, 4, 0.5)
    flowgen.add_cellular(ph, kmax, 3, 4, 0.4, 0.3, 0.7)
    shifted = ph * ((-1.0) ** np.arange(-kmax, kmax + 1))[None, :]       # psi(x + pi, y)

    def run(spec):
        q = flowgen.Problem(kappa=kap, kmax=kmax, psi_hat=spec, thresh=[2], n_cells=[16, 16],
                            n_global=[16, 32], lattice=[1, 2])
        return oracle.run_hierarchy(q)

    a, b = run(ph), run(shifted)
    kids = [j for j, d in enumerate(a.domains) if d.level == 1]
    assert len(kids) == 4
    assert np.max(np.abs(a.R[kids[0]] - a.R[kids[1]])) >= 1e-3 * np.max(np.abs(a.R[kids[0]]))
    np.testing.assert_allclose(b.K_total(), a.K_total(), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("c", [0.0, -0.4, 0.4])
def test_macro_plan_is_the_fewest_stable_steps(c):
    """The macro grid's checkerboard is an eigenvector of its diffusion with
    rate 4 (K11 + K22) / h^2 whatever K12 (the cross differences vanish on
    it).  With dt_frac = 1 one planned step keeps its amplitude within RK4's
    stability region, and for an isotropic K one step fewer over the same
    time does not."""
    N, kap, T = 8, 0.05, 100.0
    K = np.array([kap, c * kap, kap])
    cb = np.fromfunction(lambda j, i: (-1.0) ** (i + j), (N, N))
    dt, ns = oracle.macro_plan(N, np.tile(K, (N * N, 1)), 0.0, 1.0, T)
    g = oracle.macro_run(N, None, None, K, cb, dt, 1) / cb
    assert np.ptp(g) <= 1e-12 and abs(g[0, 0]) <= 1.0
    if c == 0.0:
        g = oracle.macro_run(N, None, None, K, cb, T / (ns - 1), 1) / cb
        assert abs(g[0, 0]) > 1.0


def test_macro_step_with_a_k_field_commutes_with_the_grid_symmetries():
    """A random SPD K field at cell centres: the macro step must not prefer a
    side.  Reflecting the grid in x or in y (with K12 negated) or transposing
    it (with K11 and K22 exchanged) maps the evolved field to the evolved
    reflected or transposed field, which holds when every face takes the
    mean of the two cells it separates."""
    rng = np.random.default_rng(4)
    N, dt, ns = 12, 0.05, 7
    Kc = np.zeros((N, N, 3))
    Kc[..., 0] = rng.uniform(0.02, 0.2, (N, N))
    Kc[..., 2] = rng.uniform(0.02, 0.2, (N, N))
    Kc[..., 1] = 0.3 * np.sqrt(Kc[..., 0] * Kc[..., 2]) * rng.uniform(-1, 1, (N, N))
    u0 = rng.standard_normal((N, N))

    def run(K, u):
        return oracle.macro_run(N, None, None, np.ascontiguousarray(K).reshape(-1, 3), np.ascontiguousarray(u),
                                dt, ns)

    base = run(Kc, u0)
    Kx = Kc[:, ::-1].copy()
    Kx[..., 1] *= -1
    assert np.max(np.abs(run(Kx, u0[:, ::-1]) - base[:, ::-1])) <= 1e-14
    Ky = Kc[::-1].copy()
    Ky[..., 1] *= -1
    assert np.max(np.abs(run(Ky, u0[::-1]) - base[::-1])) <= 1e-14
    Kt = Kc.transpose(1, 0, 2)[..., ::-1]
    assert np.max(np.abs(run(Kt, u0.T) - base.T)) <= 1e-14


def test_macro_dirichlet_operator_is_second_order_up_to_the_walls():
    """u = g0 + (g1 - g0) x / 2 pi + A sin(x / 2) sin y meets both wall values
    and varies along the walls; with an anisotropic K (K12 != 0) one tiny
    step gives the discrete operator, which must approach
    K11 u_xx + 2 K12 u_xy + K22 u_yy at second order in every column, the
    wall columns included (their tangential differences use ghost values
    continued linearly through the wall)."""
    g0, g1, A = 0.3, 1.1, 0.7
    K = np.array([0.4, 0.15, 0.25])
    errs = []
    for N in (16, 32, 64):
        h = 2 * np.pi / N
        c = (np.arange(N) + 0.5) * h
        X, Y = np.meshgrid(c, c, indexing="xy")
        u0 = g0 + (g1 - g0) * X / (2 * np.pi) + A * np.sin(X / 2) * np.sin(Y)
        exact = (K[0] * (-A / 4) * np.sin(X / 2) * np.sin(Y) + 2 * K[1] * (A / 2) * np.cos(X / 2) * np.cos(Y)
                 + K[2] * (-A) * np.sin(X / 2) * np.sin(Y))
        dt = 1e-6
        u1 = oracle.macro_run(N, None, None, K, u0, dt, 1, dirichlet_x=(g0, g1))
        errs.append(np.max(np.abs((u1 - u0) / dt - exact)))
    assert errs[0] <= 1e-2
    assert errs[1] <= 0.3 * errs[0] and errs[2] <= 0.3 * errs[1], errs


def test_macro_dirichlet_time_stepping_is_fourth_order():
    """Halving dt twice over the same time: the successive differences of
    the Dirichlet macro solution shrink by about 2^4 (classic RK4)."""
    g0, g1 = 0.3, 1.1
    K = np.array([0.4, 0.15, 0.25])
    N, T = 16, 2.0
    h = 2 * np.pi / N
    c = (np.arange(N) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    u0 = g0 + (g1 - g0) * X / (2 * np.pi) + 0.7 * np.sin(X / 2) * np.sin(Y) + 0.3 * np.sin(X) * np.cos(2 * Y)
    u = [oracle.macro_run(N, None, None, K, u0, T / m, m, dirichlet_x=(g0, g1)) for m in (40, 80, 160)]
    ratio = np.max(np.abs(u[0] - u[1])) / np.max(np.abs(u[1] - u[2]))
    assert 12.0 <= ratio <= 20.0, ratio


def test_macro_rk4_matches_fourier_closed_form():
    """v = 0, constant K: each Fourier mode is multiplied by R(dt mu_k)^nsteps,
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 (classic RK4), mu_k the symbol of the
    9-point operator K11 dxx + K22 dyy + 2 K12 dxdy."""
    N = 32
    h = 2 * np.pi / N
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal((N, N))
    K = np.array([0.3, 0.12, 0.2])
    dt, ns = oracle.macro_plan(N, K, 0.0, 0.2, 0.4)
    u = oracle.macro_run(N, None, None, K, u0, dt, ns)
    th = 2 * np.pi * np.fft.fftfreq(N)
    TX, TY = np.meshgrid(th, th, indexing="xy")
    mu = -(K[0] * 4 * np.sin(TX / 2) ** 2 + K[2] * 4 * np.sin(TY / 2) ** 2
           + 2 * K[1] * np.sin(TX) * np.sin(TY)) / h ** 2
    z = dt * mu
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    exact = np.real(np.fft.ifft2(np.fft.fft2(u0) * R ** ns))
    assert np.max(np.abs(u - exact)) <= 1e-12 * np.max(np.abs(u0))


def test_macro_conserves_mass_with_advection_and_field():
    N = 24
    h = 2 * np.pi / N
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    vx, vy, _, _ = oracle.staggered(np.sin(X) * np.sin(Y), h)
    Kc = np.stack([0.1 + 0.05 * np.cos(X), 0.01 * np.sin(Y), 0.2 + 0.0 * X], -1)
    u0 = flowgen.macro_initial_gaussian(N)
    dt, ns = oracle.macro_plan(N, Kc, 2.0, 0.2, 0.3)
    u = oracle.macro_run(N, vx, vy, Kc, u0, dt, ns)
    assert abs(u.sum() - u0.sum()) <= 1e-13 * abs(u0.sum())


def _heat_series(x, t, K11, terms=4000):
    """u_t = K11 u_xx on [0, L], u(0) = 1, u(L) = 0, u(x, 0) = 1 for x <= L/2
    else 0 (the step data of Section 4): the steady line plus the sine series
    of the initial deviation, whose coefficients are -2 cos(m pi / 2) / (m pi)."""
    L = 2 * np.pi
    u = 1 - x / L
    for m in range(1, terms + 1):
        b = -2.0 * math.cos(m * math.pi / 2) / (m * math.pi)
        if b != 0.0:
            u = u + b * np.sin(m * math.pi * x / L) * math.exp(-K11 * (m * math.pi / L) ** 2 * t)
    return u


def test_macro_dirichlet_step_converges_to_the_heat_series():
    """Dirichlet in x, periodic in y (Section 4), pure diffusion from the step
    data: second-order convergence to the closed-form series solution (a
    boundary flux over the wrong distance would cost an order)."""
    K = np.array([1.0, 0.0, 1.0])
    errs = []
    for N in (32, 64, 128):
        h = 2 * np.pi / N
        x = (np.arange(N) + 0.5) * h
        u0 = np.tile((x <= np.pi).astype(float), (N, 1))
        dt, ns = oracle.macro_plan(N, K, 0.0, 0.2, 0.5)
        u = oracle.macro_run(N, None, None, K, u0, dt, ns, dirichlet_x=(1.0, 0.0))
        assert np.max(np.abs(u - u[0:1])) == 0.0           # stays independent of y
        errs.append(float(np.max(np.abs(u - _heat_series(x, 0.5, 1.0)[None, :]))))
    assert errs[2] <= 1e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.6 <= a / b <= 4.4, errs


def test_macro_dirichlet_linear_profile_is_steady():
    """The linear profile between the two boundary values is a steady state of
    the Dirichlet scheme for any constant K (cross term included): every
    x-face, boundary faces over h/2 included, carries the same flux, and the
    ghost values continue the line."""
    N = 16
    h = 2 * np.pi / N
    x = (np.arange(N) + 0.5) * h
    g0, g1 = 1.0, 0.25
    u0 = np.tile(g0 + (g1 - g0) * x / (2 * np.pi), (N, 1))
    u = oracle.macro_run(N, None, None, np.array([0.3, 0.12, 0.2]), u0, 0.01, 50, dirichlet_x=(g0, g1))
    assert np.max(np.abs(u - u0)) <= 1e-13


def test_macro_dirichlet_shear_along_the_boundary_does_not_act():
    """A shear v = (0, V sin kx) carries a field that depends on x alone along
    its own level lines: with the Dirichlet boundaries the solution is the
    pure-diffusion one; a constant field stays constant under a divergence-free
    flow with both boundary values equal to it."""
    N = 32
    h = 2 * np.pi / N
    x = (np.arange(N) + 0.5) * h
    xf = np.arange(N) * h
    K = np.array([0.7, 0.0, 0.7])
    u0 = np.tile((x <= np.pi).astype(float), (N, 1))
    vy = np.tile(1.5 * np.sin(3 * (xf + 0.5 * h)), (N, 1))   # y-faces sit at x = (i + 1/2) h
    vx = np.zeros((N, N))
    dt, ns = oracle.macro_plan(N, K, 3.0, 0.2, 0.4)
    ref = oracle.macro_run(N, None, None, K, u0, dt, ns, dirichlet_x=(1.0, 0.0))
    got = oracle.macro_run(N, vx, vy, K, u0, dt, ns, dirichlet_x=(1.0, 0.0))
    assert np.max(np.abs(got - ref)) <= 1e-13
    X, Y = np.meshgrid(xf, xf, indexing="xy")
    wx, wy, _, _ = oracle.staggered(np.sin(X) * np.sin(2 * Y) + 0.3 * np.cos(2 * X + Y), h)
    c = np.full((N, N), 0.4)
    cst = oracle.macro_run(N, wx, wy, K, c, dt, ns, dirichlet_x=(0.4, 0.4))
    assert np.max(np.abs(cst - 0.4)) <= 1e-13


def test_macro_dirichlet_uniform_flow_reaches_the_discrete_steady_state():
    """A uniform flow vx = V with Dirichlet boundaries: the scheme's steady
    state carries one flux C through every x-face, boundary faces included
    (face value = boundary value, gradient over h/2).  Marching that relation
    from x = 0 gives u as an affine function of C and the last face fixes C:
    an independent 1-D computation the long-time oracle solution must reach."""
    N, K, V, g0, g1 = 16, 0.8, 0.6, 1.0, 0.2
    h = 2 * np.pi / N

    def march(C):
        u = np.zeros(N)
        u[0] = g0 + (C - V * g0) * h / (2 * K)
        for i in range(1, N):
            u[i] = (C - u[i - 1] * (V / 2 - K / h)) / (V / 2 + K / h)
        return u, V * g1 + K * (g1 - u[N - 1]) / (h / 2) - C

    (_, ra), (_, rb) = march(0.0), march(1.0)
    u_ss, _ = march(-ra / (rb - ra))
    Kv = np.array([K, 0.0, K])
    dt, ns = oracle.macro_plan(N, Kv, 2 * V, 0.4, 120.0)
    u = oracle.macro_run(N, np.full((N, N), V), np.zeros((N, N)), Kv, np.zeros((N, N)), dt, ns,
                         dirichlet_x=(g0, g1))
    assert np.max(np.abs(u - u_ss[None, :])) <= 1e-12


def test_interpolate_centres_is_separable_periodic_linear_interpolation():
    """The lattice-to-grid interpolation of the macro K field: bilinear and
    periodic means linear interpolation in x then in y with wrap-around, which
    numpy's interp with a period computes independently; where a cell centre
    falls on a lattice centre (N / M odd) the lattice value comes back exactly."""
    rng = np.random.default_rng(3)
    M, N = 4, 12
    Kc = rng.uniform(0.5, 2.0, (M, M, 3))
    got = oracle.interpolate_centres(Kc, M, N)
    lat = np.arange(M) + 0.5                      # lattice centres in lattice units
    pos = (np.arange(N) + 0.5) / N * M            # cell centres in lattice units
    for q in range(3):
        rows = np.array([np.interp(pos, lat, Kc[r, :, q], period=M) for r in range(M)])      # along x
        want = np.array([np.interp(pos, lat, rows[:, i], period=M) for i in range(N)]).T    # along y
        np.testing.assert_allclose(got[:, :, q], want, rtol=1e-14, atol=1e-14)
    assert np.array_equal(got[1::3, 1::3], Kc)
    M, N = 3, 16                                   # a ratio that is not an integer
    Kc = rng.uniform(0.5, 2.0, (M, M, 3))
    got = oracle.interpolate_centres(Kc, M, N)
    lat = np.arange(M) + 0.5
    pos = (np.arange(N) + 0.5) / N * M
    rows = np.array([np.interp(pos, lat, Kc[r, :, 0], period=M) for r in range(M)])
    want = np.array([np.interp(pos, lat, rows[:, i], period=M) for i in range(N)]).T
    np.testing.assert_allclose(got[:, :, 0], want, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------- quasi-stationary stop

def test_quasi_stationary_stop_keeps_k_within_its_bound():
    """HMM step 2 evolves each local problem until it is quasi-stationary.  The
    adaptive stop ends a solve once the change of the correctors over a chunk
    bounds the remaining error of K below delta times the base; against the
    steady K (a plan to delta = 1e-12) the stopped K must be inside that
    bound (relative to K), with fewer steps than the a-priori plan to
    delta = 1e-6."""
    p = flowgen.config_four_level_cellular(n=32, lattice=2)
    r = oracle.run_hierarchy(p)
    lv, pt = oracle.band_split(p.kmax, p.thresh)
    for d in (0, 4, 8, 12):                          # one patch per level
        D = r.domains[d]
        psi = oracle.synth_patch(p.psi_hat, p.kmax, oracle.band_mask(lv, pt, D.level, DIAG), D.N, D.I0, D.J0, D.n)
        vx, vy, f1, f2 = oracle.staggered(psi, D.h)
        Kb = r.K_base[d]
        vb = oracle.advection_bound(vx, vy)
        dt6, ns6 = oracle.plan_steps(D.n, D.h, Kb, vb, 0.5, 1e-6)
        dt12, ns12 = oracle.plan_steps(D.n, D.h, Kb, vb, 0.5, 1e-12)
        w, taken = oracle.local_solve_adaptive(D.n, D.h, vx, vy, f1, f2, Kb, dt6, ns6, 1e-6)
        ws = oracle.local_solve_batch([D.n], [D.h], vx.ravel(), vy.ravel(), f1.ravel(), f2.ravel(), Kb[None, :],
                                      [dt12], [ns12])
        n = D.n
        K = oracle.estimate(f1, f2, w[0].reshape(n, n), w[1].reshape(n, n), Kb)
        Ks = oracle.estimate(f1, f2, ws[0].reshape(n, n), ws[1].reshape(n, n), Kb)
        assert np.max(np.abs(K - Ks)) <= 1e-6 * np.max(np.abs(K)), (d, K, Ks)
        assert taken < 0.6 * ns6, (d, taken, ns6)


@pytest.mark.parametrize("delta", [1e-6, 3e-7])
def test_quasi_stationary_stop_chunk_of_a_single_mode_shear(delta):
    """v = (0, V sin x) on the whole period: the second corrector is driven by
    the single lowest mode, which decays at exactly the Poincare rate
    mu = kappa 4 sin^2(pi / n) / h^2 of the isotropic base, so w_2(t) =
    (1 - e^(-mu t)) chi with chi = f_2 / mu, and the remaining error of K22
    is e^(-mu t) <f_2 chi> (the Cauchy-Schwarz bound is an equality for one
    mode).  The stop must come at the first chunk of ceil(nsteps / chunks)
    steps where that error is at most delta times K22(t), no earlier and no
    later."""
    n, kap, V = 16, 0.05, 1.0
    h = 2 * np.pi / n
    x = np.arange(n) * h
    psi = np.tile(-V * np.cos(x), (n, 1))
    vx, vy, f1, f2 = oracle.staggered(psi, h)
    assert not np.any(vx) and not np.any(f1)
    mu = kap * 4 * math.sin(math.pi / n) ** 2 / h ** 2
    dt, nsteps, chunks = 0.2, 3301, 32
    C = 104                                            # ceil(3301 / 32)
    fc = float(np.mean(f2 * f2)) / mu                  # <f_2 chi>

    def ratio(c):                                      # remaining error over delta K22 after c chunks
        e = math.exp(-mu * c * C * dt)
        return e * fc / (delta * (kap + (1 - e) * fc))

    c = next(c for c in range(1, nsteps) if ratio(c) <= 1.0)
    assert c * C < nsteps and ratio(c) < 0.9 and ratio(c - 1) > 1.1     # clear of the threshold
    w, taken = oracle.local_solve_adaptive(n, h, vx, vy, f1, f2, [kap, 0.0, kap], dt, nsteps, delta, chunks)
    assert taken == c * C


# ---------------------------------------------------------------- Section 4, Tests 2 and 3

def _paper_gap(test):
    """Relative gap between the two-level SHMM K (decomposition factor 5) and
    the direct cell problem of the full flow, for the Section 4 example with
    the velocity scaled by 2 pi, wavenumbers divided by 5 (the same
    homogenized K), 64^2 whole-domain patches."""
    scale = 2 * math.pi
    shmm = oracle.run_hierarchy(flowgen.config_paper_cellular(test, scale, n=64, levels=2, divide=5))
    direct = oracle.run_hierarchy(flowgen.config_paper_cellular(test, scale, n=64, levels=1, divide=5))
    a, b = shmm.K_total()[0], direct.K_total()[0]
    assert abs(a[1]) < 1e-12 and abs(b[1]) < 1e-12 and abs(a[0] - a[2]) < 1e-12 * a[0]   # diagonal, isotropic
    return float(np.max(np.abs(a - b)) / b[0]), b[0]


def test_section4_separated_cellular_modes_match_the_direct_cell_problem():
    """Test 2 (Table 1): two well-separated cellular modes have no off-diagonal
    part, and the paper reports SHMM within 0.05% of the reference; the
    oracle's SHMM and its direct solve agree to the same order."""
    gap, K = _paper_gap(2)
    assert K > 1.5                 # an O(1) enhancement, so the agreement is not trivial
    assert gap <= 1e-3, gap


def test_section4_off_diagonal_cellular_modes_cost_about_five_percent():
    """Test 3 (Table 2): with off-diagonal modes (5, 45) and (45, 5) the closed
    form of Algorithm 1 misses part of their interaction with the other
    scales; the paper reports errors of about 5%."""
    gap, K = _paper_gap(3)
    assert K > 1.3
    assert 0.03 <= gap <= 0.10, gap


# ---------------------------------------------------------------- bookkeeping

def test_domain_table_geometry():
    p = flowgen.config_four_level_cellular(n=32, lattice=4)
    doms = oracle.domain_table(p)
    assert len(doms) == 4 * 16
    for d in doms:
        # the centre 2 pi (c + 1/2)/M is the patch middle: I0 + n/2 == N (c + 1/2)/M mod N
        assert (2 * (d.I0 + d.n // 2) * 4) % (2 * d.N) == (d.N * (2 * d.cx + 1)) % (2 * d.N)
        if d.level > 0:
            par = doms[d.parent]
            assert par.level == d.level - 1 and (par.cx, par.cy) == (d.cx, d.cy)
    assert doms[-1].offset + doms[-1].n ** 2 == sum(d.n ** 2 for d in doms)
    with pytest.raises(oracle.BookkeepingError):
        bad = flowgen.config_four_level_cellular(n=32, lattice=4)
        bad.lattice = [3, 4, 4, 4]
        oracle.domain_table(bad)


# ---------------------------------------------------------------- step plan

def _dense(vx, vy, K, h, n):
    """The discrete operator u -> div(v u + K grad u) as a dense matrix, column by column."""
    A = np.zeros((n * n, n * n))
    for c in range(n * n):
        e = np.zeros(n * n)
        e[c] = 1.0
        A[:, c] = oracle.operator(vx, vy, K, None, e.reshape(n, n), h).ravel()
    return A


def _random_flow(n, seed, amp):
    rng = np.random.default_rng(seed)
    h = 2 * np.pi / n
    psi = np.zeros((n, n))
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    for _ in range(4):
        k1, k2 = rng.integers(-3, 4, 2)
        psi += amp * rng.standard_normal() * np.cos(k1 * X + k2 * Y + rng.uniform(0, 2 * np.pi))
    return oracle.staggered(psi, h)[:2] + (h,)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_advection_bound_bounds_the_spectrum(seed):
    """The eigenvalues of the discrete advection operator (zero diffusion) are
    imaginary and no larger than advection_bound / h; a uniform flow reaches it."""
    n = 8
    vx, vy, h = _random_flow(n, seed, 1.0)
    ev = np.linalg.eigvals(_dense(vx, vy, [0.0, 0.0, 0.0], h, n))
    bound = oracle.advection_bound(vx, vy) / h
    assert np.max(np.abs(ev.real)) <= 1e-10 * bound
    assert np.max(np.abs(ev)) <= bound * (1 + 1e-12)
    V = 0.7
    ev = np.linalg.eigvals(_dense(np.full((n, n), V), np.zeros((n, n)), [0.0, 0.0, 0.0], h, n))
    assert abs(np.max(np.abs(ev)) - oracle.advection_bound(np.full((n, n), V), np.zeros((n, n))) / h) \
        <= 1e-12 * V / h


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_step_plan_is_stable_and_decays_by_delta(seed):
    """For random flows and random SPD bases, independently of the plan's
    formula: (i) every eigenvalue of the discrete operator times dt lies in the
    classic RK4 stability region (|1 + z + z^2/2 + z^3/6 + z^4/24| <= 1); (ii)
    the slowest decaying non-constant mode has decayed by delta or more at
    T = nsteps dt."""
    rng = np.random.default_rng(100 + seed)
    n = 8
    vx, vy, h = _random_flow(n, seed, 0.3 + 3.0 * rng.uniform())
    a, b = rng.uniform(0.02, 0.3, 2)
    c = rng.uniform(-0.9, 0.9) * np.sqrt(a * b)
    K = [a, c, b]
    delta = 1e-6
    dt, ns = oracle.plan_steps(n, h, K, oracle.advection_bound(vx, vy), 0.9, delta)
    ev = np.linalg.eigvals(_dense(vx, vy, K, h, n))
    z = dt * ev
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    assert np.max(np.abs(R)) <= 1 + 1e-12
    decay = np.sort(-ev.real)
    assert abs(decay[0]) <= 1e-10 * np.max(np.abs(ev))       # the constant mode
    assert np.exp(-decay[1] * dt * ns) <= delta * (1 + 1e-9)


def test_step_plan_decay_is_tight_for_pure_diffusion():
    """Without flow and with an isotropic base the slowest mode decays at
    exactly the plan's bound, so the planned time brings it to delta, no less."""
    n, kap, delta = 8, 0.07, 1e-6
    h = 2 * np.pi / n
    z = np.zeros((n, n))
    dt, ns = oracle.plan_steps(n, h, [kap, 0.0, kap], oracle.advection_bound(z, z), 0.5, delta)
    ev = np.linalg.eigvals(_dense(z, z, [kap, 0.0, kap], h, n))
    slow = np.sort(-ev.real)[1]
    assert abs(np.exp(-slow * dt * ns) / delta - 1) <= 1e-9


def _rk4_gain(z):
    """|R(z)| of classic RK4, R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24."""
    return np.abs(1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24)


@pytest.mark.parametrize("delta", [1e-6, 1e-3])
def test_step_plan_is_the_fewest_stable_steps_for_pure_diffusion(delta):
    """dt_frac = 1, no flow, isotropic base: the fastest mode (the
    checkerboard, 8 kappa / h^2) is where the plan's diffusion bound is exact,
    so the planned step keeps it inside RK4's real stability interval
    (about -2.785) and one step fewer over the same time leaves it.  A cross
    term of either sign leaves the fastest mode where it is, and the step
    stays stable."""
    n, kap = 8, 0.05
    h = 2 * np.pi / n
    z0 = np.zeros((n, n))
    fast = 8 * kap / h ** 2
    dt, ns = oracle.plan_steps(n, h, [kap, 0.0, kap], oracle.advection_bound(z0, z0), 1.0, delta)
    ev = np.linalg.eigvals(_dense(z0, z0, [kap, 0.0, kap], h, n))
    assert abs(np.max(np.abs(ev)) - fast) <= 1e-12 * fast
    assert _rk4_gain(-dt * fast) <= 1.0
    assert ns >= 2 and _rk4_gain(-dt * ns / (ns - 1) * fast) > 1.0
    for c in (-0.4, 0.4, -0.9):
        K = [kap, c * kap, kap]
        dt, ns = oracle.plan_steps(n, h, K, 0.0, 1.0, delta)
        ev = np.linalg.eigvals(_dense(z0, z0, K, h, n))
        assert abs(np.max(np.abs(ev)) - fast) <= 1e-12 * fast, c
        assert np.max(_rk4_gain(dt * ev)) <= 1 + 1e-12, c


def test_step_plan_meets_the_imaginary_stability_edge_for_a_moving_row():
    """One row of cells moving along x at speed U, everything else at rest,
    and a negligible base: the advection eigenvalues are i U sin(theta) / h,
    so the fastest is U / h, which the advection bound reaches.  With
    dt_frac = 1 the step puts it on RK4's imaginary stability edge
    (2 sqrt 2, where |R| = 1) to within the plan's rounded constant."""
    n, U = 8, 0.8
    h = 2 * np.pi / n
    vx = np.zeros((n, n))
    vx[3, :] = U
    vy = np.zeros((n, n))
    K = [1e-9, 0.0, 1e-9]
    dt, ns = oracle.plan_steps(n, h, K, oracle.advection_bound(vx, vy), 1.0, 1e-6)
    ev = np.linalg.eigvals(_dense(vx, vy, K, h, n))
    top = ev[np.argmax(np.abs(ev))]
    assert abs(abs(top) - U / h) <= 1e-9 * U / h
    assert 0.995 <= _rk4_gain(dt * top) <= 1.0
    assert np.max(_rk4_gain(dt * ev)) <= 1 + 1e-12


def test_macro_diffusivity_uses_the_level_base():
    """A shear v = (0, V sin 4x) in level 0's off-21 band and a cellular mode
    in level 1's diagonal band: the finer level raises level 0's base K_net
    above K_in = kappa I, and the macro diffusivity is the shear's Taylor
    value on that base, K22 = K_b22 + V^2 / (2 k^2 K_b11), with K_b11 and
    K_b12 passing through."""
    kmax, k, V, kap = 6, 4, 1.0, 0.05
    ph = np.zeros((2 * kmax + 1, 2 * kmax + 1), complex)
    flowgen.add_cos_x(ph, kmax, k, -V / k)
    flowgen.add_cellular(ph, kmax, 6, 6, 0.3)
    p = flowgen.Problem(kappa=kap, kmax=kmax, psi_hat=ph, thresh=[2], n_cells=[32, 32], n_global=[32, 32],
                        lattice=[1, 1])
    r = oracle.run_hierarchy(p)
    i = next(j for j, d in enumerate(r.domains) if d.level == 0)
    Kb = r.K_base[i]
    assert np.max(np.abs(Kb - r.K_in[i])) >= 0.1 * kap          # the base is not K_in
    Km = oracle.macro_diffusivity(r, i)
    assert abs(Km[0] - Kb[0]) <= 1e-16 and abs(Km[1] - Kb[1]) <= 1e-16
    assert abs(Km[2] - (Kb[2] + V * V / (2 * k * k * Kb[0]))) <= 1e-13 * Km[2]


def test_macro_diffusivity_of_a_resolved_shear_is_the_taylor_value():
    """v = (0, sin 16x) with band edge 8: the mode lies in level 0's off-21
    band, which a macro grid does not resolve, so the macro diffusivity is the
    closed-form shear value K_yy = kappa + V^2/(2 kappa k^2) = 0.2053125 with
    K_xx = kappa; and the additive rule R = K_solve + macro - K_base holds."""
    p = flowgen.config_shear(k=16, V=1.0, kappa=1e-2, n=32, levels=2, thresh=[8])
    r = oracle.run_hierarchy(p)
    for i, d in enumerate(r.domains):
        if d.level != 0:
            continue
        Km = oracle.macro_diffusivity(r, i)
        assert abs(Km[2] - 0.2053125) <= 1e-14 and abs(Km[0] - 0.01) <= 1e-16 and abs(Km[1]) <= 1e-16
        np.testing.assert_allclose(r.R[i], r.K_solve[i] + Km - r.K_base[i], rtol=1e-14, atol=1e-16)


def test_one_level_hierarchy_is_the_direct_cell_problem():
    """With a single level the band filter is the identity, so the hierarchy's
    K is the discrete cell problem of the full flow on the whole domain,
    solved directly (dense LU) from psi sampled at the grid nodes."""
    n = 8
    kmax = 3
    ph = flowgen.random_power_spectrum(seed=4, radius=kmax, p=-2.0, amp=0.15)
    p = flowgen.Problem(kappa=0.05, kmax=kmax, psi_hat=ph, thresh=[], n_cells=[n], n_global=[n],
                        lattice=[1], dt_frac=0.5, delta=1e-12, name="one-level")
    r = oracle.run_hierarchy(p)
    h = 2 * np.pi / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    kk = np.arange(-kmax, kmax + 1)
    psi = np.zeros((n, n))
    for b, k2 in enumerate(kk):
        for a, k1 in enumerate(kk):
            psi += (ph[b, a] * np.exp(1j * (k1 * X + k2 * Y))).real
    vx, vy, f1, f2 = oracle.staggered(psi, h)
    K = oracle.cell_problem_dense(vx, vy, f1, f2, [0.05, 0.0, 0.05], h)
    assert len(r.domains) == 1
    np.testing.assert_allclose(r.K_total()[0], K, rtol=1e-9, atol=1e-13)


def test_window_estimate_is_centred_and_normalised_on_its_cells():
    """An indicator corrector: w_1 = 1 on exactly the centred m x m cells of an
    n x n patch and f_1 = 1 everywhere, so the windowed K11 gains exactly 1,
    while the whole-patch estimate gains m^2 / n^2.  A window that is not
    centred, or not normalised by its own cell count, fails."""
    n, m = 16, 6
    a = (n - m) // 2
    w1 = np.zeros((n, n))
    w1[a:a + m, a:a + m] = 1.0
    one = np.ones((n, n))
    zero = np.zeros((n, n))
    Kb = [0.3, 0.01, 0.2]
    Kw = oracle.estimate_window(one, zero, w1, zero, Kb, m)
    np.testing.assert_allclose(Kw, [1.3, 0.01, 0.2], rtol=0, atol=1e-15)
    Kf = oracle.estimate_window(one, zero, w1, zero, Kb, 0)
    np.testing.assert_allclose(Kf, [0.3 + m * m / n / n, 0.01, 0.2], rtol=0, atol=1e-15)
    # shifting the indicator by one cell takes it off the window's edge rows
    w1s = np.roll(w1, 1, axis=1)
    assert oracle.estimate_window(one, zero, w1s, zero, Kb, m)[0] == pytest.approx(0.3 + (m - 1) / m, abs=1e-15)


def test_window_over_one_period_of_a_periodic_flow_is_the_whole_patch():
    """For a flow whose period divides the patch (psi = 0.3 sin 2x sin 2y on a
    32^2 patch of side 2 pi, period 16 cells), the correctors inherit the
    period, so the average over the centred 16^2 window (one period) equals
    the whole-patch average up to summation order."""
    n = 32
    h = 2 * np.pi / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    psi = 0.3 * np.sin(2 * X) * np.sin(2 * Y)
    vx, vy, f1, f2 = oracle.staggered(psi, h)
    Kb = [0.05, 0.01, 0.04]
    dt, _ = oracle.plan_steps(n, h, Kb, oracle.advection_bound(vx, vy), 0.5, 1e-6)
    w = oracle.local_solve_batch([n], [h], vx.ravel(), vy.ravel(), f1.ravel(), f2.ravel(), np.array([Kb]),
                                 [dt], [300])
    w1, w2 = w[0].reshape(n, n), w[1].reshape(n, n)
    assert np.abs(w1).max() > 1e-3
    Kfull = oracle.estimate(f1, f2, w1, w2, Kb)
    Kwin = oracle.estimate_window(f1, f2, w1, w2, Kb, 16)
    np.testing.assert_allclose(Kwin, Kfull, rtol=1e-12, atol=1e-15)
    # a window that is not a whole number of periods differs
    K12 = oracle.estimate_window(f1, f2, w1, w2, Kb, 12)
    assert np.abs(K12 - Kfull).max() > 1e-6 * np.abs(Kfull - Kb).max()


def test_taper_weights_shape_and_symmetry():
    """The taper is 0 at the seam node, sin^2 on its ramp, 1 inside and
    symmetric under i -> n - i; taper 0 is no taper."""
    w = oracle.taper_weights(16, 4)
    assert w[0] == 0.0 and np.all(w[4:13] == 1.0)
    np.testing.assert_allclose(w[1:4], np.sin(0.5 * np.pi * np.arange(1, 4) / 4) ** 2, rtol=0, atol=1e-16)
    np.testing.assert_array_equal(w[1:], w[1:][::-1])
    assert np.all(oracle.taper_weights(16, 0) == 1.0)


def test_windowed_fields_are_divergence_free_and_untouched_inside():
    """The tapered stream function's face velocities have zero discrete
    divergence (they are differences of one node field), see only their
    inner node across the seam (the tapered field is 0 on the seam nodes),
    and equal the untapered ones on every face whose two nodes both carry
    weight 1."""
    n, taper = 32, 6
    h = 2 * np.pi / n
    rng = np.random.default_rng(2)
    psi = rng.standard_normal((n, n))
    vx, vy, f1, f2 = oracle.staggered(psi, h)
    wx, wy, g1, g2 = oracle.windowed_staggered(psi, h, taper)
    assert np.abs(oracle.divergence(wx, wy, h)).max() <= 1e-12 * np.abs(wx).max()
    w = oracle.taper_weights(n, taper)
    W = np.outer(w, w)
    full = W == 1.0
    # x-face (j, i) pairs nodes (j, i) and (j + 1, i); y-face pairs (j, i) and (j, i + 1)
    fx = full & np.roll(full, -1, axis=0)
    fy = full & np.roll(full, -1, axis=1)
    assert fx.sum() > 0 and fy.sum() > 0
    np.testing.assert_array_equal(wx[fx], vx[fx])
    np.testing.assert_array_equal(wy[fy], vy[fy])
    # the tapered stream function vanishes on the seam nodes (row and column
    # 0), so the seam faces see only their inner node
    np.testing.assert_allclose(wx[n - 1, :], w[n - 1] * w * psi[n - 1, :] / h, rtol=1e-14, atol=0)
    np.testing.assert_allclose(wy[:, n - 1], -w * w[n - 1] * psi[:, n - 1] / h, rtol=1e-14, atol=0)


def test_zero_frame_local_problem_is_the_dirichlet_mode_in_closed_form():
    """Zero-frame local problem with no flow, K = kappa I and the forcing one
    eigenvector of the Dirichlet Laplacian on the inner (n-1)^2 cells,
    g = sin(pi p (i+1)/n) sin(pi q (j+1)/n) (zero on the frame row and column,
    which the periodic wrap also puts beside cell 0).  Each RK4 step of
    w' = lambda w + g with lambda = -(4 kappa / h^2)(sin^2(pi p/2n) +
    sin^2(pi q/2n)) gives w_s = (g / -lambda)(1 - R(lambda dt)^s), R the RK4
    stability polynomial; the frame stays exactly zero.  The periodic problem
    differs."""
    n, p_, q_, kap = 16, 2, 3, 0.07
    h = 2 * np.pi / n
    i = np.arange(n)
    s1 = np.where(i < n - 1, np.sin(np.pi * p_ * (i + 1) / n), 0.0)
    s2 = np.where(i < n - 1, np.sin(np.pi * q_ * (i + 1) / n), 0.0)
    g = np.outer(s2, s1)                     # [y][x]
    lam = -(4 * kap / h ** 2) * (np.sin(np.pi * p_ / (2 * n)) ** 2 + np.sin(np.pi * q_ / (2 * n)) ** 2)
    dt, steps = 2.0 / (8 * kap / h ** 2), 37          # every mode inside the RK4 stability interval
    z = lam * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    zero = np.zeros(n * n)
    w = oracle.local_solve_batch([n], [h], zero, zero, g.ravel(), zero, np.array([[kap, 0.0, kap]]), [dt], [steps],
                                 frame=True)
    want = g / -lam * (1 - R ** steps)
    np.testing.assert_allclose(w[0].reshape(n, n), want, rtol=0, atol=1e-12 * np.abs(want).max())
    assert np.all(w[0].reshape(n, n)[n - 1, :] == 0.0) and np.all(w[0].reshape(n, n)[:, n - 1] == 0.0)
    wp = oracle.local_solve_batch([n], [h], zero, zero, g.ravel(), zero, np.array([[kap, 0.0, kap]]), [dt], [steps])
    assert np.abs(wp[0] - w[0]).max() > 1e-3 * np.abs(want).max()
