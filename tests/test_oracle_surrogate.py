"""Pins of the surrogate oracle (features, network, loss, Adam, gate) against
closed forms and independent library implementations (torch float64 on the
CPU, scipy)."""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S


def _mode(n, a, b, A, B, quadrature=False):
    i = np.arange(n)
    I, J = np.meshgrid(i, i, indexing="xy")
    ph = 2 * np.pi * (a * I + b * J) / n
    vx = A * np.cos(ph)
    vy = B * (np.sin(ph) if quadrature else np.cos(ph))
    return vx, vy


def test_octave_bins_at_their_edges():
    """Bin b holds 2^b <= |k| < 2^(b+1): hand values on the edges (|k| = 2^b
    exactly, the largest |k| of a 256^2 patch, the first |k| past bin 7), and
    every (k1, k2) of [-300, 300]^2 against a search over b in integers."""
    hand = {(0, 0): -1, (1, 0): 0, (0, -1): 0, (1, 1): 0, (2, 0): 1, (-1, 2): 1, (3, 3): 2,
            (4, 0): 2, (0, 8): 3, (127, 0): 6, (128, 0): 7, (-128, -128): 7, (181, 181): 7,
            (255, 0): 7, (256, 0): -1, (182, 181): -1}
    for (k1, k2), b in hand.items():
        assert S.bin_of(k1, k2) == b, (k1, k2)
    for k1 in range(-300, 301):
        for k2 in range(-300, 301):
            q2 = k1 * k1 + k2 * k2
            want = -1
            for b in range(S.N_RADIAL):
                if 4 ** b <= q2 < 4 ** (b + 1):
                    want = b
            assert S.bin_of(k1, k2) == want, (k1, k2)


def test_features_single_mode_closed_form():
    """One Fourier mode in phase in both components: every channel by hand."""
    n, N = 32, 128
    a, b, A, B = 3, 2, 0.7, -0.3
    vx, vy = _mode(n, a, b, A, B)
    Kb = [0.02, 0.005, 0.03]
    f = S.patch_features(vx, vy, n, N, Kb)
    q2 = a * a + b * b
    bq = int(math.floor(math.log2(math.sqrt(q2))))          # |k| = 3.6 -> octave bin 1
    assert bq == 1
    s = (n / N) ** 2 / q2                                   # (L / 2 pi)^2 / |k|^2
    # cos splits into +-k with amplitude 1/2 each: sum over the pair of |c/2|^2 = c^2/2
    E = [A * A / 2 * s, B * B / 2 * s, (A + B) ** 2 / 4 * s, (A - B) ** 2 / 4 * s]
    Etot = E[0] + E[1]
    fl = 1e-8 * Etot + 1e-30
    det = 0.02 * 0.03 - 0.005 ** 2
    expect = np.full(S.N_IN, math.log(fl / det))
    for c in range(4):
        expect[8 * c + bq] = math.log((E[c] + fl) / det)
    expect[32] = 0.5 * math.log(det)
    expect[33:35] = S.log_base_anisotropy(Kb)
    np.testing.assert_allclose(f, expect, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,N,a,V", [(32, 128, 3, 0.4), (64, 64, 5, 1.3), (128, 2048, 20, 0.05)])
def test_features_carry_the_taylor_dispersion_of_a_shear_flow(n, N, a, V):
    """v = (0, V sin(k x)) on a patch (k = a N / n in the units of the global
    grid): the local problem of a shear flow is solved by K_yy = kappa +
    V^2 / (2 kappa k^2) at every Peclet number (Taylor dispersion), and the
    channel-1 energies summed over the bins, over kappa, give exactly that
    enhancement; channel 0 is empty and the cross channels are equal."""
    kappa = 0.013
    i = np.arange(n)
    X = np.tile(i, (n, 1))
    vx = np.zeros((n, n))
    vy = V * np.sin(2 * np.pi * a * X / n)
    E = S.channel_energies(vx, vy, n, N)
    k = a * N / n
    assert abs(E[1].sum() / kappa - V * V / (2 * kappa * k * k)) <= 1e-12 * V * V / (2 * kappa * k * k)
    assert E[0].sum() <= 1e-30
    np.testing.assert_allclose(E[2], E[3], rtol=1e-12, atol=1e-30)


def test_features_scale_invariance():
    """Scaling velocity by c and the base by c shifts feature 32 by log c and
    leaves the 32 band features unchanged (squared Peclet numbers)."""
    rng = np.random.default_rng(8)
    n, N, c = 32, 64, 7.5
    vx, vy = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    Kb = np.array([0.03, -0.004, 0.02])
    f = S.patch_features(vx, vy, n, N, Kb)
    g = S.patch_features(c * vx, c * vy, n, N, c * Kb)
    np.testing.assert_allclose(g[:32], f[:32], rtol=0, atol=1e-12)
    assert abs(g[32] - f[32] - math.log(c)) <= 1e-12
    np.testing.assert_allclose(g[33:], f[33:], rtol=0, atol=1e-12)


def _rot(theta, a, b):
    c, s = math.cos(theta), math.sin(theta)
    return [a * c * c + b * s * s, (a - b) * c * s, a * s * s + b * c * c]


@pytest.mark.parametrize("theta", [0.0, 0.3, -1.2, math.pi / 2, 2.5])
def test_base_anisotropy_features_closed_form(theta):
    """Features 33-34 of a base with eigenvalues a > b along the angle theta:
    log K_b = R diag(ln a, ln b) R^T, whose traceless part is
    (1/2) ln(a / b) [[cos 2 theta, sin 2 theta], [sin 2 theta, -cos 2 theta]]."""
    a, b = 0.07, 0.013
    t11, t12 = S.log_base_anisotropy(_rot(theta, a, b))
    h = 0.5 * math.log(a / b)
    assert abs(t11 - h * math.cos(2 * theta)) <= 1e-14
    assert abs(t12 - h * math.sin(2 * theta)) <= 1e-14


def test_base_anisotropy_features_isotropic_and_scale_free():
    """An isotropic base gives zero; scaling the base leaves the pair unchanged;
    exchanging the axes (K11 <-> K22) flips the sign of the first entry."""
    assert S.log_base_anisotropy([0.02, 0.0, 0.02]) == pytest.approx((0.0, 0.0), abs=1e-15)
    K = [0.031, -0.004, 0.012]
    f = np.array(S.log_base_anisotropy(K))
    np.testing.assert_allclose(S.log_base_anisotropy([9.0 * v for v in K]), f, rtol=0, atol=1e-14)
    g = np.array(S.log_base_anisotropy([K[2], K[1], K[0]]))
    np.testing.assert_allclose(g, [-f[0], f[1]], rtol=0, atol=1e-14)


def test_features_quadrature_has_no_cross_spectrum():
    """vx = A cos, vy = B sin: the +-45 degree channels carry equal energy."""
    n, N = 32, 32
    vx, vy = _mode(n, 1, 4, 0.5, 0.8, quadrature=True)
    E = S.channel_energies(vx, vy, n, N)
    b = int(math.floor(math.log2(math.sqrt(17))))          # |k| = 4.1 -> octave bin 2
    assert b == 2
    np.testing.assert_allclose(E[2, b], E[3, b], rtol=1e-12)
    np.testing.assert_allclose(E[2, b], (E[0, b] + E[1, b]) / 2, rtol=1e-12)


def test_features_symmetries():
    """Swapping the components swaps channels 0 and 1; negating vy swaps 2 and 3;
    channels 2 + 3 equal 0 + 1 in every bin (a random field, several bins)."""
    rng = np.random.default_rng(5)
    n, N = 32, 64
    vx, vy = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    E = S.channel_energies(vx, vy, n, N)
    Es = S.channel_energies(vy, vx, n, N)
    En = S.channel_energies(vx, -vy, n, N)
    np.testing.assert_allclose(Es[[1, 0, 2, 3]], E, rtol=1e-12)
    np.testing.assert_allclose(En[[0, 1, 3, 2]], E, rtol=1e-12)
    np.testing.assert_allclose(E[2] + E[3], E[0] + E[1], rtol=1e-12)
    # bin populations: a flat spectrum puts sum of 1 / q^2 over the modes with
    # 2^b <= q < 2^(b+1) into bin b (N = n: unit spacing of the wavenumbers);
    # every mode but the mean is counted once
    ones = np.zeros((n, n))
    ones[0, 0] = n * n                    # delta at the origin: flat spectrum |X|^2 = 1
    Ef = S.channel_energies(ones, np.zeros((n, n)), n, n)
    k = np.arange(-n // 2, n // 2)
    K1, K2 = np.meshgrid(k, k)
    q2 = (K1 ** 2 + K2 ** 2).astype(float)
    w = np.where(q2 > 0, 1.0 / np.maximum(q2, 1.0), 0.0)
    for b in range(8):
        sel = (q2 >= 4 ** b) & (q2 < 4 ** (b + 1))
        np.testing.assert_allclose(Ef[0, b], np.sum(w[sel]), rtol=1e-12)
    np.testing.assert_allclose(Ef[0].sum(), np.sum(w), rtol=1e-12)


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10
    x[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 65504.0]      # ties
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)


def _torch_net(net):
    W = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in net.W]
    b = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in net.b]
    return W, b


def test_forward_backward_match_torch_autograd():
    rng = np.random.default_rng(1)
    net = S.init_net(3)
    net.mu = rng.standard_normal(S.N_IN)
    net.sigma = rng.uniform(0.5, 2.0, S.N_IN)
    B = 7
    x = rng.standard_normal((B, S.N_IN))
    Kb = np.stack([rng.uniform(0.01, 0.1, B), rng.uniform(-0.002, 0.002, B), rng.uniform(0.01, 0.1, B)], 1)
    Kt = Kb * rng.uniform(1.0, 3.0, (B, 1))
    o, cache = S.forward(net, x)
    loss, go = S.loss_and_grad_o(o, Kb, Kt)
    gW, gb = S.backward(net, cache, go)
    W, b = _torch_net(net)
    h = (torch.tensor(x) - torch.tensor(net.mu)) / torch.tensor(net.sigma)
    for l in range(4):
        h = h @ W[l].T + b[l]
        if l < 3:
            h = torch.nn.functional.gelu(h, approximate="none")
    Kbt = torch.tensor(Kb)
    s = torch.sqrt(Kbt[:, 0] * Kbt[:, 2] - Kbt[:, 1] ** 2)
    l11, l21, l22 = torch.exp(h[:, 0]), h[:, 1], torch.exp(h[:, 2])
    Kh = Kbt + torch.stack([s * l11 * l11, s * l11 * l21, s * (l21 * l21 + l22 * l22)], 1)
    Ktt = torch.tensor(Kt)
    d = Kh - Ktt
    L = torch.mean((d[:, 0] ** 2 + 2 * d[:, 1] ** 2 + d[:, 2] ** 2)
                   / (Ktt[:, 0] ** 2 + 2 * Ktt[:, 1] ** 2 + Ktt[:, 2] ** 2))
    L.backward()
    np.testing.assert_allclose(o, h.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert abs(loss - L.item()) <= 1e-12 * abs(L.item())
    for l in range(4):
        np.testing.assert_allclose(gW[l], W[l].grad.numpy(), rtol=1e-9, atol=1e-14)
        np.testing.assert_allclose(gb[l], b[l].grad.numpy(), rtol=1e-9, atol=1e-14)


def test_head_closed_form_and_enhancement_psd():
    Kb = np.array([[0.02, 0.0, 0.08]])
    np.testing.assert_allclose(S.head(np.zeros((1, 3)), Kb), [[0.06, 0.0, 0.12]], rtol=1e-15)
    o = np.random.default_rng(2).standard_normal((100, 3))
    Kb = np.tile([0.05, 0.01, 0.03], (100, 1))
    D = S.head(o, Kb) - Kb
    assert np.all(D[:, 0] > 0) and np.all(D[:, 0] * D[:, 2] - D[:, 1] ** 2 > -1e-15)


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    p = [rng.standard_normal((5, 3)), rng.standard_normal(4)]
    pt = [torch.tensor(a.copy(), requires_grad=True) for a in p]
    opt = torch.optim.Adam(pt, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    ad = S.Adam(lr=1e-2)
    for it in range(5):
        g = [rng.standard_normal(a.shape) for a in p]
        ad.step(p, g)
        for t, gg in zip(pt, g):
            t.grad = torch.tensor(gg)
        opt.step()
    for a, t in zip(p, pt):
        np.testing.assert_allclose(a, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_gate_flags():
    Km = np.array([[[1.0, 0.0, 1.0], [1.0, 0.0, 1.0]], [[1.0, 0.0, 1.0], [1.02, 0.0, 1.0]]])
    f = np.array([[0.5, 0.5], [0.5, 2.0]])
    K, flag, spread = S.ensemble_gate(Km, f, np.zeros(2), np.ones(2), 0.005)
    assert list(flag) == [False, True]
    f2 = np.array([[0.5, 0.5], [0.5, 0.5]])
    K, flag, spread = S.ensemble_gate(Km, f2, np.zeros(2), np.ones(2), 0.005)
    assert list(flag) == [False, True] and spread[1] > 0.005
    K, flag, spread = S.ensemble_gate(Km, f2, np.zeros(2), np.ones(2), 0.05)
    assert list(flag) == [False, False]
    # members that agree: only the training range decides, on either side of it
    same = np.array([[[1.0, 0.0, 1.0]] * 3] * 2)
    f3 = np.array([[0.5, 1.5], [-0.5, 0.5], [0.0, 1.0]])
    _, flag, spread = S.ensemble_gate(same, f3, np.zeros(2), np.ones(2), 0.005)
    assert list(flag) == [True, True, False] and not spread.any()


def test_gate_spread_is_the_largest_member_deviation():
    """Three members with K11 = 1, 1, 1.03 (K12 = 0, K22 = 1): the mean is
    1.01, the deviations 0.01, 0.01, 0.02, so the spread is 0.02 over
    |K_mean| = sqrt(1.01^2 + 1) (their mean, 0.0133, would pass tau = 0.012)."""
    Km = np.array([[[1.0, 0.0, 1.0]], [[1.0, 0.0, 1.0]], [[1.03, 0.0, 1.0]]])
    f = np.full((1, 2), 0.5)
    K, flag, spread = S.ensemble_gate(Km, f, np.zeros(2), np.ones(2), 0.012)
    assert abs(spread[0] - 0.02 / math.sqrt(1.01 ** 2 + 1.0)) <= 1e-12
    np.testing.assert_allclose(K[0], [1.01, 0.0, 1.0], rtol=0, atol=1e-15)
    assert list(flag) == [True]
    _, flag, _ = S.ensemble_gate(Km, f, np.zeros(2), np.ones(2), 0.015)
    assert list(flag) == [False]


def test_gate_flags_large_enhancement():
    """The enhancement limit: |K - K_b| / |K_b| above emax falls back."""
    Kb = np.array([[1.0, 0.0, 1.0], [1.0, 0.0, 1.0]])
    Km = np.array([[[1.05, 0.0, 1.05], [1.5, 0.0, 1.5]]] * 2)      # enhancements 0.05 and 0.5
    f = np.full((2, 2), 0.5)
    _, flag, _ = S.ensemble_gate(Km, f, np.zeros(2), np.ones(2), 0.01, Kb, 0.1)
    assert list(flag) == [False, True]
    _, flag, _ = S.ensemble_gate(Km, f, np.zeros(2), np.ones(2), 0.01, Kb, 1.0)
    assert list(flag) == [False, False]


def test_adam_clipping_matches_torch():
    """Global-norm clipping before Adam equals torch's clip_grad_norm_ + Adam
    (torch adds 1e-6 to the norm, hence the tolerance)."""
    rng = np.random.default_rng(6)
    p = [rng.standard_normal((5, 3)), rng.standard_normal(4)]
    pt = [torch.tensor(a.copy(), requires_grad=True) for a in p]
    opt = torch.optim.Adam(pt, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    ad = S.Adam(lr=1e-2)
    for it in range(5):
        g = [rng.standard_normal(a.shape) * (10.0 if it % 2 else 0.1) for a in p]
        ad.step(p, g, clip=1.0)
        for t, gg in zip(pt, g):
            t.grad = torch.tensor(gg)
        torch.nn.utils.clip_grad_norm_(pt, 1.0)
        opt.step()
    for a, t in zip(p, pt):
        np.testing.assert_allclose(a, t.detach().numpy(), rtol=1e-6, atol=1e-12)
