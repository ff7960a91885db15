"""Pins of the surrogate oracle (features, network, loss, Adam, gate) against
closed forms and independent library implementations (torch float64 on the
CPU, scipy)."""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S


def test_features_single_mode_closed_form():
    n, N = 32, 128
    a, b, A = 3, 2, 0.7
    i = np.arange(n)
    I, J = np.meshgrid(i, i, indexing="xy")
    vx = A * np.cos(2 * np.pi * (a * I + b * J) / n)
    vy = np.zeros_like(vx)
    Kb = [0.02, 0.005, 0.03]
    f = S.patch_features(vx, vy, n, N, Kb)
    q = math.hypot(a, b)
    edges = S.bin_edges()
    bq = int(np.searchsorted(edges, q, side="right") - 1)
    Etot = A * A / 2 * (n / N) ** 2
    expect = np.full(33, math.log(1e-8 * Etot + 1e-30))
    expect[bq] = math.log(Etot + 1e-8 * Etot + 1e-30)
    expect[32] = 0.5 * math.log(0.02 * 0.03 - 0.005 ** 2)
    np.testing.assert_allclose(f, expect, rtol=1e-12, atol=1e-12)


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
    net.mu = rng.standard_normal(33)
    net.sigma = rng.uniform(0.5, 2.0, 33)
    B = 7
    x = rng.standard_normal((B, 33))
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
    Kh = torch.stack([s * l11 * l11, s * l11 * l21, s * (l21 * l21 + l22 * l22)], 1)
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


def test_head_closed_form_and_spd():
    Kb = np.array([[0.02, 0.0, 0.08]])
    np.testing.assert_allclose(S.head(np.zeros((1, 3)), Kb), [[0.04, 0.0, 0.04]], rtol=1e-15)
    o = np.random.default_rng(2).standard_normal((100, 3))
    K = S.head(o, np.tile([0.05, 0.01, 0.03], (100, 1)))
    assert np.all(K[:, 0] > 0) and np.all(K[:, 0] * K[:, 2] - K[:, 1] ** 2 > 0)


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
