"""Parity of the surrogate kernels (features, BF16 matrix-core network, training
step, gate, fallback) with the FP64 oracle.

Tolerances: features 1e-4 absolute (logs of FP32 energies, relative error
~1e-6).  Network outputs: the GPU evaluates GELU in FP32 and rounds hidden
activations to bfloat16, the oracle does the same roundings from FP64 values,
so a rounding decision can flip where the two differ (about one element in
1e5); one flipped activation moves K by at most a few 1e-4 relative, hence
2e-3.  Gradients: FP32 accumulation over the batch versus FP64 plus the same
flips: 1e-2 relative L2 per layer.  Loss: 1e-4 relative.
"""
import sys

import numpy as np
import pytest

import flowgen
import oracle
from oracle import DIAG
from oracle import surrogate as OS
from paper_1510_00451_amd import abi

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _patches(n, lattice=2, seed=3, amp=0.4):
    p = flowgen.config_continuous(seed=seed, radius=max(2, n // 8), p=-1.5, kappa=0.05, n=n,
                                  lattice=lattice, levels=1)
    p.psi_hat *= amp
    p.n_global = [n * lattice]
    return p


@pytest.mark.parametrize("n", [32, 64, 128, 256])
def test_patch_features_parity(torch, n):
    from paper_1510_00451_amd.hierarchy import Hierarchy
    p = _patches(n)
    say("case features n=%d" % n)
    H = Hierarchy(p)
    H.band_filter()
    rng = np.random.default_rng(n)
    Kb = np.stack([rng.uniform(0.01, 0.1, H.nd), rng.uniform(-0.003, 0.003, H.nd),
                   rng.uniform(0.01, 0.1, H.nd)], 1)
    H.K_base.copy_(torch.from_numpy(Kb))
    feats = torch.zeros(H.nd, abi.SURR_IN, dtype=torch.float32, device="cuda")
    H.ctx.shmm_patch_features(0, H.nd, H.vx.data_ptr(), H.vy.data_ptr(), H.K_base.data_ptr(),
                              feats.data_ptr(), H.stream())
    torch.cuda.synchronize()
    got = feats.cpu().numpy()
    lv, pt = oracle.band_split(p.kmax, p.thresh)
    mask = oracle.band_mask(lv, pt, 0, DIAG)
    for d in range(H.nd):
        D = H.table[d]
        psi = oracle.synth_patch(p.psi_hat, p.kmax, mask, int(D["N"]), int(D["I0"]), int(D["J0"]), n)
        vx, vy, _, _ = oracle.staggered(psi, float(D["h"]))
        ref = OS.patch_features(vx, vy, n, int(D["N"]), Kb[d])
        assert np.max(np.abs(got[d] - ref)) <= 1e-4, (d, np.abs(got[d] - ref).max())
    H.close()


def _random_member(seed, rng):
    net = OS.init_net(seed)
    for l in range(4):
        net.b[l] = rng.standard_normal(net.b[l].shape) * 0.05
    net.mu = rng.standard_normal(abi.SURR_IN)
    net.sigma = rng.uniform(0.5, 2.0, abi.SURR_IN)
    return net


def _pack(torch, nets):
    from paper_1510_00451_amd import surrogate as GS
    host = np.concatenate([GS.pack_params(n.W, n.b, n.mu, n.sigma) for n in nets])
    return torch.from_numpy(host).to("cuda")


def _to32(net):
    """The oracle side of a model stored as FP32 parameters on the device."""
    n = net.copy()
    n.W = [w.astype(np.float32).astype(np.float64) for w in n.W]
    n.b = [v.astype(np.float32).astype(np.float64) for v in n.b]
    n.mu = n.mu.astype(np.float32).astype(np.float64)
    n.sigma = n.sigma.astype(np.float32).astype(np.float64)
    return n


def test_inference_and_gate_parity(torch):
    from paper_1510_00451_amd import abi
    rng = np.random.default_rng(7)
    nets = [_to32(_random_member(s, rng)) for s in (11, 12)]
    B = 200                                  # not a multiple of the 64-row tile
    x = rng.standard_normal((B, abi.SURR_IN)).astype(np.float32).astype(np.float64)
    Kb = np.stack([rng.uniform(0.01, 0.1, B), rng.uniform(-0.003, 0.003, B), rng.uniform(0.01, 0.1, B)], 1)
    lo = np.full(abi.SURR_IN, -3.5, np.float32)
    hi = np.full(abi.SURR_IN, 3.5, np.float32)
    say("case inference")
    ctx = abi.Context(0)
    models = _pack(torch, nets)
    s = torch.cuda.current_stream().cuda_stream
    for e in range(2):
        ctx.shmm_surrogate_refresh(models.data_ptr() + e * abi.SURR_MODEL_BYTES, s)
    dx = torch.tensor(x, dtype=torch.float32, device="cuda")
    dKb = torch.tensor(Kb, dtype=torch.float64, device="cuda")
    K = torch.empty(B, 3, dtype=torch.float64, device="cuda")
    flags = torch.empty(B, dtype=torch.uint8, device="cuda")
    spread = torch.empty(B, dtype=torch.float64, device="cuda")
    Km = torch.empty(2, B, 3, dtype=torch.float64, device="cuda")
    dlo = torch.tensor(lo, device="cuda")
    dhi = torch.tensor(hi, device="cuda")
    ref_members = np.stack([OS.head(OS.forward(n, x, bf16_mode=True)[0], Kb) for n in nets])
    tau = float(np.median(OS.ensemble_gate(ref_members, x, lo, hi, 1.0)[2]))   # about half flagged
    mean = ref_members.mean(axis=0)
    fro = lambda a: np.sqrt(a[:, 0] ** 2 + 2 * a[:, 1] ** 2 + a[:, 2] ** 2)
    enh = fro(mean - Kb) / fro(Kb)
    emax = float(np.quantile(enh, 0.8))     # a fifth more flagged by the enhancement limit
    ctx.shmm_surrogate_infer(models.data_ptr(), 2, dx.data_ptr(), dKb.data_ptr(), B, dlo.data_ptr(),
                             dhi.data_ptr(), tau, emax, K.data_ptr(), flags.data_ptr(), spread.data_ptr(),
                             Km.data_ptr(), s)
    torch.cuda.synchronize()
    got_members = Km.cpu().numpy()
    rel = np.abs(got_members - ref_members).max(axis=2) / np.abs(ref_members).max(axis=2)
    assert rel.max() <= 2e-3, rel.max()
    Kref, fref, sref = OS.ensemble_gate(ref_members, x, lo.astype(np.float64), hi.astype(np.float64), tau,
                                        Kb, emax)
    np.testing.assert_allclose(K.cpu().numpy(), Kref, rtol=2e-3)
    g = flags.cpu().numpy().astype(bool)
    near = (np.abs(sref - tau) <= 5e-3 * tau) | (np.abs(enh - emax) <= 5e-3 * emax)
    assert np.array_equal(g[~near], fref[~near])
    assert 0 < g.sum() < B                   # both outcomes occur in this case
    ctx.close()


@pytest.mark.parametrize("B", [96, 2500, 4096])
def test_train_step_parity(torch, B):
    """One training step (forward, loss, backward, gradient norm, Adam) and a
    second one with clipping active, against the oracle fed the same
    BF16-rounded operands.  B = 2500 and 4096 (the training batch) take the
    split-K path of the weight-gradient products (K = B >= 2048 over 16 output
    tiles: 16 slices added in a fixed order)."""
    from paper_1510_00451_amd import abi
    rng = np.random.default_rng(5)
    net = _to32(_random_member(21, rng))
    x = rng.standard_normal((B, abi.SURR_IN)).astype(np.float32).astype(np.float64)
    Kb = np.stack([rng.uniform(0.01, 0.1, B), rng.uniform(-0.003, 0.003, B), rng.uniform(0.01, 0.1, B)], 1)
    Kt = Kb * rng.uniform(1.0, 2.5, (B, 1))
    say("case train step, B =", B)
    ctx = abi.Context(0)
    model = _pack(torch, [net])
    s = torch.cuda.current_stream().cuda_stream
    ctx.shmm_surrogate_refresh(model.data_ptr(), s)
    adam = torch.zeros(2 * abi.SURR_PARAMS_PADDED, dtype=torch.float32, device="cuda")
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    grad = torch.zeros(abi.SURR_PARAMS, dtype=torch.float32, device="cuda")
    dx = torch.tensor(x, dtype=torch.float32, device="cuda")
    dKb = torch.tensor(Kb, device="cuda")
    dKt = torch.tensor(Kt, device="cuda")
    lr = 1e-3
    ctx.shmm_surrogate_train_step(model.data_ptr(), adam.data_ptr(), dx.data_ptr(), dKb.data_ptr(),
                                  dKt.data_ptr(), B, lr, 0.0, 1, loss.data_ptr(), grad.data_ptr(), s)
    torch.cuda.synchronize()
    o, cache = OS.forward(net, x, bf16_mode=True)
    l_ref, go = OS.loss_and_grad_o(o, Kb, Kt)
    gW, gb = OS.backward(net, cache, go, bf16_mode=True)
    assert abs(loss.cpu().numpy()[0] - l_ref) <= 1e-4 * l_ref
    g = grad.cpu().numpy().astype(np.float64)
    off = 0
    for l in range(4):
        for ref in (gW[l].reshape(-1), gb[l]):
            got = g[off:off + ref.size]
            off += ref.size
            assert np.linalg.norm(got - ref) <= 1e-2 * np.linalg.norm(ref), (l, ref.size)
    # Adam step from zero moments: p - lr g / (|g| + eps) elementwise
    from paper_1510_00451_amd import surrogate as GS
    W1, b1, _, _ = GS.unpack_params(model.cpu().numpy())
    flat_new = np.concatenate([np.concatenate([w.reshape(-1), v]) for w, v in zip(W1, b1)])
    flat_old = np.concatenate([np.concatenate([w.reshape(-1), v]) for w, v in zip(net.W, net.b)])
    gref = np.concatenate([np.concatenate([gW[l].reshape(-1), gb[l]]) for l in range(4)])
    big = np.abs(gref) > 1e-3 * np.abs(gref).max()
    expect = flat_old - lr * gref / (np.abs(gref) + 1e-8)
    assert np.max(np.abs(flat_new - expect)[big]) <= 1e-6
    assert abs(loss.cpu().numpy()[1] - np.linalg.norm(gref)) <= 1e-2 * np.linalg.norm(gref)
    # second step with clipping active: the oracle's Adam from the device's
    # moments and parameters, on its own gradient at those parameters
    net2 = net.copy()
    net2.W, net2.b = [w.copy() for w in W1], [v.copy() for v in b1]
    mv = adam.cpu().numpy().astype(np.float64)
    P = abi.SURR_PARAMS_PADDED
    o2, cache2 = OS.forward(net2, x, bf16_mode=True)
    _, go2 = OS.loss_and_grad_o(o2, Kb, Kt)
    gW2, gb2 = OS.backward(net2, cache2, go2, bf16_mode=True)
    g2 = np.concatenate([np.concatenate([gW2[l].reshape(-1), gb2[l]]) for l in range(4)])
    clip = 0.3 * float(np.linalg.norm(g2))
    ctx.shmm_surrogate_train_step(model.data_ptr(), adam.data_ptr(), dx.data_ptr(), dKb.data_ptr(),
                                  dKt.data_ptr(), B, lr, clip, 2, loss.data_ptr(), 0, s)
    torch.cuda.synchronize()
    ad = OS.Adam(lr=lr)
    ad.t = 1
    ad.m = [mv[:abi.SURR_PARAMS].copy()]
    ad.v = [mv[P:P + abi.SURR_PARAMS].copy()]
    p2 = [flat_new.copy()]
    ad.step(p2, [g2], clip=clip)
    W3, b3, _, _ = GS.unpack_params(model.cpu().numpy())
    flat3 = np.concatenate([np.concatenate([w.reshape(-1), v]) for w, v in zip(W3, b3)])
    moved = np.abs(p2[0] - flat_new) > 0.3 * lr
    assert moved.sum() > 1000
    assert np.max(np.abs(flat3 - p2[0])[moved]) <= 0.05 * lr
    assert abs(loss.cpu().numpy()[1] - np.linalg.norm(g2)) <= 1e-2 * np.linalg.norm(g2)
    ctx.close()


def test_fallback_equals_plain_solve(torch):
    from paper_1510_00451_amd.hierarchy import Hierarchy
    p = _patches(32, lattice=4)
    say("case fallback")
    H = Hierarchy(p, keep_psi=False)
    H.band_filter()
    Kb = np.tile([0.05, 0.0, 0.05], (H.nd, 1))
    H.K_base.copy_(torch.from_numpy(Kb))
    H.ctx.shmm_plan_steps(0, H.nd, Kb)
    s = H.stream()
    H.w.zero_()
    H.ctx.shmm_local_solve_batch(0, H.nd, H.vx.data_ptr(), H.vy.data_ptr(), H.f1.data_ptr(),
                                 H.f2.data_ptr(), H.K_base.data_ptr(), H.w.data_ptr(), 0, 2 ** 31 - 1, 0, s)
    H.ctx.shmm_effective_diffusivity(0, H.nd, H.f1.data_ptr(), H.f2.data_ptr(), H.w.data_ptr(),
                                     H.K_base.data_ptr(), H.K_solve.data_ptr(), 0, 0, 0, s)
    torch.cuda.synchronize()
    plain = H.K_solve.cpu().numpy().copy()
    flags = torch.zeros(H.nd, dtype=torch.uint8, device="cuda")
    flags[::3] = 1
    Kout = torch.full((H.nd, 3), -1.0, dtype=torch.float64, device="cuda")
    H.status.zero_()
    H.w.fill_(7.0)                           # the fallback must clear the correctors itself
    H.ctx.shmm_fallback_solve(0, H.nd, flags.data_ptr(), H.vx.data_ptr(), H.vy.data_ptr(), H.f1.data_ptr(),
                              H.f2.data_ptr(), H.K_base.data_ptr(), H.w.data_ptr(), Kout.data_ptr(), 0, 0.0,
                              H.status.data_ptr(), s)
    torch.cuda.synchronize()
    got = Kout.cpu().numpy()
    f = flags.cpu().numpy().astype(bool)
    assert np.array_equal(got[f], plain[f])
    assert np.all(got[~f] == -1.0)
    st = H.status.cpu().numpy()
    assert np.all((st[f] & 8) == 8) and np.all(st[~f] == 0)
    # the same fallback with the quasi-stationary stop: K within the parity
    # bar of the planned solve, fewer steps for the flagged patches only
    planned = H.ctx.shmm_ctx_table()[0]["nsteps"].copy()
    Kad = torch.full((H.nd, 3), -1.0, dtype=torch.float64, device="cuda")
    H.w.fill_(7.0)
    H.ctx.shmm_fallback_solve(0, H.nd, flags.data_ptr(), H.vx.data_ptr(), H.vy.data_ptr(), H.f1.data_ptr(),
                              H.f2.data_ptr(), H.K_base.data_ptr(), H.w.data_ptr(), Kad.data_ptr(), 32, 0.0, 0, s)
    torch.cuda.synchronize()
    ga = Kad.cpu().numpy()
    assert np.all(ga[~f] == -1.0)
    assert np.max(np.abs(ga[f] - plain[f])) <= 1e-5 * np.max(np.abs(plain[f]))
    taken = H.ctx.shmm_ctx_table()[0]["nsteps"]
    assert np.array_equal(taken[~f], planned[~f]) and taken[f].sum() < planned[f].sum()
    H.close()


def test_training_reduces_loss(torch):
    """A few hundred steps on a smooth synthetic target fall well below the
    initial loss (the kernels learn, not only match one step)."""
    from paper_1510_00451_amd import abi
    from paper_1510_00451_amd import surrogate as GS
    rng = np.random.default_rng(9)
    S = 2048
    x = rng.standard_normal((S, abi.SURR_IN))
    Kb = np.tile([0.02, 0.0, 0.02], (S, 1))
    enh = 1.5 + 0.5 * np.tanh(x[:, 0]) + 0.2 * x[:, 1] ** 2     # K >= K_b, as the head requires
    Kt = Kb * enh[:, None]
    say("case training")
    ctx = abi.Context(0)
    ens = GS.Ensemble(ctx, 1, np.zeros(abi.SURR_IN), np.ones(abi.SURR_IN), seed0=3)
    data = GS.Dataset(torch.tensor(x, dtype=torch.float32, device="cuda"), torch.tensor(Kb, device="cuda"),
                      torch.tensor(Kt, device="cuda"))
    hist = GS.train(ens, data, steps=300, batch=256, lr0=3e-3, log=lambda *a: None, clip=1.0)
    K, flags, spread = GS.infer(ens, data.x, data.Kb, torch.full((abi.SURR_IN,), -1e9, device="cuda"),
                                torch.full((abi.SURR_IN,), 1e9, device="cuda"), 1.0)
    torch.cuda.synchronize()
    err = np.abs(K.cpu().numpy()[:, 0] - Kt[:, 0]) / Kt[:, 0]
    assert np.median(err) < 0.02, np.median(err)
    ctx.close()


def test_surrogate_form_gates_and_falls_back(torch):
    """The surrogate-with-fallback form of a phase: with every patch flagged it
    returns the plain result bit for bit; with none flagged it returns the
    ensemble estimate unchanged and runs no solve."""
    from paper_1510_00451_amd import abi
    from paper_1510_00451_amd import surrogate as GS
    p = _patches(32, lattice=4)
    say("case surrogate form")
    ph = GS.IsotropicPhase([p])
    ph.prepare()
    plain = ph.plain().cpu().numpy().copy()
    ctx = abi.Context(0)
    ens = GS.Ensemble(ctx, 2, np.zeros(abi.SURR_IN), np.ones(abi.SURR_IN), seed0=4)
    wide_lo = torch.full((abi.SURR_IN,), -1e30, dtype=torch.float32, device="cuda")
    wide_hi = torch.full((abi.SURR_IN,), 1e30, dtype=torch.float32, device="cuda")
    K_all = ph.surrogate(ens, wide_lo, wide_hi, -1.0).cpu().numpy().copy()
    assert ph.flags.cpu().numpy().all()
    assert np.array_equal(K_all, plain)
    ph.H.status.zero_()
    K_none = ph.surrogate(ens, wide_lo, wide_hi, 1e300, 1e300).cpu().numpy().copy()
    assert not ph.flags.cpu().numpy().any()
    K_ref, _, _ = GS.infer(ens, ph.x, ph.K_base(), wide_lo, wide_hi, 1e300, 1e300)
    assert np.array_equal(K_none, K_ref.cpu().numpy())
    assert not (ph.H.status.cpu().numpy() & 8).any()
    ctx.close()
    ph.close()


def test_ensemble_prune_drops_a_member_that_failed(torch):
    """Pruning keeps members within a factor of the best held-out loss: a member
    with untrained weights is dropped, and the kept blocks are the originals."""
    from paper_1510_00451_amd import abi
    from paper_1510_00451_amd import surrogate as GS
    rng = np.random.default_rng(12)
    S = 1024
    x = rng.standard_normal((S, abi.SURR_IN))
    Kb = np.tile([0.02, 0.0, 0.02], (S, 1))
    Kt = Kb * (1.5 + 0.5 * np.tanh(x[:, :1]))
    say("case prune")
    ctx = abi.Context(0)
    ens = GS.Ensemble(ctx, 3, np.zeros(abi.SURR_IN), np.ones(abi.SURR_IN), seed0=5)
    data = GS.Dataset(torch.tensor(x, dtype=torch.float32, device="cuda"), torch.tensor(Kb, device="cuda"),
                      torch.tensor(Kt, device="cuda"))
    GS.train(ens, data, steps=200, batch=256, lr0=3e-3)
    words = abi.SURR_MODEL_BYTES // 4
    fresh = GS.Ensemble(ctx, 1, np.zeros(abi.SURR_IN), np.ones(abi.SURR_IN), seed0=99)
    ens.buf[words:2 * words] = fresh.buf        # member 1 reverts to untrained weights
    keep0, keep2 = ens.buf[:words].clone(), ens.buf[2 * words:].clone()
    losses = ens.prune(data)
    assert losses[1] > 3 * min(losses[0], losses[2])
    assert ens.E == 2
    assert torch.equal(ens.buf[:words], keep0) and torch.equal(ens.buf[words:], keep2)
    ctx.close()


def test_feature_stats_and_rescale(torch):
    """Column statistics of a feature matrix (the standardisation and the gate
    range) against numpy in FP64, bitwise reproducible; rescaled labels: K
    and K_b times c, the band features unchanged, feature 32 moved by ln c."""
    from paper_1510_00451_amd import abi
    rng = np.random.default_rng(9)
    B = 5000
    x = (rng.standard_normal((B, abi.SURR_IN)) * rng.uniform(0.1, 3.0, abi.SURR_IN) + rng.uniform(-5, 5, abi.SURR_IN)).astype(np.float32)
    say("case feature statistics and rescaling")
    ctx = abi.Context(0)
    s = torch.cuda.current_stream().cuda_stream
    dx = torch.tensor(x, device="cuda")
    st = torch.empty(4, abi.SURR_IN, dtype=torch.float64, device="cuda")
    ctx.shmm_feature_stats(dx.data_ptr(), B, st.data_ptr(), s)
    torch.cuda.synchronize()
    got = st.cpu().numpy()
    xd = x.astype(np.float64)
    np.testing.assert_allclose(got[0], xd.mean(0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got[1], xd.std(0, ddof=1), rtol=1e-11)
    assert np.array_equal(got[2], xd.min(0)) and np.array_equal(got[3], xd.max(0))
    ctx.shmm_feature_stats(dx.data_ptr(), B, st.data_ptr(), s)
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy(), got)
    Kb = np.stack([rng.uniform(0.01, 0.1, B), rng.uniform(-0.003, 0.003, B), rng.uniform(0.01, 0.1, B)], 1)
    Kt = Kb * rng.uniform(1.0, 2.5, (B, 1))
    lc = rng.uniform(-1.5, 1.5, B)
    dKb, dKt, dlc = (torch.tensor(a, device="cuda") for a in (Kb, Kt, lc))
    xo = torch.empty_like(dx)
    Kbo, Kto = torch.empty_like(dKb), torch.empty_like(dKt)
    ctx.shmm_surrogate_rescale(dx.data_ptr(), dKb.data_ptr(), dKt.data_ptr(), dlc.data_ptr(), B, xo.data_ptr(),
                               Kbo.data_ptr(), Kto.data_ptr(), s)
    torch.cuda.synchronize()
    c = 10.0 ** lc
    np.testing.assert_allclose(Kbo.cpu().numpy(), Kb * c[:, None], rtol=1e-14)
    np.testing.assert_allclose(Kto.cpu().numpy(), Kt * c[:, None], rtol=1e-14)
    xg = xo.cpu().numpy()
    assert np.array_equal(xg[:, :32], x[:, :32])
    np.testing.assert_allclose(xg[:, 32], x[:, 32].astype(np.float64) + np.log(c), rtol=0, atol=2e-6)
    ctx.close()


def test_chain_gate_rule(torch):
    """shmm_surrogate_chain_gate on hand-built inputs: a domain with a parent
    is flagged when its predicted change of the base plus its spread times
    |K_hat| exceeds tol times the smallest lambda_min(K_in) over its
    ancestors; a flag already set stays set, and domains without a parent are
    left alone."""
    from paper_1510_00451_amd.hierarchy import Hierarchy
    H = Hierarchy(flowgen.config_four_level_cellular(n=16, lattice=2), keep_psi=False)
    say("case chain gate rule")
    rng = np.random.default_rng(3)
    table = H.table
    nd, tol = H.nd, 1e-2
    K_in = np.empty((nd, 3))
    lam_in = rng.uniform(0.5, 2.0, nd)
    K_in[:, 0] = lam_in + rng.uniform(0.0, 1.0, nd)
    K_in[:, 2] = lam_in + rng.uniform(0.0, 1.0, nd)
    K_in[:, 1] = rng.uniform(-0.3, 0.3, nd)
    d_K_in = torch.from_numpy(K_in).cuda()
    m_, q_ = 0.5 * (K_in[:, 0] + K_in[:, 2]), 0.5 * (K_in[:, 0] - K_in[:, 2])
    lam_dom = m_ - np.sqrt(q_ * q_ + K_in[:, 1] ** 2)
    lam_anc = np.full(nd, np.inf)                 # smallest over the parent and its ancestors
    for i in range(nd):
        a = int(table["parent"][i])
        while a >= 0:
            lam_anc[i] = min(lam_anc[i], lam_dom[a])
            a = int(table["parent"][a])
    checked, raised = 0, 0
    for p_ in range(len(H.phase) - 1):
        first, count = int(H.phase[p_]), int(H.phase[p_ + 1] - H.phase[p_])
        Kb = np.stack([rng.uniform(1, 2, count), rng.uniform(-0.1, 0.1, count), rng.uniform(1, 2, count)], 1)
        dK = rng.normal(size=(count, 3)) * 10.0 ** rng.uniform(-4, -1, (count, 1))
        Kh = Kb + dK
        spread = 10.0 ** rng.uniform(-5, -2, count)
        par = table["parent"][first:first + count]
        lam = lam_anc[first:first + count]
        fro = lambda A: np.sqrt(A[:, 0] ** 2 + 2 * A[:, 1] ** 2 + A[:, 2] ** 2)
        ratio = (fro(Kh - Kb) + spread * fro(Kh)) / (tol * lam)
        keep = np.abs(ratio - 1.0) > 1e-6          # away from the threshold: FMA contraction may differ
        pre = (rng.uniform(size=count) < 0.2).astype(np.uint8)
        want = pre.copy()
        want[(par >= 0) & (ratio > 1.0)] = 1
        flags = torch.from_numpy(pre.copy()).cuda()
        d_Kh, d_Kb, d_sp = (torch.from_numpy(a).cuda() for a in (Kh, Kb, spread))   # held until the call ends
        H.ctx.shmm_surrogate_chain_gate(first, count, d_Kh.data_ptr(), d_Kb.data_ptr(), d_sp.data_ptr(),
                                        d_K_in.data_ptr(), tol, flags.data_ptr(), H.stream())
        torch.cuda.synchronize()
        got = flags.cpu().numpy()
        assert np.array_equal(got[keep], want[keep]), p_
        if (par < 0).all():
            assert np.array_equal(got, pre)
        free = (par >= 0) & keep & (pre == 0)
        checked += int(free.sum())
        raised += int((free & (ratio > 1.0)).sum())
    assert 0 < raised < checked      # both outcomes were exercised
    with pytest.raises(abi.ShmmError):
        H.ctx.shmm_surrogate_chain_gate(0, 1, d_K_in.data_ptr(), d_K_in.data_ptr(), d_K_in.data_ptr(),
                                        d_K_in.data_ptr(), 0.0, d_K_in.data_ptr(), H.stream())
    H.close()


def test_surrogate_through_every_level(torch):
    """The surrogate in place of every phase's local solves (Hierarchy.use_surrogate):
    with a gate that flags every patch the pass is the plain pass bit for bit
    (the fallback runs the same solves and moments); with a gate that flags
    none, every level result follows the network on the chain's own bases."""
    from paper_1510_00451_amd import surrogate as GS
    from paper_1510_00451_amd.hierarchy import Hierarchy
    p = flowgen.config_four_level_cellular(n=16, lattice=2)
    say("case surrogate through every level")
    H = Hierarchy(p, keep_psi=False)
    H.run()
    plain = H.result()
    ens = GS.Ensemble(H.ctx, 2, np.zeros(abi.SURR_IN), np.ones(abi.SURR_IN), seed0=7)
    big = torch.full((abi.SURR_IN,), 1e30, dtype=torch.float32, device="cuda")
    H.use_surrogate(ens.buf.data_ptr(), ens.E, big, big, 1.0, float("inf"))
    H.run()
    r = H.result()
    assert np.array_equal(r.R, plain.R)
    assert all(f.all() for f in H.surrogate_flags.values()) and len(H.surrogate_flags) == 4
    H.use_surrogate(ens.buf.data_ptr(), ens.E, -big, big, float("inf"), float("inf"))
    H.run()
    r = H.result()
    assert not any(f.any() for f in H.surrogate_flags.values())
    assert np.isfinite(r.R).all() and not np.array_equal(r.R, plain.R)
    # the chain-aware gate with a vanishing tolerance sends every patch that
    # has a parent to the plain solve and leaves the coarsest level alone
    H.use_surrogate(ens.buf.data_ptr(), ens.E, -big, big, float("inf"), float("inf"), chain_tol=1e-300)
    H.run()
    lev = H.table["level"]
    for p_, f in H.surrogate_flags.items():
        assert f.all() == (lev[int(H.phase[p_])] > 0) and f.any() == (lev[int(H.phase[p_])] > 0), p_
    # ... and with a huge one it flags nothing
    H.use_surrogate(ens.buf.data_ptr(), ens.E, -big, big, float("inf"), float("inf"), chain_tol=1e300)
    H.run()
    r = H.result()
    assert not any(f.any() for f in H.surrogate_flags.values())
    # the finest phase's estimates are the ensemble's on its features and bases
    first, count = int(H.phase[0]), int(H.phase[1] - H.phase[0])
    x = torch.zeros(count, abi.SURR_IN, dtype=torch.float32, device="cuda")
    H.ctx.shmm_patch_features(first, count, H.vx.data_ptr(), H.vy.data_ptr(), H.K_base.data_ptr(), x.data_ptr(),
                              H.stream())
    K, flags, _ = GS.infer(ens, x, H.K_base[first:first + count], -big, big, float("inf"), float("inf"))
    torch.cuda.synchronize()
    assert np.array_equal(K.cpu().numpy(), r.K_solve[first:first + count])
    H.close()
