"""The seeded synthetic inputs follow their stated recipes: the counter-based
generator is splitmix64 as published, spectra are real-field power laws with
random phases, and the workload generators draw their parameters from the
stated ranges.  Inputs only: none of the method's arithmetic is involved."""
import math

import numpy as np

import flowgen

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def test_splitmix64_reproduces_the_published_sequence():
    """From state 0 the generator's first three outputs are the published
    0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f (the state
    advances by the golden-ratio increment before each output)."""
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [flowgen.splitmix64((i * GAMMA) & MASK) for i in range(3)] == want


def test_uniform01_is_uniform_on_the_unit_interval():
    u = np.array([flowgen.uniform01(9, c) for c in range(40000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) <= 5 * math.sqrt(1 / 12 / u.size)
    hist, _ = np.histogram(u, bins=10, range=(0, 1))
    assert np.all(np.abs(hist - u.size / 10) <= 5 * math.sqrt(u.size / 10))
    assert flowgen.uniform01(9, 5) != flowgen.uniform01(10, 5)      # seeds give distinct streams


def test_power_spectrum_is_a_real_field_power_law():
    """|psi_hat(k)| = amp |k|^p for 1 <= |k| <= radius and 0 elsewhere, with
    psi_hat(-k) = conj psi_hat(k), so the synthesised stream function is real."""
    radius, p, amp = 20, -7.0 / 3.0, 0.8
    ph = flowgen.random_power_spectrum_fast(3, radius, p, amp)
    k = np.arange(-radius, radius + 1)
    q2 = (k[None, :] ** 2 + k[:, None] ** 2).astype(float)
    inside = (q2 >= 1) & (q2 <= radius * radius)
    np.testing.assert_allclose(np.abs(ph[inside]), amp * q2[inside] ** (0.5 * p), rtol=1e-14)
    assert not np.any(ph[~inside])
    np.testing.assert_array_equal(ph[::-1, ::-1], np.conj(ph))
    psi = np.fft.ifft2(np.fft.ifftshift(np.pad(ph, 4)))
    assert np.max(np.abs(psi.imag)) <= 1e-14 * np.max(np.abs(psi.real))
    phases = np.angle(ph[inside & (k[:, None] > 0)])
    assert abs(np.mean(np.cos(phases))) < 0.1 and abs(np.mean(np.sin(phases))) < 0.1


def test_uneven_batch_draws_follow_the_recipe():
    """kappa log-uniform on [1e-3, 1e-1], L uniform in {2..5}, slope s uniform
    in [-3, -5/3] with p = (s - 3) / 2, n uniform in {32, 64, 128, 256}; the
    spectrum reaches radius 2 4^(L-1) and the band edges are 4^l.  Overriding
    n or the lattice leaves every draw unchanged."""
    seen_n, seen_L = set(), set()
    for seed in range(256):
        q = flowgen.config_batched_instance(seed)
        L = q.n_levels
        assert 1e-3 <= q.kappa <= 1e-1
        assert 2 <= L <= 5 and q.thresh == [4 ** l for l in range(1, L)]
        assert q.kmax == 2 * 4 ** (L - 1)
        n = q.n_cells[0]
        assert n in (32, 64, 128, 256) and q.n_cells == [n] * L
        assert q.n_global == [n * 4 ** l for l in range(L)] and q.lattice == [4] * L
        seen_n.add(n)
        seen_L.add(L)
        r = flowgen.config_batched_instance(seed, n=64, lattice=2)
        assert r.kappa == q.kappa and r.kmax == q.kmax and np.array_equal(r.psi_hat, q.psi_hat)
    assert seen_n == {32, 64, 128, 256} and seen_L == {2, 3, 4, 5}
    # slope: |psi_hat| falls as |k|^p with p = (s - 3) / 2 in [-3, -7/3]
    q = flowgen.config_batched_instance(7)
    a, b = abs(q.psi_hat[q.kmax, q.kmax + 1]), abs(q.psi_hat[q.kmax, q.kmax + 2])
    p = math.log(b / a) / math.log(2.0)
    assert -3.0 - 1e-12 <= p <= -7.0 / 3.0 + 1e-12


def test_continuous_spectrum_workload_recipe():
    """Five levels of 16 x 16 patches of 128^2, kappa 1e-3, 1 <= |k| <= 512 with
    |psi_hat| = |k|^(-7/3), band edges 4, 16, 64, 256."""
    q = flowgen.config_continuous(seed=0)
    assert q.kappa == 1e-3 and q.kmax == 512 and q.thresh == [4, 16, 64, 256]
    assert q.n_cells == [128] * 5 and q.lattice == [16] * 5
    assert q.n_global == [128 * 4 ** l for l in range(5)]
    assert abs(abs(q.psi_hat[512, 512 + 3]) - 3.0 ** (-7.0 / 3.0)) <= 1e-15
    assert q.psi_hat[512, 512] == 0 and q.psi_hat[512 + 512, 512 + 1] == 0      # |k| > 512 is empty
