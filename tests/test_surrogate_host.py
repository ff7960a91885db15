"""Host logic of the surrogate driver on the CPU: the model block layout, the
relative Frobenius error of packed 2 x 2 tensors, and the gate calibration's
choice of (tau, emax) (its per-patch inputs stubbed, no GPU call)."""
import math

import numpy as np

from paper_1510_00451_amd import abi
from paper_1510_00451_amd import surrogate as GS


def test_model_block_layout_round_trips():
    """35 -> 256 -> 256 -> 256 -> 3 weights and biases fill SURR_PARAMS words;
    the input standardisation sits after the padded parameters."""
    assert sum(fi * fo + fo for fi, fo in GS.LAYERS) == abi.SURR_PARAMS
    assert abi.SURR_PARAMS_PADDED >= abi.SURR_PARAMS
    W, b = GS.init_params(5)
    rng = np.random.default_rng(1)
    mu, sigma = rng.standard_normal(abi.SURR_IN), rng.uniform(0.5, 2.0, abi.SURR_IN)
    block = GS.pack_params(W, b, mu, sigma)
    W2, b2, mu2, sg2 = GS.unpack_params(block)
    for a, c in zip(W + b, W2 + b2):
        np.testing.assert_array_equal(c, np.asarray(a, np.float32).astype(np.float64))
    np.testing.assert_array_equal(mu2, mu.astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(sg2, sigma.astype(np.float32).astype(np.float64))
    assert b[-1][0] == b[-1][2] == -2.0 and not np.any(b[0])


def test_relative_frobenius_counts_the_off_diagonal_twice():
    A = np.array([[1.0, 0.0, 1.0], [1.0, 1.0, 1.0], [2.0, 0.5, 3.0]])
    B = np.array([[1.0, 0.0, 2.0], [1.0, 0.0, 1.0], [2.0, 0.5, 3.0]])
    got = GS.relative_frobenius(A, B)
    np.testing.assert_allclose(got, [math.sqrt(1 / 5), 1.0, 0.0], rtol=1e-15)


def _stub(monkeypatch, err, enh, spread, inside):
    monkeypatch.setattr(GS, "gate_inputs", lambda ens, data, lo, hi: (np.asarray(err), np.asarray(enh),
                                                                      np.asarray(spread), np.asarray(inside)))


def test_gate_calibration_takes_the_largest_accepted_set_and_the_larger_thresholds(monkeypatch):
    """Four patches; patch 2 is wrong by 5%.  Keeping it out leaves two
    accepted patches either way: {0, 1} with 2e-3 <= tau < 5e-3 and emax >=
    0.5, or {0, 3} with tau >= 1e-2 and 0.05 <= emax < 0.1.  Among equal
    acceptance the larger thresholds win: tau = 0.03 and emax = 0.07."""
    _stub(monkeypatch, err=[0.001, 0.002, 0.05, 0.003], enh=[0.01, 0.5, 0.1, 0.05],
          spread=[1e-4, 2e-3, 5e-3, 1e-2], inside=[True] * 4)
    tau, emax, frac = GS.calibrate_gate(None, None, None, None, target=0.01, quantile=1.0)
    assert (tau, emax, frac) == (0.03, 0.07, 0.5)
    # a patch outside the training range is never accepted, whatever the thresholds
    _stub(monkeypatch, err=[0.001, 0.002, 0.003], enh=[0.01, 0.01, 0.01], spread=[1e-4] * 3,
          inside=[True, False, True])
    tau, emax, frac = GS.calibrate_gate(None, None, None, None, target=0.01, quantile=1.0)
    assert frac == 2 / 3 and tau == 0.03 and emax == math.inf


def test_gate_calibration_with_no_admissible_pair_flags_every_patch(monkeypatch):
    """No pair keeps the errors within the target: the thresholds returned
    flag every patch under the gate's rule (spread > tau or enhancement >
    emax), also for a single-member ensemble whose spread is 0."""
    _stub(monkeypatch, err=[0.5, 0.6], enh=[0.0, 0.001], spread=[0.0, 1e-5], inside=[True, True])
    tau, emax, frac = GS.calibrate_gate(None, None, None, None, target=0.01, quantile=0.99)
    assert frac == 0.0
    spread, enh = np.array([0.0, 1e-5]), np.array([0.0, 0.001])
    assert np.all((spread > tau) | ~(enh <= emax))
