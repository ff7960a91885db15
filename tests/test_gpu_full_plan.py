"""Full-plan parity at the production sizes: whole passes of the hot path on
the GPU (band filter, Algorithm 2, every phase's plan, local solves to the
quasi-stationary state of the step plan, FP64 estimates, Algorithm 3) against
the FP64 oracle on sampled centres.

The oracle takes minutes to hours per chain of levels at 128^2 and 256^2 with
3e4 to 4e5 RK4 steps per solve, so its values are stored: they are written by
tests/golden/make_full_plan.py, which runs only oracle/ on flowgen inputs
(tests/golden/full_plan_<case>.json).  The GPU runs its own plan: step counts
agree within one step plus the relative difference of the bases (the
advection bound is reduced from FP32 faces on the GPU, FP64 faces in the
oracle, and a coarse level's base comes from each side's own finer results;
the stopping time depends on the base, not on the advection bound).

Bar: every K tensor of every sampled domain (K_base, the local solve's K and
the level result R; R at level 0 is K_total) within 1e-5 of the oracle's,
relative to its largest entry; no status bit set.  Printed beside it: the
largest relative error and the error of the enhancement K - K_b relative to
the enhancement, which is what the FP32 solve actually computes.
"""
import json
import os
import sys

import numpy as np
import pytest

import flowgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
sys.path.insert(0, GOLDEN)
import make_full_plan as golden_cases  # noqa: E402  (case definitions only; runs nothing on import)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


def _golden(case):
    path = os.path.join(GOLDEN, f"full_plan_{case}.json")
    with open(path) as f:
        return json.load(f)


def _compare(res, table, status, gold, index_of=None):
    """res: PassResult of the GPU pass; gold: the stored oracle values.
    index_of maps a golden entry to the GPU table index (default: the same
    index, when both ran the same problem list)."""
    worst, worst_enh = 0.0, 0.0
    assert gold["clamped"] == []
    for g in gold["domains"]:
        i = g["index"] if index_of is None else index_of(g)
        D = table[i]
        assert (int(D["level"]), int(D["cx"]), int(D["cy"]), int(D["n"])) == (g["level"], g["cx"], g["cy"], g["n"])
        # the plan follows the domain's own base: the GPU's base is within the
        # K bar of the oracle's, and nsteps ~ 1 / lambda_min(K_base)
        assert abs(int(res.nsteps[i]) - g["nsteps"]) <= 1 + 2e-5 * g["nsteps"], (i, int(res.nsteps[i]), g["nsteps"])
        for name, got in (("K_base", res.K_base[i]), ("K_solve", res.K_solve[i]), ("R", res.R[i])):
            want = np.array(g[name])
            err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
            worst = max(worst, err)
            assert err <= 1e-5, (name, i, g["level"], got, want, err)
        enh = np.array(g["K_solve"]) - np.array(g["K_base"])
        if np.max(np.abs(enh)) > 0:
            got_enh = res.K_solve[i] - res.K_base[i]
            worst_enh = max(worst_enh, float(np.max(np.abs(got_enh - enh)) / np.max(np.abs(enh))))
        assert int(status[i]) == 0, (i, int(status[i]))
    return worst, worst_enh


def _run(torch, probs):
    import time
    from paper_1510_00451_amd.hierarchy import Hierarchy
    H = Hierarchy(probs, keep_psi=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.run()
    res = H.result()
    el = time.perf_counter() - t0
    say("  pass %.2f s, %.4g point-steps, %.1f Gpoint-steps/s" % (el, res.point_steps, res.point_steps / el / 1e9))
    return H, res


@pytest.mark.timeout(300)
def test_full_plan_four_level_cellular(torch):
    """The four-level cellular flow at its full size (64 patches of 128^2 per
    level), four sampled chains of levels against the oracle."""
    gold = _golden("cellular4")
    probs, _ = golden_cases.case("cellular4")
    say("case full plan four-level cellular")
    H, res = _run(torch, probs)
    worst, worst_enh = _compare(res, H.table, H.status.cpu().numpy(), gold)
    say("  max rel err %.2e, enhancement %.2e" % (worst, worst_enh))
    H.close()


@pytest.mark.timeout(300)
def test_full_plan_five_level_continuous(torch):
    """The five-level continuous-spectrum flow at its full size (256 patches of
    128^2 per level, 1 <= |k| <= 512, kappa 1e-3): four sampled chains of
    five levels against the oracle, from the finest level's base to K_total."""
    gold = _golden("continuous5")
    probs, _ = golden_cases.case("continuous5")
    say("case full plan five-level continuous")
    H, res = _run(torch, probs)
    worst, worst_enh = _compare(res, H.table, H.status.cpu().numpy(), gold)
    say("  max rel err %.2e, enhancement %.2e" % (worst, worst_enh))
    H.close()


@pytest.mark.timeout(900)
def test_full_plan_uneven_batch_stratified_64(torch):
    """64 instances of the uneven-batch generator, stratified by patch size
    (the first 16 seeds drawing each of n = 32, 64, 128, 256; 4 x 4 patches
    per level, 2-5 levels, kappa and slope as drawn), in one pass at full
    plans: every phase holds all four sizes (the 256^2 patches on the
    ring-exchange bands first, the others concurrently after them).  Every
    domain of the n = 32 and n = 64 instances, and one sampled chain of
    levels in each of two n = 128 and two n = 256 instances, against the
    oracle."""
    seeds = (golden_cases.SEEDS_N32 + golden_cases.SEEDS_N64 + golden_cases.SEEDS_N128 +
             golden_cases.SEEDS_N256)
    probs = [flowgen.config_batched_instance(q) for q in seeds]
    say("case full plan uneven batch, 64 instances")
    H, res = _run(torch, probs)
    where = {}
    for i, D in enumerate(H.table):
        where[(int(D["instance"]), int(D["level"]), int(D["cx"]), int(D["cy"]))] = i
    status = H.status.cpu().numpy()
    report = []
    for case, case_seeds in (("uneven_small", golden_cases.SEEDS_N32 + golden_cases.SEEDS_N64),
                             ("uneven_large", golden_cases.LARGE_SEEDS)):
        gold = _golden(case)
        if case == "uneven_small":
            assert len(gold["domains"]) == sum(1 for D in H.table if int(D["instance"]) < 32)
        index_of = lambda g: where[(seeds.index(case_seeds[g["instance"]]), g["level"], g["cx"], g["cy"])]
        report.append(_compare(res, H.table, status, gold, index_of))
    say("  max rel err (small, large) %s" % ["%.2e / enhancement %.2e" % r for r in report])
    H.close()
