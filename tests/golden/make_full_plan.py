"""Stored oracle values for the full-plan parity tests (tests/test_gpu_full_plan.py).

The local solves of the production workloads run 3e4 to 4e5 RK4 steps on
128^2 and 256^2 patches; the FP64 oracle takes minutes to hours for one chain
of levels there, too long for a test.  This script runs the oracle once, over
sampled centres, and writes what it computed to tests/golden/full_plan_<case>.json.
It imports only oracle/ (the FP64 reference) and flowgen/ (the seeded inputs);
nothing here comes from the HIP path.

For every computed domain the file holds its table entry (instance, level,
cx, cy, n), the step plan (nsteps, dt) and the FP64 tensors K_in, K_off,
K_base, K_solve and R of Algorithm 3 extended to L levels (K_total = R at
level 0).  A sampled centre is a level-0 domain; the oracle computes it and
every domain below it (oracle.run_hierarchy with roots), which is everything
its level results depend on.

Cases (each a workload at its full size, full step plans, delta = 1e-6):
  cellular4     the four-level cellular flow (64 patches of 128^2 per level),
                4 sampled centres;
  continuous5   the five-level continuous-spectrum flow (256 patches of 128^2
                per level, 1 <= |k| <= 512, kappa 1e-3), 4 sampled centres;
  uneven_small  32 instances of the uneven-batch generator (the first 16 seeds
                drawing n = 32 and the first 16 drawing n = 64), every domain;
  uneven_large  sampled chains of instances drawing n = 128 and n = 256.

Usage: python tests/golden/make_full_plan.py [case ...]   (OMP_NUM_THREADS sets the threads)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import flowgen  # noqa: E402
import oracle   # noqa: E402

# first 16 seeds of the uneven-batch generator drawing each patch size
SEEDS_N32 = [3, 8, 9, 10, 11, 19, 20, 23, 24, 27, 34, 39, 43, 45, 46, 49]
SEEDS_N64 = [1, 2, 6, 18, 21, 32, 35, 36, 37, 38, 41, 44, 52, 55, 56, 59]
SEEDS_N128 = [0, 4, 5, 15, 26, 30, 31, 40, 42, 51, 54, 58, 63, 65, 69, 71]
SEEDS_N256 = [7, 12, 13, 14, 16, 17, 22, 25, 28, 29, 33, 47, 48, 60, 68, 70]
# sampled instances of the two larger strata (one centre each)
LARGE_SEEDS = [40, 51, 14, 12]
LARGE_CENTRES = [(1, 2), (3, 0), (2, 1), (0, 3)]


def _level0(doms, inst, cx, cy):
    for i, d in enumerate(doms):
        if d.instance == inst and d.level == 0 and d.cx == cx and d.cy == cy:
            return i
    raise KeyError((inst, cx, cy))


def case(name):
    """(problems, roots) of one case."""
    if name == "cellular4":
        probs = [flowgen.config_four_level_cellular(seed=0, n=128, lattice=8)]
        centres = [(0, 0), (5, 2), (3, 6), (7, 7)]
    elif name == "continuous5":
        probs = [flowgen.config_continuous(seed=0)]
        centres = [(0, 0), (9, 4), (5, 13), (15, 15)]
    elif name == "uneven_small":
        probs = [flowgen.config_batched_instance(s) for s in SEEDS_N32 + SEEDS_N64]
        return probs, None
    elif name == "uneven_large":
        probs = [flowgen.config_batched_instance(s) for s in LARGE_SEEDS]
        doms = oracle.domain_table(probs)
        return probs, [_level0(doms, q, cx, cy) for q, (cx, cy) in enumerate(LARGE_CENTRES)]
    else:
        raise KeyError(name)
    doms = oracle.domain_table(probs)
    return probs, [_level0(doms, 0, cx, cy) for cx, cy in centres]


def run(name):
    probs, roots = case(name)
    t0 = time.time()
    res = oracle.run_hierarchy(probs, roots=roots)
    el = time.time() - t0
    keep = [i for i in range(len(res.domains)) if res.K_in[i][0] > 0]   # the computed domains
    out = {"case": name, "roots": roots, "oracle_seconds": round(el, 1),
           "clamped": list(res.clamped or []),
           "domains": []}
    for i in keep:
        d = res.domains[i]
        out["domains"].append({
            "index": i, "instance": d.instance, "level": d.level, "cx": d.cx, "cy": d.cy, "n": d.n,
            "nsteps": int(res.nsteps[i]), "dt": float(res.dt[i]),
            "K_in": [float(v) for v in res.K_in[i]], "K_off": [float(v) for v in res.K_off[i]],
            "K_base": [float(v) for v in res.K_base[i]], "K_solve": [float(v) for v in res.K_solve[i]],
            "R": [float(v) for v in res.R[i]]})
    path = os.path.join(HERE, f"full_plan_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}: {len(keep)} domains, {el:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["cellular4", "continuous5", "uneven_small", "uneven_large"]:
        run(n)
