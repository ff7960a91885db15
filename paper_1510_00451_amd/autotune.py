"""Autotuner for the local-solve kernels: times every kernel variant the
library offers for each patch size of a phase, on that phase's own patches,
with HIP events on the launch stream, and selects the fastest through
shmm_ctx_tune.  Variants differ only in work decomposition, so they agree to
rounding (the GPU parity tests run every variant against the oracle)."""
from __future__ import annotations

import json
import os
from typing import Dict

import numpy as np


def tune_solve(H, phase: int = 0, steps: int = 200, repeats: int = 2) -> Dict[int, dict]:
    """Tune the solve kernel for every patch size in `phase` of Hierarchy H.

    The phase must have a step plan (for example after one pass).  Leaves the
    correctors of the phase overwritten; run the pass again afterwards.
    """
    torch = H.torch
    first, count = int(H.phase[phase]), int(H.phase[phase + 1] - H.phase[phase])
    table = H.ctx.shmm_ctx_table()[0]
    ns = sorted(set(int(v) for v in table["n"][first:first + count]))
    a, b = H.cell_range(first, count)
    out = {}
    s = H.stream()
    for n in ns:
        nv = H.ctx.solve_variants(n)
        if nv <= 1:
            continue
        ms = []
        for v in range(nv):
            H.ctx.shmm_ctx_tune(n, v)
            best = float("inf")
            for rep in range(repeats + 1):
                H.w.view(2, H.cells)[:, a:b].zero_()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                H.ctx.shmm_local_solve_batch(first, count, H.vx.data_ptr(), H.vy.data_ptr(),
                                             H.f1.data_ptr(), H.f2.data_ptr(), H.K_base.data_ptr(),
                                             H.w.data_ptr(), 0, steps, 0, s)
                e1.record()
                torch.cuda.synchronize()
                if rep:                       # the first launch warms caches and code
                    best = min(best, e0.elapsed_time(e1))
            ms.append(best)
        choice = int(np.argmin(ms))
        H.ctx.shmm_ctx_tune(n, choice)
        out[n] = {"variant": choice, "ms": [round(x, 3) for x in ms], "steps": steps}
    return out


def save(results: Dict[int, dict], path: str) -> None:
    with open(path, "w") as f:
        json.dump({str(k): v for k, v in results.items()}, f, indent=1)


def load(path: str) -> Dict[int, int]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return {int(k): int(v["variant"]) for k, v in json.load(f).items()}
