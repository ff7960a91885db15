"""Autotuner for the local-solve kernels.

Two choices are tuned, both timed with HIP events on the launch stream on a
phase's own patches:
  * the kernel variant per patch size n (shmm_ctx_tune): every variant the
    library offers for that size, the fastest kept;
  * the steps per launch of a phase's local solves: the solve of a given
    number of steps issued as one launch per chunk of that many steps
    (shmm_local_solve_batch with step_begin, steps), the fastest chunk kept.
Variants and chunkings differ only in work decomposition, so they agree to
rounding (the GPU parity tests run every variant against the oracle, and the
chunked calls against the single launch).

Results are cached in a JSON file keyed by the GPU architecture and n
(tuned.json beside this module unless another path is given), so a process
that finds its sizes in the cache applies them without timing anything.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Sequence

import numpy as np

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def arch(device: int = 0) -> str:
    """Architecture name of the device (gfx950 on MI355X), without feature flags."""
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def load(path: str = CACHE) -> Dict[str, dict]:
    """The whole cache: {arch: {str(n): {"variant": v, ...}, "chunk": {...}}}."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(cache: Dict[str, dict], path: str = CACHE) -> None:
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply_cached(ctx, sizes: Iterable[int], device: int = 0, path: str = CACHE) -> Dict[int, dict]:
    """Select the cached variant of every size in `sizes` that the cache holds
    for this device's architecture; returns {n: entry} for those."""
    entries = load(path).get(arch(device), {})
    out = {}
    for n in sizes:
        e = entries.get(str(int(n)))
        if e is not None and 0 <= int(e["variant"]) < ctx.solve_variants(int(n)):
            ctx.shmm_ctx_tune(int(n), int(e["variant"]))
            out[int(n)] = e
    return out


def record(results: Dict[int, dict], device: int = 0, path: str = CACHE, workload: str = "") -> None:
    """Merge tuning results {n: {"variant": v, "ms": [...], ...}} into the cache."""
    cache = load(path)
    a = cache.setdefault(arch(device), {})
    for n, r in results.items():
        e = dict(r)
        if workload:
            e["workload"] = workload
        a[str(int(n))] = e
    save(cache, path)


def _time_solve(H, first, count, chunks: Sequence[tuple], repeats: int):
    """Best-of-`repeats` HIP-event time (ms) of the solve of [first, first +
    count) issued as the given (step_begin, steps) launches, correctors reset
    to zero before each repeat (the first, untimed, warms caches and code)."""
    torch = H.torch
    a, b = H.cell_range(first, count)
    s = H.stream()
    best = float("inf")
    for rep in range(repeats + 1):
        H.w.view(2, H.cells)[:, a:b].zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for s0, c in chunks:
            H.ctx.shmm_local_solve_batch(first, count, H.vx.data_ptr(), H.vy.data_ptr(),
                                         H.f1.data_ptr(), H.f2.data_ptr(), H.K_base.data_ptr(),
                                         H.w.data_ptr(), s0, c, 0, s)
        e1.record()
        torch.cuda.synchronize()
        if rep:
            best = min(best, e0.elapsed_time(e1))
    return best


def tune_solve(H, phase: int = 0, steps: int = 200, repeats: int = 2,
               sizes: Optional[Iterable[int]] = None) -> Dict[int, dict]:
    """Tune the solve kernel variant for every patch size in `phase` of
    Hierarchy H (or only `sizes`), `steps` RK4 steps on the phase's patches.

    The phase must have a step plan (for example after one pass).  Leaves the
    correctors of the phase overwritten; run the pass again afterwards.
    """
    first, count = int(H.phase[phase]), int(H.phase[phase + 1] - H.phase[phase])
    table = H.ctx.shmm_ctx_table()[0]
    ns = sorted(set(int(v) for v in table["n"][first:first + count]))
    if sizes is not None:
        ns = [n for n in ns if n in set(int(v) for v in sizes)]
    out = {}
    for n in ns:
        nv = H.ctx.solve_variants(n)
        if nv <= 1:
            continue
        # the whole phase is timed; the other sizes keep their variant
        ms = []
        for v in range(nv):
            H.ctx.shmm_ctx_tune(n, v)
            ms.append(_time_solve(H, first, count, [(0, steps)], repeats))
        choice = int(np.argmin(ms))
        H.ctx.shmm_ctx_tune(n, choice)
        out[n] = {"variant": choice, "ms": [round(x, 3) for x in ms], "steps": steps}
    return out


def tune_chunk(H, phase: int, steps: int, candidates: Sequence[int] = (0, 1000, 250, 50),
               repeats: int = 1) -> dict:
    """Steps per launch for the local solves of `phase`: `steps` RK4 steps
    issued as launches of c steps each (0: one launch for all), for each c in
    `candidates`; returns {"chunk": best c, "ms": {c: time}}."""
    first, count = int(H.phase[phase]), int(H.phase[phase + 1] - H.phase[phase])
    ms = {}
    for c in candidates:
        per = steps if c <= 0 else c
        launches = [(s0, min(per, steps - s0)) for s0 in range(0, steps, per)]
        ms[int(c)] = round(_time_solve(H, first, count, launches, repeats), 3)
    best = min(ms, key=lambda c: (ms[c], c != 0))
    return {"chunk": best, "ms": {str(k): v for k, v in ms.items()}, "steps": steps}
