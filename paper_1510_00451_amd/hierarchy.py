"""One pass of the SHMM hot path on the GPU: band filter, top-down Algorithm 2,
then phase by phase (finest level first) the local solves, the effective
diffusivity and the level combination of Algorithm 3.

PyTorch supplies device memory and the stream; every numeric step runs in
libshmm.so.  The only host work between phases is the step plan, which needs
the phase's base diffusivities (24 bytes per domain) on the host.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import abi

MODE_TOPDOWN, MODE_BASE, MODE_RESULT, MODE_MACRO = 0, 1, 2, 3


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the SHMM hot path needs a HIP device; no CPU fallback exists")
    return torch


@dataclass
class PassResult:
    K_total: np.ndarray      # [instances * coarsest-lattice][3], level-0 results
    R: np.ndarray            # [nd][3] level results
    K_base: np.ndarray
    K_solve: np.ndarray
    K_in: np.ndarray
    K_off: np.ndarray
    nsteps: np.ndarray
    dt: np.ndarray
    point_steps: int         # sum over domains of n^2 * nsteps


class Hierarchy:
    """Device buffers and phase schedule for a batch of flow instances."""

    def __init__(self, problems, device: int = 0, keep_psi: bool = False):
        torch = _torch()
        self.torch = torch
        self.problems = problems if isinstance(problems, (list, tuple)) else [problems]
        self.device = torch.device("cuda", device)
        self.ctx = abi.Context(device)
        self.ctx.shmm_ctx_set_problem(self.problems)
        self.table, self.cells, self.lines_total, self.phase = self.ctx.shmm_ctx_table()
        nd = len(self.table)
        self.nd = nd
        f32 = dict(dtype=torch.float32, device=self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.psi = torch.zeros(self.cells, **f32) if keep_psi else None
        self.vx = torch.zeros(self.cells, **f32)
        self.vy = torch.zeros(self.cells, **f32)
        self.f1 = torch.zeros(self.cells, **f32)
        self.f2 = torch.zeros(self.cells, **f32)
        self.w = torch.zeros(2 * self.cells, **f32)
        self.lines = torch.zeros(max(1, self.lines_total), **f64)
        self.K_in = torch.zeros(nd, 3, **f64)
        self.K_off = torch.zeros(nd, 3, **f64)
        self.K_base = torch.zeros(nd, 3, **f64)
        self.K_solve = torch.zeros(nd, 3, **f64)
        self.R = torch.zeros(nd, 3, **f64)
        self.K_energy = torch.zeros(nd, 3, **f64)
        self.mass = torch.zeros(nd, 2, **f64)
        self.status = torch.zeros(nd, dtype=torch.int32, device=self.device)
        self.host_K = np.zeros((nd, 3))
        self.level0 = np.flatnonzero(self.table["level"] == 0)
        # optional callable(first, count, launch) wrapped around each solve launch
        self.solve_hook = None
        # quasi-stationary stop: chunks per plan, tolerance (0: each instance's delta)
        self.adaptive_chunks = 32
        self.adaptive_tol = 0.0
        # oversampled patches: average the estimator over the centred inner x
        # inner cells of each patch (0: the whole patch; the energy form and
        # the mass are then not formed)
        self.estimator_inner = 0
        # windowed patches: taper the stream function over this many nodes at
        # each patch edge after the band filter (needs keep_psi)
        self.patch_taper = 0
        # steps per launch of the planned local solves (0: one call for all;
        # the autotuner's chunk)
        self.solve_chunk = 0
        # replay each phase's planned local solves from a captured HIP graph:
        # the first pass runs them eagerly (which also sets up the launch lists
        # and the workspace), later passes capture once and replay
        self.graph_solves = False
        self._graphs = {}
        self._graph_seen = set()
        # learned surrogate in place of the planned local solves (see
        # use_surrogate); per-phase flags of the patches it sent to the plain solve
        self.surrogate = None
        self.surrogate_flags = {}

    # -- pieces -------------------------------------------------------------
    def stream(self) -> int:
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def cell_range(self, first: int, count: int):
        t = self.table
        a = int(t["offset"][first])
        b = int(t["offset"][first + count - 1] + t["n"][first + count - 1] ** 2)
        return a, b

    def band_filter(self) -> None:
        s = self.stream()
        nph = len(self.phase) - 1
        if self.patch_taper and self.psi is None:
            raise ValueError("windowed patches need the stream function (keep_psi=True)")
        for p in range(nph):
            first, count = int(self.phase[p]), int(self.phase[p + 1] - self.phase[p])
            self.ctx.shmm_band_filter(first, count, self.psi.data_ptr() if self.psi is not None else 0,
                                      self.vx.data_ptr(), self.vy.data_ptr(), self.f1.data_ptr(),
                                      self.f2.data_ptr(), self.lines.data_ptr(), s)
            if self.patch_taper:
                n = self.table["n"]
                i = first
                while i < first + count:   # runs of one patch size
                    j = i
                    while j < first + count and n[j] == n[i]:
                        j += 1
                    self.ctx.shmm_window_patches(i, j - i, self.patch_taper, self.psi.data_ptr(),
                                                 self.vx.data_ptr(), self.vy.data_ptr(), self.f1.data_ptr(),
                                                 self.f2.data_ptr(), s)
                    i = j

    def top_down(self) -> None:
        s = self.stream()
        nph = len(self.phase) - 1
        for p in range(nph - 1, -1, -1):
            first, count = int(self.phase[p]), int(self.phase[p + 1] - self.phase[p])
            self.ctx.shmm_level_chain(first, count, MODE_TOPDOWN, self.lines.data_ptr(),
                                      self.K_in.data_ptr(), self.K_off.data_ptr(), stream=s)

    def use_surrogate(self, models_ptr: int, E: int, lo, hi, tau: float, emax: float,
                      chain_tol: Optional[float] = None) -> None:
        """Replace every phase's planned local solves by the ensemble surrogate
        (shmm_patch_features, shmm_surrogate_infer) with the plain solve as
        its fallback for the flagged patches (shmm_fallback_solve); the bases
        are the level chain's own (Algorithm 3), anisotropic in general.
        models_ptr: E members back to back (device); lo, hi: device [35]
        feature range of the gate.  chain_tol: also flag a patch whose
        predicted change of its base plus ensemble spread, in absolute
        terms, exceeds chain_tol times the smallest eigenvalue of the K_in
        of its ancestors (shmm_surrogate_chain_gate: the accuracy Algorithm 3
        needs of a finer result, which enters the parent's base after K_off
        is subtracted and from there the bases above it)."""
        torch = self.torch
        self.surrogate = (models_ptr, E, lo, hi, tau, emax, chain_tol)
        self._x = torch.zeros(self.nd, abi.SURR_IN, dtype=torch.float32, device=self.device)
        self._flags = torch.zeros(self.nd, dtype=torch.uint8, device=self.device)
        self._spread = torch.zeros(self.nd, dtype=torch.float64, device=self.device)

    def _surrogate_phase(self, first: int, count: int, s: int) -> None:
        c = self.ctx
        models, E, lo, hi, tau, emax, chain_tol = self.surrogate
        t = c.shmm_ctx_table()[0]
        if np.any(t["nsteps"][first:first + count] == 0):
            raise NotImplementedError("a phase with an empty diagonal band: its exact result is the base")
        n = t["n"]
        i = first
        while i < first + count:          # features: runs of one patch size
            j = i
            while j < first + count and n[j] == n[i]:
                j += 1
            c.shmm_patch_features(i, j - i, self.vx.data_ptr(), self.vy.data_ptr(), self.K_base.data_ptr(),
                                  self._x[i].data_ptr(), s)
            i = j
        c.shmm_surrogate_infer(models, E, self._x[first].data_ptr(), self.K_base[first].data_ptr(), count,
                               lo.data_ptr(), hi.data_ptr(), tau, emax, self.K_solve[first].data_ptr(),
                               self._flags[first].data_ptr(), self._spread[first].data_ptr(), 0, s)
        if chain_tol is not None:
            c.shmm_surrogate_chain_gate(first, count, self.K_solve[first].data_ptr(), self.K_base[first].data_ptr(),
                                        self._spread[first].data_ptr(), self.K_in.data_ptr(), chain_tol,
                                        self._flags[first].data_ptr(), s)
        c.shmm_fallback_solve(first, count, self._flags[first].data_ptr(), self.vx.data_ptr(), self.vy.data_ptr(),
                              self.f1.data_ptr(), self.f2.data_ptr(), self.K_base.data_ptr(), self.w.data_ptr(),
                              self.K_solve.data_ptr(), 0, 0.0, self.status.data_ptr(), s)

    def phase_solve(self, p: int, steps: Optional[int] = None, adaptive: bool = False) -> None:
        s = self.stream()
        first, count = int(self.phase[p]), int(self.phase[p + 1] - self.phase[p])
        c = self.ctx
        c.shmm_level_chain(first, count, MODE_BASE, self.lines.data_ptr(), self.K_in.data_ptr(),
                           self.K_off.data_ptr(), self.K_base.data_ptr(), 0, self.R.data_ptr(),
                           self.status.data_ptr(), s)
        # step plan on the host (bit-reproducible bookkeeping)
        self.host_K[first:first + count] = self.K_base[first:first + count].cpu().numpy()
        c.shmm_plan_steps(first, count, self.host_K)
        a, b = self.cell_range(first, count)
        self.w.view(2, self.cells)[:, a:b].zero_()
        if self.surrogate is not None and steps is None and not adaptive:
            self._surrogate_phase(first, count, s)
            self.surrogate_flags[p] = self._flags[first:first + count].cpu().numpy().copy()
            c.shmm_level_chain(first, count, MODE_RESULT, self.lines.data_ptr(), self.K_in.data_ptr(),
                               self.K_off.data_ptr(), self.K_base.data_ptr(), self.K_solve.data_ptr(),
                               self.R.data_ptr(), self.status.data_ptr(), s)
            return
        def launch():
            if adaptive:
                # quasi-stationary stop (plans cut to the steps taken)
                c.shmm_local_solve_adaptive(first, count, self.vx.data_ptr(), self.vy.data_ptr(),
                                            self.f1.data_ptr(), self.f2.data_ptr(), self.K_base.data_ptr(),
                                            self.w.data_ptr(), self.adaptive_chunks, self.adaptive_tol,
                                            self.status.data_ptr(), s)
                return
            self._planned_solve(first, count, steps, s)

        if self.graph_solves and not adaptive:
            key = (p, steps)
            if key in self._graphs:
                launch = self._graphs[key].replay
            elif key in self._graph_seen:
                self._graphs[key] = self._capture(lambda st: self._planned_solve(first, count, steps, st))
                launch = self._graphs[key].replay
            else:
                self._graph_seen.add(key)
        if self.solve_hook is None:
            launch()
        else:
            self.solve_hook(first, count, launch)
        if self.estimator_inner:
            c.shmm_effective_diffusivity_window(first, count, self.estimator_inner, self.f1.data_ptr(),
                                                self.f2.data_ptr(), self.w.data_ptr(), self.K_base.data_ptr(),
                                                self.K_solve.data_ptr(), self.status.data_ptr(), s)
        else:
            c.shmm_effective_diffusivity(first, count, self.f1.data_ptr(), self.f2.data_ptr(),
                                         self.w.data_ptr(), self.K_base.data_ptr(),
                                         self.K_solve.data_ptr(), self.K_energy.data_ptr(),
                                         self.mass.data_ptr(), self.status.data_ptr(), s)
        c.shmm_level_chain(first, count, MODE_RESULT, self.lines.data_ptr(), self.K_in.data_ptr(),
                           self.K_off.data_ptr(), self.K_base.data_ptr(), self.K_solve.data_ptr(),
                           self.R.data_ptr(), self.status.data_ptr(), s)

    def _planned_solve(self, first: int, count: int, steps: Optional[int], stream: int) -> None:
        """The planned local solves of [first, first + count): steps [0, steps)
        of each plan (all of it when steps is None), in launches of
        solve_chunk steps (one launch when 0)."""
        total = 2 ** 31 - 1 if steps is None else steps
        if steps is None and self.solve_chunk > 0:
            t = self.ctx.shmm_ctx_table()[0]
            total = int(t["nsteps"][first:first + count].max()) if count else 0
        per = total if self.solve_chunk <= 0 else self.solve_chunk
        for s0 in range(0, max(total, 1), max(per, 1)):
            self.ctx.shmm_local_solve_batch(first, count, self.vx.data_ptr(), self.vy.data_ptr(),
                                            self.f1.data_ptr(), self.f2.data_ptr(), self.K_base.data_ptr(),
                                            self.w.data_ptr(), s0, min(per, total - s0),
                                            self.status.data_ptr(), stream)

    def _capture(self, issue):
        """A HIP graph of the launches that issue(stream) enqueues, captured on
        a side stream (the library's work for the range is already set up)."""
        torch = self.torch
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.graph(g, stream=side):
            issue(torch.cuda.current_stream(self.device).cuda_stream)
        torch.cuda.current_stream(self.device).wait_stream(side)
        return g

    def run(self, steps: Optional[int] = None, adaptive: bool = False) -> None:
        """One pass of the hot path (asynchronous apart from the per-phase plan;
        with `adaptive`, the local solves stop at the quasi-stationary test)."""
        self.status.zero_()
        self.band_filter()
        self.top_down()
        for p in range(len(self.phase) - 1):
            self.phase_solve(p, steps, adaptive)

    # -- results ------------------------------------------------------------
    def result(self) -> PassResult:
        self.torch.cuda.synchronize(self.device)
        table, _, _, _ = self.ctx.shmm_ctx_table()
        R = self.R.cpu().numpy()
        return PassResult(K_total=R[self.level0], R=R, K_base=self.K_base.cpu().numpy(),
                          K_solve=self.K_solve.cpu().numpy(), K_in=self.K_in.cpu().numpy(),
                          K_off=self.K_off.cpu().numpy(), nsteps=table["nsteps"].copy(),
                          dt=table["dt"].copy(),
                          point_steps=int(np.sum(table["n"].astype(np.int64) ** 2
                                                 * table["nsteps"].astype(np.int64))))

    def close(self):
        self._graphs.clear()
        self.ctx.close()
