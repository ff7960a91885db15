"""ctypes binding of libshmm.so.  Argument marshalling only: every step of the
method runs inside the library.  Device pointers are plain integers (for
example ``tensor.data_ptr()``); streams are hipStream_t handles as integers.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshmm.so")

SHMM_OK, SHMM_EINVAL, SHMM_ERANGE, SHMM_ENOTSPD, SHMM_EDEVICE, SHMM_ENOMEM = 0, -1, -2, -3, -4, -5
ERRORS = {SHMM_EINVAL: "SHMM_EINVAL", SHMM_ERANGE: "SHMM_ERANGE", SHMM_ENOTSPD: "SHMM_ENOTSPD",
          SHMM_EDEVICE: "SHMM_EDEVICE", SHMM_ENOMEM: "SHMM_ENOMEM"}
DOM_NONFINITE, DOM_NOT_SPD, DOM_FALLBACK = 1, 2, 8
MAX_LEVELS = 8

EXPORTS = ["shmm_ctx_create", "shmm_ctx_destroy", "shmm_build_levels", "shmm_ctx_set_problem",
           "shmm_ctx_table", "shmm_band_tags", "shmm_plan_steps", "shmm_band_filter",
           "shmm_local_solve_batch", "shmm_local_solve_adaptive", "shmm_effective_diffusivity",
           "shmm_effective_diffusivity_window", "shmm_window_patches", "shmm_ctx_set_local_bc",
           "shmm_level_chain",
           "shmm_macro_step", "shmm_macro_step_noalloc", "shmm_ctx_tune", "shmm_patch_features", "shmm_surrogate_refresh",
           "shmm_surrogate_train_step", "shmm_surrogate_infer", "shmm_fallback_solve",
           "shmm_feature_stats", "shmm_surrogate_rescale", "shmm_surrogate_chain_gate"]

BC_PERIODIC, BC_DIRICHLET_X = 0, 1
LOCAL_PERIODIC, LOCAL_ZERO_FRAME = 0, 1
TUNE_SOLVE_VARIANT_COUNT, TUNE_RING_SPIN_CAP = 0, -1
MACRO_NOALLOC_MAX_N = 512
SURR_BINS, SURR_IN, SURR_WIDTH, SURR_OUT = 32, 35, 256, 3
SURR_PARAMS, SURR_PARAMS_PADDED = 141571, 141824
SURR_MODEL_BYTES = 4 * SURR_PARAMS_PADDED + 4 * 128 + 2 * SURR_PARAMS_PADDED


class ShmmError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed: {ERRORS.get(code, code)}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("kmax", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("psi_hat", ctypes.c_void_p), ("thresh", ctypes.c_void_p),
                ("n_cells", ctypes.c_void_p), ("n_global", ctypes.c_void_p),
                ("lattice", ctypes.c_void_p), ("dt_frac", ctypes.c_double),
                ("delta", ctypes.c_double)]


DOMAIN_DTYPE = np.dtype([("instance", "<i4"), ("level", "<i4"), ("cx", "<i4"), ("cy", "<i4"),
                         ("n", "<i4"), ("N", "<i4"), ("I0", "<i4"), ("J0", "<i4"),
                         ("parent", "<i4"), ("nsteps", "<i4"), ("offset", "<i8"),
                         ("line_offset", "<i8"), ("h", "<f8"), ("dt", "<f8")])
assert DOMAIN_DTYPE.itemsize == 72

_lib = None


def lib() -> ctypes.CDLL:
    """Load libshmm.so (built in-tree by ``build.py``).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1510_00451_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "shmm_ctx_create": [ctypes.POINTER(P), ctypes.c_int],
            "shmm_ctx_destroy": [P],
            "shmm_build_levels": [P, i32, P, P, P, P],
            "shmm_ctx_set_problem": [P, P, i32],
            "shmm_ctx_table": [P, P, P, P, P, P, P],
            "shmm_band_tags": [P, i32, P, P],
            "shmm_plan_steps": [P, i64, i64, P, P],
            "shmm_band_filter": [P, i64, i64, P, P, P, P, P, P, P],
            "shmm_local_solve_batch": [P, i64, i64, P, P, P, P, P, P, i32, i32, P, P],
            "shmm_local_solve_adaptive": [P, i64, i64, P, P, P, P, P, P, i32, f64, P, P],
            "shmm_effective_diffusivity": [P, i64, i64, P, P, P, P, P, P, P, P, P],
            "shmm_effective_diffusivity_window": [P, i64, i64, i32, P, P, P, P, P, P, P],
            "shmm_window_patches": [P, i64, i64, i32, P, P, P, P, P, P],
            "shmm_ctx_set_local_bc": [P, i32],
            "shmm_level_chain": [P, i64, i64, i32, P, P, P, P, P, P, P, P],
            "shmm_macro_step": [P, i32, i32, f64, f64, P, P, P, i32, f64, i32, P, i32, P],
            "shmm_macro_step_noalloc": [P, i32, i32, f64, f64, P, P, P, i32, f64, i32, P, i32, P],
            "shmm_ctx_tune": [P, i32, i32],
            "shmm_patch_features": [P, i64, i64, P, P, P, P, P],
            "shmm_surrogate_refresh": [P, P, P],
            "shmm_surrogate_train_step": [P, P, P, P, P, P, i64, ctypes.c_float, ctypes.c_float, i32, P, P, P],
            "shmm_surrogate_infer": [P, P, i32, P, P, i64, P, P, f64, f64, P, P, P, P, P],
            "shmm_fallback_solve": [P, i64, i64, P, P, P, P, P, P, P, P, i32, f64, P, P],
            "shmm_feature_stats": [P, P, i64, P, P],
            "shmm_surrogate_rescale": [P, P, P, P, P, i64, P, P, P, P],
            "shmm_surrogate_chain_gate": [P, i64, i64, P, P, P, P, f64, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc: int, what: str) -> None:
    if rc != SHMM_OK:
        raise ShmmError(rc, what)


class ProblemSet:
    """ctypes array of shmm_problem plus the numpy buffers it points into."""

    def __init__(self, problems):
        self.keep: List[np.ndarray] = []
        self.arr = (Problem * len(problems))()
        for q, p in enumerate(problems):
            ph = np.ascontiguousarray(np.asarray(p.psi_hat, np.complex128)).view(np.float64).reshape(-1)
            th = np.ascontiguousarray(list(p.thresh) + [0], np.int32)
            nc = np.ascontiguousarray(p.n_cells, np.int32)
            ng = np.ascontiguousarray(p.n_global, np.int32)
            la = np.ascontiguousarray(p.lattice, np.int32)
            self.keep += [ph, th, nc, ng, la]
            s = self.arr[q]
            s.kappa = float(p.kappa)
            s.kmax = int(p.kmax)
            s.n_levels = len(p.n_cells)
            s.psi_hat = ph.ctypes.data
            s.thresh = th.ctypes.data
            s.n_cells = nc.ctypes.data
            s.n_global = ng.ctypes.data
            s.lattice = la.ctypes.data
            s.dt_frac = float(p.dt_frac)
            s.delta = float(p.delta)

    @property
    def ptr(self) -> int:
        return ctypes.addressof(self.arr)

    def __len__(self) -> int:
        return len(self.arr)


def shmm_build_levels(problems) -> Tuple[np.ndarray, int, int]:
    """Host-only bookkeeping: (domain table as a structured array, cells, lines)."""
    ps = ProblemSet(problems if isinstance(problems, (list, tuple)) else [problems])
    nd, cells, lines = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib().shmm_build_levels(ps.ptr, len(ps), None, ctypes.byref(nd), ctypes.byref(cells),
                                  ctypes.byref(lines)), "shmm_build_levels")
    out = np.zeros(nd.value, DOMAIN_DTYPE)
    check(lib().shmm_build_levels(ps.ptr, len(ps), out.ctypes.data, None, None, None),
          "shmm_build_levels")
    return out, cells.value, lines.value


class Context:
    """Owns one shmm_ctx on one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        check(lib().shmm_ctx_create(ctypes.byref(h), int(device)), "shmm_ctx_create")
        self.h = h
        self.problems = None

    def close(self):
        if self.h:
            lib().shmm_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shmm_ctx_set_problem(self, problems) -> None:
        self.problems = ProblemSet(problems if isinstance(problems, (list, tuple)) else [problems])
        check(lib().shmm_ctx_set_problem(self.h, self.problems.ptr, len(self.problems)),
              "shmm_ctx_set_problem")

    def shmm_ctx_table(self):
        tab, nd, cells, lines = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        pf, nph = ctypes.c_void_p(), ctypes.c_int32()
        check(lib().shmm_ctx_table(self.h, ctypes.byref(tab), ctypes.byref(nd), ctypes.byref(cells),
                                   ctypes.byref(lines), ctypes.byref(pf), ctypes.byref(nph)),
              "shmm_ctx_table")
        table = np.frombuffer((ctypes.c_char * (nd.value * DOMAIN_DTYPE.itemsize)).from_address(tab.value),
                              DOMAIN_DTYPE).copy() if nd.value else np.zeros(0, DOMAIN_DTYPE)
        phase = np.frombuffer((ctypes.c_int64 * (nph.value + 1)).from_address(pf.value), np.int64).copy()
        return table, cells.value, lines.value, phase

    def shmm_band_tags(self, inst: int, d_tags: int, stream: int = 0) -> None:
        check(lib().shmm_band_tags(self.h, inst, d_tags, stream), "shmm_band_tags")

    def shmm_plan_steps(self, first: int, count: int, K_base_host: np.ndarray,
                        vmax_host: "np.ndarray | None" = None) -> None:
        K = np.ascontiguousarray(K_base_host, np.float64)
        V = None if vmax_host is None else np.ascontiguousarray(vmax_host, np.float64)
        check(lib().shmm_plan_steps(self.h, first, count, K.ctypes.data,
                                    None if V is None else V.ctypes.data), "shmm_plan_steps")

    def shmm_band_filter(self, first, count, d_psi, d_vx, d_vy, d_f1, d_f2, d_lines, stream=0):
        check(lib().shmm_band_filter(self.h, first, count, d_psi or None, d_vx, d_vy, d_f1, d_f2,
                                     d_lines, stream), "shmm_band_filter")

    def shmm_local_solve_batch(self, first, count, d_vx, d_vy, d_f1, d_f2, d_K_base, d_w,
                               step_begin=0, steps=2 ** 31 - 1, d_status=0, stream=0):
        check(lib().shmm_local_solve_batch(self.h, first, count, d_vx, d_vy, d_f1, d_f2, d_K_base,
                                           d_w, int(step_begin), int(steps), d_status or None,
                                           stream), "shmm_local_solve_batch")

    def shmm_local_solve_adaptive(self, first, count, d_vx, d_vy, d_f1, d_f2, d_K_base, d_w,
                                  chunks=32, tol=0.0, d_status=0, stream=0):
        check(lib().shmm_local_solve_adaptive(self.h, first, count, d_vx, d_vy, d_f1, d_f2, d_K_base, d_w,
                                              int(chunks), float(tol), d_status or None, stream),
              "shmm_local_solve_adaptive")

    def shmm_effective_diffusivity(self, first, count, d_f1, d_f2, d_w, d_K_base, d_K_out,
                                   d_K_energy=0, d_mass=0, d_status=0, stream=0):
        check(lib().shmm_effective_diffusivity(self.h, first, count, d_f1, d_f2, d_w, d_K_base,
                                               d_K_out, d_K_energy or None, d_mass or None,
                                               d_status or None, stream),
              "shmm_effective_diffusivity")

    def shmm_ctx_set_local_bc(self, bc):
        check(lib().shmm_ctx_set_local_bc(self.h, int(bc)), "shmm_ctx_set_local_bc")

    def shmm_window_patches(self, first, count, taper, d_psi, d_vx, d_vy, d_f1, d_f2, stream=0):
        check(lib().shmm_window_patches(self.h, first, count, int(taper), d_psi, d_vx, d_vy, d_f1, d_f2, stream),
              "shmm_window_patches")

    def shmm_effective_diffusivity_window(self, first, count, inner, d_f1, d_f2, d_w, d_K_base, d_K_out,
                                          d_status=0, stream=0):
        check(lib().shmm_effective_diffusivity_window(self.h, first, count, int(inner), d_f1, d_f2, d_w,
                                                      d_K_base, d_K_out, d_status or None, stream),
              "shmm_effective_diffusivity_window")

    def shmm_level_chain(self, first, count, mode, d_lines, d_K_in, d_K_off, d_K_base=0,
                         d_K_solve=0, d_R=0, d_status=0, stream=0):
        check(lib().shmm_level_chain(self.h, first, count, mode, d_lines, d_K_in, d_K_off,
                                     d_K_base or None, d_K_solve or None, d_R or None,
                                     d_status or None, stream), "shmm_level_chain")

    def shmm_ctx_tune(self, key: int, value: int) -> int:
        rc = lib().shmm_ctx_tune(self.h, int(key), int(value))
        if rc < 0:
            raise ShmmError(rc, "shmm_ctx_tune")
        return rc

    def solve_variants(self, n: int) -> int:
        return self.shmm_ctx_tune(0, n)

    def shmm_patch_features(self, first, count, d_vx, d_vy, d_K_base, d_features, stream=0):
        check(lib().shmm_patch_features(self.h, first, count, d_vx, d_vy, d_K_base, d_features, stream),
              "shmm_patch_features")

    def shmm_surrogate_refresh(self, d_model, stream=0):
        check(lib().shmm_surrogate_refresh(self.h, d_model, stream), "shmm_surrogate_refresh")

    def shmm_surrogate_train_step(self, d_model, d_adam, d_x, d_K_base, d_K_true, B, lr, clip, t, d_loss,
                                  d_grad=0, stream=0):
        check(lib().shmm_surrogate_train_step(self.h, d_model, d_adam, d_x, d_K_base, d_K_true, int(B),
                                              float(lr), float(clip), int(t), d_loss, d_grad or None, stream),
              "shmm_surrogate_train_step")

    def shmm_surrogate_infer(self, d_models, E, d_x, d_K_base, B, d_lo, d_hi, tau, emax, d_K_out, d_flags,
                             d_spread=0, d_K_members=0, stream=0):
        check(lib().shmm_surrogate_infer(self.h, d_models, int(E), d_x, d_K_base, int(B), d_lo, d_hi,
                                         float(tau), float(emax), d_K_out, d_flags, d_spread or None,
                                         d_K_members or None, stream), "shmm_surrogate_infer")

    def shmm_fallback_solve(self, first, count, d_flags, d_vx, d_vy, d_f1, d_f2, d_K_base, d_w, d_K_out,
                            chunks=0, tol=0.0, d_status=0, stream=0):
        check(lib().shmm_fallback_solve(self.h, first, count, d_flags, d_vx, d_vy, d_f1, d_f2, d_K_base,
                                        d_w, d_K_out, int(chunks), float(tol), d_status or None, stream),
              "shmm_fallback_solve")

    def shmm_surrogate_chain_gate(self, first, count, d_K_hat, d_K_base, d_spread, d_K_in, tol, d_flags, stream=0):
        check(lib().shmm_surrogate_chain_gate(self.h, first, count, d_K_hat, d_K_base, d_spread, d_K_in, float(tol),
                                              d_flags, stream), "shmm_surrogate_chain_gate")

    def shmm_feature_stats(self, d_x, B, d_stats, stream=0):
        check(lib().shmm_feature_stats(self.h, d_x, int(B), d_stats, stream), "shmm_feature_stats")

    def shmm_surrogate_rescale(self, d_x, d_K_base, d_K_true, d_log10c, B, d_x_out, d_K_base_out, d_K_true_out,
                               stream=0):
        check(lib().shmm_surrogate_rescale(self.h, d_x, d_K_base, d_K_true, d_log10c, int(B), d_x_out,
                                           d_K_base_out, d_K_true_out, stream), "shmm_surrogate_rescale")

    def shmm_macro_step(self, N, bc, g0, g1, d_vx, d_vy, d_K, K_is_field, dt, nsteps, d_u, dtype, stream=0):
        check(lib().shmm_macro_step(self.h, N, int(bc), float(g0), float(g1), d_vx or None, d_vy or None, d_K,
                                    int(K_is_field), float(dt), int(nsteps), d_u, int(dtype), stream),
              "shmm_macro_step")

    def shmm_macro_step_noalloc(self, N, bc, g0, g1, d_vx, d_vy, d_K, K_is_field, dt, nsteps, d_u, dtype,
                                stream=0):
        check(lib().shmm_macro_step_noalloc(self.h, N, int(bc), float(g0), float(g1), d_vx or None,
                                            d_vy or None, d_K, int(K_is_field), float(dt), int(nsteps), d_u,
                                            int(dtype), stream), "shmm_macro_step_noalloc")
