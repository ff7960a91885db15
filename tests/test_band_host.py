"""The band-filter block code of the HIP path, compiled for the host and run
with one thread per block, against the FP64 oracle (no GPU needed).

Checks the in-house Stockham FFT, the pruned two-pass synthesis at the patch
nodes, the difference-symbol velocities and the line energies."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import flowgen
import oracle
from oracle import DIAG, OFF12, OFF21

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_SO = None


def harness():
    global _SO
    if _SO is None:
        out = os.path.join(tempfile.gettempdir(), "shmm_band_host_%d.so" % os.getpid())
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-x", "hip", "--cuda-host-only", "-O2",
                               "-std=c++17", "-fPIC", "-shared",
                               "-I", os.path.join(ROOT, "include"),
                               "-I", os.path.join(ROOT, "paper_1510_00451_amd", "csrc"),
                               os.path.join(ROOT, "tests", "band_host_harness.cpp"), "-o", out],
                              stderr=subprocess.DEVNULL)
        _SO = ctypes.CDLL(out)
        _SO.band_host_run.restype = ctypes.c_int
        _SO.seam_host.restype = None
    return _SO


def run_group(p, table, level):
    from paper_1510_00451_amd import abi
    rows = np.flatnonzero(table["level"] == level)
    first = int(rows[0])
    M = p.lattice[level]
    n, N = p.n_cells[level], p.n_global[level]
    lv, pt = oracle.band_split(p.kmax, p.thresh)
    diag = (lv == level) & (pt == DIAG) & (p.psi_hat != 0)
    k = np.arange(-p.kmax, p.kmax + 1)
    kb1 = int(np.max(np.abs(k)[None, :].repeat(len(k), 0)[diag])) if diag.any() else 0
    kb2 = int(np.max(np.abs(k)[:, None].repeat(len(k), 1)[diag])) if diag.any() else 0
    I0 = np.ascontiguousarray([table["I0"][first + c] for c in range(M)], np.int32)
    J0 = np.ascontiguousarray([table["J0"][first + c * M] for c in range(M)], np.int32)
    cells = int(table["offset"][-1] + table["n"][-1] ** 2)
    psi = np.zeros(cells, np.float32)
    vx = np.zeros(cells, np.float32)
    vy = np.zeros(cells, np.float32)
    lines = np.zeros(int(table["line_offset"][-1] + 2 * table["n"][-1]))
    ph = np.ascontiguousarray(p.psi_hat.astype(np.complex128)).view(np.float64).reshape(-1)
    th = np.ascontiguousarray(list(p.thresh) + [0], np.int32)
    tab = np.ascontiguousarray(table)
    P = ctypes.c_void_p
    harness().band_host_run(P(ph.ctypes.data), p.kmax, len(p.n_cells), P(th.ctypes.data), level,
                            N, n, M, P(I0.ctypes.data), P(J0.ctypes.data), P(tab.ctypes.data),
                            ctypes.c_int64(first), kb1, kb2, P(psi.ctypes.data), P(vx.ctypes.data),
                            P(vy.ctypes.data), P(lines.ctypes.data))
    periodic = all((k1 * n) % N == 0 and (k2 * n) % N == 0
                   for k2, k1 in zip(*np.nonzero(diag)) for k1, k2 in [(k1 - p.kmax, k2 - p.kmax)])
    if not periodic:
        for d in rows:
            o = int(table["offset"][d])
            harness().seam_host(n, ctypes.c_double(float(table["h"][d])), P(psi[o:].ctypes.data),
                                P(vx[o:].ctypes.data), P(vy[o:].ctypes.data))
    return rows, psi, vx, vy, lines, (lv, pt)


CASES = [
    ("two-level", lambda: flowgen.config_two_level_cellular()),
    ("four-level-small", lambda: flowgen.config_four_level_cellular(n=16, lattice=2)),
    ("continuous", lambda: flowgen.config_continuous(seed=2, radius=40, n=16, lattice=2, levels=3)),
]


@pytest.mark.parametrize("name,make", CASES)
def test_band_filter_block_code_matches_oracle(name, make):
    from paper_1510_00451_amd import abi
    p = make()
    table, _, _ = abi.shmm_build_levels(p)
    for level in range(len(p.n_cells)):
        rows, psi, vx, vy, lines, (lv, pt) = run_group(p, table, level)
        mask = oracle.band_mask(lv, pt, level, DIAG)
        for d in rows:
            D = table[d]
            n, o = int(D["n"]), int(D["offset"])
            ref = oracle.synth_patch(p.psi_hat, p.kmax, mask, int(D["N"]), int(D["I0"]), int(D["J0"]), n)
            rvx, rvy, _, _ = oracle.staggered(ref, float(D["h"]))
            scale = max(np.abs(ref).max(), 1e-300)
            got = psi[o:o + n * n].reshape(n, n)
            assert np.abs(got - ref).max() <= 2e-6 * scale + 1e-30, (name, level, d)
            vs = max(np.abs(rvx).max(), np.abs(rvy).max(), 1e-300)
            assert np.abs(vx[o:o + n * n].reshape(n, n) - rvx).max() <= 2e-6 * vs + 1e-30
            assert np.abs(vy[o:o + n * n].reshape(n, n) - rvy).max() <= 2e-6 * vs + 1e-30
            lo = int(D["line_offset"])
            s12 = oracle.line_energies(p.psi_hat, p.kmax, oracle.band_mask(lv, pt, level, OFF12),
                                       int(D["N"]), int(D["I0"]), n, 0)
            s21 = oracle.line_energies(p.psi_hat, p.kmax, oracle.band_mask(lv, pt, level, OFF21),
                                       int(D["N"]), int(D["J0"]), n, 1)
            np.testing.assert_allclose(lines[lo:lo + n], s12, rtol=1e-11, atol=1e-300)
            np.testing.assert_allclose(lines[lo + n:lo + 2 * n], s21, rtol=1e-11, atol=1e-300)
