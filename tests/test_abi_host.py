"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-only bookkeeping reproduces the oracle's domain table bit for bit.
No GPU compute is called here."""
import os
import re

import pytest

import flowgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    from paper_1510_00451_amd import abi
    if not os.path.exists(abi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return abi


def test_library_exports_every_declared_symbol():
    abi = _lib_or_skip()
    header = open(os.path.join(ROOT, "include", "shmm.h")).read()
    declared = set(re.findall(r"^int\s+(shmm_\w+)\s*\(", header, re.M))
    assert declared, "no declarations found"
    lib = abi.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(abi.EXPORTS)


WORKLOADS = [
    lambda: flowgen.config_two_level_cellular(),
    lambda: flowgen.config_four_level_cellular(n=128, lattice=8),
    lambda: flowgen.config_continuous(seed=1, radius=64, n=32, lattice=4, levels=3),
    lambda: [flowgen.config_batched_instance(s) for s in range(6)],
]


@pytest.mark.parametrize("make", WORKLOADS)
def test_build_levels_matches_oracle_bit_for_bit(make):
    abi = _lib_or_skip()
    probs = make()
    table, cells, lines = abi.shmm_build_levels(probs)
    ref = oracle.domain_table(probs)
    assert len(table) == len(ref)
    for row, d in zip(table, ref):
        assert (row["instance"], row["level"], row["cx"], row["cy"], row["n"], row["N"],
                row["I0"], row["J0"], row["parent"], row["offset"], row["line_offset"]) == \
               (d.instance, d.level, d.cx, d.cy, d.n, d.N, d.I0, d.J0, d.parent, d.offset,
                d.line_offset)
        assert row["h"] == d.h      # same double, bit for bit
    assert cells == sum(d.n * d.n for d in ref)
    assert lines == sum(2 * d.n for d in ref)


def test_build_levels_rejects_bad_geometry():
    abi = _lib_or_skip()
    p = flowgen.config_four_level_cellular(n=32, lattice=4)
    p.lattice = [3, 4, 4, 4]
    with pytest.raises(abi.ShmmError) as e:
        abi.shmm_build_levels(p)
    assert e.value.code == abi.SHMM_EINVAL
    q = flowgen.config_four_level_cellular(n=32, lattice=4)
    q.n_cells = [24, 32, 32, 32]
    with pytest.raises(abi.ShmmError):
        abi.shmm_build_levels(q)
    r = flowgen.config_four_level_cellular(n=32, lattice=4)
    r.kappa = 0.0
    with pytest.raises(abi.ShmmError):
        abi.shmm_build_levels(r)
    # the rest of the documented malformed geometry, one field at a time
    bad = [("thresh", lambda t: [t.thresh[1], t.thresh[0]] + list(t.thresh[2:])),   # edges not increasing
           ("dt_frac", lambda t: 0.0), ("dt_frac", lambda t: 1.5),
           ("delta", lambda t: 0.0), ("delta", lambda t: 1.0),
           ("n_global", lambda t: [t.n_global[0] + 1] + list(t.n_global[1:]))]          # origin off the grid
    for field, value in bad:
        t = flowgen.config_four_level_cellular(n=32, lattice=4)
        setattr(t, field, value(t))
        with pytest.raises(abi.ShmmError) as e:
            abi.shmm_build_levels(t)
        assert e.value.code == abi.SHMM_EINVAL, field
        if field in ("thresh", "n_global"):        # geometry the oracle's table refuses too
            with pytest.raises(oracle.BookkeepingError):
                oracle.domain_table(t)
