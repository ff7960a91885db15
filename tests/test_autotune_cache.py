"""The autotuner's cache on the CPU: the shipped entries name the fastest
variant they timed, and record / load / apply_cached round-trip through a
JSON file keyed by architecture and patch size (the device's architecture
name stubbed, no GPU call)."""
import json

import numpy as np
import pytest

from paper_1510_00451_amd import autotune


def test_shipped_cache_names_the_fastest_timed_variant():
    cache = autotune.load()
    assert "gfx950" in cache
    for n, e in cache["gfx950"].items():
        assert int(n) in (8, 16, 32, 64, 128, 256)
        assert e["variant"] == int(np.argmin(e["ms"])), n
        assert e["steps"] > 0 and all(t > 0 for t in e["ms"])


class _Ctx:
    """Stands in for the library context: variant counts and the last tune."""

    def __init__(self, counts):
        self.counts = counts
        self.tuned = {}

    def solve_variants(self, n):
        return self.counts.get(n, 1)

    def shmm_ctx_tune(self, n, v):
        self.tuned[n] = v


def test_record_load_apply_round_trip(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "arch", lambda device=0: "gfx950")
    path = str(tmp_path / "tuned.json")
    assert autotune.load(path) == {}
    autotune.record({128: {"variant": 7, "ms": [2.0, 1.0], "steps": 10}}, path=path, workload="w128")
    autotune.record({64: {"variant": 9, "ms": [1.0], "steps": 10}}, path=path)
    with open(path) as f:
        raw = json.load(f)
    assert raw["gfx950"]["128"]["workload"] == "w128" and raw["gfx950"]["64"]["variant"] == 9
    ctx = _Ctx({128: 9, 64: 7})
    got = autotune.apply_cached(ctx, [32, 64, 128], path=path)
    assert ctx.tuned == {128: 7}                 # 64's cached variant is out of range; 32 is not cached
    assert set(got) == {128}
    monkeypatch.setattr(autotune, "arch", lambda device=0: "gfx942")
    ctx = _Ctx({128: 9})
    assert autotune.apply_cached(ctx, [128], path=path) == {} and ctx.tuned == {}


@pytest.mark.parametrize("bad", [-1, 9])
def test_apply_cached_ignores_a_variant_the_library_does_not_offer(tmp_path, monkeypatch, bad):
    monkeypatch.setattr(autotune, "arch", lambda device=0: "gfx950")
    path = str(tmp_path / "tuned.json")
    autotune.save({"gfx950": {"128": {"variant": bad, "ms": [1.0], "steps": 1}}}, path)
    ctx = _Ctx({128: 9})
    assert autotune.apply_cached(ctx, [128], path=path) == {} and ctx.tuned == {}
