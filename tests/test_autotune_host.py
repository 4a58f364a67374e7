"""Host-side checks of the autotuner (no GPU): the candidate space per shape, the cache
keys, and that the frozen cache shipped with the package was tuned on the current
library sources (an entry keyed by another source hash is never used)."""
import json
import os

import pytest

from paper_2510_20929_amd import autotune


@pytest.fixture
def mi355x(monkeypatch):
    monkeypatch.setattr(autotune, "_cus", lambda: 256)
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")


def test_candidates_on_chip(mi355x):
    c = autotune.plan_candidates(128, 4, 1, K=2000, split_ok=True, E=1)
    layouts = {(x["variant"], x["recompute"], x["grid"]) for x in c if "mode_groups" not in x and "probe_stage" not in x}
    assert layouts == {(v, r, g) for v in range(5) for r in (0, 1) for g in (0, 512)} | {(5, 1, 0), (6, 1, 0)}
    # the LDS-resident layouts only where they apply (one slice, far field, bilinear patch)
    assert not any(x["variant"] >= 5 for x in autotune.plan_candidates(128, 4, 1, K=2000, lds_ok=False))
    assert not any(x["variant"] >= 5 for x in autotune.plan_candidates(64, 4, 1, K=2000))
    assert not any("mode_groups" in x for x in c)          # 2000 positions fill the GPU
    assert any(x.get("probe_stage") == 1 for x in c)         # one eigenprobe, one slice
    few = autotune.plan_candidates(128, 30, 1, K=50, split_ok=True, E=1)
    groups = sorted({x["mode_groups"] for x in few if "mode_groups" in x})
    assert groups == [min(30, -(-256 // 50)), min(30, -(-512 // 50))]   # one or two items per CU
    assert not any("mode_groups" in x for x in autotune.plan_candidates(128, 30, 1, K=50, split_ok=False))


def test_candidates_four_step_and_multislice(mi355x):
    c = autotune.plan_candidates(512, 15, 1, K=16, split_ok=True, E=3)
    assert {x["variant"] for x in c} == {0, 1}
    assert {x["mode_groups"] for x in c if "mode_groups" in x} == {15}
    assert not any("probe_stage" in x for x in c)            # several eigenprobes are staged anyway
    ms = autotune.plan_candidates(128, 2, 8, K=100, split_ok=True, E=1)
    assert not any("mode_groups" in x or "probe_stage" in x for x in ms)
    assert {(x["variant"], x["recompute"]) for x in ms if x["variant"] >= 5} == {(5, 0), (5, 1)}


def test_shape_key_buckets_positions(mi355x):
    key = autotune.shape_key(128, 4, 1, 1, "poisson", ("pos", "obj", "probe"), 2000)
    assert key.startswith("gfx950|src") and key.endswith("|N128|M4|E1|S1|poisson|obj+pos+probe|K2048")
    for K, b in ((1, 1), (16, 16), (50, 64), (2000, 2048), (6732, 8192)):
        assert autotune.shape_key(64, 1, 1, 1, "amplitude", ("obj",), K).endswith(f"|K{b}")


def test_source_hash_is_stable():
    h = autotune.source_hash()
    assert len(h) == 12 and int(h, 16) >= 0
    autotune._SRC_HASH = None
    assert autotune.source_hash() == h


def test_frozen_cache_matches_the_sources():
    path = os.path.join(os.path.dirname(autotune.__file__), "tune_cache.json")
    with open(path) as fh:
        cache = json.load(fh)
    assert cache, "empty tune cache"
    h = autotune.source_hash()
    stale = [k for k in cache if f"|src{h}|" not in k]
    assert not stale, f"entries tuned on other sources: {stale}"
    headline = [k for k in cache if "|N128|M4|E1|S1|poisson|obj+pos+probe|K2048" in k]
    assert headline and all("tune" in cache[k] and "ms" in cache[k] for k in cache)
