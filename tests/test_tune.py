"""Autotuner: plan keys, candidate sets and the JSON cache (CPU), and a
tuned run against the oracle (GPU)."""

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def tune():
    from paper_1604_06697_amd import tune as t

    return t


def test_plan_key_rounds_to_powers_of_two(tune):
    assert tune.plan_key(1 << 28, 1, 1, 0) == "dtype1:v0:n2^28:k2^0"
    assert tune.plan_key(1_904_612_016, 20_000, 1, 0) == "dtype1:v0:n2^31:k2^14"
    assert tune.plan_key(3 << 20, 3, 6, 4) == "dtype6:v4:n2^22:k2^2"


def test_candidates_follow_compiled_shapes(tune):
    i32 = tune.candidates(1, 0)
    assert {c["tile_ept"] for c in i32} == {8, 16, 32}
    assert {c["small_cutoff"] for c in i32} == set(tune.CUTOFF_CHOICES)
    assert {c["multiway"] for c in i32} == {0, 1}
    # two-way plans with each pivot strategy, multiway plans with the default
    assert {c["pivot_mode"] for c in i32 if not c["multiway"]} == set(tune.PIVOT_CHOICES)
    assert {c["pivot_mode"] for c in i32 if c["multiway"]} == {0}
    per_step = len(tune.EPT_CHOICES) * len(tune.CUTOFF_CHOICES)
    assert len(i32) == per_step * len(tune.PIVOT_CHOICES) + per_step
    # other key types and pairs compile one tile shape (0 = library default)
    assert {c["tile_ept"] for c in tune.candidates(6, 0)} == {0}
    assert {c["tile_ept"] for c in tune.candidates(1, 4)} == {0}
    assert {c["multiway"] for c in tune.candidates(1, 4)} == {0}


def test_cache_round_trip(tune, tmp_path):
    path = str(tmp_path / "plans.json")
    assert tune.lookup(1 << 20, 1, 1, 0, path) is None
    cache = {tune.plan_key(1 << 20, 1, 1, 0): {"plan": {"tile_ept": 16, "small_cutoff": 2048}, "ms": 1.5}}
    tune.save_cache(cache, path)
    assert tune.lookup(1 << 20, 1, 1, 0, path) == {"tile_ept": 16, "small_cutoff": 2048}
    # same shape class: n within a factor sqrt(2)
    assert tune.lookup(1_200_000, 1, 1, 0, path) == {"tile_ept": 16, "small_cutoff": 2048}
    assert tune.lookup(1 << 24, 1, 1, 0, path) is None
    (tmp_path / "bad.json").write_text("{not json")
    assert tune.load_cache(str(tmp_path / "bad.json")) == {}


def test_tuned_context_applies_cached_plan(tune, tmp_path):
    path = str(tmp_path / "plans.json")
    tune.save_cache({tune.plan_key(1 << 20, 1, 1, 0): {"plan": {"tile_ept": 8, "small_cutoff": 1024,
                                                                "multiway": 1}, "ms": 1.0}}, path)
    ctx = tune.tuned_context(1 << 20, 1, 1, 0, path, graph=1)
    assert ctx.get_param("tile_ept") == 8
    assert ctx.get_param("small_cutoff") == 1024
    assert ctx.get_param("multiway") == 1
    assert ctx.get_param("graph") == 1
    assert tune.tuned_context(1 << 10, 1, 1, 0, path).get_param("tile_ept") == 0


@pytest.mark.gpu
def test_autotune_segments_matches_oracle(tune, oracle, tmp_path):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    keys, offsets = W.segmented_i32(400, 3, 4.0, 15.0)
    print(f"[case] autotune segments n={keys.size}", flush=True)
    t = torch.from_numpy(keys).cuda()
    o = torch.from_numpy(offsets).cuda()
    path = str(tmp_path / "plans.json")
    res = tune.autotune(t, o, graph=True, reps=1, path=path)
    assert res["plan"] in tune.candidates(1, 0)
    assert len(res["table"]) == len(tune.candidates(1, 0))
    ref = oracle.sort_segments(keys, offsets)
    assert np.array_equal(t.cpu().numpy(), ref)
    # the cached plan sorts a fresh copy identically
    ctx = tune.tuned_context(keys.size, 400, 1, 0, path)
    t2 = torch.from_numpy(keys).cuda()
    ctx.sort_segments(t2, o)
    torch.cuda.synchronize()
    assert np.array_equal(t2.cpu().numpy(), ref)
