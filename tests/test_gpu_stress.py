"""GPU stress tests of the device protocols, each checked against the CPU
oracle: the decoupled look-back with tiles claimed out of order and delayed
publication; per-level work lists too small for the recursion (the overflow
must be reported, nothing written past a list); a tiny depth limit (every
pivot then comes from the largest sample)."""

import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def bqs():
    import paper_1604_06697_amd as bqs_mod

    return bqs_mod


def dev(torch, a):
    hold = {np.dtype(np.uint64): np.int64}.get(a.dtype)
    return torch.from_numpy(np.ascontiguousarray(a.view(hold) if hold is not None else a)).cuda()


@pytest.mark.parametrize("mode", [0, 1])
def test_shuffled_lookback_matches_oracle(torch_mod, bqs, oracle, mode):
    """Tiles take their tiles in reverse order inside windows of 64 tickets
    and pause before publishing: every look-back then waits on tiles claimed
    after it.  Keys (look-back claims) and pairs (always look-back) come
    out as the oracle's."""
    torch = torch_mod
    for fam, n in (("uniform", 1 << 20), ("few_distinct", 3_000_001), ("sorted", 8192 * 64 + 5)):
        a = W.I32_FAMILIES[fam](n, 71)
        ctx = bqs.Context(shuffle=1, lookback=1, mode=mode, small_cutoff=1024)
        note(f"shuffled look-back, mode {mode}, {fam} n={n}")
        t = dev(torch, a)
        ctx.sort(t)
        ctx.synchronize()
        assert np.array_equal(t.cpu().numpy(), oracle.sort(a))
    k, v = W.uniform_u64_pairs(1 << 20, 72)
    ctx = bqs.Context(shuffle=1, mode=mode)
    note(f"shuffled look-back, mode {mode}, pairs")
    tk, tv = dev(torch, k), dev(torch, v.view(np.int32))
    ctx.sort_pairs(tk, tv, key_type="u64")
    ctx.synchronize()
    ko = tk.cpu().numpy().view(np.uint64)
    vo = tv.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(ko, oracle.sort(k))
    assert np.array_equal(np.sort(vo), np.arange(k.size))
    assert np.array_equal(k[vo], ko)


@pytest.mark.parametrize("mode", [0, 1])
def test_list_capacity_overflow_is_reported(torch_mod, bqs, oracle, mode):
    """Per-level lists capped at 4 entries: a recursion that needs more room
    reports BQS_EOVERFLOW (6) and writes nothing past a list; one that fits
    is still sorted; the context is usable afterwards."""
    torch = torch_mod
    ctx = bqs.Context(list_cap=4, mode=mode)
    a = W.uniform_i32(1 << 20, 73)
    note(f"list cap 4, mode {mode}, 2^20 keys")
    t = dev(torch, a)
    with pytest.raises(bqs.BqsError) as e:
        ctx.sort(t)  # host-driven mode reports at once, the default mode at synchronize()
        ctx.synchronize()
    assert e.value.status == 6
    small = W.uniform_i32(5000, 74)
    note(f"list cap 4, mode {mode}, 5000 keys (one small segment)")
    t = dev(torch, small)
    ctx.sort(t)
    ctx.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.sort(small))
    ctx.set_param("list_cap", 0)
    t = dev(torch, a)
    ctx.sort(t)
    ctx.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.sort(a))
    # segments: more level-0 segments than the lists hold
    keys, offsets = W.segmented_i32(50, 75, 4.0, 16.0)
    ctx = bqs.Context(list_cap=4, mode=mode)
    note(f"list cap 4, mode {mode}, 50 segments")
    t = dev(torch, keys)
    with pytest.raises(bqs.BqsError) as e:
        ctx.sort_segments(t, torch.from_numpy(offsets).cuda())
        ctx.synchronize()
    assert e.value.status == 6


def test_depth_limit_override_stays_correct(torch_mod, bqs, oracle):
    """Depth limit 1: from the second level on every pivot is the median of
    the largest sample, whatever the strategy asked for; keys are the
    oracle's and the recursion is no deeper than with the default limit."""
    torch = torch_mod
    for params in ({"depth_limit": 1}, {"depth_limit": 1, "pivot_skew": 16}, {"depth_limit": 1, "pivot_mode": 3}):
        for fam in ("uniform", "sorted", "few_distinct"):
            a = W.I32_FAMILIES[fam](1_000_003, 76)
            ctx = bqs.Context(small_cutoff=512, **params)
            note(f"depth limit {params} {fam}")
            t = dev(torch, a)
            ctx.sort(t)
            ctx.synchronize()
            assert np.array_equal(t.cpu().numpy(), oracle.sort(a))
            assert ctx.stats()["levels"] <= 20
