"""GPU parity of the in-place step (BQS_PARAM_INPLACE = 1): keys and payloads
never leave the caller's buffers; every sort is compared with the CPU oracle
element by element.  Sizes straddle the 4096-key tile (ragged last tiles,
boundaries inside a tile), distributions cover the equal-key paths (a
segment of one value, a pivot with many copies, the pivot as the smallest
key), and the call forms cover keys, pairs, segments, records, the
host-driven mode, graph replays and the one-workgroup tail."""

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


_KT = {np.dtype(np.int32): "i32", np.dtype(np.uint32): "u32", np.dtype(np.float32): "f32",
       np.dtype(np.int64): "i64", np.dtype(np.uint64): "u64", np.dtype(np.float64): "f64"}
_HOLD = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}


def to_dev(torch, a):
    hold = _HOLD.get(a.dtype)
    return torch.from_numpy(np.ascontiguousarray(a.view(hold) if hold is not None else a)).cuda()


def host(t, dtype):
    return t.cpu().numpy().view(dtype)


def same_bits(got, expect):
    u = f"u{got.itemsize}"
    diff = np.flatnonzero(got.view(u) != expect.view(u))
    assert diff.size == 0, f"{diff.size} positions differ, first at {diff[:8]}"


def sort_inplace(torch, ctx, a):
    t = to_dev(torch, a)
    ptr = t.data_ptr()
    ctx.sort(t, key_type=_KT[a.dtype])
    ctx.synchronize()
    assert t.data_ptr() == ptr
    return host(t, a.dtype)


SIZES = [2, 3, 4095, 4096, 4097, 8191, 8193, 16385, 16384 * 3 + 7, 100_003, 1 << 20]


@pytest.mark.parametrize("family", ["uniform", "sorted", "reverse", "few_distinct", "all_equal"])
def test_int32_families_match_oracle(torch_mod, bqs, oracle, family):
    ctx = bqs.Context(inplace=1)
    for n in SIZES:
        a = W.I32_FAMILIES[family](n, n + 3)
        note(f"in-place int32 {family} n={n}")
        same_bits(sort_inplace(torch_mod, ctx, a), oracle.sort(a))


@pytest.mark.parametrize("family", ["permutation", "uniform_sqrt", "half_zero_one", "random_zero_one",
                                    "neighbour_swaps"])
def test_paper_families_match_oracle(torch_mod, bqs, oracle, family):
    gen = {**W.I32_FAMILIES, **W.I32_EXTRA_FAMILIES}[family]
    ctx = bqs.Context(inplace=1)
    for n in (50_000, 1_000_003):
        a = gen(n, 5)
        note(f"in-place paper family {family} n={n}")
        same_bits(sort_inplace(torch_mod, ctx, a), oracle.sort(a))


def test_key_types_and_special_values(torch_mod, bqs, oracle):
    """Float keys with +-0, +-inf, subnormals and extremes; every integer
    width.  Bit-exact (so -0.0 precedes +0.0)."""
    ctx = bqs.Context(inplace=1)
    for n in (5000, 300_001):
        f = W.special_f64(n, 9)
        cases = [f, f.astype(np.float32), W.uniform_i32(n, 10).astype(np.int64) * 7919,
                 np.random.default_rng(11).integers(0, 2**64 - 1, n, dtype=np.uint64),
                 np.random.default_rng(12).integers(0, 2**32 - 1, n, dtype=np.uint32),
                 W.normal_f64(n, 13)]
        for a in cases:
            note(f"in-place {a.dtype} n={n}")
            same_bits(sort_inplace(torch_mod, ctx, a), oracle.sort(a))


@pytest.mark.parametrize("cutoff", [256, 1024])
def test_deep_recursion_and_small_cutoffs(torch_mod, bqs, oracle, cutoff):
    """Small cutoffs make many levels with many small segments of a few
    tiles each (boundaries inside tiles at every level)."""
    for params in ({}, {"pivot_mode": 3}, {"pivot_skew": 8}, {"depth_limit": 1}):
        ctx = bqs.Context(inplace=1, small_cutoff=cutoff, **params)
        for fam in ("uniform", "few_distinct"):
            a = W.I32_FAMILIES[fam](700_001, 14)
            note(f"in-place cutoff {cutoff} {params} {fam}")
            same_bits(sort_inplace(torch_mod, ctx, a), oracle.sort(a))


def test_pairs_match_oracle(torch_mod, bqs, oracle):
    """Pairs (u64 keys with u32 payloads, i32 keys with u64 payloads, tied
    keys): keys bit for bit the oracle's, payloads a permutation, each next to
    its own key; two runs give the same payload order."""
    torch = torch_mod
    ctx = bqs.Context(inplace=1)
    for n in (4097, 100_003, 1 << 20):
        for name, (k, v) in (("u64/u32", W.uniform_u64_pairs(n, 15)), ("tied u64/u32", W.tied_u64_pairs(n, 16)),
                             ("i32/u64", (W.few_distinct_i32(n, 17), np.arange(n, dtype=np.uint64)))):
            note(f"in-place pairs {name} n={n}")
            outs = []
            for _ in range(2):
                tk, tv = to_dev(torch, k), to_dev(torch, v)
                ctx.sort_pairs(tk, tv, key_type=_KT[k.dtype])
                ctx.synchronize()
                outs.append((host(tk, k.dtype), host(tv, v.dtype).astype(np.int64)))
            ko, vo = outs[0]
            same_bits(ko, oracle.sort(k))
            assert np.array_equal(np.sort(vo), np.arange(n))
            same_bits(k[vo], ko)
            assert np.array_equal(outs[1][1], vo)  # deterministic


def test_segments_match_oracle(torch_mod, bqs, oracle):
    """Segmented keys and pairs (log-uniform sizes, empty and one-key
    segments included) against the oracle's per-segment sort."""
    torch = torch_mod
    ctx = bqs.Context(inplace=1)
    keys, offsets = W.segmented_i32(400, 18, 0.0, 17.0)
    note(f"in-place segments k=400 n={keys.size}")
    t = to_dev(torch, keys)
    ctx.sort_segments(t, torch.from_numpy(offsets).cuda())
    ctx.synchronize()
    same_bits(host(t, np.int32), oracle.sort_segments(keys, offsets))
    n = keys.size
    k = W.tied_u64_pairs(n, 19)[0]
    v = np.arange(n, dtype=np.uint32)
    note(f"in-place segment pairs n={n}")
    tk, tv = to_dev(torch, k), to_dev(torch, v)
    ctx.sort_segments_pairs(tk, tv, torch.from_numpy(offsets).cuda(), key_type="u64")
    ctx.synchronize()
    ko, vo = host(tk, np.uint64), host(tv, np.uint32).astype(np.int64)
    same_bits(ko, oracle.sort_segments(k, offsets))
    assert np.array_equal(np.sort(vo), np.arange(n))
    for i in range(offsets.size - 1):
        lo, hi = offsets[i], offsets[i + 1]
        assert np.all((vo[lo:hi] >= lo) & (vo[lo:hi] < hi))
    same_bits(k[vo], ko)


def test_records_match_oracle(torch_mod, bqs, oracle):
    torch = torch_mod
    ctx = bqs.Context(inplace=1)
    r = np.random.default_rng(20).integers(-2**31, 2**31 - 1, size=(200_003, 21), dtype=np.int32)
    r[:, 0] = np.random.default_rng(21).integers(-500, 500, size=r.shape[0])
    note("in-place records")
    got = ctx.sort_records(torch.from_numpy(r).cuda())
    ctx.synchronize()
    g = got.cpu().numpy()
    assert np.array_equal(g[:, 0], oracle.sort_records(r)[:, 0])
    assert np.array_equal(np.unique(g, axis=0), np.unique(r, axis=0))


def test_modes_graph_and_tail(torch_mod, bqs, oracle):
    """The host-driven mode, graph replays (refilled buffer), and one or two
    enqueued levels with the one-workgroup tail doing the rest."""
    torch = torch_mod
    a = W.uniform_i32(600_001, 22)
    b = W.few_distinct_i32(600_001, 23)
    expect_a, expect_b = oracle.sort(a), oracle.sort(b)
    ctx = bqs.Context(inplace=1, mode=bqs.MODE_LEVELS)
    note("in-place host-driven levels")
    same_bits(sort_inplace(torch, ctx, a), expect_a)
    same_bits(sort_inplace(torch, ctx, b), expect_b)
    ctx = bqs.Context(inplace=1, graph=1)
    t = to_dev(torch, a)
    for rep in range(3):
        note(f"in-place graph replay {rep}")
        t.copy_(to_dev(torch, a if rep != 1 else b))
        ctx.sort(t)
        ctx.synchronize()
        same_bits(host(t, np.int32), expect_a if rep != 1 else expect_b)
    for levels in (1, 2):
        for arr, expect in ((a, expect_a), (b, expect_b)):
            ctx = bqs.Context(inplace=1, enqueue_levels=levels, small_cutoff=512)
            note(f"in-place tail after {levels} levels")
            same_bits(sort_inplace(torch, ctx, arr), expect)
        k, v = W.tied_u64_pairs(300_000, 24)
        ctx = bqs.Context(inplace=1, enqueue_levels=levels)
        note(f"in-place pairs tail after {levels} levels")
        tk, tv = to_dev(torch, k), to_dev(torch, v)
        ctx.sort_pairs(tk, tv, key_type="u64")
        ctx.synchronize()
        ko, vo = host(tk, np.uint64), host(tv, np.uint32).astype(np.int64)
        same_bits(ko, oracle.sort(k))
        assert np.array_equal(np.sort(vo), np.arange(k.size))


def test_persistent_mode_is_rejected(torch_mod, bqs):
    torch = torch_mod
    ctx = bqs.Context(inplace=1, mode=bqs.MODE_PERSISTENT)
    t = to_dev(torch, W.uniform_i32(100_000, 25))
    note("in-place persistent rejected")
    with pytest.raises(bqs.BqsError) as e:
        ctx.sort(t)
        ctx.synchronize()
    assert e.value.status == 1


def test_full_size_2p28_matches_oracle(torch_mod, bqs, oracle):
    """2^28 uniform int32 keys in place, bit for bit the oracle's; the
    workspace is a small fraction of the default one."""
    torch = torch_mod
    n = 1 << 28
    a = W.uniform_i32(n, 0)
    ctx = bqs.Context(inplace=1)
    ws = bqs.lib.bqs_workspace_bytes
    assert ws(ctx._h, n, bqs.I32, 0, 1) < 0.1 * ws(None, n, bqs.I32, 0, 1)
    note("in-place 2^28 int32 uniform")
    got = sort_inplace(torch, ctx, a)
    same_bits(got, oracle.sort(a))
