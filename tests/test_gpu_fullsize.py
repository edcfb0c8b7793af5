"""Full-size parity: the benchmark's workloads at their real sizes, sorted by
the HIP library in the launch configuration the benchmark times, compared
element by element with the CPU oracle on the same seeded input.

* 2^28 int32 keys in each of the five single-array distributions;
* 2^27 float64 keys (uniform, normal, sorted with 1 % random pair swaps) and
  2^26 uint64 keys with uint32 payloads (payload = original index);
* 20,000 int32 arrays of log-uniform sizes in [16, 2^20] (about 1.9e9 keys),
  sorted by one segmented call with the default plan and by graph replays of
  the multiway plan, against the oracle's per-segment sort;
* 2^25 + 4097 uint32, float32 and int64 keys, large enough for every
  per-level partition tile size, in the default, graph and host-driven
  modes.

The oracle is single-threaded; independent oracle sorts run in threads (its
ctypes calls release the interpreter lock), so a test takes seconds.
"""

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N28 = 1 << 28


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


@pytest.fixture(scope="module")
def pool():
    with ThreadPoolExecutor(max_workers=16) as ex:
        yield ex


_KT = {np.dtype(np.int32): "i32", np.dtype(np.float64): "f64", np.dtype(np.uint64): "u64",
       np.dtype(np.uint32): "u32", np.dtype(np.float32): "f32", np.dtype(np.int64): "i64"}
_HOLD = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32}


def to_dev(torch, a):
    hold = _HOLD.get(a.dtype)
    return torch.from_numpy(a.view(hold) if hold is not None else a).cuda()


def first_difference(got, expect):
    u = f"u{got.itemsize}"
    diff = np.flatnonzero(got.view(u) != expect.view(u))
    return f"{diff.size} positions differ, first at {diff[:8]}"


def gpu_sort_host(torch, ctx, a):
    t = to_dev(torch, a)
    ctx.sort(t, key_type=_KT[a.dtype])
    torch.cuda.synchronize()
    out = t.cpu().numpy().view(a.dtype)
    del t
    return out


SINGLE_I32 = ("uniform", "sorted", "reverse", "few_distinct", "all_equal")


@pytest.mark.parametrize("family", SINGLE_I32)
def test_2p28_int32_matches_oracle(torch_mod, bqs, oracle, pool, family):
    """2^28 int32 keys, one of the five distributions of the single-array
    benchmark, default plan: bit for bit the oracle's output."""
    a = W.I32_FAMILIES[family](N28, 0)
    expect = pool.submit(oracle.sort, a)
    note(f"2^28 int32 {family}")
    ctx = bqs.Context(timing=2)  # the benchmark's context
    got = gpu_sort_host(torch_mod, ctx, a)
    ctx.close()
    ref = expect.result()
    assert np.array_equal(got, ref), first_difference(got, ref)


@pytest.mark.parametrize("family", ("uniform", "normal", "sorted_swaps"))
def test_2p27_float64_matches_oracle(torch_mod, bqs, oracle, pool, family):
    """2^27 float64 keys (uniform [0, 1), normal(0, 1), sorted with 1 % random
    pair swaps): bit for bit the oracle's output."""
    a = W.F64_FAMILIES[family](N28 // 2, 1)
    expect = pool.submit(oracle.sort, a)
    note(f"2^27 float64 {family}")
    got = gpu_sort_host(torch_mod, bqs.default_context(), a)
    ref = expect.result()
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), first_difference(got, ref)


def test_2p26_u64_u32_pairs_match_oracle(torch_mod, bqs, oracle, pool):
    """2^26 uint64 keys with uint32 payloads (payload = original index): keys
    bit for bit the oracle's, payloads a permutation of the indexes, and
    every payload next to its own key."""
    torch = torch_mod
    n = N28 // 4
    k, v = W.uniform_u64_pairs(n, 1)
    expect = pool.submit(oracle.sort, k)
    note("2^26 u64/u32 pairs")
    tk, tv = to_dev(torch, k), to_dev(torch, v)
    bqs.sort_pairs(tk, tv, key_type="u64")
    torch.cuda.synchronize()
    ko = tk.cpu().numpy().view(np.uint64)
    vo = tv.cpu().numpy().view(np.uint32).astype(np.int64)
    del tk, tv
    ref = expect.result()
    assert np.array_equal(ko, ref), first_difference(ko, ref)
    assert np.array_equal(np.sort(vo), np.arange(n))
    assert np.array_equal(k[vo], ko)


@pytest.mark.parametrize("mode", ["default", "graph", "levels"])
def test_per_level_tiles_match_oracle(torch_mod, bqs, oracle, pool, mode):
    """Arrays large enough for every partition tile size of the enqueued
    levels (16384-key tiles on the first levels, 4096-key tiles once a level
    can hold 256 segments, 8192 in between and on the last levels): uint32,
    float32 and int64 keys of a ragged length, bit for bit the oracle's.
    Graph mode replays its captured levels twice on refilled buffers; the
    host-driven mode keeps one tile size, the same keys."""
    n = (1 << 25) + 4097
    cases = [np.random.default_rng(31).integers(0, 2**32, n, dtype=np.uint32),
             W.normal_f64(n, 32).astype(np.float32),
             W.few_distinct_i32(n, 33).astype(np.int64) * 7919 - (1 << 40)]
    expects = [pool.submit(oracle.sort, a) for a in cases]
    plan = {"default": {}, "graph": {"graph": 1}, "levels": {"mode": bqs.MODE_LEVELS}}[mode]
    torch = torch_mod
    for a, expect in zip(cases, expects):
        ctx = bqs.Context(**plan)
        ref = expect.result()
        src = to_dev(torch, a)
        t = torch.empty_like(src)
        for rep in range(2 if mode == "graph" else 1):
            note(f"per-level tiles, {mode}, {a.dtype} n={n}, call {rep}")
            t.copy_(src)
            ctx.sort(t, key_type=_KT[a.dtype])
            torch.cuda.synchronize()
            got = t.cpu().numpy().view(a.dtype)
            assert np.array_equal(got.view(f"u{a.itemsize}"), ref.view(f"u{a.itemsize}")), first_difference(got, ref)
        ctx.close()
        del src, t


def oracle_segments_parallel(oracle, pool, keys, offsets, chunks=16):
    """The oracle's per-segment sort, with the segments split into `chunks`
    contiguous groups sorted in parallel threads."""
    k = offsets.size - 1
    cuts = np.linspace(0, k, chunks + 1).astype(np.int64)
    out = np.empty_like(keys)

    def part(i):
        s0, s1 = int(cuts[i]), int(cuts[i + 1])
        lo, hi = int(offsets[s0]), int(offsets[s1])
        out[lo:hi] = oracle.sort_segments(keys[lo:hi], offsets[s0:s1 + 1] - lo)

    list(pool.map(part, range(chunks)))
    return out


def test_batched_20000_arrays_match_oracle(torch_mod, bqs, oracle, pool):
    """The batched workload at full size (20,000 int32 arrays, sizes
    log-uniform in [16, 2^20], about 1.9e9 keys, int64 offsets): one
    segmented call with the default plan, and two graph replays of the
    multiway plan the autotuner picks for this shape, each bit for bit the
    oracle's per-segment sort."""
    torch = torch_mod
    keys, offsets = W.segmented_i32(20_000, 7)
    expect = pool.submit(oracle_segments_parallel, oracle, pool, keys, offsets)
    off_d = torch.from_numpy(offsets).cuda()
    pristine = torch.from_numpy(keys).cuda()
    work = torch.empty_like(pristine)
    plans = [("default", {}), ("multiway graph", {"graph": 1, "multiway": 1, "small_cutoff": 8192})]
    results = []
    for name, plan in plans:
        ctx = bqs.Context(**plan)
        for rep in range(2 if plan.get("graph") else 1):
            note(f"batched 20000 arrays, {name} plan, call {rep}")
            work.copy_(pristine)
            ctx.sort_segments(work, off_d)
            torch.cuda.synchronize()
            results.append((f"{name} call {rep}", work.cpu().numpy()))
        ctx.close()
    del work, pristine, off_d
    ref = expect.result()
    for name, got in results:
        assert np.array_equal(got, ref), f"{name}: {first_difference(got, ref)}"
