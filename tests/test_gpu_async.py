"""GPU tests of the call contract: calls only enqueue (the host gets control
back while the sort still runs), device-detected errors are latched and
returned by the context's synchronisation, the NaN check mode, and the
single-workgroup tail that finishes whatever recursion the enqueued levels
did not reach.  Sorted keys are compared with the CPU oracle throughout."""

import sys
import time

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


_HOLD = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32}
_KT = {np.dtype(np.int32): "i32", np.dtype(np.float32): "f32", np.dtype(np.float64): "f64",
       np.dtype(np.uint64): "u64"}


def to_dev(torch, a):
    hold = _HOLD.get(a.dtype)
    return torch.from_numpy(np.ascontiguousarray(a.view(hold) if hold is not None else a)).cuda()


def host(t, dtype):
    return t.cpu().numpy().view(dtype)


def test_call_returns_before_the_stream_is_idle(torch_mod, bqs, oracle):
    """A 2^27-key sort: the call returns while the stream still runs it, and
    after the stream has passed it the keys are the oracle's."""
    torch = torch_mod
    a = W.uniform_i32(1 << 27, 21)
    expect = oracle.sort(a)
    ctx = bqs.Context()
    t = to_dev(torch, a)
    warm = t.clone()
    ctx.sort(warm)  # first call: code objects, pinned slots
    ctx.synchronize()
    del warm
    torch.cuda.synchronize()
    note("async 2^27 int32: call time against completion time")
    t0 = time.perf_counter()
    ctx.sort(t)
    t_call = time.perf_counter() - t0
    busy = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    t_done = time.perf_counter() - t0
    ctx.synchronize()
    print(f"call {t_call * 1e3:.3f} ms, sorted after {t_done * 1e3:.3f} ms", flush=True)
    assert busy, "the stream was idle when the call returned"
    assert t_call < 0.5 * t_done
    assert np.array_equal(host(t, np.int32), expect)
    st = ctx.stats()
    assert st["partitioned_keys"] >= a.size and st["small_sorted_keys"] > 0


def test_calls_pipeline_on_one_context(torch_mod, bqs, oracle):
    """Several calls enqueued back to back on one context and one stream
    (different inputs and sizes) each come out sorted."""
    torch = torch_mod
    ctx = bqs.Context()
    arrays = [W.uniform_i32(n, 30 + i) for i, n in enumerate((1 << 20, 300_001, 1 << 22, 17, 9000))]
    devs = [to_dev(torch, a) for a in arrays]
    note("five calls enqueued before one synchronisation")
    for d in devs:
        ctx.sort(d)
    ctx.synchronize()
    for a, d in zip(arrays, devs):
        assert np.array_equal(host(d, np.int32), oracle.sort(a))


def test_bad_offsets_latched_until_synchronize(torch_mod, bqs):
    """Malformed offsets are found on the device: the call returns OK, the
    error comes from synchronize(), and the latch is cleared after it."""
    torch = torch_mod
    ctx = bqs.Context()
    keys = to_dev(torch, W.uniform_i32(1000, 0))
    bad = torch.tensor([0, 600, 500, 1000], dtype=torch.int64, device="cuda")
    note("bad offsets, asynchronous")
    before = keys.clone()
    ctx.sort_segments(keys, bad)
    with pytest.raises(bqs.BqsError) as e:
        ctx.synchronize()
    assert e.value.status == 1
    assert torch.equal(keys, before)  # nothing ran
    ctx.synchronize()  # cleared
    good = torch.tensor([0, 500, 600, 1000], dtype=torch.int64, device="cuda")
    ctx.sort_segments(keys, good)
    ctx.synchronize()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_nan_check_mode(torch_mod, bqs, oracle, dtype):
    """Check mode: an input with a NaN is reported as BQS_ENAN (5); without
    a NaN the sort is the oracle's; without check mode no error is raised."""
    torch = torch_mod
    a = W.normal_f64(200_003, 5).astype(dtype)
    ctx = bqs.Context(check_nan=1)
    note(f"check mode, no NaN, {dtype.__name__}")
    t = to_dev(torch, a)
    ctx.sort(t, key_type=_KT[np.dtype(dtype)])
    ctx.synchronize()
    assert np.array_equal(host(t, dtype).view(f"u{a.itemsize}"), oracle.sort(a).view(f"u{a.itemsize}"))
    for pos in (0, 123_457, a.size - 1):
        b = a.copy()
        b[pos] = np.nan
        note(f"check mode, NaN at {pos}, {dtype.__name__}")
        t = to_dev(torch, b)
        ctx.sort(t, key_type=_KT[np.dtype(dtype)])
        with pytest.raises(bqs.BqsError) as e:
            ctx.synchronize()
        assert e.value.status == 5
        # found before anything moved: the keys are as they were
        assert np.array_equal(host(t, dtype).view(f"u{a.itemsize}"), b.view(f"u{a.itemsize}"))
    # a negative NaN and a signalling NaN pattern are NaNs too
    b = a.copy()
    b.view(f"u{a.itemsize}")[7] = (0xFFF0000000000001 if a.itemsize == 8 else 0xFF800001)
    t = to_dev(torch, b)
    ctx.sort(t, key_type=_KT[np.dtype(dtype)])
    with pytest.raises(bqs.BqsError) as e:
        ctx.synchronize()
    assert e.value.status == 5
    # infinities are keys, not NaNs
    b = a.copy()
    b[3], b[4] = np.inf, -np.inf
    t = to_dev(torch, b)
    ctx.sort(t, key_type=_KT[np.dtype(dtype)])
    ctx.synchronize()
    assert np.array_equal(host(t, dtype).view(f"u{a.itemsize}"), oracle.sort(b).view(f"u{a.itemsize}"))
    # pairs and segments are checked as well
    k = to_dev(torch, a.copy())
    k.view(torch.int64 if a.itemsize == 8 else torch.int32)[11] = -1  # all ones: a NaN
    v = torch.arange(a.size, dtype=torch.int32, device="cuda")
    ctx.sort_pairs(k, v, key_type=_KT[np.dtype(dtype)])
    with pytest.raises(bqs.BqsError) as e:
        ctx.synchronize()
    assert e.value.status == 5


def test_tail_finishes_what_the_enqueued_levels_leave(torch_mod, bqs, oracle):
    """Only one or two levels enqueued: the single-workgroup tail runs the
    rest of the recursion (for the multiway step it first gives the listed
    segments two-way tiles); keys are the oracle's either way."""
    torch = torch_mod
    cases = [("uniform", W.uniform_i32(300_000, 41), {}),
             ("few distinct", W.few_distinct_i32(300_000, 42), {}),
             ("pairs", None, {}),
             ("multiway", W.uniform_i32(400_000, 43), {"multiway": 1}),
             ("multiway small cutoff", W.uniform_i32(400_000, 44), {"multiway": 1, "small_cutoff": 256}),
             ("segments", None, {})]
    for name, a, params in cases:
        for levels in (1, 2):
            ctx = bqs.Context(enqueue_levels=levels, **params)
            note(f"tail: {name}, {levels} enqueued levels")
            if name == "pairs":
                k, v = W.uniform_u64_pairs(200_000, 45)
                tk, tv = to_dev(torch, k), to_dev(torch, v)
                ctx.sort_pairs(tk, tv, key_type="u64")
                ctx.synchronize()
                ko, vo = host(tk, np.uint64), host(tv, np.uint32).astype(np.int64)
                assert np.array_equal(ko, oracle.sort(k))
                assert np.array_equal(np.sort(vo), np.arange(k.size))
                assert np.array_equal(k[vo], ko)
            elif name == "segments":
                keys, offsets = W.segmented_i32(300, 46, 4.0, 17.0)
                t = to_dev(torch, keys)
                ctx.sort_segments(t, torch.from_numpy(offsets).cuda())
                ctx.synchronize()
                assert np.array_equal(host(t, np.int32), oracle.sort_segments(keys, offsets))
            else:
                t = to_dev(torch, a)
                ctx.sort(t)
                ctx.synchronize()
                assert np.array_equal(host(t, np.int32), oracle.sort(a))
            st = ctx.stats()
            assert st["partition_launches"] == levels and st["levels"] >= 1


def test_depth_follows_the_last_call(torch_mod, bqs, oracle):
    """Skewed pivots make a deep recursion: the first call's estimate falls
    short and the tail finishes it; the next call of the same shape enqueues
    the depth the first one needed.  Both sorts are the oracle's."""
    torch = torch_mod
    a = W.uniform_i32(1 << 20, 47)
    expect = oracle.sort(a)
    # look-back claims lay every level out the same way on every run, so the
    # recursion (and its depth) repeats exactly
    ctx = bqs.Context(pivot_skew=16, small_cutoff=512, lookback=1)
    for rep in range(2):
        note(f"skewed pivots, call {rep}")
        t = to_dev(torch, a)
        ctx.sort(t)
        ctx.synchronize()
        assert np.array_equal(host(t, np.int32), expect)
        st = ctx.stats()
        if rep == 0:
            first = st
        else:
            assert st["levels"] == first["levels"]
            assert st["partition_launches"] >= st["levels"] + 1


def test_segment_completion_clock(torch_mod, bqs, oracle):
    """bqs_ctx_set_segment_ticks: every segment's completion time is at or
    after the call's start, segments of at most one key complete at the
    start, the latest completion is no later than the host saw the call end,
    and the keys are the oracle's -- for the default, in-place, multiway,
    host-driven, graph and persistent forms."""
    torch = torch_mod
    keys, offsets = W.segmented_i32(300, 48, 0.0, 17.0)
    sizes = np.diff(offsets)
    k = sizes.size
    expect = oracle.sort_segments(keys, offsets)
    off = torch.from_numpy(offsets).cuda()
    forms = [("default", {}), ("in-place", {"inplace": 1}), ("multiway", {"multiway": 1}),
             ("host-driven", {"mode": bqs.MODE_LEVELS}), ("graph", {"graph": 1}),
             ("persistent", {"mode": bqs.MODE_PERSISTENT})]
    for name, params in forms:
        ctx = bqs.Context(**params)
        ticks = torch.full((k + 1,), -1, dtype=torch.int64, device="cuda")
        ctx.set_segment_ticks(ticks)
        for rep in range(2 if params.get("graph") else 1):
            note(f"completion clock, {name}, call {rep}")
            t = to_dev(torch, keys)
            ticks.fill_(-1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sort_segments(t, off)
            ctx.synchronize()
            torch.cuda.synchronize()
            wall_ticks = (time.perf_counter() - t0) * 1e8  # 100 MHz
            assert np.array_equal(host(t, np.int32), expect), name
            tk = ticks.cpu().numpy()
            start = tk[k]
            assert start > 0, name
            done = tk[:k]
            assert np.all(done >= start), (name, np.flatnonzero(done < start)[:8])
            assert np.all(done[sizes <= 1] == start), name
            assert np.all(done[sizes > 4096] > start), name
            assert done.max() - start <= wall_ticks, (name, done.max() - start, wall_ticks)
        # too short an array is an argument error
        ctx.set_segment_ticks(ticks[:k])
        with pytest.raises(bqs.BqsError):
            ctx.sort_segments(to_dev(torch, keys), off)
        ctx.set_segment_ticks(None)
        ctx.close()
