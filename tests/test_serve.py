"""Serving loop: batching rule, HBM budget and traces on the CPU; on the
GPU, every request of a mixed trace gives the same result in the mix as
sorted alone."""

import threading
from collections import deque

import numpy as np
import pytest


@pytest.fixture(scope="module")
def serve():
    from paper_1604_06697_amd import serve as s

    return s


def test_form_batch_takes_oldest_kind_in_arrival_order(serve):
    R = serve.Request
    w = deque([R(0, "f64", 10, 0.0), R(1, "i32", 5, 0.1), R(2, "f64", 7, 0.2),
               R(3, "pairs", 3, 0.3), R(4, "f64", 100, 0.4), R(5, "f64", 1, 0.5)])
    b = serve.form_batch(w, max_keys=20)
    # f64 requests 0 and 2 fit (17 keys), 4 would exceed 20, 5 still fits
    assert [r.rid for r in b] == [0, 2, 5]
    # the others keep their order
    assert [r.rid for r in w] == [1, 3, 4]
    b = serve.form_batch(w, max_keys=20)
    assert [r.rid for r in b] == [1]
    # an oversized oldest request is taken alone
    b = serve.form_batch(w, max_keys=1)
    assert [r.rid for r in b] == [3]
    assert [r.rid for r in w] == [4]
    assert serve.form_batch(deque(), 10) == []


def test_form_batch_stops_where_the_ring_slots_do_not_follow(serve):
    R = serve.Request
    # ring positions: 0, 10 follow each other; 17 does not follow 10 + 5 = 15
    # (a wrap or another type's slots in between); 15 does
    w = deque([R(0, "i32", 10, 0.0, pos=0), R(1, "i32", 5, 0.1, pos=10), R(2, "i32", 3, 0.2, pos=17),
               R(3, "i32", 4, 0.3, pos=15)])
    b = serve.form_batch(w, max_keys=100)
    assert [r.rid for r in b] == [0, 1, 3]
    assert [r.rid for r in w] == [2]


def test_ring_allocates_in_order_wraps_and_reuses_released_space(serve):
    ring = serve.Ring(100)
    a = ring.alloc(40)
    b = ring.alloc(40)
    assert (a, b) == (0, 40)
    assert ring.try_alloc(30) is None          # 20 free at the end, 0 at the start
    ring.release(b)                            # out of order: the oldest is still live
    assert ring.used == 40 and ring.try_alloc(30) is None
    ring.release(a)                            # now everything is free again
    assert ring.used == 0
    c = ring.alloc(70)
    assert c == 0
    d = ring.try_alloc(30)
    assert d == 70
    ring.release(c)
    e = ring.alloc(50)                         # wraps to the start, before d
    assert e == 0
    assert ring.try_alloc(21) is None          # 20 free between e and d
    f = ring.alloc(20)
    assert f == 50
    assert ring.peak == 100
    with pytest.raises(ValueError):
        ring.alloc(101)


def test_ring_alloc_blocks_until_release(serve):
    ring = serve.Ring(100)
    a = ring.alloc(60)
    got = []
    t = threading.Thread(target=lambda: got.append(ring.alloc(50)))
    t.start()
    t.join(0.1)
    assert not got
    ring.release(a)
    t.join(2.0)
    assert got == [0] and ring.used == 50 and ring.peak == 60


def test_footprint_is_the_request_in_the_arena(serve):
    assert serve.footprint("i32", 1000) == 1000 * 4
    assert serve.footprint("f64", 1000) == 1000 * 8
    assert serve.footprint("pairs", 1000) == 1000 * 12


def test_trace_shape(serve):
    tr = serve.make_trace(20000, qps=1000.0, seed=3)
    sizes = np.array([r.n for r in tr])
    assert sizes.min() >= 2 ** 10 and sizes.max() <= 2 ** 24
    # log-uniform: the median is near 2^17
    assert 2 ** 16 < np.median(sizes) < 2 ** 18
    kinds = np.array([r.kind for r in tr])
    for k, p in zip(serve.KINDS, (0.5, 0.3, 0.2)):
        assert abs(np.mean(kinds == k) - p) < 0.02
    arr = np.array([r.arrival for r in tr])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    # Poisson: mean gap 1/qps
    assert abs(np.mean(np.diff(arr)) - 1e-3) < 5e-5
    # same seed, same trace
    tr2 = serve.make_trace(20000, qps=1000.0, seed=3)
    assert [(r.n, r.kind, r.arrival) for r in tr2] == [(r.n, r.kind, r.arrival) for r in tr]


def test_latency_summary_nearest_rank(serve):
    R = serve.Request
    tr = []
    for i in range(100):
        r = R(i, "i32", 10, 0.0)
        r.done = (i + 1) * 1e-3
        tr.append(r)
    s = serve.latency_summary(tr, makespan=0.1)
    assert s["p50_ms"] == 50.0 and s["p99_ms"] == 99.0
    assert s["keys"] == 1000 and s["requests"] == 100 and s["makespan_s"] == 0.1


@pytest.mark.gpu
@pytest.mark.parametrize("params", [None, {"inplace": 1}], ids=["default", "inplace"])
def test_results_same_alone_and_in_the_mix(serve, oracle, params):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_06697_amd as bqs

    trace = serve.make_trace(240, qps=4000.0, seed=5, lo_exp=10, hi_exp=17)
    print(f"[case] serving mix of {len(trace)} requests, params {params}", flush=True)
    trace, makespan, svc = serve.run_service(trace, budget_bytes=1 << 30, workers=3, seed_base=100,
                                             keep_inputs=[r.rid for r in trace], params=params)
    assert svc.batches < len(trace)  # requests were batched together
    assert svc.peak_bytes() <= 1 << 30
    alone = bqs.Context()
    for r in trace:
        assert r.done >= r.arrival
        k = r.input_keys.clone()
        if r.kind == "pairs":
            v = r.input_vals.clone()
            alone.sort_pairs(k, v, key_type="u64")
            torch.cuda.synchronize()
            assert torch.equal(r.out_keys, k), f"request {r.rid}"
            # payload = index into the request's input: every payload moved with its key
            assert torch.equal(r.input_keys[r.out_vals.long()], r.out_keys), f"request {r.rid}"
        else:
            alone.sort(k)
            torch.cuda.synchronize()
            assert torch.equal(r.out_keys, k), f"request {r.rid}"
        if r.rid % 24 == 0:  # and a sample against the oracle
            a = r.input_keys.cpu().numpy()
            if r.kind == "pairs":
                a = a.view(np.uint64)
            ref = oracle.sort(a)
            got = r.out_keys.cpu().numpy()
            assert np.array_equal(got.view(ref.dtype), ref), f"request {r.rid}"
