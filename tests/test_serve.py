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


def test_budget_blocks_until_release(serve):
    b = serve.Budget(100)
    assert b.try_acquire(60)
    assert not b.try_acquire(50)
    got = []
    t = threading.Thread(target=lambda: (b.acquire(50), got.append(1)))
    t.start()
    t.join(0.1)
    assert not got
    b.release(60)
    t.join(2.0)
    assert got == [1] and b.used == 50 and b.peak == 60
    # a request larger than the whole budget is admitted alone
    b.release(50)
    assert b.try_acquire(1000)


def test_footprint_counts_input_batch_and_workspace(serve):
    assert serve.footprint("i32", 1000) == 1000 * (2 * 4 + 4)
    assert serve.footprint("f64", 1000) == 1000 * (2 * 8 + 8)
    assert serve.footprint("pairs", 1000) == 1000 * (2 * 12 + 8 + 8)


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
def test_results_same_alone_and_in_the_mix(serve, oracle):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_06697_amd as bqs

    trace = serve.make_trace(240, qps=4000.0, seed=5, lo_exp=10, hi_exp=17)
    print(f"[case] serving mix of {len(trace)} requests", flush=True)
    trace, makespan, svc = serve.run_service(trace, budget_bytes=1 << 30, workers=3, seed_base=100,
                                             keep_inputs=[r.rid for r in trace])
    assert svc.batches < len(trace)  # requests were batched together
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
