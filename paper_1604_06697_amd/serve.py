"""Continuous-batching sort service on one GPU.

Sort requests (keys, optionally with payloads) arrive over time.  The
service admits each one when its device memory fits the HBM budget, keeps
admitted requests in a FIFO queue, and hands batches to worker threads.  A
worker takes the key type of the oldest waiting request, packs every waiting
request of that type (in arrival order, up to a batch size) into one
segmented batch, and sorts it with one segmented call of the library on its
own HIP stream -- so batches of different workers run on the device at the
same time, and requests that arrive while others are on the GPU join the
next batch as soon as a worker frees up.  A request completes when its
batch's call returns; its result is its slice of the batch.

Keys come out bit for bit as a request sorted alone would give them (the
sorted sequence of a totally ordered key set is unique); for pairs, every
payload travels with its key.

The queue, the budget and the batching rule are plain host logic
(`form_batch`, `Budget`); the device work is the library's.
"""

from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import Context

KINDS = ("i32", "f64", "pairs")
KEY_BYTES = {"i32": 4, "f64": 8, "pairs": 8}
VAL_BYTES = {"i32": 0, "f64": 0, "pairs": 4}


@dataclass
class Request:
    rid: int
    kind: str                    # "i32", "f64" or "pairs" (uint64 key + uint32 payload)
    n: int
    arrival: float               # seconds on the service clock
    keys: torch.Tensor | None = None
    vals: torch.Tensor | None = None
    ready: torch.cuda.Event | None = None   # the request's data is on the device
    admitted: float = math.nan
    done: float = math.nan
    out_keys: torch.Tensor | None = None
    out_vals: torch.Tensor | None = None
    batch: int = -1
    error: str | None = None


def footprint(kind: str, n: int) -> int:
    """Device bytes a request holds while it is in the service: its input,
    its slice of the batch arena, and its share of the sort's workspace
    (second key buffer, and for pairs the second payload buffer and the
    side buffer)."""
    kb, vb = KEY_BYTES[kind], VAL_BYTES[kind]
    return n * (2 * (kb + vb) + kb + 2 * vb)


def form_batch(waiting: deque, max_keys: int) -> list:
    """Removes and returns the next batch: the oldest waiting request and
    every later waiting request of its key type, in arrival order, while the
    batch stays within max_keys (the oldest is always taken)."""
    if not waiting:
        return []
    kind = waiting[0].kind
    batch, keep, total = [], deque(), 0
    while waiting:
        r = waiting.popleft()
        if r.kind == kind and (not batch or total + r.n <= max_keys):
            batch.append(r)
            total += r.n
        else:
            keep.append(r)
    waiting.extend(keep)
    return batch


class Budget:
    """HBM budget shared by admission (acquire) and completion (release)."""

    def __init__(self, limit: int):
        self.limit = int(limit)
        self.used = 0
        self.peak = 0
        self._cv = threading.Condition()

    def try_acquire(self, nbytes: int) -> bool:
        with self._cv:
            if self.used + nbytes > self.limit and self.used > 0:
                return False
            self.used += nbytes
            self.peak = max(self.peak, self.used)
            return True

    def acquire(self, nbytes: int, stop=lambda: False):
        with self._cv:
            while self.used + nbytes > self.limit and self.used > 0 and not stop():
                self._cv.wait(0.01)
            self.used += nbytes
            self.peak = max(self.peak, self.used)

    def release(self, nbytes: int):
        with self._cv:
            self.used -= nbytes
            self._cv.notify_all()


def make_request_data(kind: str, n: int, seed: int, device="cuda"):
    """Seeded device-generated request data: int32 uniform over the full
    range; float64 uniform in [0, 1) with 53 random bits; pairs: uint64 key
    uniform over the full range (held in an int64 tensor) with the uint32
    payload = index."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if kind == "i32":
        return torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device=device, generator=g), None
    if kind == "f64":
        u = torch.randint(0, 2**53, (n,), dtype=torch.int64, device=device, generator=g)
        return u.to(torch.float64) * (2.0 ** -53), None
    hi = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int64, device=device, generator=g)
    lo = torch.randint(0, 2**32, (n,), dtype=torch.int64, device=device, generator=g)
    return (hi << 32) | lo, torch.arange(n, dtype=torch.int32, device=device)


class SortService:
    """Admission, FIFO queue and `workers` batch workers (one stream and
    one library context each)."""

    def __init__(self, budget_bytes: int, workers: int = 3, max_batch_keys: int = 1 << 27,
                 clock=time.perf_counter, keep_output=lambda r: True,
                 params=None):
        # library parameters of the workers' contexts; keys-only batches use
        # the multiway partition step by default (pairs ignore it)
        self.params = dict(multiway=1) if params is None else dict(params)
        self.keep_output = keep_output  # results of other requests are dropped once done
        self.budget = Budget(budget_bytes)
        self.max_batch_keys = int(max_batch_keys)
        self.clock = clock
        self.t0 = clock()
        self.waiting: deque = deque()
        self.done: list = []
        self.batches = 0
        self._cv = threading.Condition()
        self._closing = False
        self._errors: list = []
        self._ingest = torch.cuda.Stream()
        self._workers = [threading.Thread(target=self._work, args=(i,), daemon=True)
                         for i in range(workers)]
        for w in self._workers:
            w.start()

    def now(self) -> float:
        return self.clock() - self.t0

    # ---------------------------------------------------------- admission --
    def submit(self, req: Request, data=None, seed: int = 0):
        """Admits a request (blocking while the budget is exhausted): its
        data is `data` (keys, vals) or generated on the device from `seed`."""
        self.budget.acquire(footprint(req.kind, req.n), stop=lambda: bool(self._errors))
        req.admitted = self.now()
        req.ready = torch.cuda.Event()
        if data is None:
            with torch.cuda.stream(self._ingest):
                req.keys, req.vals = make_request_data(req.kind, req.n, seed)
                req.ready.record(self._ingest)
        else:
            # the caller produced the data on its current stream
            req.keys, req.vals = data
            req.ready.record(torch.cuda.current_stream())
        with self._cv:
            self.waiting.append(req)
            self._cv.notify()

    def close(self):
        """Waits until every submitted request is done, then stops the workers."""
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        for w in self._workers:
            w.join()
        if self._errors:
            raise self._errors[0]

    # ------------------------------------------------------------ workers --
    def _work(self, wid: int):
        stream = torch.cuda.Stream()
        ctx = Context(**self.params)
        try:
            while True:
                with self._cv:
                    while not self.waiting and not self._closing:
                        self._cv.wait(0.01)
                    if not self.waiting and self._closing:
                        return
                    batch = form_batch(self.waiting, self.max_batch_keys)
                    bid = self.batches
                    self.batches += 1
                self._run_batch(batch, bid, stream, ctx)
        except Exception as e:  # surfaced by close()
            self._errors.append(e)
            with self._cv:
                self._closing = True
                self._cv.notify_all()

    def _run_batch(self, batch, bid, stream, ctx):
        kind = batch[0].kind
        sizes = np.array([r.n for r in batch], dtype=np.int64)
        offsets = np.zeros(len(batch) + 1, dtype=np.int64)
        np.cumsum(sizes, out=offsets[1:])
        with torch.cuda.stream(stream):
            for r in batch:
                stream.wait_event(r.ready)
                # the inputs are read on this stream: keep the allocator from
                # handing their memory out again before that work is done
                r.keys.record_stream(stream)
                if r.vals is not None:
                    r.vals.record_stream(stream)
            keys = torch.cat([r.keys for r in batch]) if len(batch) > 1 else batch[0].keys
            vals = None
            if kind == "pairs":
                vals = torch.cat([r.vals for r in batch]) if len(batch) > 1 else batch[0].vals
            off = torch.from_numpy(offsets).to("cuda", non_blocking=False)
            if kind == "pairs":
                ctx.sort_segments_pairs(keys, vals, off, key_type="u64")
            else:
                ctx.sort_segments(keys, off)
            stream.synchronize()
            ctx.synchronize()  # raises for an error the device latched
        t = self.now()
        for i, r in enumerate(batch):
            lo, hi = int(offsets[i]), int(offsets[i + 1])
            if self.keep_output(r):
                r.out_keys = keys[lo:hi]
                r.out_vals = None if vals is None else vals[lo:hi]
            r.keys = r.vals = None  # the input buffer is free once the batch holds a copy
            r.done = t
            r.batch = bid
        with self._cv:
            self.done.extend(batch)
        for r in batch:
            self.budget.release(footprint(r.kind, r.n))


# ---------------------------------------------------------------- traces --

def make_trace(count: int, qps: float, seed: int, lo_exp: int = 10, hi_exp: int = 24,
               mix=(0.5, 0.3, 0.2)):
    """Poisson arrivals at `qps`; sizes log-uniform in [2^lo, 2^hi]; key
    types drawn with probabilities `mix` over (i32, f64, pairs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=count) if qps > 0 else np.zeros(count)
    arrivals = np.cumsum(gaps) - (gaps[0] if count else 0.0)
    u = rng.random(count)
    sizes = np.minimum(np.floor(2.0 ** (lo_exp + (hi_exp - lo_exp) * u)), 2.0 ** hi_exp).astype(np.int64)
    kinds = rng.choice(len(KINDS), size=count, p=np.asarray(mix) / np.sum(mix))
    return [Request(rid=i, kind=KINDS[kinds[i]], n=int(sizes[i]), arrival=float(arrivals[i]))
            for i in range(count)]


def _drive(trace, submit, clock, t0):
    """Submits each request at its arrival time (on the given clock)."""
    for r in trace:
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        submit(r)


def run_service(trace, budget_bytes: int, workers: int = 3, seed_base: int = 0,
                max_batch_keys: int = 1 << 27, keep_inputs=()):
    """Replays the trace through a SortService; returns (requests, makespan,
    service).  Requests whose rid is in keep_inputs keep a copy of their
    input in `.input_keys` / `.input_vals` for checking."""
    keep = set(keep_inputs)
    # a delivered result leaves the device; only the checked ones are kept
    svc = SortService(budget_bytes, workers=workers, max_batch_keys=max_batch_keys,
                      keep_output=lambda r: r.rid in keep)

    def submit(r):
        data = make_request_data(r.kind, r.n, seed_base + r.rid)
        if r.rid in keep:
            r.input_keys = data[0].clone()
            r.input_vals = None if data[1] is None else data[1].clone()
        svc.submit(r, data=data)

    torch.cuda.synchronize()
    svc.t0 = svc.clock()
    _drive(trace, submit, svc.clock, svc.t0)
    svc.close()
    makespan = max(r.done for r in trace) - min(r.arrival for r in trace)
    return trace, makespan, svc


def run_one_per_launch(trace, seed_base: int = 0, keep_inputs=()):
    """Baseline on the same trace: one plain sort call per request, in
    arrival order, on one stream."""
    ctx = Context()
    keep = set(keep_inputs)
    torch.cuda.synchronize()
    clock = time.perf_counter
    t0 = clock()
    for r in trace:
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        keys, vals = make_request_data(r.kind, r.n, seed_base + r.rid)
        if r.rid in keep:
            r.input_keys = keys.clone()
            r.input_vals = None if vals is None else vals.clone()
        r.admitted = clock() - t0
        if r.kind == "pairs":
            ctx.sort_pairs(keys, vals, key_type="u64")
        else:
            ctx.sort(keys)
        torch.cuda.current_stream().synchronize()
        ctx.synchronize()
        r.done = clock() - t0
        if r.rid in keep:
            r.out_keys, r.out_vals = keys, vals
    makespan = max(r.done for r in trace) - min(r.arrival for r in trace)
    return trace, makespan


def latency_summary(trace, makespan: float) -> dict:
    """Nearest-rank p50 / p99 of arrival-to-completion latency, and keys/s
    over the makespan."""
    lat = np.sort(np.array([r.done - r.arrival for r in trace]))

    def rank(p):  # nearest rank: the ceil(p * N / 100)-th smallest, in integers
        return float(lat[max(0, -(-p * len(lat) // 100) - 1)])

    keys = sum(r.n for r in trace)
    return {"requests": len(trace), "keys": int(keys), "makespan_s": round(makespan, 4),
            "p50_ms": round(1e3 * rank(50), 3), "p99_ms": round(1e3 * rank(99), 3),
            "Gkeys/s": round(keys / makespan / 1e9, 3)}
