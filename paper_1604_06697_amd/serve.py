"""Continuous-batching sort service on one GPU.

Sort requests (keys, optionally with payloads) arrive over time.  Admission
places each request's data in a device arena -- one ring of slots per key
type, so that consecutive requests of a type sit next to each other -- and
blocks while its ring has no room.  Admitted requests wait in a FIFO queue;
worker threads take batches: a worker takes the key type of the oldest
waiting request and every later waiting request of that type whose slots
continue the batch's range of the ring (in arrival order, up to a batch
size), and sorts that range in place with one segmented call of the library
(the request boundaries are the segment offsets) on its own HIP stream.
Nothing is copied to form a batch.  The worker records an event after the
call and waits for that event before it takes the next batch (one batch
in flight per worker, so that requests arriving meanwhile join the next
batch); a batch's requests complete at the device time the event records,
and their slots go back to the ring then.

Keys come out bit for bit as a request sorted alone would give them (the
sorted sequence of a totally ordered key set is unique); for pairs, every
payload travels with its key.

Device memory is fixed when the service starts: the rings, sized from the
HBM budget by the expected mix of key types, and each worker's workspace
for the largest batch.  With the out-of-place steps (the default here) that
workspace is a second copy of the batch; with the library's in-place step
(params=dict(inplace=1)) it is a few percent of a batch.

The queue, the rings and the batching rule are plain host logic
(`form_batch`, `Ring`); the device work is the library's.
"""

from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass

import numpy as np
import torch

from . import I32, F64, U64, Context

KINDS = ("i32", "f64", "pairs")
KEY_BYTES = {"i32": 4, "f64": 8, "pairs": 8}
VAL_BYTES = {"i32": 0, "f64": 0, "pairs": 4}
KEY_DTYPE = {"i32": torch.int32, "f64": torch.float64, "pairs": torch.int64}
KEY_CODE = {"i32": I32, "f64": F64, "pairs": U64}
MIX = (0.5, 0.3, 0.2)  # expected share of requests per key type


@dataclass
class Request:
    rid: int
    kind: str                    # "i32", "f64" or "pairs" (uint64 key + uint32 payload)
    n: int
    arrival: float               # seconds on the service clock
    pos: int = -1                # first slot in its type's ring
    ready: torch.cuda.Event | None = None   # the request's data is in the arena
    admitted: float = math.nan
    done: float = math.nan
    out_keys: torch.Tensor | None = None
    out_vals: torch.Tensor | None = None
    batch: int = -1
    error: str | None = None


def footprint(kind: str, n: int) -> int:
    """Arena bytes a request holds from admission to completion: its keys
    and payloads (it is sorted where it sits)."""
    return n * (KEY_BYTES[kind] + VAL_BYTES[kind])


def form_batch(waiting: deque, max_keys: int) -> list:
    """Removes and returns the next batch: the oldest waiting request and
    every later waiting request of its key type, in arrival order, while the
    batch stays within max_keys (the oldest is always taken) and, for
    requests placed in a ring (pos >= 0), while each one's slots follow the
    previous one's."""
    if not waiting:
        return []
    kind = waiting[0].kind
    batch, keep, total = [], deque(), 0
    while waiting:
        r = waiting.popleft()
        follows = (not batch or r.pos < 0 or batch[-1].pos < 0 or r.pos == batch[-1].pos + batch[-1].n)
        if r.kind == kind and follows and (not batch or total + r.n <= max_keys):
            batch.append(r)
            total += r.n
        else:
            keep.append(r)
    waiting.extend(keep)
    return batch


class Ring:
    """Allocator of contiguous slot ranges in [0, capacity): ranges are
    handed out in order (wrapping to the start when the end has no room)
    and released in any order; space returns once every older range has
    been released."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.live: deque = deque()   # [start, n, released, lap] in allocation order
        self.used = 0                # slots of live ranges
        self.peak = 0
        self._cv = threading.Condition()

    def _place(self, n: int):
        if not self.live:
            return (0, 0) if n <= self.capacity else None
        first, last = self.live[0], self.live[-1]
        end = last[0] + last[1]
        if first[3] == last[3]:
            # live slots [first.start, end): room after them, else at the start
            if end + n <= self.capacity:
                return end, last[3]
            if n <= first[0]:
                return 0, last[3] + 1
            return None
        # wrapped: live slots [first.start, ...) and [0, end)
        return (end, last[3]) if end + n <= first[0] else None

    def try_alloc(self, n: int):
        with self._cv:
            at = self._place(n)
            if at is None:
                return None
            self.live.append([at[0], n, False, at[1]])
            self.used += n
            self.peak = max(self.peak, self.used)
            return at[0]

    def alloc(self, n: int, stop=lambda: False) -> int:
        if n > self.capacity:
            raise ValueError(f"request of {n} slots exceeds the ring's {self.capacity}")
        with self._cv:
            while True:
                at = self._place(n)
                if at is not None or stop():
                    break
                self._cv.wait(0.01)
            if at is None:
                raise RuntimeError("service stopped")
            self.live.append([at[0], n, False, at[1]])
            self.used += n
            self.peak = max(self.peak, self.used)
            return at[0]

    def release(self, start: int):
        with self._cv:
            for e in self.live:
                if e[0] == start and not e[2]:
                    e[2] = True
                    self.used -= e[1]
                    break
            else:
                raise KeyError(start)
            while self.live and self.live[0][2]:
                self.live.popleft()
            self._cv.notify_all()


def fill_request(kind: str, keys: torch.Tensor, vals: torch.Tensor | None, seed: int):
    """Seeded device-generated request data, written into `keys` (and
    `vals`): int32 uniform over the full range; float64 uniform in [0, 1)
    with 53 random bits; pairs: uint64 key uniform over the full range (held
    in an int64 tensor) with the uint32 payload = index."""
    n = keys.numel()
    g = torch.Generator(device=keys.device)
    g.manual_seed(seed)
    if kind == "i32":
        torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device=keys.device, generator=g, out=keys)
    elif kind == "f64":
        u = torch.randint(0, 2**53, (n,), dtype=torch.int64, device=keys.device, generator=g)
        torch.mul(u.to(torch.float64), 2.0 ** -53, out=keys)
    else:
        hi = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int64, device=keys.device, generator=g)
        lo = torch.randint(0, 2**32, (n,), dtype=torch.int64, device=keys.device, generator=g)
        torch.bitwise_or(hi << 32, lo, out=keys)
        torch.arange(n, dtype=torch.int32, device=keys.device, out=vals)


def make_request_data(kind: str, n: int, seed: int, device="cuda"):
    """The same data as fill_request, in fresh tensors."""
    keys = torch.empty(n, dtype=KEY_DTYPE[kind], device=device)
    vals = torch.empty(n, dtype=torch.int32, device=device) if kind == "pairs" else None
    fill_request(kind, keys, vals, seed)
    return keys, vals


class SortService:
    """Admission into the arena, FIFO queue and `workers` batch workers (one
    stream and one library context each)."""

    def __init__(self, budget_bytes: int, workers: int = 3, max_batch_keys: int = 1 << 27,
                 clock=time.perf_counter, keep_output=lambda r: True, params=None, mix=MIX):
        # library parameters of the workers' contexts: the multiway step by
        # default (keys-only batches; pairs take the two-way step); with
        # dict(inplace=1) the workspace shrinks to a few percent of a batch
        self.params = dict(multiway=1) if params is None else dict(params)
        self.keep_output = keep_output  # results of other requests are dropped once done
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
        self._start = torch.cuda.Event(enable_timing=True)
        self._start.record()
        # workspace of every worker, for the largest batch of any key type;
        # the largest batch shrinks (by halves, down to 2^16 keys) until the
        # workspaces take at most half the budget.  A request larger than the
        # batch size is sorted alone and grows its worker's workspace.
        self._ctxs = [Context(**self.params) for _ in range(workers)]

        def workspace(keys):
            segs = max(1, keys >> 10)  # requests hold at least 2^10 keys
            return max(self._ctxs[0].workspace_bytes(keys, KEY_CODE[k], VAL_BYTES[k], segs) for k in KINDS)

        while self.max_batch_keys > (1 << 16) and workers * workspace(self.max_batch_keys) > budget_bytes // 2:
            self.max_batch_keys //= 2
        ws = workspace(self.max_batch_keys)
        for c in self._ctxs:
            c.reserve(ws)
        self.workspace_bytes = ws * workers
        # rings: the rest of the budget, split by the bytes the mix brings in
        arena = int(budget_bytes) - self.workspace_bytes
        weight = {k: m * (KEY_BYTES[k] + VAL_BYTES[k]) for k, m in zip(KINDS, mix)}
        total_w = sum(weight.values())
        self.rings, self.keys, self.vals = {}, {}, {}
        for k in KINDS:
            slots = max(1 << 10, int(arena * weight[k] / total_w) // (KEY_BYTES[k] + VAL_BYTES[k]))
            self.rings[k] = Ring(slots)
            self.keys[k] = torch.empty(slots, dtype=KEY_DTYPE[k], device="cuda")
            self.vals[k] = torch.empty(slots, dtype=torch.int32, device="cuda") if VAL_BYTES[k] else None
        self.arena_bytes = sum(r.capacity * (KEY_BYTES[k] + VAL_BYTES[k]) for k, r in self.rings.items())
        torch.cuda.synchronize()
        self._workers = [threading.Thread(target=self._work, args=(i,), daemon=True) for i in range(workers)]
        for w in self._workers:
            w.start()

    def now(self) -> float:
        return self.clock() - self.t0

    def restart_clock(self):
        """Makes now() and the device completion times count from here."""
        torch.cuda.synchronize()
        self._start.record()
        self.t0 = self.clock()

    def peak_bytes(self) -> int:
        """Most arena bytes held at once, plus the workspaces."""
        return self.workspace_bytes + sum(r.peak * (KEY_BYTES[k] + VAL_BYTES[k]) for k, r in self.rings.items())

    def slots(self, r: Request):
        """The request's keys (and payloads) in the arena."""
        k = self.keys[r.kind][r.pos:r.pos + r.n]
        v = self.vals[r.kind][r.pos:r.pos + r.n] if self.vals[r.kind] is not None else None
        return k, v

    # ---------------------------------------------------------- admission --
    def submit(self, req: Request, seed: int = 0, keep_input: bool = False):
        """Admits a request (blocking while its ring has no room): its data
        is generated from `seed` into its slots on the ingest stream.  With
        keep_input, a copy of the input is kept in `.input_keys` /
        `.input_vals`."""
        req.pos = self.rings[req.kind].alloc(req.n, stop=lambda: bool(self._errors))
        req.admitted = self.now()
        req.ready = torch.cuda.Event()
        with torch.cuda.stream(self._ingest):
            keys, vals = self.slots(req)
            fill_request(req.kind, keys, vals, seed)
            if keep_input:
                req.input_keys = keys.clone()
                req.input_vals = None if vals is None else vals.clone()
            req.ready.record(self._ingest)
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
        for c in self._ctxs:
            c.close()
        if self._errors:
            raise self._errors[0]

    # ------------------------------------------------------------ workers --
    def _work(self, wid: int):
        stream = torch.cuda.Stream()
        ctx = self._ctxs[wid]
        pending: deque = deque()  # (batch, event, pinned offsets) in launch order
        try:
            while True:
                with self._cv:
                    while not self.waiting and not self._closing and not pending:
                        self._cv.wait(0.01)
                    batch = form_batch(self.waiting, self.max_batch_keys) if self.waiting else []
                    if batch:
                        bid = self.batches
                        self.batches += 1
                    elif self._closing and not pending:
                        return
                if batch:
                    pending.append(self._launch(batch, bid, stream, ctx))
                # one batch in flight per worker: requests that arrive while
                # it runs join the next batch instead of each taking a small
                # batch of its own (three workers keep the device busy)
                while pending:
                    self._finish(*pending.popleft(), stream, ctx)
        except Exception as e:  # surfaced by close()
            self._errors.append(e)
            with self._cv:
                self._closing = True
                self._cv.notify_all()

    def _launch(self, batch, bid, stream, ctx):
        kind = batch[0].kind
        sizes = np.array([r.n for r in batch], dtype=np.int64)
        off_h = torch.zeros(len(batch) + 1, dtype=torch.int64, pin_memory=True)
        np.cumsum(sizes, out=off_h.numpy()[1:])
        lo, hi = batch[0].pos, batch[-1].pos + batch[-1].n
        keys = self.keys[kind][lo:hi]
        vals = self.vals[kind][lo:hi] if self.vals[kind] is not None else None
        ev = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            for r in batch:
                stream.wait_event(r.ready)
            off = off_h.to("cuda", non_blocking=True)
            if kind == "pairs":
                ctx.sort_segments_pairs(keys, vals, off, key_type="u64")
            else:
                ctx.sort_segments(keys, off)
            ev.record(stream)
        for r in batch:
            r.batch = bid
        return batch, ev, off_h

    def _finish(self, batch, ev, off_h, stream, ctx):
        ev.synchronize()
        ctx.poll()  # raises for an error the device latched in a completed call
        t = self._start.elapsed_time(ev) * 1e-3  # device time of the batch's end
        kept = [r for r in batch if self.keep_output(r)]
        if kept:
            with torch.cuda.stream(stream):
                for r in kept:
                    k, v = self.slots(r)
                    r.out_keys = k.clone()
                    r.out_vals = None if v is None else v.clone()
            stream.synchronize()  # the copies leave the slots before they are reused
        for r in batch:
            r.done = t
            self.rings[r.kind].release(r.pos)
        with self._cv:
            self.done.extend(batch)


# ---------------------------------------------------------------- traces --

def make_trace(count: int, qps: float, seed: int, lo_exp: int = 10, hi_exp: int = 24,
               mix=MIX):
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
    for r in trace:
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        submit(r)


def run_service(trace, budget_bytes: int, workers: int = 3, seed_base: int = 0,
                max_batch_keys: int = 1 << 27, keep_inputs=(), params=None):
    """Replays the trace through a SortService; returns (requests, makespan,
    service).  Requests whose rid is in keep_inputs keep a copy of their
    input in `.input_keys` / `.input_vals` for checking."""
    keep = set(keep_inputs)
    # a delivered result leaves the device; only the checked ones are kept
    svc = SortService(budget_bytes, workers=workers, max_batch_keys=max_batch_keys,
                      keep_output=lambda r: r.rid in keep, params=params)
    svc.restart_clock()
    _drive(trace, lambda r: svc.submit(r, seed=seed_base + r.rid, keep_input=r.rid in keep), svc.clock, svc.t0)
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
    ctx.close()
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
