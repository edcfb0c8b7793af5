"""Benchmark of the block-partition sort on one MI355X.

One step = one complete sort of a fresh copy of the workload (every
partition pass, the small-segment sorts and the equal-key fills).  The
headline workload is a single array of 2^28 uniform random int32 keys; the
other single-array distributions of the same size class are reported in
`distributions`.  Inputs are generated on the device (seeded) and are
resident in HBM before the timed region starts: each step sorts its own
pre-made copy, so no copy runs inside the timed region.

Prints one JSON line (see the README of the repository for the fields).
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
N_HEADLINE = 1 << 28
PAPER_CPU_GKEYS = 1.0 / 45.0  # 45 ns per element at n = 2^28 (i5-2500K), context only


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N_HEADLINE, help="keys of the headline workload")
    ap.add_argument("--no-dists", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched segmented workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving loop")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the persistent-mode line (a cooperative launch, which some profilers "
                         "do not shut down cleanly)")
    ap.add_argument("--serve-requests", type=int, default=100_000)
    return ap.parse_args()


def make_inputs(torch, kind: str, n: int, copies: int, seed: int):
    """`copies` device arrays holding the same seeded input."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dev = "cuda"
    if kind == "i32_uniform":
        src = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device=dev, generator=g)
    elif kind == "i32_sorted":
        src = torch.arange(n, dtype=torch.int32, device=dev)
    elif kind == "i32_reverse":
        src = torch.arange(n - 1, -1, -1, dtype=torch.int32, device=dev)
    elif kind == "i32_few_distinct":
        src = torch.randint(0, 1024, (n,), dtype=torch.int32, device=dev, generator=g)
    elif kind == "i32_all_equal":
        src = torch.full((n,), 0x2A, dtype=torch.int32, device=dev)
    elif kind == "f64_uniform":
        u = torch.randint(0, 2**53, (n,), dtype=torch.int64, device=dev, generator=g)
        src = u.to(torch.float64) * (2.0 ** -53)
    elif kind == "f64_normal":
        src = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
    elif kind == "f64_sorted_swaps":
        u = torch.randint(0, 2**53, (n,), dtype=torch.int64, device=dev, generator=g)
        src = torch.sort(u.to(torch.float64) * (2.0 ** -53)).values
        k = n // 100
        # floor(n/100) swaps of disjoint, uniformly drawn index pairs
        perm = torch.randperm(n, device=dev, generator=g)[: 2 * k]
        i, j = perm[:k], perm[k:]
        vi, vj = src[i].clone(), src[j].clone()
        src[i] = vj
        src[j] = vi
    else:
        raise ValueError(kind)
    out = [src] + [src.clone() for _ in range(copies - 1)]
    return out


def make_pairs(torch, n: int, copies: int, seed: int):
    """uint64 keys uniform over the full range (held in an int64 tensor),
    uint32 payload = original index."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    hi = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int64, device="cuda", generator=g)
    lo = torch.randint(0, 2**32, (n,), dtype=torch.int64, device="cuda", generator=g)
    k = (hi << 32) | lo
    v = torch.arange(n, dtype=torch.int32, device="cuda")
    return [(k.clone(), v.clone()) for _ in range(copies)]


def run_workload(torch, bqs, ctx, kind, n, steps, warmup, seed=0, keep=None):
    """Times `steps` sorts; returns (ms_per_step, stats dict, per-level list,
    partition ms and keys per step, correct).  With `keep` (a list), the last
    step's sorted keys are appended to it as a host array."""
    pairs = kind == "pairs_u64_u32"
    copies = steps + warmup
    data = make_pairs(torch, n, copies, seed) if pairs else make_inputs(torch, kind, n, copies, seed)

    def one(i):
        if pairs:
            ctx.sort_pairs(data[i][0], data[i][1], key_type="u64")
        else:
            ctx.sort(data[i])

    # reference of the last step's input, taken before it is sorted
    last = data[-1][0] if pairs else data[-1]
    sign = torch.tensor(-(2**63), dtype=torch.int64, device="cuda")
    if pairs:
        keys_in = last.clone()
        ref = torch.sort(last ^ sign).values ^ sign  # unsigned order of the uint64 keys
    else:
        ref = torch.sort(last).values
    for i in range(warmup):
        one(i)
    ctx.synchronize()
    torch.cuda.synchronize()
    # the timed steps only enqueue (the library's calls are asynchronous);
    # the barrier after the last one ends the timed region
    t0 = time.perf_counter()
    for i in range(warmup, copies):
        one(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.synchronize()
    # every step sorts the same input: the last step's statistics and
    # kernel times stand for each step
    levels = ctx.levels()
    st = ctx.stats()
    part_ms, part_keys = st["partition_ms"] * steps, st["partitioned_keys"] * steps
    # the last step against the reference: keys bit for bit; pairs also carry
    # their payload (payload = original index)
    ok = bool(torch.equal(last, ref))
    if pairs:
        vals = data[-1][1].to(torch.int64) & 0xFFFFFFFF
        ok = ok and bool(torch.equal(keys_in[vals], last))
    del ref
    if keep is not None:
        keep.append(last.cpu().numpy())
    del data
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    return ms, st, levels, part_ms / steps, part_keys / steps, ok


def batched_segments(torch, bqs, steps, warmup, k=20000, seed=7, per_array=True, cpu=True):
    """k int32 arrays, sizes log-uniform in [16, 2^20] (uniform keys),
    concatenated with an int64 offsets array: one sort_segments call per
    step, against one sort call per array on the same stream."""
    import workloads as W

    sizes = W.log_uniform_sizes(k, seed)
    offsets = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    n = int(offsets[-1])
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    pristine = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device="cuda", generator=g)
    work = torch.empty_like(pristine)
    off_d = torch.from_numpy(offsets).cuda()
    # the plan (tile shape, small cutoff) from the autotuner, measured on this
    # input in graph mode (untimed); then the warm-up call captures the
    # launches and the timed calls replay them
    from paper_1604_06697_amd import tune

    work.copy_(pristine)
    tuned = tune.autotune(work, off_d, graph=True, reps=1, path=None)
    progress(f"batched: autotuner picked {tuned['plan']}")
    ctx = bqs.Context(graph=1, **tuned["plan"])
    times = []
    for i in range(warmup + steps):
        work.copy_(pristine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.sort_segments(work, off_d)
        torch.cuda.synchronize()
        if i >= warmup:
            times.append(time.perf_counter() - t0)
    st = ctx.stats()
    ok = check_segments(torch, pristine, work, offsets)
    ms = 1e3 * float(np.median(times))
    # bytes the method moves: 8 B per key and two-way pass (read + write),
    # 12 B per key and multiway pass (two reads + write), 8 B per small-sorted
    # key, 4 B per key of an equal run
    pass_b = 12 if tuned["plan"].get("multiway") else 8
    alg_b = pass_b * st["partitioned_keys"] + 8 * st["small_sorted_keys"] + 4 * st["filled_keys"]
    # per-phase breakdown: one more call with the same plan, every launch
    # timed (outside the timed steps)
    bctx = bqs.Context(timing=1, **tuned["plan"])
    work.copy_(pristine)
    bctx.sort_segments(work, off_d)
    bctx.synchronize()
    bst = bctx.stats()
    bctx.close()
    # per-array completion inside one call: the device clock when each
    # array's last key became final (bqs_ctx_set_segment_ticks), one more
    # graph replay with the same plan
    tctx = bqs.Context(graph=1, **tuned["plan"])
    ticks = torch.zeros(k + 1, dtype=torch.int64, device="cuda")
    tctx.set_segment_ticks(ticks)
    tms = []
    for i in range(2):  # capture, then the measured replay
        work.copy_(pristine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tctx.sort_segments(work, off_d)
        torch.cuda.synchronize()
        tms.append(1e3 * (time.perf_counter() - t0))
    tctx.synchronize()
    tk = ticks.cpu().numpy()
    done_ms = (tk[:k] - tk[k]) * 1e-5  # 100 MHz clock
    t_ok = check_segments(torch, pristine, work, offsets)
    tctx.close()
    out = {
        "workload": f"{k} int32 arrays, sizes log-uniform in [16, 2^20], {n} keys, int64 offsets",
        "k": k, "n": n, "seed": seed,
        "batched": {"ms": round(ms, 3), "ms_min": round(1e3 * min(times), 3),
                    "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3),
                    "alg_GBps": round(alg_b / (ms * 1e-3) / 1e9, 1),
                    "frac": round(alg_b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "levels": st["levels"], "graph_replay": bool(st["graph_launches"]),
                    "breakdown": {"partition_ms": round(bst["partition_ms"], 3),
                                  "small_ms": round(bst["small_ms"], 3), "plan_ms": round(bst["plan_ms"], 3)},
                    # from the call's first kernel to each array's last
                    # key in place (device clock), in a separate replay
                    "array_done_p50_ms": round(float(np.percentile(done_ms, 50, method="nearest")), 3),
                    "array_done_p99_ms": round(float(np.percentile(done_ms, 99, method="nearest")), 3),
                    "array_done_max_ms": round(float(done_ms.max()), 3),
                    "clocked_call_ms": round(tms[-1], 3), "clocked_correct": t_ok},
        "correct": ok,
        "plan": tuned["plan"],
        "tuner_table": tuned["table"],
    }
    if per_array:
        # baseline: one sort call per array, in order, on one stream
        work.copy_(pristine)
        torch.cuda.synchronize()
        views = [work[int(offsets[i]):int(offsets[i + 1])] for i in range(k)]
        ctx = bqs.Context()
        done = np.empty(k)
        t0 = time.perf_counter()
        for i, v in enumerate(views):
            if v.numel() > 1:
                ctx.sort(v)
            done[i] = time.perf_counter() - t0
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        ok_pa = check_segments(torch, pristine, work, offsets)
        out["per_array"] = {"ms": round(1e3 * total, 1), "Gkeys/s": round(n / total / 1e9, 3),
                            "array_done_p50_ms": round(1e3 * float(np.percentile(done, 50, method="nearest")), 1),
                            "array_done_p99_ms": round(1e3 * float(np.percentile(done, 99, method="nearest")), 1),
                            "correct": ok_pa}
        out["speedup_vs_per_array"] = round(total * 1e3 / ms, 2)
    if cpu:
        out["cpu_oracle"] = cpu_segments(pristine.cpu().numpy(), offsets)
    del work, pristine
    torch.cuda.empty_cache()
    return out


def check_segments(torch, pristine, work, offsets):
    """Every segment ascending, and per segment the same multiset of keys
    as the input (sum of a 64-bit mix of each key, per segment)."""
    k = len(offsets) - 1
    n = int(offsets[-1])
    sizes = torch.from_numpy(np.diff(offsets)).cuda()
    seg = torch.repeat_interleave(torch.arange(k, device="cuda"), sizes)
    up = work[1:] >= work[:-1]
    first = torch.zeros(n, dtype=torch.bool, device="cuda")
    starts = torch.from_numpy(offsets[:-1][np.diff(offsets) > 0]).cuda()
    first[starts] = True
    ok = bool((up | first[1:]).all())

    def mix(x):
        z = x.to(torch.int64) * -7046029254386353131  # 0x9e3779b97f4a7c15 as int64
        z = z ^ (z >> 29)
        return z * -4658895280553007687  # 0xbf58476d1ce4e5b9 as int64

    a = torch.zeros(k, dtype=torch.int64, device="cuda").index_add_(0, seg, mix(pristine))
    b = torch.zeros(k, dtype=torch.int64, device="cuda").index_add_(0, seg, mix(work))
    return ok and bool(torch.equal(a, b))


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy of `nbytes` (one read + one write per byte):
    the practical HBM ceiling, reported as context beside the 8 TB/s peak."""
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(7)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = None
    for _ in range(reps):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        ev[1].synchronize()
        ms = ev[0].elapsed_time(ev[1])
        best = ms if best is None else min(best, ms)
    del src, dst
    return {"bytes": nbytes, "ms": round(best, 4), "GBps": round(2 * nbytes / (best * 1e-3) / 1e9, 1)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_partition_i32_2p28_uniform_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1604_06697_amd", "csrc", "bqs_kernels.hpp")


def measured_traffic():
    """HBM bytes per partition launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a copy of known
    size), or None when the kernel source changed since it was taken."""
    import hashlib

    try:
        fields = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    fields[k.strip()] = v.strip()
        with open(KERNEL_SOURCE, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if fields.get("kernel_source_sha256") != digest:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def serving(torch, requests, seed=11, budget=64 << 30, workers=3):
    """Serving loop: Poisson arrivals of mixed requests (sizes log-uniform in
    [2^10, 2^24]; 50 % int32, 30 % float64, 20 % uint64+uint32 pairs), placed
    in a device arena under an HBM budget, batched continuously and sorted
    where they sit (the service's default step: multiway for keys, two-way
    for pairs).  The arrival rate is 0.7 x the service's saturated capacity,
    measured first on a burst of requests that all arrive at once.  The
    same burst is served with the in-place step (workspace a few percent of
    a batch), and the trace is replayed with one plain sort call per
    request, in arrival order on one stream."""
    from paper_1604_06697_amd import serve

    def fresh(tr):
        return [serve.Request(r.rid, r.kind, r.n, r.arrival) for r in tr]

    # a warm-up burst (kernel code objects, allocator pools), then the median
    # of three calibration bursts
    warm = serve.make_trace(max(50, requests // 200), qps=0.0, seed=seed + 2)
    serve.run_service(warm, budget, workers=workers, seed_base=1 << 41)
    caps = []
    for rep in range(3):
        burst = serve.make_trace(max(200, requests // 50), qps=0.0, seed=seed + 1)
        _, mk, _ = serve.run_service(burst, budget, workers=workers, seed_base=(1 << 40) + rep)
        caps.append((mk, serve.latency_summary(burst, mk)))
    caps.sort(key=lambda c: c[0])
    mk, cap = caps[1]
    qps = 0.7 * len(burst) / mk
    progress(f"serving: saturated capacity {cap['Gkeys/s']} Gkeys/s")
    trace = serve.make_trace(requests, qps=qps, seed=seed)
    sample = [r.rid for r in trace if r.rid % 100 == 0]
    trace, mk, svc = serve.run_service(trace, budget, workers=workers, seed_base=0, keep_inputs=sample)
    ok = check_requests(torch, [trace[i] for i in sample])
    out = {
        "workload": f"{requests} requests, Poisson arrivals at {qps:.0f}/s (0.7 x saturated capacity), "
                    "sizes log-uniform [2^10, 2^24], 50% int32 / 30% float64 / 20% uint64+uint32 pairs, "
                    f"{budget >> 30} GiB HBM budget, {workers} batch workers",
        "qps": round(qps, 1),
        "saturated": {"requests": cap["requests"], "Gkeys/s": cap["Gkeys/s"],
                      "bursts_Gkeys/s": sorted(c[1]["Gkeys/s"] for c in caps)},
        "service": dict(serve.latency_summary(trace, mk), batches=svc.batches,
                        step="multiway (pairs: two-way), out of place",
                        workspace_GiB=round(svc.workspace_bytes / 2**30, 3),
                        peak_device_GiB=round(svc.peak_bytes() / 2**30, 2)),
        "correct_sample": ok,
    }
    progress(f"serving: service p50 {out['service']['p50_ms']} ms")
    # the in-place step on the calibration burst: capacity and device memory
    ib = fresh(burst)
    ib, mk_i, isvc = serve.run_service(ib, budget, workers=workers, seed_base=(1 << 40) + 1,
                                       keep_inputs=[r.rid for r in ib if r.rid % 50 == 0], params=dict(inplace=1))
    out["inplace_saturated"] = dict(serve.latency_summary(ib, mk_i), step="in-place",
                                    workspace_GiB=round(isvc.workspace_bytes / 2**30, 3),
                                    peak_device_GiB=round(isvc.peak_bytes() / 2**30, 2),
                                    correct_sample=check_requests(torch, [r for r in ib if r.rid % 50 == 0]))
    progress(f"serving: in-place burst {out['inplace_saturated']['Gkeys/s']} Gkeys/s")
    base = fresh(trace)
    base, mk_b = serve.run_one_per_launch(base, seed_base=0, keep_inputs=sample)
    out["one_per_launch"] = dict(serve.latency_summary(base, mk_b),
                                 correct_sample=check_requests(torch, [base[i] for i in sample]))
    return out


def check_requests(torch, reqs):
    """Each sampled request's output against torch.sort of its input (for
    pairs: the unsigned order of the keys, and payload = index into the
    input)."""
    sign = torch.tensor(-(2**63), dtype=torch.int64, device="cuda")
    for r in reqs:
        if r.kind == "pairs":
            ref = torch.sort(r.input_keys ^ sign).values ^ sign
            if not (torch.equal(r.out_keys, ref) and
                    torch.equal(r.input_keys[r.out_vals.long()], r.out_keys)):
                return False
        elif not torch.equal(r.out_keys, torch.sort(r.input_keys).values):
            return False
        r.input_keys = r.input_vals = None
    return True


def paper_families(torch, bqs, n=1 << 26, reps=3):
    """The int32 input families of the paper's benchmark (random
    permutation, few-distinct and structured inputs), n keys each, default
    plan; each timed call sorts a fresh copy of the input."""
    import workloads as W

    out = {}
    ctx = bqs.Context()
    for fam, gen in W.I32_EXTRA_FAMILIES.items():
        pristine = torch.from_numpy(gen(n, 3)).cuda()
        ref = torch.sort(pristine).values
        t = torch.empty_like(pristine)
        times = []
        for r in range(reps + 1):
            t.copy_(pristine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sort(t)
            torch.cuda.synchronize()
            if r:
                times.append(time.perf_counter() - t0)
        ms = 1e3 * min(times)
        st = ctx.stats()
        out[fam] = {"ms": round(ms, 3), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3), "levels": st["levels"],
                    "correct": bool(torch.equal(t, ref))}
        del pristine, ref, t
    return {"n": n, "families": out}


PIVOT_STRATEGIES = (
    ("median_of_3", {"pivot_mode": 3}),
    ("median_of_5", {"pivot_mode": 5}),
    ("median_of_23", {"pivot_mode": 23}),
    ("mo3_of_mo3", {"pivot_mode": 33}),
    ("mo3_of_mo5", {"pivot_mode": 35}),
    ("mo5_of_mo5", {"pivot_mode": 55}),
    ("median_of_sqrt_n", {"pivot_mode": 1}),
    ("median_of_sample", {}),
    ("skew_4", {"pivot_skew": 4}),
    ("skew_16", {"pivot_skew": 16}),
)


def pivot_study(torch, bqs, n, reps=3):
    """The paper's pivot strategies (Section 4: median of 3, 5, 23; medians
    of medians; median of sqrt(n); skewed pivots, here the 1/s quantile of
    the default sample) against the default median of a sample, on the
    headline input."""
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    pristine = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device="cuda", generator=g)
    t = torch.empty_like(pristine)
    out = {}
    for name, params in PIVOT_STRATEGIES:
        ctx = bqs.Context(timing=1, **params)
        times = []
        for r in range(reps + 1):
            t.copy_(pristine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sort(t)
            torch.cuda.synchronize()
            if r:
                times.append(time.perf_counter() - t0)
        st = ctx.stats()
        out[name] = {"ms": round(1e3 * min(times), 3), "levels": st["levels"],
                     "partitioned_keys": st["partitioned_keys"],
                     "partition_ms": round(st["partition_ms"], 3)}
    del pristine, t
    return out


def records(torch, bqs, n=1 << 23, reps=3):
    """The paper's large element types: Vector (10 doubles, by the sum of
    squares) and Record (21 int32, by the first component), n records each;
    every call sorts from a pristine input into an output buffer."""
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    out = {}
    for name, src in (("vector", torch.randn((n, 10), dtype=torch.float64, device="cuda", generator=g)),
                      ("record", torch.randint(-(2**31), 2**31, (n, 21), dtype=torch.int32, device="cuda",
                                               generator=g))):
        dst = torch.empty_like(src)
        ctx = bqs.Context()
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sort_records(src, dst)
            torch.cuda.synchronize()
            if r:
                times.append(time.perf_counter() - t0)
        ms = 1e3 * min(times)
        if name == "vector":
            k = dst[:, 0] * dst[:, 0]
            for i in range(1, 10):
                k = k + dst[:, i] * dst[:, i]
        else:
            k = dst[:, 0]
        ok = bool((k[1:] >= k[:-1]).all())
        out[name] = {"n": n, "record_bytes": src.shape[1] * src.element_size(), "ms": round(ms, 3),
                     "Mrecords/s": round(n / (ms * 1e-3) / 1e6, 1), "sorted": ok}
        del src, dst
    return out


def record_bytes(kind):
    if kind.startswith("i32"):
        return 4
    if kind.startswith("f64"):
        return 8
    return 12  # u64 key + u32 payload


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(torch, n: int, gpu_sorted):
    """The CPU oracle (single-threaded BlockQuicksort, the paper's algorithm)
    on the headline's own input: the same 2^28 seeded keys the timed GPU
    steps sorted, copied to the host.  The host's std::sort is timed beside
    it on the same bytes (the paper's comparison, Section 4), and the
    oracle's output is compared bit for bit with the GPU's."""
    import oracle

    orc = oracle.default()
    host = make_inputs(torch, "i32_uniform", n, 1, 0)[0].cpu().numpy()
    t0 = time.perf_counter()
    out = orc.sort(host)
    t_or = time.perf_counter() - t0
    t0 = time.perf_counter()
    progress("cpu baseline: oracle timed")
    ref = orc.std_sort(host)
    t_std = time.perf_counter() - t0
    same = bool(np.array_equal(out, ref)) and (gpu_sorted is None or bool(np.array_equal(out, gpu_sorted)))
    return {
        "value": round(n / t_or / 1e9, 5),
        "unit": "Gkeys/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the headline input ({n} uniform int32 keys, device seed 0) copied to the host, "
                  f"single-threaded BlockQuicksort oracle, {t_or:.1f} s",
        "ns_per_key": round(t_or / n * 1e9, 2),
        "std_sort": {"Gkeys/s": round(n / t_std / 1e9, 5), "ns_per_key": round(t_std / n * 1e9, 2),
                     "s": round(t_std, 2), "oracle_speedup_over_std_sort": round(t_std / t_or, 3)},
        "matches_gpu_bit_for_bit": same,
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
    }


def cpu_segments(keys, offsets, every=10):
    """The CPU oracle on a bounded sample of the batched workload (every
    `every`-th array): one core, and all host cores with one array per
    task (threads; the oracle's calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    orc = oracle.default()
    pick = np.arange(0, offsets.size - 1, every)
    arrays = [keys[offsets[i]:offsets[i + 1]].copy() for i in pick]
    nk = sum(a.size for a in arrays)
    t0 = time.perf_counter()
    for a in arrays:
        orc.sort(a)
    t1 = time.perf_counter() - t0
    cores = min(os.cpu_count() or 1, 64)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(orc.sort, arrays))
    tc = time.perf_counter() - t0
    return {"sample": f"every {every}th array ({len(arrays)} arrays, {nk} keys)", "keys": nk,
            "one_core": {"Gkeys/s": round(nk / t1 / 1e9, 5), "s": round(t1, 2), "cores": 1},
            "all_cores": {"Gkeys/s": round(nk / tc / 1e9, 5), "s": round(tc, 2), "cores": cores},
            "cpu_model": cpu_model()}


def _csv_rows(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def trace_summary(trace_dir: str, bench_json: str | None, counters: list[str]) -> str:
    """Markdown summary of a rocprofv3 run of this benchmark (written to
    profiles/): per-kernel statistics from --kernel-trace --stats, the
    dispatches of one headline sort with the partition kernel's rate per
    level (keys per level from the benchmark's JSON line of the same run),
    and, from --pmc runs, the HBM bytes of a partition launch (FETCH_SIZE and
    WRITE_SIZE scaled by what they read on the benchmark's 1 GiB copy)."""
    import glob

    out = []
    stats = glob.glob(os.path.join(trace_dir, "*kernel_stats.csv"))
    trace = glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))
    passes = None
    if bench_json:
        with open(bench_json) as f:
            line = [ln for ln in f.read().splitlines() if ln.startswith("{")][-1]
        passes = json.loads(line).get("passes")
    if stats:
        rows = _csv_rows(stats[0])
        out.append("| kernel | calls | total ms | average us |\n|---|---|---|---|")
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
            name = r["Name"].split("(")[0].replace("void ", "")
            name = name if len(name) <= 70 else name[:67] + "..."
            out.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                       f"{float(r['AverageNs']) / 1e3:.2f} |")
    if trace:
        rows = sorted(_csv_rows(trace[0]), key=lambda r: int(r["Start_Timestamp"]))
        starts = [i for i, r in enumerate(rows) if "k_init_single" in r["Kernel_Name"]]
        if len(starts) >= 2:
            # the last sort of the timed headline steps: the third init of a
            # run with one warm-up and two steps
            i0 = starts[min(2, len(starts) - 2)]
            i1 = next((i + 1 for i in range(i0, len(rows)) if "k_persist" in rows[i]["Kernel_Name"]),
                      starts[starts.index(i0) + 1])
            sort = rows[i0:i1]
            t0 = int(sort[0]["Start_Timestamp"])
            t1 = max(int(r["End_Timestamp"]) for r in sort)
            parts = [r for r in sort if "k_partition" in r["Kernel_Name"]]
            out.append(f"\nOne headline sort: {len(sort)} dispatches, {(t1 - t0) / 1e6:.3f} ms first start "
                       f"to last end (under the profiler), "
                       f"{sum(int(r['End_Timestamp']) - int(r['Start_Timestamp']) for r in sort) / 1e6:.3f} ms "
                       "of kernel time.\n")
            out.append("| level | partition us | keys | GB/s (8 B per key) |\n|---|---|---|---|")
            for lv, r in enumerate(parts):
                us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                keys = passes[lv]["keys"] if passes and lv < len(passes) else None
                gbs = f"{8 * keys / (us * 1e-6) / 1e9:.0f}" if keys else "-"
                out.append(f"| {lv} | {us:.1f} | {keys if keys is not None else '-'} | {gbs} |")
            if passes and len(starts) >= 3:
                # the partition launches with tiles of the timed sorts (the
                # second and third inits), the launches bench.py averages
                durs = []
                for j in (1, 2):
                    a0 = starts[j]
                    a1 = next((i for i in range(a0, len(rows)) if "k_persist" in rows[i]["Kernel_Name"]), len(rows))
                    ps = [r for r in rows[a0:a1] if "k_partition" in r["Kernel_Name"]][:len(passes)]
                    durs += [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in ps]
                avg = json.loads(line).get("roofline", {}).get("avg_launch_ms")
                out.append(f"\nk_partition launches with tiles in the two timed sorts: {len(durs)}, average "
                           f"{sum(durs) / len(durs):.1f} us (bench.py's HIP events, same run: "
                           f"{avg * 1e3 if avg else float('nan'):.1f} us)")
    hbm = 0.0
    for cdir in counters:
        rows = _csv_rows(glob.glob(os.path.join(cdir, "*counter_collection.csv"))[0])
        byname = {}
        for r in rows:
            byname.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
        if any(c.startswith("SQ_") for _, c in byname):
            # instruction-mix counters: per-launch means over the launches
            # that did work (wave cycles above 1 % of the kernel's largest)
            kernels = sorted({k for k, _ in byname})
            cnames = sorted({c for _, c in byname})
            out.append("\n| kernel | launches | " + " | ".join(c.replace("SQ_", "") for c in cnames) +
                       " |\n|---|---|" + "---|" * len(cnames))
            for k in kernels:
                wc = byname.get((k, "SQ_WAVE_CYCLES"))
                keep = [i for i, v in enumerate(wc) if v > 0.01 * max(wc)] if wc else None
                cells = []
                for c in cnames:
                    v = byname.get((k, c), [])
                    v = [v[i] for i in keep] if keep is not None else v
                    cells.append(f"{sum(v) / len(v):.3g}" if v else "-")
                name = k.split("(")[0].replace("void ", "")
                out.append(f"| `{name}` | {len(keep) if keep is not None else '-'} | " + " | ".join(cells) + " |")
            continue
        copy = {c: max(v) for (k, c), v in byname.items() if "copyBuffer" in k}
        order = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
        for cname in sorted({c for _, c in byname}):
            # the benchmark's largest copy moves 1 GiB each way: the counter's
            # scale factor
            factor = (1 << 20) / copy[cname] if copy.get(cname) else float("nan")
            # every partition launch of every sort, over the launches that
            # had tiles (more than 64 KiB moved): bench.py's launch count
            total, launches, empty = 0.0, 0, 0
            for r in order:
                if r["Counter_Name"] != cname or "k_partition" not in r["Kernel_Name"]:
                    continue
                v = float(r["Counter_Value"])
                total += v
                launches += v > 64.0
                empty += v <= 64.0
            if not launches:
                continue
            per_launch = total / launches * 1024 * factor
            hbm += per_launch
            out.append(f"- `{cname}` k_partition: {total:.0f} KiB over {launches} launches with tiles "
                       f"(+{empty} without), scale {factor:.4f} (1 GiB copy: "
                       f"{copy.get(cname, float('nan')):.1f} KiB) -> {per_launch:.0f} B per launch")
    if hbm:
        out.append(f"- HBM bytes per partition launch (fetch + write): {hbm:.0f}")
    return "\n".join(out) + "\n"


def progress(msg: str):
    """One line per finished bench section on stderr (the JSON line stays
    alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def inplace_lines(torch, bqs, n, steps):
    """The in-place step (BQS_PARAM_INPLACE) on the headline input and on
    the pairs workload: time, rate and workspace against the default step.
    Algorithmic bytes per in-place level: the count pass reads every key,
    the exchange reads and writes the tiles that hold misplaced keys (about
    every tile on random input): 3 r per partitioned key."""
    out = {}
    for kind, nn, r, vb, code in (("i32_uniform", n, 4, 0, bqs.I32), ("pairs_u64_u32", n // 4, 12, 4, bqs.U64)):
        ctx = bqs.Context(timing=1, inplace=1)
        ms, st, _, part_ms, part_keys, ok = run_workload(torch, bqs, ctx, kind, nn, steps, 1)
        ws_in = bqs.lib.bqs_workspace_bytes(ctx._h, nn, code, vb, 1)
        ws_out = bqs.lib.bqs_workspace_bytes(None, nn, code, vb, 1)
        ab = 3 * r * st["partitioned_keys"] + 2 * r * st["small_sorted_keys"]
        out[kind] = {"n": nn, "ms": round(ms, 3), "Gkeys/s": round(nn / (ms * 1e-3) / 1e9, 3),
                     "alg_GBps": round(ab / (ms * 1e-3) / 1e9, 1),
                     "frac": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "partition_ms": round(st["partition_ms"], 3), "small_ms": round(st["small_ms"], 3),
                     "plan_ms": round(st["plan_ms"], 3), "levels": st["levels"],
                     "workspace_bytes": int(ws_in), "default_workspace_bytes": int(ws_out),
                     "workspace_saved_bytes": int(ws_out - ws_in), "correct": ok}
        ctx.close()
    return out


def main():
    if "--trace-summary" in sys.argv:
        ap = argparse.ArgumentParser()
        ap.add_argument("--trace-summary", required=True, help="rocprofv3 --output-format csv directory")
        ap.add_argument("--bench-json", help="this benchmark's output of the same run")
        ap.add_argument("--counters", nargs="*", default=[], help="rocprofv3 --pmc csv directories")
        a = ap.parse_args()
        print(trace_summary(a.trace_summary, a.bench_json, a.counters), end="")
        return
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the sort runs on one GPU; --gpus must be 1 "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1604_06697_amd as bqs

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    # the timed region records HIP events around the partition kernels only
    ctx = bqs.Context(timing=2)

    kept = [] if not args.no_cpu else None
    ms, st, levels, part_ms, part_keys, ok = run_workload(
        torch, bqs, ctx, "i32_uniform", args.n, args.steps, args.warmup, keep=kept)
    n = args.n
    value = n / (ms * 1e-3) / 1e9
    r = 4
    # dominant kernel: the partition pass; algorithmic bytes = read + write of
    # every key of every partitioned segment (2 * 4 B per key)
    achieved = 2 * r * part_keys / (part_ms * 1e-3) / 1e9 if part_ms > 0 else None
    launches = st["levels"]  # partition launches that had tiles
    passes = [{"level": i, "keys": k, "ms": round(t, 4),
               "GBps": round(2 * r * k / (t * 1e-3) / 1e9, 1) if t > 0 else None}
              for i, (k, t) in enumerate(levels)]
    alg_bytes = 2 * r * (st["partitioned_keys"] + st["small_sorted_keys"]) + r * st["filled_keys"]
    out = {
        "metric": "Gkeys/s and HBM GB/s fraction per distribution; batched p50/p99 latency",
        "value": round(value, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"single array of {n} uniform random int32 keys (full range), "
                               "sorted ascending in place",
                   "n": n, "distribution": "uniform", "seed": 0},
        "correct": ok,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": measured_traffic(),
            "kernel": "k_partition (int32 keys; by level 16384-key tiles of 512 threads, 8192 or 4096 of 256)",
            "bytes_per_launch": round(2 * r * part_keys / max(launches, 1)),
            "avg_launch_ms": round(part_ms / max(launches, 1), 4),
        },
        "whole_sort": {
            "algorithmic_GBps": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
            "frac_of_hbm_peak": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "effective_passes": round(alg_bytes / (2 * r * n), 2),
            "partition_ms": round(part_ms, 3),
            "levels": st["levels"],
        },
        "passes": passes,
        "paper_cpu_context_gkeys": round(PAPER_CPU_GKEYS, 4),
        "copy_context": copy_bandwidth(torch),
    }

    progress(f"headline: {ms:.3f} ms per sort")
    # per-phase breakdown of one more sort with every launch timed (outside
    # the timed region: the extra events cost the host time)
    bctx = bqs.Context(timing=1)
    bms, bst, _, _, _, bok = run_workload(torch, bqs, bctx, "i32_uniform", args.n, 1, 1)
    out["whole_sort"]["breakdown"] = {"ms": round(bms, 3), "partition_ms": round(bst["partition_ms"], 3),
                                      "small_ms": round(bst["small_ms"], 3), "plan_ms": round(bst["plan_ms"], 3),
                                      "correct": bok}

    # the multiway partition step (opt-in; same keys, fewer passes)
    mctx = bqs.Context(timing=1, multiway=1)
    mms, mst, _, mpart_ms, mpart_keys, mok = run_workload(
        torch, bqs, mctx, "i32_uniform", args.n, max(2, args.steps // 2), 1)
    # a multiway pass reads each key twice (count, scatter) and writes it once
    mw_bytes = 3 * r * mst["partitioned_keys"] + 2 * r * mst["small_sorted_keys"] + r * mst["filled_keys"]
    out["multiway"] = {"ms": round(mms, 3), "Gkeys/s": round(n / (mms * 1e-3) / 1e9, 3),
                       "alg_GBps": round(mw_bytes / (mms * 1e-3) / 1e9, 1),
                       "frac": round(mw_bytes / (mms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "partition_ms": round(mst["partition_ms"], 3), "small_ms": round(mst["small_ms"], 3),
                       "plan_ms": round(mst["plan_ms"], 3), "levels": mst["levels"],
                       "partitioned_keys": mst["partitioned_keys"], "small_cutoff": 8192, "correct": mok}

    progress("breakdown and multiway done")
    # the in-place step: keys never leave the caller's buffer, the workspace
    # holds one class bit per key instead of a second copy of the keys
    out["inplace"] = inplace_lines(torch, bqs, n, max(2, args.steps // 2))

    if not args.no_dists:
        dists = {}
        for kind, nn in [("i32_sorted", n), ("i32_reverse", n), ("i32_few_distinct", n),
                         ("i32_all_equal", n), ("f64_uniform", n // 2), ("f64_normal", n // 2),
                         ("f64_sorted_swaps", n // 2), ("pairs_u64_u32", n // 4)]:
            dms, dst, _, dpart_ms, dpart_keys, dok = run_workload(
                torch, bqs, ctx, kind, nn, max(2, args.steps // 2), 1, seed=1)
            rb = record_bytes(kind)
            # equal runs: keys are written once; pairs also park and restore
            # their payloads (side write + side read + final write)
            fill_b = rb if kind != "pairs_u64_u32" else 8 + 3 * 4
            ab = 2 * rb * (dst["partitioned_keys"] + dst["small_sorted_keys"]) + fill_b * dst["filled_keys"]
            dists[kind] = {
                "n": nn, "ms": round(dms, 3), "Gkeys/s": round(nn / (dms * 1e-3) / 1e9, 3),
                "alg_GBps": round(ab / (dms * 1e-3) / 1e9, 1),
                "frac": round(ab / (dms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "partition_GBps": round(2 * rb * dpart_keys / (dpart_ms * 1e-3) / 1e9, 1)
                if dpart_ms > 0 else None,
                "levels": dst["levels"], "correct": dok,
            }
        out["distributions"] = dists

    progress("in-place and distributions done")
    if not args.no_dists:
        out["paper_families"] = paper_families(torch, bqs)
        out["pivot_study"] = pivot_study(torch, bqs, n)
        out["records"] = records(torch, bqs)

    progress("paper families, pivot study and records done")
    if not args.no_batched:
        out["segmented"] = batched_segments(torch, bqs, max(2, args.steps // 3), 2, cpu=not args.no_cpu)

    progress("batched segments done")
    if not args.no_serve:
        out["serving"] = serving(torch, args.serve_requests)
        progress("serving done")

    # persistent mode: every level in one cooperative launch, one host wait.
    # Runs after the serving loop: once a process has made a cooperative
    # launch, its later work on several streams overlaps less (measured:
    # serving capacity 18 -> 11 Gkeys/s).
    if not args.no_persistent:
        pctx = bqs.Context(mode=bqs.MODE_PERSISTENT)
        pms, pst, _, _, _, pok = run_workload(
            torch, bqs, pctx, "i32_uniform", args.n, max(2, args.steps // 2), 1)
        out["persistent"] = {"ms": round(pms, 3), "Gkeys/s": round(n / (pms * 1e-3) / 1e9, 3),
                             "levels": pst["levels"], "partition_launches": pst["partition_launches"],
                             "small_cutoff": pst["small_cutoff"], "correct": pok}

    progress("persistent done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(torch, n, kept[0] if kept else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
