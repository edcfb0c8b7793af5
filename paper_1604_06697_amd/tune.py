"""Autotuner for the launch plan of the block-partition sort.

A plan is (keys per thread in a partition tile, small-segment cutoff,
partition step, pivot strategy).  The tile size sets how many keys one
workgroup scans and how many output-range claims a pass makes; the cutoff
sets where the recursion stops and the in-LDS sort takes over (the paper's
Insertionsort threshold, Section 2); the step is the paper's two-way block
partition or the multiway (sample-sort) step for keys-only int32 sorts; the
pivot strategy is one of the paper's (Section 4).  None of them changes the
result: keys come out bit for bit the same under every plan.

`autotune` times every candidate plan on the caller's own input (sorted from
a pristine copy each time, in the same mode the caller will use) and keeps
the fastest.  Results are cached in a JSON file keyed by key type, payload
width and the powers of two of the key and segment counts, so that inputs of
the same shape class reuse the measurement.
"""

from __future__ import annotations

import json
import math
import os
import time

import torch

from . import BqsError, Context, _key_code

EPT_CHOICES = (8, 16, 32)
CUTOFF_CHOICES = (1024, 2048, 4096, 8192, 16384)
PIVOT_CHOICES = (0, 55)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_plans.json")


def plan_key(n: int, k: int, key_code: int, val_bytes: int) -> str:
    """Shape class of a call: key type, payload width, and n and k rounded
    to the nearest power of two."""
    ln = int(round(math.log2(max(n, 1))))
    lk = int(round(math.log2(max(k, 1))))
    return f"dtype{key_code}:v{val_bytes}:n2^{ln}:k2^{lk}"


def candidates(key_code: int, val_bytes: int) -> list[dict]:
    """Plans the library compiles for this key type: the tile shape is
    selectable for int32 keys only; the cutoff is clamped by the library to
    the largest in-LDS size it compiles for the type; keys-only int32 sorts
    also try the multiway partition step; two-way plans try the default
    sampled median and the median of five medians of five (Section 4's
    fastest strategy for int keys) as pivot."""
    i32 = key_code == 1 and val_bytes == 0
    epts = EPT_CHOICES if i32 else (0,)
    out = [{"tile_ept": e, "small_cutoff": c, "multiway": 0, "pivot_mode": pm}
           for pm in PIVOT_CHOICES for e in epts for c in CUTOFF_CHOICES]
    if i32:
        out += [{"tile_ept": e, "small_cutoff": c, "multiway": 1, "pivot_mode": 0}
                for e in epts for c in CUTOFF_CHOICES]
    return out


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(n: int, k: int, key_code: int, val_bytes: int = 0, path: str = DEFAULT_CACHE):
    """The cached plan for this shape class, or None."""
    entry = load_cache(path).get(plan_key(n, k, key_code, val_bytes))
    return None if entry is None else dict(entry["plan"])


def _time_plan(plan, keys, vals, offsets, pristine_k, pristine_v, key_type, graph, reps):
    ctx = Context(graph=1 if graph else 0, **plan)
    times = []
    for r in range(reps + 1):
        keys.copy_(pristine_k)
        if vals is not None:
            vals.copy_(pristine_v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if offsets is not None:
            ctx.sort_segments(keys, offsets, key_type=key_type)
        elif vals is not None:
            ctx.sort_pairs(keys, vals, key_type=key_type)
        else:
            ctx.sort(keys, key_type=key_type)
        torch.cuda.synchronize()
        if r > 0:  # the first run warms up (and captures, in graph mode)
            times.append(time.perf_counter() - t0)
    times.sort()
    return 1e3 * times[len(times) // 2]


def autotune(keys: torch.Tensor, offsets: torch.Tensor | None = None, vals: torch.Tensor | None = None,
             key_type=None, graph: bool = False, reps: int = 2, path: str | None = DEFAULT_CACHE) -> dict:
    """Times every candidate plan on this input and returns
    {"key", "plan", "ms", "table"}; `keys` (and `vals`) are left sorted.
    With `path`, the result is stored in the cache file."""
    code = _key_code(keys, key_type)
    vb = 0 if vals is None else vals.element_size()
    k = 1 if offsets is None else offsets.numel() - 1
    pristine_k = keys.clone()
    pristine_v = None if vals is None else vals.clone()
    table = []
    for plan in candidates(code, vb):
        try:
            ms = _time_plan(plan, keys, vals, offsets, pristine_k, pristine_v, key_type, graph, reps)
        except BqsError:
            continue  # a plan this key type does not compile
        table.append({"plan": plan, "ms": round(ms, 4)})
    if not table:
        raise BqsError(2, "autotune: no candidate plan runs for this key type")
    best = min(table, key=lambda e: e["ms"])
    out = {"key": plan_key(keys.numel(), k, code, vb), "plan": best["plan"], "ms": best["ms"], "table": table}
    if path:
        cache = load_cache(path)
        cache[out["key"]] = {"plan": best["plan"], "ms": best["ms"]}
        save_cache(cache, path)
    return out


def tuned_context(n: int, k: int, key_code: int, val_bytes: int = 0, path: str = DEFAULT_CACHE,
                  **extra) -> Context:
    """A context with the cached plan for this shape class (library defaults
    when none is cached) plus any extra parameters."""
    plan = lookup(n, k, key_code, val_bytes, path) or {}
    plan.update(extra)
    return Context(**plan)
