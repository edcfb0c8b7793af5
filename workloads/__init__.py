"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds no sorting arithmetic: it only draws numbers.

Every generator takes an explicit seed and uses numpy's PCG64, so the GPU
library and the CPU oracle sort identical bytes.  The input families follow
the ones the BlockQuicksort paper measures (Section 4 and the appendix
figures): random permutations and uniform integers, few distinct values,
sorted / reversed / transposed permutations, neighbour swaps, constant and
0-1 arrays, and the modular families i mod floor(sqrt n), (i^2 + n/2) mod n,
(i^8 + n/2) mod n.  The float64 and key-value families are the workloads the
library is benchmarked on.
"""

from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- int32 ----

def uniform_i32(n: int, seed: int) -> np.ndarray:
    """Uniform over the whole int32 range."""
    return rng(seed).integers(-(2**31), 2**31, size=n, dtype=np.int32)


def sorted_i32(n: int, seed: int = 0) -> np.ndarray:
    return np.arange(n, dtype=np.int32)


def reverse_i32(n: int, seed: int = 0) -> np.ndarray:
    return np.arange(n - 1, -1, -1, dtype=np.int32)


def few_distinct_i32(n: int, seed: int, distinct: int = 1024) -> np.ndarray:
    """Uniform key reduced to its non-negative residue mod `distinct`
    (a power of two): values 0 .. distinct-1."""
    u = rng(seed).integers(0, 2**32, size=n, dtype=np.uint32)
    return (u & np.uint32(distinct - 1)).astype(np.int32)


def all_equal_i32(n: int, seed: int = 0, value: int = 0x2A) -> np.ndarray:
    return np.full(n, value, dtype=np.int32)


def random_permutation_i32(n: int, seed: int) -> np.ndarray:
    return rng(seed).permutation(n).astype(np.int32)


def uniform_sqrt_i32(n: int, seed: int) -> np.ndarray:
    """Random values between 0 and sqrt(n)."""
    return rng(seed).integers(0, int(math.isqrt(max(n, 1))) + 1, size=n, dtype=np.int32)


def mod_sqrt_i32(n: int, seed: int = 0) -> np.ndarray:
    """A[i] = i mod floor(sqrt n)."""
    m = max(1, math.isqrt(max(n, 1)))
    return (np.arange(n, dtype=np.int64) % m).astype(np.int32)


def square_mod_i32(n: int, seed: int = 0) -> np.ndarray:
    """A[i] = (i^2 + n/2) mod n, in 64-bit arithmetic."""
    i = np.arange(n, dtype=np.uint64)
    nn = np.uint64(max(n, 1))
    return (((i * i) % nn + np.uint64(n // 2)) % nn).astype(np.int32)


def eighth_power_mod_i32(n: int, seed: int = 0) -> np.ndarray:
    """A[i] = (i^8 + n/2) mod n; i^8 mod n by repeated squaring mod n."""
    nn = np.uint64(max(n, 1))
    x = np.arange(n, dtype=np.uint64) % nn
    for _ in range(3):
        # n <= 2^32 keeps x*x below 2^64
        x = (x * x) % nn
    return ((x + np.uint64(n // 2)) % nn).astype(np.int32)


def transposition_i32(n: int, seed: int = 0) -> np.ndarray:
    """A[i] = (i + n/2) mod n."""
    return ((np.arange(n, dtype=np.int64) + n // 2) % max(n, 1)).astype(np.int32)


def neighbour_swaps_i32(n: int, seed: int, k: int | None = None) -> np.ndarray:
    """Sorted permutation with k random swaps of neighbouring elements."""
    a = np.arange(n, dtype=np.int32)
    if n < 2:
        return a
    k = n if k is None else k
    pos = rng(seed).integers(0, n - 1, size=k)
    for p in pos:  # sequential by definition; only used at test sizes
        a[p], a[p + 1] = a[p + 1], a[p]
    return a


def half_zero_one_i32(n: int, seed: int = 0) -> np.ndarray:
    a = np.zeros(n, dtype=np.int32)
    a[n // 2:] = 1
    return a


def random_zero_one_i32(n: int, seed: int) -> np.ndarray:
    return rng(seed).integers(0, 2, size=n, dtype=np.int32)


I32_FAMILIES = {
    "uniform": uniform_i32,
    "sorted": sorted_i32,
    "reverse": reverse_i32,
    "few_distinct": few_distinct_i32,
    "all_equal": all_equal_i32,
}

I32_EXTRA_FAMILIES = {
    "permutation": random_permutation_i32,
    "uniform_sqrt": uniform_sqrt_i32,
    "mod_sqrt": mod_sqrt_i32,
    "square_mod": square_mod_i32,
    "eighth_power_mod": eighth_power_mod_i32,
    "transposition": transposition_i32,
    "neighbour_swaps": neighbour_swaps_i32,
    "half_zero_one": half_zero_one_i32,
    "random_zero_one": random_zero_one_i32,
}


# -------------------------------------------------------------- float64 ----

def uniform_f64(n: int, seed: int) -> np.ndarray:
    """Uniform [0,1) with 53 random bits: (u64 >> 11) * 2^-53."""
    u = rng(seed).integers(0, 2**64, size=n, dtype=np.uint64)
    return (u >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal_f64(n: int, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(n)


def sorted_swaps_f64(n: int, seed: int, fraction: float = 0.01) -> np.ndarray:
    """Sorted uniform [0,1) with floor(fraction*n) swaps of disjoint,
    uniformly drawn index pairs (the first 2k entries of a random
    permutation give the k pairs)."""
    g = rng(seed)
    u = g.integers(0, 2**64, size=n, dtype=np.uint64)
    a = np.sort((u >> np.uint64(11)).astype(np.float64) * (2.0 ** -53))
    k = int(fraction * n)
    if n >= 2 and k:
        perm = g.permutation(n)[: 2 * k]
        i, j = perm[:k], perm[k:]
        a[i], a[j] = a[j].copy(), a[i].copy()
    return a


def special_f64(n: int, seed: int) -> np.ndarray:
    """Adversarial float64 keys: +-0, +-inf, subnormals, extremes and random
    non-NaN bit patterns, shuffled."""
    g = rng(seed)
    fixed = np.array([0.0, -0.0, np.inf, -np.inf, 5e-324, -5e-324, 2.2250738585072014e-308,
                      -2.2250738585072014e-308, 1.7976931348623157e308, -1.7976931348623157e308,
                      1.0, -1.0, 0.5, -0.5], dtype=np.float64)
    bits = g.integers(0, 2**64, size=n, dtype=np.uint64)
    vals = bits.view(np.float64).copy()
    nan = np.isnan(vals)
    vals[nan] = 0.0
    reps = g.integers(0, fixed.size, size=n)
    pick = g.random(n) < 0.5
    vals[pick] = fixed[reps[pick]]
    return vals


F64_FAMILIES = {
    "uniform": uniform_f64,
    "normal": normal_f64,
    "sorted_swaps": sorted_swaps_f64,
}


# ---------------------------------------------------------------- pairs ----

def uniform_u64_pairs(n: int, seed: int):
    """uint64 keys uniform over the full range, uint32 payload = index."""
    keys = rng(seed).integers(0, 2**64, size=n, dtype=np.uint64)
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


def tied_u64_pairs(n: int, seed: int, distinct: int = 64):
    keys = rng(seed).integers(0, distinct, size=n, dtype=np.uint64)
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


# ------------------------------------------------------------- segments ----

def log_uniform_sizes(k: int, seed: int, lo_exp: float = 4.0, hi_exp: float = 20.0) -> np.ndarray:
    """size = min(2^hi, floor(2^lo * (2^(hi-lo))^U)), U ~ U[0,1)."""
    u = rng(seed).random(k)
    sizes = np.floor((2.0 ** lo_exp) * (2.0 ** (hi_exp - lo_exp)) ** u).astype(np.int64)
    return np.minimum(sizes, int(2 ** hi_exp))


def segmented_i32(k: int, seed: int, lo_exp: float = 4.0, hi_exp: float = 20.0):
    """k int32 arrays, sizes log-uniform in [2^lo, 2^hi], uniform keys,
    concatenated; returns (keys, offsets[k+1])."""
    sizes = log_uniform_sizes(k, seed, lo_exp, hi_exp)
    offsets = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    keys = uniform_i32(int(offsets[-1]), seed + 1_000_003)
    return keys, offsets
