"""Pins for the CPU oracle.

The oracle is checked against things it does not compute itself:
  * brute force: every permutation of n <= 8 and every sequence in
    {0..n-1}^n for n <= 6 must come out as the unique ascending sequence;
  * a library routine reached by a special case: numpy's sort of the keys
    (for floats: of the IEEE-754 totalOrder bit transform, written out here
    from the standard, not from the oracle's comparator);
  * closed forms of the paper's input families (sorted output of
    A[i] = i mod m, of permutations, of constant arrays);
  * the partition postcondition of Section 2 (left <= pivot <= right, pivot
    at its rank);
  * the paper's average comparison count for median-of-three Quicksort
    (about 1.18 n log2 n, Section 3.1);
  * the IEEE totalOrder fixture in tests/golden.
A mutation test then plants plausible mistakes into the oracle and checks
that these pins catch every one of them.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as oracle_mod
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (B, insertion threshold): the paper's (128, 16) plus tiny ones so that
# arrays of a handful of elements reach every branch of the final phase.
PARAMS = [(128, 16), (1, 2), (2, 2), (3, 3), (4, 2), (2, 5)]


def all_permutations(n):
    return np.array(list(itertools.permutations(range(n))), dtype=np.int32).reshape(-1)


def all_sequences(n):
    return np.array(list(itertools.product(range(n), repeat=n)), dtype=np.int32).reshape(-1)


def f64_order_bits(a):
    """IEEE 754 totalOrder for non-NaN binary64 as an unsigned integer:
    positive values get the sign bit set, negative values are inverted."""
    b = a.view(np.uint64)
    neg = (b >> np.uint64(63)) == 1
    return np.where(neg, ~b, b | np.uint64(1 << 63))


def check_exhaustive(orc, n, block, is_thresh, seqs=False):
    data = all_sequences(n) if seqs else all_permutations(n)
    k = data.size // n
    offsets = np.arange(k + 1, dtype=np.int64) * n
    out = orc.sort_segments(data, offsets, block=block, is_thresh=is_thresh, check=True)
    expect = np.sort(data.reshape(k, n), axis=1).reshape(-1)
    return np.array_equal(out, expect)


@pytest.mark.parametrize("block,is_thresh", PARAMS)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6, 7, 8])
def test_exhaustive_permutations(oracle, n, block, is_thresh):
    if n == 0:
        assert oracle.sort(np.zeros(0, np.int32)).size == 0
        return
    assert check_exhaustive(oracle, n, block, is_thresh)


@pytest.mark.parametrize("block,is_thresh", PARAMS)
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_exhaustive_sequences_with_duplicates(oracle, n, block, is_thresh):
    assert check_exhaustive(oracle, n, block, is_thresh, seqs=True)


SIZES = [0, 1, 2, 3, 16, 17, 18, 255, 256, 257, 258, 384, 511, 513, 1000, 4099]


@pytest.mark.parametrize("family", sorted({**W.I32_FAMILIES, **W.I32_EXTRA_FAMILIES}))
def test_families_against_numpy(oracle, family):
    gen = {**W.I32_FAMILIES, **W.I32_EXTRA_FAMILIES}[family]
    for n in SIZES:
        for seed in range(3):
            a = gen(n, seed)
            for block, is_thresh in [(128, 16), (4, 2)]:
                out, st = oracle.sort(a, block=block, is_thresh=is_thresh, check=True,
                                      return_stats=True)
                assert np.array_equal(out, np.sort(a)), (family, n, seed, block)
                assert st.check_failures == 0


def test_uniform_large_against_numpy(oracle):
    for seed in range(20):
        a = W.uniform_i32(100_000, seed)
        assert np.array_equal(oracle.sort(a), np.sort(a))
    a = W.uniform_i32(1_000_000, 0)
    assert np.array_equal(oracle.sort(a), np.sort(a))


@pytest.mark.parametrize("dtype", [np.int32, np.uint32, np.int64, np.uint64])
def test_integer_dtypes(oracle, dtype):
    info = np.iinfo(dtype)
    g = W.rng(7)
    a = g.integers(info.min, info.max, size=5000, dtype=dtype, endpoint=True)
    a[:4] = [info.min, info.max, info.min, info.max]
    assert np.array_equal(oracle.sort(a), np.sort(a))


def test_closed_forms(oracle):
    n = 4096
    m = int(math.isqrt(n))
    out = oracle.sort(W.mod_sqrt_i32(n))
    # each residue 0..m-1 occurs n/m times
    assert np.array_equal(out, np.repeat(np.arange(m, dtype=np.int32), n // m))
    for gen in (W.reverse_i32, W.transposition_i32, W.random_permutation_i32):
        assert np.array_equal(oracle.sort(gen(n, 3)), np.arange(n, dtype=np.int32))
    assert np.array_equal(oracle.sort(W.all_equal_i32(n)), np.full(n, 0x2A, np.int32))
    z = oracle.sort(W.random_zero_one_i32(n, 5))
    ones = int(W.random_zero_one_i32(n, 5).sum())
    assert np.array_equal(z, np.r_[np.zeros(n - ones, np.int32), np.ones(ones, np.int32)])


def test_f64_total_order_golden(oracle):
    rows = [ln.split()[0] for ln in open(os.path.join(GOLDEN, "f64_total_order.txt"))
            if ln.strip() and not ln.startswith("#")]
    ordered = np.array([int(h, 16) for h in rows], dtype=np.uint64).view(np.float64)
    g = W.rng(11)
    for _ in range(50):
        shuffled = ordered[g.permutation(ordered.size)]
        out = oracle.sort(np.repeat(shuffled, 9), block=2, is_thresh=2)
        assert np.array_equal(out.view(np.uint64), np.repeat(ordered, 9).view(np.uint64))


def test_f64_special_values_against_bit_transform(oracle):
    for seed in range(5):
        a = W.special_f64(20_000, seed)
        out = oracle.sort(a)
        expect = a[np.argsort(f64_order_bits(a), kind="stable")]
        assert np.array_equal(out.view(np.uint64), expect.view(np.uint64))
    zeros = np.array([0.0, -0.0] * 50)
    out = oracle.sort(zeros)
    assert np.all(np.signbit(out[:50])) and not np.any(np.signbit(out[50:]))


def test_f32_total_order(oracle):
    with np.errstate(over="ignore"):
        a = W.special_f64(5000, 1).astype(np.float32)
    a = np.where(np.isnan(a), np.float32(0), a)
    b = a.view(np.uint32)
    key = np.where((b >> np.uint32(31)) == 1, ~b, b | np.uint32(1 << 31))
    assert np.array_equal(oracle.sort(a).view(np.uint32), a[np.argsort(key, kind="stable")].view(np.uint32))


def test_nan_rejected(oracle):
    with pytest.raises(oracle_mod.OracleError):
        oracle.sort(np.array([1.0, np.nan, 0.0]))


def test_float_families(oracle):
    for name, gen in W.F64_FAMILIES.items():
        a = gen(50_000, 2)
        assert np.array_equal(oracle.sort(a), np.sort(a)), name


def test_partition_postcondition(oracle):
    g = W.rng(3)
    for n in [3, 4, 5, 17, 64, 255, 256, 257, 258, 300, 1000, 5000]:
        for block in [1, 2, 3, 128]:
            for dist in range(3):
                if dist == 0:
                    a = g.integers(-50, 50, size=n).astype(np.int32)
                elif dist == 1:
                    a = g.permutation(n).astype(np.int32)
                else:
                    a = np.full(n, 7, np.int32)
                out, cut = oracle.partition(a, block=block)
                assert np.array_equal(np.sort(out), np.sort(a))
                p = out[cut]
                assert np.all(out[:cut] <= p) and np.all(out[cut + 1:] >= p)
                assert p == np.sort(a)[cut]  # pivot sits at its rank


def test_heapsort_fallback(oracle):
    a = W.uniform_i32(10_000, 4)
    out, st = oracle.sort(a, depth_limit=0, return_stats=True)
    assert st.heapsorts == 1 and st.partitions == 0
    assert np.array_equal(out, np.sort(a))
    out, st = oracle.sort(a, depth_limit=3, return_stats=True)
    assert st.heapsorts > 0 and np.array_equal(out, np.sort(a))


def test_comparison_count_matches_paper(oracle):
    consts = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    c = consts["median_of_3_comparisons_leading_coefficient"]["value"]
    n = 1 << 20
    ratios = []
    for seed in range(3):
        a = W.random_permutation_i32(n, seed)
        _, st = oracle.sort(a, return_stats=True)
        ratios.append(st.comparisons / (n * math.log2(n)))
    r = float(np.mean(ratios))
    # leading term c n log2 n plus an O(n) term (insertion sort, sampling)
    assert abs(r - c) < 0.12, r


def test_depth_limit_default(oracle):
    # sorted input with median-of-three never needs the fallback
    _, st = oracle.sort(W.sorted_i32(1 << 16), return_stats=True)
    assert st.heapsorts == 0


def test_pairs_payload_travels_with_key(oracle):
    for n, seed in [(0, 0), (1, 0), (17, 1), (1000, 2), (100_000, 3)]:
        keys, vals = W.uniform_u64_pairs(n, seed)
        ko, vo = oracle.sort_pairs(keys, vals)
        assert np.array_equal(ko, np.sort(keys))
        assert np.array_equal(np.sort(vo), np.arange(n, dtype=np.uint32))
        assert np.array_equal(keys[vo], ko)
    keys, vals = W.tied_u64_pairs(50_000, 9)
    ko, vo = oracle.sort_pairs(keys, vals)
    assert np.array_equal(ko, np.sort(keys)) and np.array_equal(keys[vo], ko)
    assert np.array_equal(np.sort(vo), np.arange(keys.size, dtype=np.uint32))


def test_segments(oracle):
    keys, offsets = W.segmented_i32(200, 5, 0.0, 12.0)
    out = oracle.sort_segments(keys, offsets)
    for i in range(offsets.size - 1):
        s, e = offsets[i], offsets[i + 1]
        assert np.array_equal(out[s:e], np.sort(keys[s:e]))


# --------------------------------------------------------------- mutation --

MUTANTS = range(1, 9)


def pins_pass(orc):
    """A compact run of the pins above against one oracle build."""
    try:
        for n in range(2, 8):
            for block, is_thresh in PARAMS:
                if not check_exhaustive(orc, n, block, is_thresh):
                    return False
        for n in range(2, 6):
            for block, is_thresh in PARAMS:
                if not check_exhaustive(orc, n, block, is_thresh, seqs=True):
                    return False
        for seed in range(3):
            a = W.uniform_i32(5000, seed)
            if not np.array_equal(orc.sort(a), np.sort(a)):
                return False
            if not np.array_equal(orc.sort(a, depth_limit=2), np.sort(a)):
                return False
        a = W.special_f64(2000, 0)
        expect = a[np.argsort(f64_order_bits(a), kind="stable")]
        if not np.array_equal(orc.sort(a).view(np.uint64), expect.view(np.uint64)):
            return False
    except oracle_mod.OracleError:
        return False
    return True


def test_unmutated_passes_compact_pins(oracle):
    assert pins_pass(oracle)


@pytest.mark.parametrize("mutant", MUTANTS)
def test_planted_mistakes_are_caught(tmp_path, mutant):
    path = str(tmp_path / f"liboracle_m{mutant}.so")
    oracle_mod.compile_library(path, mutant=mutant)
    orc = oracle_mod.Oracle(path)
    assert orc.mutant() == mutant
    assert not pins_pass(orc), f"mutant {mutant} survived the pins"


# ------------------------------------------------------------------ records --
# The paper's Vector (10 x float64, by the sum of squares) and Record
# (21 x int32, by the first component) types.

def _sum_sq(v):
    # left to right, every product and sum rounded, as the comparator does
    s = v[:, 0] * v[:, 0]
    for i in range(1, 10):
        s = s + v[:, i] * v[:, i]
    return s


def _rows_sorted(a):
    return a[np.lexsort(a.T[::-1])]


@pytest.mark.parametrize("n", [0, 1, 2, 17, 1000, 50_000])
def test_oracle_vector_records(oracle, n):
    v = np.random.default_rng(n + 5).standard_normal((n, 10))
    out = oracle.sort_records(v, check=True)
    assert oracle.last.check_failures == 0
    k = _sum_sq(out)
    assert np.all(k[1:] >= k[:-1])
    assert np.array_equal(k, np.sort(_sum_sq(v)))
    assert np.array_equal(_rows_sorted(out), _rows_sorted(v))


@pytest.mark.parametrize("n", [0, 1, 3, 1000, 60_000])
def test_oracle_record_records_with_ties(oracle, n):
    rng = np.random.default_rng(n + 9)
    r = rng.integers(-2**31, 2**31 - 1, size=(n, 21), dtype=np.int32)
    r[:, 0] = rng.integers(-8, 8, size=n)  # many equal keys
    out = oracle.sort_records(r, check=True)
    assert oracle.last.check_failures == 0
    assert np.array_equal(out[:, 0], np.sort(r[:, 0]))
    assert np.array_equal(_rows_sorted(out), _rows_sorted(r))
    # the order among equal keys is a valid one: only the first field is compared
    assert np.all(np.diff(out[:, 0].astype(np.int64)) >= 0)


def test_oracle_records_reject_other_shapes(oracle):
    import oracle as O

    with pytest.raises(O.OracleError):
        oracle.sort_records(np.zeros((4, 9)))
    with pytest.raises(O.OracleError):
        oracle.sort_records(np.zeros((4, 21), dtype=np.int64))
