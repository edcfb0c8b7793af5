"""GPU parity tests: the HIP library against the CPU oracle, element by
element, on the same seeded inputs.  Keys must match bit for bit (the sorted
sequence of a totally ordered key set is unique).  For key-value pairs the
keys must match and every payload must travel with its key (the order of
payloads among equal keys is not unique: Quicksort is unstable).
"""

import sys

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


_KT = {np.dtype(np.int32): "i32", np.dtype(np.uint32): "u32", np.dtype(np.float32): "f32",
       np.dtype(np.int64): "i64", np.dtype(np.uint64): "u64", np.dtype(np.float64): "f64"}
_HOLD = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}


def to_dev(torch, a):
    hold = _HOLD.get(a.dtype)
    src = a.view(hold) if hold is not None else a
    return torch.from_numpy(np.ascontiguousarray(src)).cuda()


def from_dev(t, dtype):
    return t.cpu().numpy().view(dtype)


def gpu_sort(torch, bqs, a, ctx=None):
    t = to_dev(torch, a)
    c = ctx or bqs.default_context()
    c.sort(t, key_type=_KT[a.dtype])
    c.synchronize()  # waits, and raises for a device-detected error
    return from_dev(t, a.dtype)


def assert_same_bits(got, expect):
    assert got.dtype == expect.dtype and got.shape == expect.shape
    if not np.array_equal(got.view(f"u{got.itemsize}"), expect.view(f"u{expect.itemsize}")):
        diff = np.flatnonzero(got.view(f"u{got.itemsize}") != expect.view(f"u{expect.itemsize}"))
        raise AssertionError(f"{diff.size} positions differ, first at {diff[:8]}: "
                             f"got {got[diff[:4]]} expect {expect[diff[:4]]}")


# ------------------------------------------------------------------ keys --

def test_config0_million_uniform_int32(torch_mod, bqs, oracle):
    """1,000,000 uniform int32 keys: the oracle with the paper's parameters
    (median-of-three, B = 128, insertion sort <= 16) against the GPU, with
    both the default pivot sample and median-of-three on the GPU."""
    for seed in range(3):
        a = W.uniform_i32(1_000_000, seed)
        expect = oracle.sort(a)
        note(f"config0 seed={seed} default plan")
        assert_same_bits(gpu_sort(torch_mod, bqs, a), expect)
        note(f"config0 seed={seed} median-of-3")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, bqs.Context(pivot_mode=3)), expect)


RAGGED = [0, 1, 2, 3, 5, 17, 64, 65, 100, 1000, 4095, 4096, 4097, 8191, 8192, 8193, 8194,
          12295, 16384, 65537, 100_003, (1 << 20) + 13]


@pytest.mark.parametrize("family", sorted(W.I32_FAMILIES))
def test_i32_families_ragged_sizes(torch_mod, bqs, oracle, family):
    gen = W.I32_FAMILIES[family]
    for n in RAGGED:
        a = gen(n, n + 1)
        note(f"i32 {family} n={n}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a), oracle.sort(a))


@pytest.mark.parametrize("family", sorted(W.I32_EXTRA_FAMILIES))
def test_i32_paper_families(torch_mod, bqs, oracle, family):
    gen = W.I32_EXTRA_FAMILIES[family]
    for n in [1000, 50_000, 300_001]:
        a = gen(n, 7) if family != "neighbour_swaps" else gen(n, 7, k=n // 10)
        note(f"i32 {family} n={n}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a), oracle.sort(a))


@pytest.mark.parametrize("cutoff,ept", [(2, 16), (16, 8), (100, 32), (300, 16), (1000, 8)])
def test_deep_recursion_small_cutoffs(torch_mod, bqs, oracle, cutoff, ept):
    """Tiny small-sort cutoffs force many partition levels, one-tile and
    multi-tile segments, and every tile shape."""
    ctx = bqs.Context(small_cutoff=cutoff, tile_ept=ept)
    for fam, n in [("uniform", 200_003), ("few_distinct", 100_000), ("sorted", 70_001),
                   ("reverse", 33_333), ("all_equal", 50_000)]:
        a = W.I32_FAMILIES[fam](n, 3)
        note(f"cutoff={cutoff} ept={ept} {fam} n={n}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))


@pytest.mark.parametrize("dtype", [np.uint32, np.int64, np.uint64])
def test_integer_dtypes(torch_mod, bqs, oracle, dtype):
    info = np.iinfo(dtype)
    for n in [3, 1000, 9000, 250_001]:
        a = W.rng(n).integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)
        a[: min(4, n)] = [info.min, info.max, info.min, info.max][: min(4, n)]
        note(f"{np.dtype(dtype).name} n={n}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a), oracle.sort(a))


def test_float64_families(torch_mod, bqs, oracle):
    for name, gen in W.F64_FAMILIES.items():
        for n in [5000, 300_007]:
            a = gen(n, 4)
            note(f"f64 {name} n={n}")
            assert_same_bits(gpu_sort(torch_mod, bqs, a), oracle.sort(a))


def test_float_special_values(torch_mod, bqs, oracle):
    for n in [100, 10_000, 200_000]:
        a = W.special_f64(n, n)
        note(f"f64 special n={n}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a), oracle.sort(a))
        with np.errstate(over="ignore"):
            f = a.astype(np.float32)
        note(f"f32 special n={n}")
        assert_same_bits(gpu_sort(torch_mod, bqs, f), oracle.sort(f))
    z = np.array([0.0, -0.0] * 6000)
    note("f64 zeros")
    out = gpu_sort(torch_mod, bqs, z)
    assert np.all(np.signbit(out[:6000])) and not np.any(np.signbit(out[6000:]))


# ----------------------------------------------------------------- pairs --

def check_pairs(keys_in, ko, vo, expect_keys):
    assert_same_bits(ko, expect_keys)
    n = keys_in.size
    assert np.array_equal(np.sort(vo.astype(np.int64)), np.arange(n))
    assert np.array_equal(keys_in[vo.astype(np.int64)].view(np.uint64 if keys_in.itemsize == 8 else np.uint32),
                          ko.view(np.uint64 if ko.itemsize == 8 else np.uint32))


def gpu_pairs(torch, bqs, k, v, ctx=None):
    tk = to_dev(torch, k)
    tv = to_dev(torch, v)
    c = ctx or bqs.default_context()
    c.sort_pairs(tk, tv, key_type=_KT[k.dtype])
    c.synchronize()
    return from_dev(tk, k.dtype), from_dev(tv, v.dtype)


@pytest.mark.parametrize("n", [2, 17, 2047, 2048, 2049, 4097, 100_000, 1 << 20])
def test_pairs_u64_u32(torch_mod, bqs, oracle, n):
    k, v = W.uniform_u64_pairs(n, n)
    note(f"pairs u64/u32 n={n}")
    ko, vo = gpu_pairs(torch_mod, bqs, k, v)
    check_pairs(k, ko, vo, oracle.sort(k))


def test_pairs_with_ties_and_payload_widths(torch_mod, bqs, oracle):
    for n in [5000, 300_000]:
        k, v = W.tied_u64_pairs(n, 3)
        note(f"pairs tied u64/u32 n={n}")
        ko, vo = gpu_pairs(torch_mod, bqs, k, v)
        check_pairs(k, ko, vo, oracle.sort(k))
        note(f"pairs tied u64/u64 n={n}")
        ko, vo = gpu_pairs(torch_mod, bqs, k, v.astype(np.uint64))
        check_pairs(k, ko, vo, oracle.sort(k))
        a = W.few_distinct_i32(n, 5)
        note(f"pairs i32/u32 few-distinct n={n}")
        ko, vo = gpu_pairs(torch_mod, bqs, a, np.arange(n, dtype=np.uint32))
        check_pairs(a, ko, vo, oracle.sort(a))
        f = W.special_f64(n, 2)
        note(f"pairs f64/u32 specials n={n}")
        ko, vo = gpu_pairs(torch_mod, bqs, f, np.arange(n, dtype=np.uint32))
        check_pairs(f, ko, vo, oracle.sort(f))


def test_pairs_deterministic(torch_mod, bqs):
    k, v = W.tied_u64_pairs(400_000, 8, distinct=16)
    note("pairs determinism")
    a = gpu_pairs(torch_mod, bqs, k, v)
    b = gpu_pairs(torch_mod, bqs, k, v)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# -------------------------------------------------------------- segments --

def gpu_segments(torch, bqs, keys, offsets, ctx=None):
    t = to_dev(torch, keys)
    o = torch.from_numpy(offsets).cuda()
    c = ctx or bqs.default_context()
    c.sort_segments(t, o, key_type=_KT[keys.dtype])
    c.synchronize()
    return from_dev(t, keys.dtype)


def test_segments_log_uniform(torch_mod, bqs, oracle):
    for k, hi in [(1, 10.0), (50, 14.0), (2000, 16.0)]:
        keys, offsets = W.segmented_i32(k, k, 0.0, hi)
        note(f"segments k={k} n={keys.size}")
        assert_same_bits(gpu_segments(torch_mod, bqs, keys, offsets),
                         oracle.sort_segments(keys, offsets))


def test_segments_with_empty_and_single(torch_mod, bqs, oracle):
    sizes = np.array([0, 1, 0, 2, 9000, 0, 1, 30_000, 3, 0], dtype=np.int64)
    offsets = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    keys = W.uniform_i32(int(offsets[-1]), 1)
    note("segments with empties")
    assert_same_bits(gpu_segments(torch_mod, bqs, keys, offsets), oracle.sort_segments(keys, offsets))


def test_segments_exhaustive_permutations(torch_mod, bqs, oracle):
    """Every permutation of 8 keys (40,320 segments) in one call."""
    import itertools

    perms = np.array(list(itertools.permutations(range(8))), dtype=np.int32).reshape(-1)
    offsets = np.arange(perms.size // 8 + 1, dtype=np.int64) * 8
    note("segments all 8! permutations")
    out = gpu_segments(torch_mod, bqs, perms, offsets)
    assert np.array_equal(out, np.tile(np.arange(8, dtype=np.int32), perms.size // 8))
    seqs = np.array(list(itertools.product(range(6), repeat=6)), dtype=np.int32).reshape(-1)
    offs = np.arange(seqs.size // 6 + 1, dtype=np.int64) * 6
    note("segments all 6^6 sequences")
    assert_same_bits(gpu_segments(torch_mod, bqs, seqs, offs), oracle.sort_segments(seqs, offs))


def test_segments_pairs_match_oracle(torch_mod, bqs, oracle):
    """Segmented pairs: per segment, keys equal the oracle's and every
    payload (the record's original index) travels with its key."""
    torch = torch_mod
    sizes = np.r_[W.log_uniform_sizes(300, 8, 0.0, 15.0), [0, 1, 2, 70_000]].astype(np.int64)
    offsets = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    n = int(offsets[-1])
    for kt, gen in (("u64", lambda: W.uniform_u64_pairs(n, 12)[0]),
                    ("u64", lambda: W.tied_u64_pairs(n, 13)[0]),
                    ("f64", lambda: W.uniform_f64(n, 14))):
        keys = gen()
        vals = np.arange(n, dtype=np.uint32)
        note(f"segments pairs {kt} n={n}")
        tk = to_dev(torch, keys)
        tv = torch.from_numpy(vals.view(np.int32)).cuda()
        bqs.sort_segments_pairs(tk, tv, torch.from_numpy(offsets).cuda(), key_type=kt)
        torch.cuda.synchronize()
        ko = from_dev(tk, keys.dtype)
        vo = tv.cpu().numpy().view(np.uint32).astype(np.int64)
        # the payloads are a permutation of the indexes: none lost, none
        # duplicated (a payload copied twice among equal keys would keep the
        # key check below green)
        assert np.array_equal(np.sort(vo), np.arange(n))
        for i in range(len(sizes)):
            lo, hi = offsets[i], offsets[i + 1]
            assert_same_bits(ko[lo:hi], oracle.sort(keys[lo:hi]))
            assert np.all((vo[lo:hi] >= lo) & (vo[lo:hi] < hi))
        assert np.array_equal(keys[vo].view(np.uint64), ko.view(np.uint64))


def test_segments_bad_offsets_reported(torch_mod, bqs):
    keys = W.uniform_i32(1000, 0)
    bad = np.array([0, 600, 500, 1000], dtype=np.int64)
    note("segments bad offsets")
    with pytest.raises(bqs.BqsError) as e:
        gpu_segments(torch_mod, bqs, keys, bad)
    assert e.value.status == 1


# ---------------------------------------------------------- claim modes --

@pytest.mark.parametrize("lookback", [0, 1])
def test_claim_modes_match_oracle(torch_mod, bqs, oracle, lookback):
    """Keys-only tiles claim their output ranges with the segment's cursors
    (default) or by decoupled look-back; both must give the oracle's keys,
    across tile-aligned and ragged sizes and duplicate-heavy inputs."""
    ctx = bqs.Context(lookback=lookback, small_cutoff=1024)
    for fam in ("uniform", "few_distinct", "sorted", "all_equal"):
        for n in (8192 * 3, 8192 * 7 + 5, 1 << 20):
            a = W.I32_FAMILIES[fam](n, 9)
            note(f"claim lookback={lookback} {fam} n={n}")
            assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    keys, offsets = W.segmented_i32(500, 2, 4.0, 16.0)
    note(f"claim lookback={lookback} segments n={keys.size}")
    assert_same_bits(gpu_segments(torch_mod, bqs, keys, offsets, ctx), oracle.sort_segments(keys, offsets))


def test_lookback_layout_is_deterministic(torch_mod, bqs):
    """With the look-back every tile's runs land in tile order, so pivots and
    the whole recursion repeat exactly: the per-level counts of two runs are
    equal."""
    a = W.uniform_i32(3_000_017, 4)
    ctx = bqs.Context(lookback=1, timing=1)
    runs = []
    for r in range(2):
        note(f"lookback determinism run {r}")
        gpu_sort(torch_mod, bqs, a, ctx)
        s = ctx.stats()
        runs.append((s["levels"], s["partitioned_keys"], s["small_sorted_keys"], [k for k, _ in ctx.levels()]))
    assert runs[0] == runs[1]


# ------------------------------------------------------------- multiway --

@pytest.mark.parametrize("cut", [256, 4096])
def test_multiway_int32_families(torch_mod, bqs, oracle, cut):
    """Multiway levels (up to 15 splitters, equal-key buckets finished at
    once) against the oracle: every int32 family of the paper's benchmark
    and the duplicate-heavy ones, tile-aligned and ragged sizes."""
    ctx = bqs.Context(multiway=1, small_cutoff=cut)
    fams = dict(W.I32_FAMILIES)
    fams.update(W.I32_EXTRA_FAMILIES)
    for fam, gen in fams.items():
        for n in (8192 * 3, 8192 * 7 + 5, 1_000_003):
            a = gen(n, 21)
            note(f"multiway cut={cut} {fam} n={n}")
            assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))


def test_multiway_key_types_and_specials(torch_mod, bqs, oracle):
    ctx = bqs.Context(multiway=1, small_cutoff=512)
    rng = np.random.Generator(np.random.PCG64(31))
    for dt in (np.uint32, np.int64, np.uint64):
        a = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=700_001, dtype=dt, endpoint=True)
        note(f"multiway {np.dtype(dt).name}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    for fam, gen in W.F64_FAMILIES.items():
        a = gen(600_007, 5)
        note(f"multiway f64 {fam}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    for n in (10_000, 200_000):
        a = W.special_f64(n, n)
        note(f"multiway f64 special n={n}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
        with np.errstate(over="ignore"):
            f = a.astype(np.float32)
        assert_same_bits(gpu_sort(torch_mod, bqs, f, ctx), oracle.sort(f))
    z = np.array([0.0, -0.0] * 60000)
    note("multiway f64 zeros")
    out = gpu_sort(torch_mod, bqs, z, ctx)
    assert np.all(np.signbit(out[:60000])) and not np.any(np.signbit(out[60000:]))


def test_multiway_segments_and_graph(torch_mod, bqs, oracle):
    torch = torch_mod
    keys, offsets = W.segmented_i32(800, 6, 4.0, 17.0)
    ctx = bqs.Context(multiway=1)
    note(f"multiway segments n={keys.size}")
    assert_same_bits(gpu_segments(torch, bqs, keys, offsets, ctx), oracle.sort_segments(keys, offsets))
    # graph replays on one set of buffers, with a deeper input after a shallow one
    gctx = bqs.Context(multiway=1, graph=1)
    buf = torch.empty(keys.size, dtype=torch.int32, device="cuda")
    off = torch.from_numpy(offsets).cuda()
    for i, (fam, seed) in enumerate([("few_distinct", 1), ("uniform", 2), ("uniform", 3), ("sorted", 0)]):
        a = W.I32_FAMILIES[fam](keys.size, seed)
        note(f"multiway graph replay {i} {fam}")
        buf.copy_(torch.from_numpy(a))
        gctx.sort_segments(buf, off)
        torch.cuda.synchronize()
        assert_same_bits(buf.cpu().numpy(), oracle.sort_segments(a, offsets))
        assert gctx.stats()["graph_launches"] == 1  # the first call captures and launches


def test_multiway_graph_single_array(torch_mod, bqs, oracle):
    """Graph replays of multiway levels on one array: a level can hold up to
    sixteen children per segment, so the captured tile grids must cover
    them (regression: grids sized for two children left tiles unsorted)."""
    torch = torch_mod
    n = 3_000_017
    ctx = bqs.Context(multiway=1, graph=1)
    buf = torch.empty(n, dtype=torch.int32, device="cuda")
    for i, (fam, seed) in enumerate([("uniform", 1), ("uniform", 2), ("few_distinct", 3), ("uniform", 4)]):
        a = W.I32_FAMILIES[fam](n, seed)
        note(f"multiway graph single array {i} {fam}")
        buf.copy_(torch.from_numpy(a))
        ctx.sort(buf)
        torch.cuda.synchronize()
        assert_same_bits(buf.cpu().numpy(), oracle.sort(a))
        if i:
            assert ctx.stats()["graph_launches"] == 1


def test_multiway_pairs_use_two_way(torch_mod, bqs, oracle):
    """Pairs keep the two-way step; the parameter only changes keys-only sorts."""
    k, v = W.tied_u64_pairs(300_000, 3)
    ctx = bqs.Context(multiway=1)
    note("multiway param with pairs")
    ko, vo = gpu_pairs(torch_mod, bqs, k, v, ctx)
    check_pairs(k, ko, vo, oracle.sort(k))


# ------------------------------------------------------------ graph mode --

def test_graph_replays_match_oracle(torch_mod, bqs, oracle):
    """Graph mode on one set of buffers: the first call runs host-driven and
    captures; later calls replay the graph.  Eager work and synchronisations
    run between the replays, and every replay is compared with the oracle.
    A uniform input after a few-distinct one needs more levels than the
    first graph holds: the host-driven loop finishes it and a deeper graph
    is captured for the next calls."""
    torch = torch_mod
    keys0, offsets = W.segmented_i32(300, 11, 4.0, 16.0)
    n = keys0.size
    ctx = bqs.Context(graph=1)
    buf = torch.empty(n, dtype=torch.int32, device="cuda")
    off = torch.from_numpy(offsets).cuda()
    seq = [("few_distinct", 3), ("uniform", 4), ("uniform", 5), ("few_distinct", 6),
           ("reverse", 0), ("all_equal", 0), ("uniform", 7)]
    for i, (fam, seed) in enumerate(seq):
        a = W.I32_FAMILIES[fam](n, seed)
        note(f"graph replay {i}: segments {fam} seed {seed} n={n}")
        buf.copy_(torch.from_numpy(a))
        junk = (buf.to(torch.float32) * 2.0).sum()  # eager work on the same stream
        ctx.sort_segments(buf, off)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert_same_bits(buf.cpu().numpy(), oracle.sort_segments(a, offsets))
        s = ctx.stats()
        assert s["graph_launches"] == 1
        assert s["small_sorted_keys"] + s["filled_keys"] <= n


def test_graph_single_array_and_pairs(torch_mod, bqs, oracle):
    torch = torch_mod
    n = 1_000_003
    ctx = bqs.Context(graph=1)
    buf = torch.empty(n, dtype=torch.int32, device="cuda")
    for r in range(3):
        a = W.uniform_i32(n, 20 + r)
        note(f"graph single array replay {r}")
        buf.copy_(torch.from_numpy(a))
        ctx.sort(buf)
        torch.cuda.synchronize()
        assert_same_bits(buf.cpu().numpy(), oracle.sort(a))
        assert ctx.stats()["graph_launches"] == 1
    m = 300_000
    kb = torch.empty(m, dtype=torch.int64, device="cuda")
    vb = torch.empty(m, dtype=torch.int32, device="cuda")
    for r in range(3):
        k, v = W.uniform_u64_pairs(m, 30 + r)
        note(f"graph pairs replay {r}")
        kb.copy_(torch.from_numpy(k.view(np.int64)))
        vb.copy_(torch.from_numpy(v.view(np.int32)))
        ctx.sort_pairs(kb, vb, key_type="u64")
        torch.cuda.synchronize()
        ko = kb.cpu().numpy().view(np.uint64)
        vo = vb.cpu().numpy().view(np.uint32)
        assert_same_bits(ko, oracle.sort(k))
        assert np.array_equal(k[vo.astype(np.int64)], ko)


def test_graph_bad_offsets_on_replay(torch_mod, bqs):
    torch = torch_mod
    keys = W.uniform_i32(100_000, 0)
    good = np.array([0, 40_000, 60_000, 100_000], dtype=np.int64)
    ctx = bqs.Context(graph=1)
    buf = to_dev(torch, keys)
    off = torch.from_numpy(good).cuda()
    note("graph capture for offsets check")
    ctx.sort_segments(buf, off)
    torch.cuda.synchronize()
    off.copy_(torch.tensor([0, 60_000, 40_000, 100_000], dtype=torch.int64))
    note("graph replay with malformed offsets")
    ctx.sort_segments(buf, off)  # enqueued; the device finds the offsets malformed
    with pytest.raises(bqs.BqsError) as e:
        ctx.synchronize()
    assert e.value.status == 1


# --------------------------------------------------------------- records --

def _sum_sq(v):
    # left to right, every product and sum rounded, as the comparator does
    s = v[:, 0] * v[:, 0]
    for i in range(1, 10):
        s = s + v[:, i] * v[:, i]
    return s


def _rows_sorted(a):
    return a[np.lexsort(a.T[::-1])]


def test_records_match_oracle(torch_mod, bqs, oracle):
    """The paper's Vector and Record types: the key sequence of the output
    equals the oracle's bit for bit, and the output holds the same records
    (records with equal keys may come in another order)."""
    torch = torch_mod
    for n in (0, 1, 2, 1000, 100_003, 1_000_000):
        v = np.random.default_rng(n + 1).standard_normal((n, 10))
        note(f"records vector n={n}")
        got = bqs.sort_records(torch.from_numpy(v).cuda())
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        e = oracle.sort_records(v)
        assert_same_bits(_sum_sq(g), _sum_sq(e))
        assert np.array_equal(_rows_sorted(g), _rows_sorted(v))
    rng = np.random.default_rng(3)
    for n, spread in ((5000, 4), (300_007, 1000), (1_000_000, 2**31 - 1)):
        r = rng.integers(-2**31, 2**31 - 1, size=(n, 21), dtype=np.int32)
        r[:, 0] = rng.integers(-spread, spread, size=n)
        note(f"records record n={n} spread={spread}")
        got = bqs.sort_records(torch.from_numpy(r).cuda())
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        e = oracle.sort_records(r)
        assert np.array_equal(g[:, 0], e[:, 0])
        assert np.array_equal(_rows_sorted(g), _rows_sorted(r))


def test_records_reject_bad_arguments(torch_mod, bqs):
    torch = torch_mod
    note("records bad arguments")
    with pytest.raises(bqs.BqsError):
        bqs.sort_records(torch.zeros((10, 9), dtype=torch.float64, device="cuda"))
    t = torch.zeros((10, 21), dtype=torch.int32, device="cuda")
    with pytest.raises(bqs.BqsError):
        bqs.sort_records(t, out=t)  # out overlaps the input


# ------------------------------------------------------------- contract --

def test_workspace_too_small_is_rejected(torch_mod, bqs):
    import ctypes

    t = to_dev(torch_mod, W.uniform_i32(100_000, 0))
    ws = torch_mod.empty(1024, dtype=torch_mod.uint8, device="cuda")
    h = ctypes.c_void_p()
    assert bqs.lib.bqs_ctx_create(ctypes.byref(h)) == 0
    try:
        assert bqs.lib.bqs_ctx_set_workspace(h, ctypes.c_void_p(ws.data_ptr()), 1024) == 0
        assert bqs.lib.bqs_sort(ctypes.c_void_p(t.data_ptr()), t.numel(), bqs.I32, h) == 1
    finally:
        bqs.lib.bqs_ctx_destroy(h)


def test_stats_account_for_every_key(torch_mod, bqs):
    ctx = bqs.Context(timing=1)
    for fam in ("uniform", "few_distinct", "all_equal"):
        a = W.I32_FAMILIES[fam](1 << 20, 0)
        note(f"stats {fam}")
        gpu_sort(torch_mod, bqs, a, ctx)
        s = ctx.stats()
        # every key ends in exactly one small segment or one equal run,
        # except single keys already in place
        done = s["small_sorted_keys"] + s["filled_keys"]
        assert 0.99 * a.size <= done <= a.size
        # the call enqueues its levels plus spare ones (empty launches)
        assert s["partition_launches"] > s["levels"] >= 1
        assert s["graph_launches"] == 0
        # per-level partitioned keys add up to the total; level 0 holds every key
        per_level = [k for k, _ in ctx.levels()]
        assert sum(per_level) == s["partitioned_keys"]
        assert per_level[0] == a.size
        assert s["partition_ms"] > 0


def test_partition_only_timing(torch_mod, bqs, oracle):
    """Timing mode 2 records events around the partition kernels only: the
    partition time is there, the other launches are not timed, and the keys
    are the oracle's."""
    a = W.uniform_i32(1 << 20, 3)
    ctx = bqs.Context(timing=2)
    note("timing mode 2")
    assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    s = ctx.stats()
    assert s["partition_ms"] > 0 and s["small_ms"] == 0 and s["plan_ms"] == 0
    assert len(ctx.levels()) == s["levels"] and all(ms > 0 for _, ms in ctx.levels())


def test_full_size_2p28_uniform_properties(torch_mod, bqs):
    """2^28 int32 keys at the benchmark's configuration: sorted, and the
    same multiset as the input (compared through torch.sort of the input as
    an independent library routine), plus sampled order statistics from
    numpy's selection."""
    torch = torch_mod
    n = 1 << 28
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    note("2^28 uniform int32")
    t = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device="cuda", generator=g)
    ref = torch.sort(t).values
    bqs.sort(t)
    torch.cuda.synchronize()
    assert bool((t[1:] >= t[:-1]).all())
    assert bool(torch.equal(t, ref))
    del ref
    idx = np.random.default_rng(0).integers(0, n, size=16)
    t.copy_(torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device="cuda",
                          generator=g.manual_seed(0)))
    host = t.cpu().numpy()
    bqs.sort(t)
    torch.cuda.synchronize()
    for i in idx[:4]:
        assert int(t[int(i)]) == int(np.partition(host, int(i))[int(i)])


# ------------------------------------------------------ pivot strategies --

@pytest.mark.parametrize("mode", [1, 3, 5, 23, 33, 35, 55])
def test_pivot_strategies_match_oracle(torch_mod, bqs, oracle, mode):
    """The paper's pivot strategies (Section 4) change only the recursion,
    never the sorted keys."""
    ctx = bqs.Context(pivot_mode=mode, small_cutoff=512)
    for fam in ("uniform", "few_distinct", "sorted", "reverse"):
        for n in (1000, 8192 * 5 + 3, 400_001):
            a = W.I32_FAMILIES[fam](n, mode)
            note(f"pivot mode {mode} {fam} n={n}")
            assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    f = W.special_f64(100_000, mode)
    note(f"pivot mode {mode} f64 specials")
    assert_same_bits(gpu_sort(torch_mod, bqs, f, ctx), oracle.sort(f))


def test_skewed_pivots_deepen_the_recursion(torch_mod, bqs, oracle):
    """Skew factor s takes the 1/s quantile of the sample as pivot: the keys
    still match the oracle, and the recursion gets deeper as s grows."""
    a = W.uniform_i32(1 << 20, 77)
    expect = oracle.sort(a)
    levels = []
    for skew in (0, 4, 16, 64):
        ctx = bqs.Context(pivot_skew=skew, small_cutoff=1024)
        note(f"pivot skew {skew}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), expect)
        levels.append(ctx.stats()["levels"])
    assert levels[0] < levels[1] < levels[2] < levels[3]
    k, v = W.tied_u64_pairs(200_000, 9)
    note("pivot skew 8 pairs")
    ko, vo = gpu_pairs(torch_mod, bqs, k, v, bqs.Context(pivot_skew=8))
    check_pairs(k, ko, vo, oracle.sort(k))


# ------------------------------------------------------- persistent mode --
# Every level in one cooperative launch (grid barriers between the steps).
# The results must be the oracle's, as in the level-by-level mode.

def _pctx(bqs, **kw):
    return bqs.Context(mode=bqs.MODE_PERSISTENT, **kw)


def test_persistent_int32_families(torch_mod, bqs, oracle):
    ctx = _pctx(bqs)
    fams = dict(W.I32_FAMILIES)
    fams.update(W.I32_EXTRA_FAMILIES)
    for fam, gen in fams.items():
        for n in (0, 1, 2, 4096, 4097, 8192 * 3, 8192 * 7 + 5, 1_000_003):
            a = gen(n, 23)
            note(f"persistent {fam} n={n}")
            assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
        s = ctx.stats()
        assert s["partition_launches"] == 1 and s["small_cutoff"] <= 4096


def test_persistent_deep_recursion_and_grids(torch_mod, bqs, oracle):
    """Small cutoffs give many levels (four barriers each); smaller grids
    give workgroups several tiles per level."""
    for cut, grid in ((2, 0), (16, 0), (300, 64), (4096, 8), (100, 1)):
        ctx = _pctx(bqs, small_cutoff=cut, grid=grid)
        a = W.uniform_i32(200_003, cut + grid)
        note(f"persistent cutoff={cut} grid={grid}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
        assert ctx.stats()["levels"] >= 1


def test_persistent_key_types_and_specials(torch_mod, bqs, oracle):
    ctx = _pctx(bqs)
    rng = np.random.Generator(np.random.PCG64(37))
    for dt in (np.uint32, np.int64, np.uint64):
        a = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=700_001, dtype=dt, endpoint=True)
        note(f"persistent {np.dtype(dt).name}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    for fam, gen in W.F64_FAMILIES.items():
        a = gen(600_007, 6)
        note(f"persistent f64 {fam}")
        assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    a = W.special_f64(200_000, 4)
    note("persistent f64/f32 specials")
    assert_same_bits(gpu_sort(torch_mod, bqs, a, ctx), oracle.sort(a))
    with np.errstate(over="ignore"):
        f = a.astype(np.float32)
    assert_same_bits(gpu_sort(torch_mod, bqs, f, ctx), oracle.sort(f))


def test_persistent_pairs(torch_mod, bqs, oracle):
    ctx = _pctx(bqs)
    for n in (2, 2049, 100_000, 1 << 20):
        k, v = W.uniform_u64_pairs(n, n + 1)
        note(f"persistent pairs u64/u32 n={n}")
        ko, vo = gpu_pairs(torch_mod, bqs, k, v, ctx)
        check_pairs(k, ko, vo, oracle.sort(k))
    k, v = W.tied_u64_pairs(300_000, 4)
    note("persistent pairs tied u64/u64")
    ko, vo = gpu_pairs(torch_mod, bqs, k, v.astype(np.uint64), ctx)
    check_pairs(k, ko, vo, oracle.sort(k))
    a = W.few_distinct_i32(300_000, 6)
    note("persistent pairs i32 few-distinct")
    ko, vo = gpu_pairs(torch_mod, bqs, a, np.arange(a.size, dtype=np.uint32), ctx)
    check_pairs(a, ko, vo, oracle.sort(a))


def test_persistent_segments(torch_mod, bqs, oracle):
    ctx = _pctx(bqs)
    for k, hi in [(1, 10.0), (50, 14.0), (2000, 16.0)]:
        keys, offsets = W.segmented_i32(k, k + 3, 0.0, hi)
        note(f"persistent segments k={k} n={keys.size}")
        assert_same_bits(gpu_segments(torch_mod, bqs, keys, offsets, ctx), oracle.sort_segments(keys, offsets))
    sizes = np.array([0, 1, 0, 2, 9000, 0, 1, 30_000, 3, 0], dtype=np.int64)
    offsets = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    keys = W.uniform_i32(int(offsets[-1]), 2)
    note("persistent segments with empties")
    assert_same_bits(gpu_segments(torch_mod, bqs, keys, offsets, ctx), oracle.sort_segments(keys, offsets))
    bad = np.array([0, 600, 500, 1000], dtype=np.int64)
    note("persistent segments bad offsets")
    with pytest.raises(bqs.BqsError) as e:
        gpu_segments(torch_mod, bqs, W.uniform_i32(1000, 0), bad, ctx)
    assert e.value.status == 1


def test_persistent_records(torch_mod, bqs, oracle):
    torch = torch_mod
    ctx = _pctx(bqs)
    v = np.random.default_rng(5).standard_normal((100_003, 10))
    note("persistent records vector")
    g = ctx.sort_records(torch.from_numpy(v).cuda()).cpu().numpy()
    assert_same_bits(_sum_sq(g), _sum_sq(oracle.sort_records(v)))
    assert np.array_equal(_rows_sorted(g), _rows_sorted(v))


def test_persistent_rejects_multiway(torch_mod, bqs):
    note("persistent + multiway rejected")
    t = to_dev(torch_mod, W.uniform_i32(100_000, 0))
    with pytest.raises(bqs.BqsError) as e:
        _pctx(bqs, multiway=1).sort(t)
    assert e.value.status == 1


def test_persistent_full_size_2p28(torch_mod, bqs):
    """2^28 int32 keys in one persistent launch: equal to torch.sort of the
    same input (an independent library routine)."""
    torch = torch_mod
    n = 1 << 28
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    note("persistent 2^28 uniform int32")
    t = torch.randint(-(2**31), 2**31, (n,), dtype=torch.int32, device="cuda", generator=g)
    ref = torch.sort(t).values
    ctx = _pctx(bqs)
    ctx.sort(t)
    torch.cuda.synchronize()
    assert bool(torch.equal(t, ref))
    s = ctx.stats()
    assert s["partition_launches"] == 1 and s["levels"] >= 15
