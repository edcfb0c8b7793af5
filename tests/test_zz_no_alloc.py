"""GPU test of bqs_sort_noalloc, the entry point for callers that cannot
allocate: called through the C ABI twice in a row (the second input
smaller than the first), it must give bit for bit what bqs_sort gives and
what the CPU oracle gives, and report BQS_OK through its status word."""

import ctypes
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


def _dev(torch, a):
    hold = {np.dtype(np.uint64): np.int64}.get(a.dtype)
    return torch.from_numpy(np.ascontiguousarray(a.view(hold) if hold is not None else a)).cuda()


CASES = [
    ("i32", np.int32, lambda n, s: W.uniform_i32(n, s), (9_000_001, 300_007)),
    ("f64", np.float64, lambda n, s: W.special_f64(n, s), (5_000_003, 70_001)),
    ("i32 few distinct", np.int32, lambda n, s: W.few_distinct_i32(n, s), (1 << 22, 8_193)),
]


@pytest.mark.parametrize("name,dtype,gen,sizes", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_bqs_sort_and_oracle(torch_mod, bqs, oracle, name, dtype, gen, sizes):
    torch = torch_mod
    code = {np.dtype(np.int32): bqs.I32, np.dtype(np.float64): bqs.F64}[np.dtype(dtype)]
    stream = torch.cuda.current_stream().cuda_stream
    for call, n in enumerate(sizes):  # the second call is the smaller one
        a = gen(n, 60 + call)
        expect = oracle.sort(a)
        ref = _dev(torch, a)
        bqs.sort(ref)  # the existing entry point, with a caller workspace
        bqs.synchronize()
        t = _dev(torch, a)
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        note(f"noalloc {name} call {call} n={n}")
        rc = bqs.lib.bqs_sort_noalloc(ctypes.c_void_p(t.data_ptr()), n, code, ctypes.c_void_p(stream),
                                      ctypes.c_void_p(status.data_ptr()))
        assert rc == 0
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        u = f"u{a.itemsize}"
        got = t.cpu().numpy().view(a.dtype)
        assert np.array_equal(got.view(u), ref.cpu().numpy().view(a.dtype).view(u))
        assert np.array_equal(got.view(u), expect.view(u))


def test_noalloc_rejects_what_does_not_fit(torch_mod, bqs):
    torch = torch_mod
    stream = torch.cuda.current_stream().cuda_stream
    big = torch.zeros(1 << 24, dtype=torch.int32, device="cuda")
    note("noalloc too large")
    assert bqs.lib.bqs_sort_noalloc(ctypes.c_void_p(big.data_ptr()), big.numel(), bqs.I32,
                                    ctypes.c_void_p(stream), None) == 7
    # trivial inputs report OK through the status word
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    assert bqs.lib.bqs_sort_noalloc(ctypes.c_void_p(big.data_ptr()), 1, bqs.I32, ctypes.c_void_p(stream),
                                    ctypes.c_void_p(status.data_ptr())) == 0
    torch.cuda.synchronize()
    assert int(status.item()) == 0
