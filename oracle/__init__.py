"""CPU BlockQuicksort oracle -- test infrastructure only.

A thin ctypes wrapper around ``bqs_oracle.cpp`` (a plain, slow, single
threaded BlockQuicksort written from Edelkamp & Weiss, arXiv 1604.06697,
Sections 2-3).  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library and does not
import it.

All functions copy their inputs; numpy arrays in, numpy arrays out.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "bqs_oracle.cpp")
LIBRARY = os.path.join(_HERE, "liboracle.so")

# dtype codes of the oracle's C interface
_DTYPES = {
    np.dtype(np.int32): 1,
    np.dtype(np.uint32): 2,
    np.dtype(np.int64): 3,
    np.dtype(np.uint64): 4,
    np.dtype(np.float32): 5,
    np.dtype(np.float64): 6,
}

_ERRORS = {1: "invalid argument", 2: "unsupported dtype", 5: "NaN key"}


class OracleError(RuntimeError):
    pass


class _Params(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int64),
        ("is_thresh", ctypes.c_int64),
        ("depth_limit", ctypes.c_int64),
        ("check", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("comparisons", ctypes.c_int64),
        ("partitions", ctypes.c_int64),
        ("heapsorts", ctypes.c_int64),
        ("check_failures", ctypes.c_int64),
    ]


@dataclass
class Stats:
    comparisons: int
    partitions: int
    heapsorts: int
    check_failures: int


def compile_library(out: str = LIBRARY, mutant: int = 0) -> str:
    """Compiles the oracle with g++ (host only).  ``mutant`` > 0 plants one of
    the numbered mistakes used to show that the pins catch them."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC", "-o", out, SOURCE]
    if mutant:
        cmd.insert(1, f"-DORACLE_MUTANT={int(mutant)}")
    subprocess.run(cmd, check=True)
    return out


class Oracle:
    def __init__(self, path: str = LIBRARY):
        if not os.path.exists(path):
            compile_library(path)
        self.lib = ctypes.CDLL(path)
        L = self.lib
        P = ctypes.POINTER(_Params)
        L.oracle_sort.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, P]
        L.oracle_sort.restype = ctypes.c_int
        L.oracle_sort_pairs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int, ctypes.c_int, P]
        L.oracle_sort_pairs.restype = ctypes.c_int
        L.oracle_sort_segments.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_int, P]
        L.oracle_sort_segments.restype = ctypes.c_int
        L.oracle_sort_records.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, P]
        L.oracle_sort_records.restype = ctypes.c_int
        L.oracle_partition.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int, P]
        L.oracle_partition.restype = ctypes.c_int64
        L.oracle_std_sort.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        L.oracle_std_sort.restype = ctypes.c_int
        L.oracle_mutant.argtypes = []
        L.oracle_mutant.restype = ctypes.c_int

    @staticmethod
    def _params(block=0, is_thresh=0, depth_limit=-1, check=False) -> _Params:
        return _Params(block, is_thresh, depth_limit, 1 if check else 0, 0, 0, 0, 0, 0)

    @staticmethod
    def _code(a: np.ndarray) -> int:
        try:
            return _DTYPES[a.dtype]
        except KeyError:
            raise OracleError(f"unsupported dtype {a.dtype}") from None

    @staticmethod
    def _stats(p: _Params) -> Stats:
        return Stats(p.comparisons, p.partitions, p.heapsorts, p.check_failures)

    def _rc(self, rc: int):
        if rc != 0:
            raise OracleError(_ERRORS.get(rc, f"error {rc}"))

    def sort(self, keys: np.ndarray, *, block=0, is_thresh=0, depth_limit=-1,
             check=False, return_stats=False):
        a = np.ascontiguousarray(keys).copy()
        p = self._params(block, is_thresh, depth_limit, check)
        self._rc(self.lib.oracle_sort(a.ctypes.data, a.size, self._code(a), ctypes.byref(p)))
        return (a, self._stats(p)) if return_stats else a

    def sort_pairs(self, keys: np.ndarray, vals: np.ndarray, *, block=0, is_thresh=0,
                   depth_limit=-1, check=False):
        k = np.ascontiguousarray(keys).copy()
        v = np.ascontiguousarray(vals).copy()
        if k.shape != v.shape:
            raise OracleError("keys and vals differ in length")
        p = self._params(block, is_thresh, depth_limit, check)
        self._rc(self.lib.oracle_sort_pairs(k.ctypes.data, v.ctypes.data, k.size, self._code(k),
                                            v.dtype.itemsize, ctypes.byref(p)))
        return k, v

    def sort_segments(self, keys: np.ndarray, offsets: np.ndarray, **kw):
        a = np.ascontiguousarray(keys).copy()
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        p = self._params(kw.get("block", 0), kw.get("is_thresh", 0), kw.get("depth_limit", -1),
                         kw.get("check", False))
        self._rc(self.lib.oracle_sort_segments(a.ctypes.data, off.ctypes.data, off.size - 1,
                                               self._code(a), ctypes.byref(p)))
        return a

    def sort_records(self, recs: np.ndarray, **kw) -> np.ndarray:
        """Sorts the paper's Vector records (n x 10 float64, by the sum of
        squares) or Record records (n x 21 int32, by the first component)."""
        a = np.ascontiguousarray(recs).copy()
        if a.ndim != 2 or (a.dtype, a.shape[1]) not in ((np.dtype(np.float64), 10), (np.dtype(np.int32), 21)):
            raise OracleError("records are n x 10 float64 (Vector) or n x 21 int32 (Record)")
        kind = 1 if a.dtype == np.float64 else 2
        p = self._params(kw.get("block", 0), kw.get("is_thresh", 0), kw.get("depth_limit", -1),
                         kw.get("check", False))
        self._rc(self.lib.oracle_sort_records(a.ctypes.data, a.shape[0], kind, ctypes.byref(p)))
        self.last = Stats(p.comparisons, p.partitions, p.heapsorts, p.check_failures)
        return a

    def partition(self, keys: np.ndarray, lo: int = 0, hi: int | None = None, *, block=0):
        """One median-of-three + block-partition step; returns (array, cut)."""
        a = np.ascontiguousarray(keys).copy()
        hi = a.size if hi is None else hi
        p = self._params(block)
        cut = self.lib.oracle_partition(a.ctypes.data, lo, hi, self._code(a), ctypes.byref(p))
        if cut < 0:
            raise OracleError("invalid partition arguments")
        return a, int(cut)

    def std_sort(self, keys: np.ndarray) -> np.ndarray:
        """The host's std::sort with the same key order (a library routine:
        the CPU context the paper compares against, not an oracle)."""
        a = np.ascontiguousarray(keys).copy()
        self._rc(self.lib.oracle_std_sort(a.ctypes.data, a.size, self._code(a)))
        return a

    def mutant(self) -> int:
        return int(self.lib.oracle_mutant())


_DEFAULT: Oracle | None = None


def default() -> Oracle:
    global _DEFAULT
    if _DEFAULT is None:
        _DEFAULT = Oracle()
    return _DEFAULT
