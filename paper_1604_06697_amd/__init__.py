"""Python binding of libbqs.so, a BlockQuicksort-style sort for MI355X.

Argument marshalling only: every step of the sort runs in the library's
HIP kernels.  PyTorch provides device memory (keys, payloads, workspace) and
the stream.  The three entry points mirror the C ABI in include/bqs.h:

    sort(keys)                 -> keys sorted ascending in place
    sort_pairs(keys, vals)     -> records sorted by key, payload follows key
    sort_segments(keys, offs)  -> every segment keys[offs[i]:offs[i+1]] sorted

Calls are asynchronous, like any kernel on PyTorch's current stream: they
return once the sort is enqueued.  ``Context.synchronize()`` waits for the
context's calls and raises ``BqsError`` for an error the device detected
(a malformed offsets array, a NaN key in check mode, ...).

The library must be built (``python -m paper_1604_06697_amd.build`` or
``__graft_entry__.build()``); importing fails loudly when it is missing.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import sys
import threading
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; BQS_LIBRARY names another build of the same library
LIBRARY = os.environ.get("BQS_LIBRARY") or os.path.join(_HERE, "libbqs.so")

I32, U32, I64, U64, F32, F64 = 1, 2, 3, 4, 5, 6

STATUS = {
    0: "ok",
    1: "invalid argument",
    2: "unsupported dtype",
    3: "out of host memory",
    4: "HIP runtime error",
    5: "NaN key",
    6: "device work list overflow",
    7: "input larger than the no-allocation scratch",
}

PARAM_SMALL_CUTOFF = 1
PARAM_SAMPLE_MAX = 2
PARAM_PIVOT_MODE = 3
PARAM_TIMING = 4
PARAM_TILE_EPT = 5
PARAM_GRID = 6
PARAM_PROFILE = 7
PARAM_MODE = 8
PARAM_GRAPH = 9
PARAM_LOOKBACK = 10
PARAM_MULTIWAY = 11
PARAM_PIVOT_SKEW = 12
PARAM_CHECK_NAN = 13
PARAM_ENQUEUE_LEVELS = 14
PARAM_DEPTH_LIMIT = 15
PARAM_LIST_CAP = 16
PARAM_SHUFFLE = 17
PARAM_INPLACE = 18
RECORD_VECTOR, RECORD_RECORD = 1, 2
MODE_ASYNC, MODE_LEVELS, MODE_PERSISTENT = 0, 1, 2

_TORCH_DTYPES = {
    torch.int32: I32,
    torch.int64: I64,
    torch.float32: F32,
    torch.float64: F64,
}
for _name, _code in (("uint32", U32), ("uint64", U64)):
    if hasattr(torch, _name):
        _TORCH_DTYPES[getattr(torch, _name)] = _code

EXPORTED = [
    "bqs_ctx_create", "bqs_ctx_destroy", "bqs_ctx_set_stream", "bqs_ctx_set_workspace",
    "bqs_ctx_set_param", "bqs_ctx_get_param", "bqs_ctx_get_stats", "bqs_ctx_get_level",
    "bqs_workspace_bytes",
    "bqs_sort", "bqs_sort_pairs", "bqs_sort_segments", "bqs_sort_segments_pairs",
    "bqs_records_workspace_bytes", "bqs_sort_records", "bqs_ctx_sync_status", "bqs_ctx_poll_status", "bqs_ctx_set_segment_ticks",
    "bqs_status_str", "bqs_version", "bqs_sort_noalloc",
]


class BqsError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int64),
        ("partitioned_keys", ctypes.c_int64),
        ("small_sorted_keys", ctypes.c_int64),
        ("filled_keys", ctypes.c_int64),
        ("tiles", ctypes.c_int64),
        ("partition_ms", ctypes.c_double),
        ("partition_launches", ctypes.c_int64),
        ("small_ms", ctypes.c_double),
        ("small_launches", ctypes.c_int64),
        ("plan_ms", ctypes.c_double),
        ("tile_keys", ctypes.c_int64),
        ("small_cutoff", ctypes.c_int64),
        ("prof_tiles", ctypes.c_int64),
        ("prof_lookback_rounds", ctypes.c_int64),
        ("prof_lookback_polls", ctypes.c_int64),
        ("prof_lookback_cycles", ctypes.c_double),
        ("prof_tile_cycles", ctypes.c_double),
        ("prof_load_cycles", ctypes.c_double),
        ("graph_launches", ctypes.c_int64),
        ("prof_small_segments", ctypes.c_int64),
        ("prof_small_cycles", ctypes.c_double * 5),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else v
        return out


def _load(path: str = LIBRARY) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_1604_06697_amd.build` "
            "(the sort has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "bqs_ctx_create": ([ctypes.POINTER(vp)], st),
        "bqs_ctx_destroy": ([vp], None),
        "bqs_ctx_set_stream": ([vp, vp], st),
        "bqs_ctx_set_workspace": ([vp, vp, sz], st),
        "bqs_ctx_set_param": ([vp, ctypes.c_int, i64], st),
        "bqs_ctx_get_param": ([vp, ctypes.c_int], i64),
        "bqs_ctx_get_stats": ([vp, ctypes.POINTER(Stats)], st),
        "bqs_ctx_get_level": ([vp, ctypes.c_int, ctypes.POINTER(i64),
                               ctypes.POINTER(ctypes.c_double)], st),
        "bqs_workspace_bytes": ([vp, i64, ctypes.c_int, i32, i64], sz),
        "bqs_sort": ([vp, i64, ctypes.c_int, vp], st),
        "bqs_sort_pairs": ([vp, vp, i64, ctypes.c_int, i32, vp], st),
        "bqs_sort_segments": ([vp, vp, i64, i64, ctypes.c_int, vp], st),
        "bqs_sort_segments_pairs": ([vp, vp, vp, i64, i64, ctypes.c_int, i32, vp], st),
        "bqs_records_workspace_bytes": ([vp, i64, ctypes.c_int], sz),
        "bqs_sort_records": ([vp, vp, i64, ctypes.c_int, vp], st),
        "bqs_ctx_sync_status": ([vp], st),
        "bqs_ctx_poll_status": ([vp], st),
        "bqs_ctx_set_segment_ticks": ([vp, vp, i64], st),
        "bqs_status_str": ([st], ctypes.c_char_p),
        "bqs_version": ([], ctypes.c_int),
        "bqs_sort_noalloc": ([vp, i64, ctypes.c_int, vp, vp], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(rc: int, where: str):
    if rc != 0:
        raise BqsError(rc, where)


KEY_TYPES = {"i32": I32, "u32": U32, "i64": I64, "u64": U64, "f32": F32, "f64": F64}
_KEY_BYTES = {I32: 4, U32: 4, F32: 4, I64: 8, U64: 8, F64: 8}


def dtype_code(dtype: torch.dtype) -> int:
    try:
        return _TORCH_DTYPES[dtype]
    except KeyError:
        raise BqsError(2, f"dtype {dtype}") from None


def _key_code(t: torch.Tensor, key_type) -> int:
    """Key type of a tensor; `key_type` ("u64", "u32", ... or a code)
    reinterprets the tensor's bytes, e.g. uint64 keys held in an int64
    tensor."""
    if key_type is None:
        return dtype_code(t.dtype)
    code = KEY_TYPES[key_type] if isinstance(key_type, str) else int(key_type)
    if _KEY_BYTES.get(code) != t.element_size():
        raise BqsError(2, f"key type {key_type} does not match {t.dtype}")
    return code


# Contexts still open.  They are closed by an exit hook, which runs before
# the interpreter (and with it PyTorch and the HIP runtime) is torn down:
# destroying a context frees pinned host memory, events and a stream, which
# must not happen after the runtime has shut down.
_LIVE: "weakref.WeakSet[Context]" = weakref.WeakSet()


class Context:
    """One library context: parameters, statistics and a workspace tensor
    taken from PyTorch's caching allocator (grown on demand).  `close()`
    releases it; contexts still open at interpreter exit are closed by an
    exit hook."""

    def __init__(self, **params):
        h = ctypes.c_void_p()
        _check(lib.bqs_ctx_create(ctypes.byref(h)), "bqs_ctx_create")
        self._h = h
        self._ws: torch.Tensor | None = None
        self._lock = threading.Lock()
        _LIVE.add(self)
        for k, v in params.items():
            self.set_param(k, v)

    def close(self):
        """Waits for the context's work and releases it (idempotent)."""
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None:
            lib.bqs_ctx_destroy(h)
        self._ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the exit hook has already closed every
        # context; a HIP call from here could run after the runtime is gone
        # (module globals may already be gone too, hence the bound default)
        if getattr(self, "_h", None) is None or _finalizing():
            return
        self.close()

    _NAMES = {
        "small_cutoff": PARAM_SMALL_CUTOFF,
        "sample_max": PARAM_SAMPLE_MAX,
        "pivot_mode": PARAM_PIVOT_MODE,
        "timing": PARAM_TIMING,
        "tile_ept": PARAM_TILE_EPT,
        "grid": PARAM_GRID,
        "profile": PARAM_PROFILE,
        "mode": PARAM_MODE,
        "graph": PARAM_GRAPH,
        "lookback": PARAM_LOOKBACK,
        "multiway": PARAM_MULTIWAY,
        "pivot_skew": PARAM_PIVOT_SKEW,
        "check_nan": PARAM_CHECK_NAN,
        "enqueue_levels": PARAM_ENQUEUE_LEVELS,
        "depth_limit": PARAM_DEPTH_LIMIT,
        "list_cap": PARAM_LIST_CAP,
        "shuffle": PARAM_SHUFFLE,
        "inplace": PARAM_INPLACE,
    }

    def set_param(self, name: str, value: int):
        _check(lib.bqs_ctx_set_param(self._h, self._NAMES[name], int(value)), f"set_param {name}")

    def get_param(self, name: str) -> int:
        return int(lib.bqs_ctx_get_param(self._h, self._NAMES[name]))

    def synchronize(self):
        """Waits for every call enqueued on this context; raises BqsError for
        the first error the device latched since the last synchronize()."""
        _check(lib.bqs_ctx_sync_status(self._h), "bqs_ctx_sync_status")

    def poll(self):
        """Raises BqsError for the first error latched by calls that have
        completed so far, without waiting for the others."""
        _check(lib.bqs_ctx_poll_status(self._h), "bqs_ctx_poll_status")

    def set_segment_ticks(self, ticks: torch.Tensor | None):
        """Completion clock of later segmented calls: `ticks` (int64 on the
        device, at least k + 1 entries) receives per segment the device
        clock (100 MHz) when it was final, and at [k] the call's start;
        None turns it off."""
        if ticks is None:
            _check(lib.bqs_ctx_set_segment_ticks(self._h, None, 0), "bqs_ctx_set_segment_ticks")
            self._ticks = None
            return
        self._check_tensor(ticks, "ticks")
        if ticks.dtype != torch.int64:
            raise BqsError(1, "ticks must be int64")
        self._ticks = ticks  # kept alive while calls may write it
        _check(lib.bqs_ctx_set_segment_ticks(self._h, ctypes.c_void_p(ticks.data_ptr()), ticks.numel()),
               "bqs_ctx_set_segment_ticks")

    def reserve(self, nbytes: int, device=None):
        """Allocates the workspace up front (at least `nbytes`), so that
        later calls of up to that size allocate nothing."""
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._prepare(dev, int(nbytes))

    def stats(self) -> dict:
        s = Stats()
        _check(lib.bqs_ctx_get_stats(self._h, ctypes.byref(s)), "bqs_ctx_get_stats")
        return s.as_dict()

    def levels(self) -> list:
        """[(keys partitioned, partition ms), ...] per level of the last call."""
        out = []
        keys, ms = ctypes.c_int64(), ctypes.c_double()
        while lib.bqs_ctx_get_level(self._h, len(out), ctypes.byref(keys), ctypes.byref(ms)) == 0:
            out.append((int(keys.value), float(ms.value)))
        return out

    def workspace_bytes(self, n: int, dtype_c: int, val_bytes: int = 0, k: int = 1) -> int:
        return int(lib.bqs_workspace_bytes(self._h, int(n), dtype_c, int(val_bytes), int(k)))

    def _prepare(self, device: torch.device, need: int):
        if self._ws is None or self._ws.device != device or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
        _check(lib.bqs_ctx_set_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()),
                                         self._ws.numel()), "bqs_ctx_set_workspace")
        stream = torch.cuda.current_stream(device)
        _check(lib.bqs_ctx_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)),
               "bqs_ctx_set_stream")

    @staticmethod
    def _check_tensor(t: torch.Tensor, what: str):
        if not t.is_cuda:
            raise BqsError(1, f"{what} must be a GPU tensor")
        if t.dim() != 1 or not t.is_contiguous():
            raise BqsError(1, f"{what} must be 1-D and contiguous")

    def sort(self, keys: torch.Tensor, key_type=None) -> torch.Tensor:
        self._check_tensor(keys, "keys")
        code = _key_code(keys, key_type)
        n = keys.numel()
        with self._lock, torch.cuda.device(keys.device):
            self._prepare(keys.device, self.workspace_bytes(n, code))
            _check(lib.bqs_sort(ctypes.c_void_p(keys.data_ptr()), n, code, self._h), "bqs_sort")
        return keys

    def sort_pairs(self, keys: torch.Tensor, vals: torch.Tensor, key_type=None):
        self._check_tensor(keys, "keys")
        self._check_tensor(vals, "vals")
        if keys.numel() != vals.numel() or keys.device != vals.device:
            raise BqsError(1, "keys and vals differ in length or device")
        vb = vals.element_size()
        code = _key_code(keys, key_type)
        n = keys.numel()
        with self._lock, torch.cuda.device(keys.device):
            self._prepare(keys.device, self.workspace_bytes(n, code, vb))
            _check(lib.bqs_sort_pairs(ctypes.c_void_p(keys.data_ptr()),
                                      ctypes.c_void_p(vals.data_ptr()), n, code, vb, self._h),
                   "bqs_sort_pairs")
        return keys, vals

    def sort_segments(self, keys: torch.Tensor, offsets: torch.Tensor, key_type=None) -> torch.Tensor:
        self._check_tensor(keys, "keys")
        self._check_tensor(offsets, "offsets")
        if offsets.dtype != torch.int64 or offsets.device != keys.device:
            raise BqsError(1, "offsets must be int64 on the keys' device")
        k = offsets.numel() - 1
        if k < 0:
            raise BqsError(1, "offsets must hold k+1 >= 1 entries")
        code = _key_code(keys, key_type)
        n = keys.numel()
        with self._lock, torch.cuda.device(keys.device):
            self._prepare(keys.device, self.workspace_bytes(n, code, 0, max(k, 1)))
            _check(lib.bqs_sort_segments(ctypes.c_void_p(keys.data_ptr()),
                                         ctypes.c_void_p(offsets.data_ptr()), k, n, code, self._h),
                   "bqs_sort_segments")
        return keys

    def sort_records(self, recs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """The paper's record types: an (n, 10) float64 tensor of Vector
        records (ordered by the sum of squares) or an (n, 21) int32 tensor of
        Record records (ordered by the first component); returns the records
        in key order in `out` (a new tensor by default)."""
        if not recs.is_cuda or recs.dim() != 2 or not recs.is_contiguous():
            raise BqsError(1, "records must be a 2-D contiguous GPU tensor")
        if recs.dtype == torch.float64 and recs.shape[1] == 10:
            kind = RECORD_VECTOR
        elif recs.dtype == torch.int32 and recs.shape[1] == 21:
            kind = RECORD_RECORD
        else:
            raise BqsError(2, "records are (n, 10) float64 or (n, 21) int32")
        if out is None:
            out = torch.empty_like(recs)
        elif out.shape != recs.shape or out.dtype != recs.dtype or not out.is_contiguous():
            raise BqsError(1, "out must match the records' shape and dtype")
        n = recs.shape[0]
        with self._lock, torch.cuda.device(recs.device):
            self._prepare(recs.device, int(lib.bqs_records_workspace_bytes(self._h, n, kind)))
            _check(lib.bqs_sort_records(ctypes.c_void_p(recs.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                                        kind, self._h), "bqs_sort_records")
        return out

    def sort_segments_pairs(self, keys: torch.Tensor, vals: torch.Tensor, offsets: torch.Tensor,
                            key_type=None):
        self._check_tensor(keys, "keys")
        self._check_tensor(vals, "vals")
        self._check_tensor(offsets, "offsets")
        if keys.numel() != vals.numel() or keys.device != vals.device:
            raise BqsError(1, "keys and vals differ in length or device")
        if offsets.dtype != torch.int64 or offsets.device != keys.device:
            raise BqsError(1, "offsets must be int64 on the keys' device")
        k = offsets.numel() - 1
        if k < 0:
            raise BqsError(1, "offsets must hold k+1 >= 1 entries")
        vb = vals.element_size()
        code = _key_code(keys, key_type)
        n = keys.numel()
        with self._lock, torch.cuda.device(keys.device):
            self._prepare(keys.device, self.workspace_bytes(n, code, vb, max(k, 1)))
            _check(lib.bqs_sort_segments_pairs(ctypes.c_void_p(keys.data_ptr()),
                                               ctypes.c_void_p(vals.data_ptr()),
                                               ctypes.c_void_p(offsets.data_ptr()), k, n, code, vb,
                                               self._h),
                   "bqs_sort_segments_pairs")
        return keys, vals


@atexit.register
def _close_all():
    for ctx in list(_LIVE):
        ctx.close()


_default: Context | None = None


def default_context() -> Context:
    global _default
    if _default is None:
        _default = Context()
    return _default


def synchronize(ctx: Context | None = None):
    (ctx or default_context()).synchronize()


def sort(keys: torch.Tensor, ctx: Context | None = None, key_type=None) -> torch.Tensor:
    return (ctx or default_context()).sort(keys, key_type)


def sort_noalloc(keys: torch.Tensor, status: torch.Tensor | None = None, key_type=None) -> torch.Tensor:
    """bqs_sort_noalloc: sorts `keys` in place on the current stream without
    any allocation (the library's fixed scratch as workspace, default
    parameters); `status`, an int32 GPU tensor of one element, receives the
    call's status on the device."""
    Context._check_tensor(keys, "keys")
    code = _key_code(keys, key_type)
    if status is not None and (not status.is_cuda or status.dtype != torch.int32 or status.numel() < 1):
        raise BqsError(1, "status must be an int32 GPU tensor")
    with torch.cuda.device(keys.device):
        stream = torch.cuda.current_stream(keys.device).cuda_stream
        _check(lib.bqs_sort_noalloc(ctypes.c_void_p(keys.data_ptr()), keys.numel(), code,
                                    ctypes.c_void_p(stream),
                                    None if status is None else ctypes.c_void_p(status.data_ptr())),
               "bqs_sort_noalloc")
    return keys


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, ctx: Context | None = None, key_type=None):
    return (ctx or default_context()).sort_pairs(keys, vals, key_type)


def sort_segments(keys: torch.Tensor, offsets: torch.Tensor, ctx: Context | None = None,
                  key_type=None):
    return (ctx or default_context()).sort_segments(keys, offsets, key_type)


def sort_segments_pairs(keys: torch.Tensor, vals: torch.Tensor, offsets: torch.Tensor,
                        ctx: Context | None = None, key_type=None):
    return (ctx or default_context()).sort_segments_pairs(keys, vals, offsets, key_type)


def sort_records(recs: torch.Tensor, out: torch.Tensor | None = None, ctx: Context | None = None):
    return (ctx or default_context()).sort_records(recs, out)
