"""Python binding of libzset.so (include/zset.h): argument marshalling only.

Every step of the enumeration runs in the HIP library; torch supplies device
memory (the output tensor) and streams.  Importing works without a GPU; the
calls that launch work need one.  If the library has not been built this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ZSET_LIB_PATH names another build of the same library (the host-sanitizer
# build of the CPU tests); by default the in-tree one.
LIB_PATH = os.environ.get("ZSET_LIB_PATH") or os.path.join(_HERE, "libzset.so")

OK, EINVAL, EOVERFLOW, ENOMEM, ECAPACITY, EDEVICE = 0, -1, -2, -3, -4, -5
MAX_D = 32

# Exported symbols, in the order include/zset.h declares them.
SYMBOLS = (
    "zset_default_opts", "zset_count", "zset_count_table", "zset_memo_build",
    "zset_memo_free", "zset_memo_read", "zset_enumerate", "zset_enumerate_ex",
    "zset_enumerate_noalloc", "zset_enumerate_async", "zset_enumerate_walk",
    "zset_batch_default_opts", "zset_batch_create", "zset_batch_info", "zset_batch_run",
    "zset_batch_times", "zset_batch_free",
    "zset_server_default_opts", "zset_server_create", "zset_server_add_set",
    "zset_server_set_info", "zset_server_count", "zset_server_submit", "zset_server_wait",
    "zset_server_release", "zset_server_stats", "zset_server_free", "zset_store_ceiling",
    "zset_strerror", "zset_selftest_host", "zset_last_error",
)


class Opts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("order", ctypes.c_int),
                ("rows_per_tile", ctypes.c_uint64), ("count_only", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("claim_pct", ctypes.c_int),
                ("memo_top", ctypes.c_uint64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_uint64), ("dispatchers", ctypes.c_int),
                ("memo_bytes", ctypes.c_uint64)]


class ServerResult(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_uint64), ("out_offset", ctypes.c_uint64),
                ("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("done_us", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("count_us", ctypes.c_double), ("memo_us", ctypes.c_double),
                ("plan_us", ctypes.c_double), ("write_us", ctypes.c_double),
                ("total_us", ctypes.c_double), ("rows", ctypes.c_uint64),
                ("memo_rows", ctypes.c_uint64), ("memo_bytes", ctypes.c_uint64),
                ("tiles", ctypes.c_uint64), ("rows_per_tile", ctypes.c_uint64),
                ("k", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchOpts(ctypes.Structure):
    _fields_ = [("count_only", ctypes.c_int), ("max_chain_steps", ctypes.c_uint32),
                ("unit_tiles", ctypes.c_uint32), ("use_graph", ctypes.c_int),
                ("stream", ctypes.c_void_p)]


class BatchStats(ctypes.Structure):
    _fields_ = [("total_us", ctypes.c_double), ("count_us", ctypes.c_double),
                ("memo_us", ctypes.c_double), ("plan_us", ctypes.c_double),
                ("write_us", ctypes.c_double), ("rows", ctypes.c_uint64),
                ("words", ctypes.c_uint64), ("tiles", ctypes.c_uint64),
                ("units", ctypes.c_uint32), ("memo_queries", ctypes.c_uint32),
                ("write_blocks", ctypes.c_uint32), ("lds_bytes", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ZsetError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        msg = f"{where}: {strerror(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)
        self.status = status


_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_lib = None


def load():
    """Load libzset.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2407_20474_amd.build` (no fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.zset_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.zset_default_opts.restype = None
    lib.zset_count.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, _u64p]
    lib.zset_count_table.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p]
    lib.zset_memo_build.argtypes = [_u32p, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]
    lib.zset_memo_free.argtypes = [ctypes.c_void_p]
    lib.zset_memo_free.restype = None
    lib.zset_memo_read.argtypes = [ctypes.c_void_p, _u64p, _u32p, _u64p,
                                   ctypes.POINTER(ctypes.c_int), _u64p]
    lib.zset_enumerate.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_void_p]
    lib.zset_enumerate_ex.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_uint64, ctypes.POINTER(Opts), ctypes.c_void_p,
                                      _u64p, _u64p, ctypes.POINTER(Stats)]
    lib.zset_enumerate_noalloc.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_uint64, ctypes.POINTER(Opts), _u64p, _u64p]
    lib.zset_enumerate_async.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_uint64, ctypes.POINTER(Opts), ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]
    lib.zset_store_ceiling.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.zset_enumerate_walk.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, _u64p]
    lib.zset_batch_default_opts.argtypes = [ctypes.POINTER(BatchOpts)]
    lib.zset_batch_default_opts.restype = None
    _i32p = ctypes.POINTER(ctypes.c_int)
    lib.zset_batch_create.argtypes = [ctypes.c_int, _u64p, _i32p, _u32p, _i32p, _u64p,
                                      ctypes.POINTER(BatchOpts), ctypes.POINTER(ctypes.c_void_p)]
    lib.zset_batch_info.argtypes = [ctypes.c_void_p, _u64p, _u64p, _u64p, _i32p, _u64p]
    lib.zset_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, _u64p,
                                   ctypes.POINTER(BatchStats)]
    lib.zset_batch_times.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.zset_batch_free.argtypes = [ctypes.c_void_p]
    lib.zset_batch_free.restype = None
    lib.zset_server_default_opts.argtypes = [ctypes.POINTER(ServerOpts)]
    lib.zset_server_default_opts.restype = None
    lib.zset_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)]
    lib.zset_server_add_set.argtypes = [ctypes.c_void_p, _u32p, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_int, _i32p]
    lib.zset_server_set_info.argtypes = [ctypes.c_void_p, ctypes.c_int, _i32p, _u64p, _u64p,
                                         _u64p, _u64p]
    lib.zset_server_count.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, _u64p]
    lib.zset_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, _u64p]
    lib.zset_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.POINTER(ServerResult)]
    lib.zset_server_release.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.zset_server_stats.argtypes = [ctypes.c_void_p, _u64p, _u64p, _u64p,
                                      ctypes.POINTER(ctypes.c_double)]
    lib.zset_server_free.argtypes = [ctypes.c_void_p]
    lib.zset_server_free.restype = None
    lib.zset_strerror.argtypes = [ctypes.c_int]
    lib.zset_strerror.restype = ctypes.c_char_p
    lib.zset_selftest_host.argtypes = []
    lib.zset_last_error.argtypes = []
    lib.zset_last_error.restype = ctypes.c_char_p
    for name in ("zset_count", "zset_count_table", "zset_memo_build", "zset_memo_read",
                 "zset_enumerate", "zset_enumerate_ex", "zset_enumerate_noalloc",
                 "zset_enumerate_async", "zset_batch_create", "zset_batch_info",
                 "zset_batch_run", "zset_batch_times", "zset_selftest_host",
                 "zset_server_create", "zset_server_add_set", "zset_server_set_info",
                 "zset_server_count", "zset_server_submit", "zset_server_wait",
                 "zset_server_release", "zset_server_stats", "zset_store_ceiling"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().zset_strerror(status).decode()


def last_error() -> str:
    return load().zset_last_error().decode()


def _check(status: int, where: str) -> None:
    if status != OK:
        raise ZsetError(status, where, last_error())


def _gens(gens) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(gens, dtype=np.uint32).reshape(-1))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def selftest_host() -> None:
    _check(load().zset_selftest_host(), "zset_selftest_host")


def count(n: int, gens) -> int:
    """|Z(n; g)|, computed on the GPU."""
    g = _gens(gens)
    out = ctypes.c_uint64(0)
    _check(load().zset_count(n, g.ctypes.data_as(_u32p), len(g), ctypes.byref(out)),
           "zset_count")
    return int(out.value)


def count_table(n: int, gens, stream=None):
    """(d+1, n+1) int64 CUDA tensor holding the uint64 count table bit patterns."""
    import torch
    g = _gens(gens)
    t = torch.empty((len(g) + 1, n + 1), dtype=torch.int64, device="cuda")
    _check(load().zset_count_table(n, g.ctypes.data_as(_u32p), len(g), t.data_ptr(),
                                   _stream_handle(stream)), "zset_count_table")
    return t


class Memo:
    """Device-resident memo of Z(p; h) for p < top (zset_memo_build)."""

    def __init__(self, h, top: int, stream=None):
        self.h = [int(x) for x in _gens(h)]
        self.k = len(self.h)
        self.top = int(top)
        g = _gens(h)
        handle = ctypes.c_void_p(None)
        _check(load().zset_memo_build(g.ctypes.data_as(_u32p), self.k, self.top,
                                      _stream_handle(stream), ctypes.byref(handle)),
               "zset_memo_build")
        self._handle = handle

    @property
    def handle(self):
        return self._handle

    def sizes(self):
        top, k, rows = ctypes.c_uint64(), ctypes.c_int(), ctypes.c_uint64()
        _check(load().zset_memo_read(self._handle, None, None, ctypes.byref(top),
                                     ctypes.byref(k), ctypes.byref(rows)), "zset_memo_read")
        return int(top.value), int(k.value), int(rows.value)

    def read(self):
        """(off[top+1] uint64, rows[R, k] uint32) copied to the host."""
        top, k, rows = self.sizes()
        off = np.empty(top + 1, dtype=np.uint64)
        data = np.empty((max(rows, 1), k), dtype=np.uint32)
        _check(load().zset_memo_read(self._handle, off.ctypes.data_as(_u64p),
                                     data.ctypes.data_as(_u32p), None, None, None),
               "zset_memo_read")
        return off, data[:rows]

    def free(self):
        if self._handle is not None and self._handle.value:
            load().zset_memo_free(self._handle)
        self._handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclass
class Result:
    rows: int
    checksum: int
    stats: dict
    out: object = None   # torch.int32 CUDA tensor (rows, d): the uint32 rows


def tuned(n: int, gens):
    """(k, rows_per_tile) from the autotuner's table for this query's bucket
    (d, decade of |Z(n)|), or (-1, 0) -- the library's own choice -- when the
    table has no entry."""
    from . import autotune
    g = _gens(gens)
    c = autotune.choose(len(g), count(n, g))
    return c if c is not None else (-1, 0)


def enumerate_ex(n: int, gens, out=None, *, k: int = -1, order: int = 0,
                 rows_per_tile: int = 0, count_only: bool = False, memo: Memo | None = None,
                 stream=None, out_rows_cap: int | None = None, claim_pct: int = -1,
                 memo_top: int = 0, stats: bool = True) -> Result:
    """Z(n; g) through zset_enumerate_ex.  `out` is an int32 CUDA tensor with at least
    |Z(n)| * d elements (allocated here when None and count_only is False).
    `claim_pct`: percent of slices claimed at run time (-1 automatic, 0 none).
    `memo_top`: 0, or the memo covers p < memo_top only (a partial memo).
    `stats`: False passes no stats structure (the call records no timing
    events); Result.stats is then empty."""
    import torch
    g = _gens(gens)
    d = len(g)
    if k == "tuned":
        k, t = tuned(n, g)
        rows_per_tile = rows_per_tile or t
    if out is None and not count_only:
        rows = count(n, g)
        out = torch.empty((max(rows, 1), d), dtype=torch.int32, device="cuda")
    if out is not None:
        cap = out.numel() // max(d, 1) if out_rows_cap is None else out_rows_cap
        ptr = out.data_ptr()
    else:
        cap, ptr = 0, None
    opts = Opts()
    load().zset_default_opts(ctypes.byref(opts))
    opts.k, opts.order, opts.rows_per_tile = k, order, rows_per_tile
    opts.count_only = 1 if count_only else 0
    opts.stream = _stream_handle(stream)
    opts.claim_pct = claim_pct
    opts.memo_top = memo_top
    rows_written, csum = ctypes.c_uint64(), ctypes.c_uint64()
    st = Stats() if stats else None
    _check(load().zset_enumerate_ex(n, g.ctypes.data_as(_u32p), d, ptr, cap, ctypes.byref(opts),
                                    memo.handle if memo is not None else None,
                                    ctypes.byref(rows_written), ctypes.byref(csum),
                                    ctypes.byref(st) if st is not None else None),
           "zset_enumerate_ex")
    r = int(rows_written.value)
    view = out[:r] if (out is not None and out.dim() == 2) else out
    return Result(rows=r, checksum=int(csum.value), stats=st.as_dict() if st is not None else {},
                  out=view)


def enumerate_noalloc(n: int, gens, out=None, *, k: int = -1, order: int = 0,
                      rows_per_tile: int = 0, count_only: bool = False, stream=None,
                      out_rows_cap: int | None = None, claim_pct: int = -1,
                      memo_top: int = 0) -> Result:
    """Z(n; g) through zset_enumerate_noalloc (scratch from the library's fixed
    device array; no device allocation by the library).  `out` as for
    enumerate_ex, but never allocated here: pass it unless count_only."""
    g = _gens(gens)
    d = len(g)
    if out is not None:
        cap = out.numel() // max(d, 1) if out_rows_cap is None else out_rows_cap
        ptr = out.data_ptr()
    else:
        cap, ptr = 0, None
    opts = Opts()
    load().zset_default_opts(ctypes.byref(opts))
    opts.k, opts.order, opts.rows_per_tile = k, order, rows_per_tile
    opts.count_only = 1 if count_only else 0
    opts.stream = _stream_handle(stream)
    opts.claim_pct = claim_pct
    opts.memo_top = memo_top
    rows_written, csum = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().zset_enumerate_noalloc(n, g.ctypes.data_as(_u32p), d, ptr, cap,
                                         ctypes.byref(opts), ctypes.byref(rows_written),
                                         ctypes.byref(csum)), "zset_enumerate_noalloc")
    r = int(rows_written.value)
    view = out[:r] if (out is not None and out.dim() == 2) else out
    return Result(rows=r, checksum=int(csum.value), stats={}, out=view)


def enumerate_async(n: int, gens, out, result, *, k: int = -1, order: int = 0,
                    count_only: bool = False, stream=None, out_rows_cap: int | None = None,
                    write_events=None) -> None:
    """Enqueue Z(n; g) through zset_enumerate_async and return without waiting.
    `result` is a pinned int64 CPU tensor of at least 3 elements, written by
    the device (read it with async_outcome once the stream is synchronised);
    `out` as for enumerate_ex, never allocated here.  `write_events`: None, or
    two torch.cuda.Event(enable_timing=True) recorded around the write pass."""
    g = _gens(gens)
    d = len(g)
    if not (result.is_pinned() and result.dtype.itemsize == 8 and result.numel() >= 3
            and result.is_contiguous()):
        raise ValueError("result must be a contiguous pinned 64-bit CPU tensor of >= 3 elements")
    if out is not None:
        cap = out.numel() // max(d, 1) if out_rows_cap is None else out_rows_cap
        ptr = out.data_ptr()
    else:
        cap, ptr = 0, None
    opts = Opts()
    load().zset_default_opts(ctypes.byref(opts))
    opts.k, opts.order = k, order
    opts.count_only = 1 if count_only else 0
    opts.stream = _stream_handle(stream)
    evs = None
    if write_events is not None:
        handles = []
        for ev in write_events:
            if not ev.cuda_event:
                ev.record()  # torch creates the event at its first record
            handles.append(ev.cuda_event)
        evs = (ctypes.c_void_p * 2)(*handles)
    _check(load().zset_enumerate_async(n, g.ctypes.data_as(_u32p), d, ptr, cap,
                                       ctypes.byref(opts), result.data_ptr(), evs),
           "zset_enumerate_async")


def async_outcome(result) -> tuple[int, int]:
    """(|Z(n)|, checksum) from the result words of a finished asynchronous
    call; raises ZsetError when the call's outcome was an error."""
    import torch
    st, rows, csum = (int(x) for x in result[:3].view(torch.int64).tolist())
    if st != OK:
        raise ZsetError(st, "zset_enumerate_async", f"outcome {strerror(st)}, |Z(n)| = {rows}")
    return rows & ((1 << 64) - 1), csum & ((1 << 64) - 1)


def store_ceiling(buf, reps: int = 5, stream=None) -> float:
    """Mean microseconds per pass of the library's store-only kernel (16-byte
    non-temporal stores, the write pass's store form) over the whole of `buf`,
    a CUDA tensor (overwritten).  A measurement of the device, not of Z(n)."""
    us = ctypes.c_double()
    _check(load().zset_store_ceiling(buf.data_ptr(), buf.numel() * buf.element_size(), reps,
                                     _stream_handle(stream), ctypes.byref(us)),
           "zset_store_ceiling")
    return float(us.value)


def enumerate_walk(n: int, gens, out, *, order: int = 0, stream=None) -> int:
    """Z(n; g) through zset_enumerate_walk (no count table) into `out`, an int32
    CUDA tensor of at least |Z(n)| * d elements; returns |Z(n)|."""
    g = _gens(gens)
    cap = out.numel() // len(g)
    rows = ctypes.c_uint64()
    _check(load().zset_enumerate_walk(n, g.ctypes.data_as(_u32p), len(g), out.data_ptr(), cap,
                                      order, _stream_handle(stream), ctypes.byref(rows)),
           "zset_enumerate_walk")
    return int(rows.value)


def enumerate(n: int, gens, out=None):
    """Z(n; g) through the plain zset_enumerate (default options, null stream)."""
    import torch
    g = _gens(gens)
    d = len(g)
    rows = count(n, g)
    if out is None:
        out = torch.empty((max(rows, 1), d), dtype=torch.int32, device="cuda")
    _check(load().zset_enumerate(n, g.ctypes.data_as(_u32p), d, out.data_ptr()),
           "zset_enumerate")
    return out[:rows]


@dataclass
class BatchResult:
    checksums: np.ndarray   # per query (count-only batches; zeros otherwise)
    stats: dict
    out: object = None      # int32 CUDA tensor of total_words elements


class Batch:
    """Many independent queries planned once (zset_batch_create) and run by one
    persistent write launch per run (zset_batch_run).  `queries` is a list of
    (n, gens); `k` and `rows_per_tile` are None (automatic) or one value per
    query (-1 / 0 = automatic)."""

    def __init__(self, queries, *, k=None, rows_per_tile=None, count_only: bool = False,
                 max_chain_steps: int = 0, unit_tiles: int = 0, use_graph: bool = True,
                 stream=None):
        self.nq = len(queries)
        if self.nq == 0:
            raise ValueError("a batch needs at least one query")
        ns = np.ascontiguousarray([int(n) for n, _ in queries], dtype=np.uint64)
        gl = [_gens(g) for _, g in queries]
        ds = np.ascontiguousarray([len(g) for g in gl], dtype=np.int32)
        gens = np.ascontiguousarray(np.concatenate(gl) if gl else np.zeros(0), dtype=np.uint32)
        self.d = ds.astype(np.int64)
        self.gens = [list(map(int, g)) for g in gl]
        self.n = ns.astype(np.int64)
        kk = None if k is None else np.ascontiguousarray(k, dtype=np.int32)
        tt = None if rows_per_tile is None else np.ascontiguousarray(rows_per_tile,
                                                                     dtype=np.uint64)
        opts = BatchOpts()
        load().zset_batch_default_opts(ctypes.byref(opts))
        opts.count_only = 1 if count_only else 0
        opts.max_chain_steps = max_chain_steps
        opts.unit_tiles = unit_tiles
        opts.use_graph = 1 if use_graph else 0
        opts.stream = _stream_handle(stream)
        self.count_only = count_only
        handle = ctypes.c_void_p(None)
        _i32p = ctypes.POINTER(ctypes.c_int)
        _check(load().zset_batch_create(
            self.nq, ns.ctypes.data_as(_u64p), ds.ctypes.data_as(_i32p),
            gens.ctypes.data_as(_u32p),
            kk.ctypes.data_as(_i32p) if kk is not None else None,
            tt.ctypes.data_as(_u64p) if tt is not None else None,
            ctypes.byref(opts), ctypes.byref(handle)), "zset_batch_create")
        self._handle = handle
        total = ctypes.c_uint64()
        self.rows = np.zeros(self.nq, dtype=np.uint64)
        self.offsets = np.zeros(self.nq, dtype=np.uint64)
        self.k = np.zeros(self.nq, dtype=np.int32)
        self.tiles = np.zeros(self.nq, dtype=np.uint64)
        _check(load().zset_batch_info(self._handle, ctypes.byref(total),
                                      self.rows.ctypes.data_as(_u64p),
                                      self.offsets.ctypes.data_as(_u64p),
                                      self.k.ctypes.data_as(_i32p),
                                      self.tiles.ctypes.data_as(_u64p)), "zset_batch_info")
        self.total_words = int(total.value)

    def alloc(self):
        import torch
        return torch.empty(max(self.total_words, 4), dtype=torch.int32, device="cuda")

    def run(self, out=None) -> BatchResult:
        if out is None and not self.count_only:
            out = self.alloc()
        cs = np.zeros(self.nq, dtype=np.uint64)
        st = BatchStats()
        ptr = out.data_ptr() if out is not None else None
        cap = out.numel() if out is not None else 0
        _check(load().zset_batch_run(self._handle, ptr, cap, cs.ctypes.data_as(_u64p),
                                     ctypes.byref(st)), "zset_batch_run")
        return BatchResult(checksums=cs, stats=st.as_dict(), out=out)

    def rows_of(self, out, q: int):
        """Query q's rows in `out` as an int32 (|Z_q|, d_q) view."""
        o, r, d = int(self.offsets[q]), int(self.rows[q]), int(self.d[q])
        return out[o:o + r * d].view(r, d)

    def times(self) -> np.ndarray:
        """Per-query completion times of the last run, microseconds from its start."""
        t = np.zeros(self.nq, dtype=np.float64)
        _check(load().zset_batch_times(self._handle,
                                       t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "zset_batch_times")
        return t

    def free(self):
        if self._handle is not None and self._handle.value:
            load().zset_batch_free(self._handle)
        self._handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Request loop over resident generator sets (zset_server_*).

    HIP runs streams on GPU_MAX_HW_QUEUES hardware queues (4 by default), which
    bounds how many queries run on the device at once: set it to the slot count
    (at most 32) in the environment before the runtime starts.

    `arena` is a contiguous int32 CUDA tensor that the outputs are carved from;
    the caller keeps it alive while the server runs.  Submission never blocks;
    wait() blocks until a query is done (the GIL is released meanwhile)."""

    def __init__(self, arena, slots: int = 8, dispatchers: int = 1, memo_bytes: int = 0):
        if arena.dtype.itemsize != 4 or not arena.is_contiguous():
            raise ValueError("arena must be a contiguous 4-byte CUDA tensor")
        self.arena = arena.reshape(-1)
        self.d = []
        opts = ServerOpts()
        load().zset_server_default_opts(ctypes.byref(opts))
        opts.slots = slots
        opts.dispatchers = dispatchers
        opts.memo_bytes = memo_bytes
        opts.arena = self.arena.data_ptr()
        opts.arena_bytes = self.arena.numel() * 4
        handle = ctypes.c_void_p(None)
        _check(load().zset_server_create(ctypes.byref(opts), ctypes.byref(handle)),
               "zset_server_create")
        self._handle = handle

    def add_set(self, gens, n_max: int, k=-1) -> int:
        """k: -1 (the library's rule), "tuned" (the autotuner's choice for the
        bucket of |Z(n_max)|), or a memo dimension."""
        g = _gens(gens)
        if k == "tuned":
            k = tuned(n_max, g)[0]
        sid = ctypes.c_int()
        _check(load().zset_server_add_set(self._handle, g.ctypes.data_as(_u32p), len(g), n_max, k,
                                          ctypes.byref(sid)), "zset_server_add_set")
        self.d.append(len(g))
        return int(sid.value)

    def set_info(self, set_id: int) -> dict:
        k, n_max, rows, nbytes = ctypes.c_int(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        top = ctypes.c_uint64()
        _check(load().zset_server_set_info(self._handle, set_id, ctypes.byref(k),
                                           ctypes.byref(n_max), ctypes.byref(rows),
                                           ctypes.byref(nbytes), ctypes.byref(top)),
               "zset_server_set_info")
        return {"k": int(k.value), "n_max": int(n_max.value), "memo_rows": int(rows.value),
                "resident_bytes": int(nbytes.value), "memo_top": int(top.value)}

    def count(self, set_id: int, n: int) -> int:
        v = ctypes.c_uint64()
        _check(load().zset_server_count(self._handle, set_id, n, ctypes.byref(v)),
               "zset_server_count")
        return int(v.value)

    def submit(self, set_id: int, n: int) -> int:
        t = ctypes.c_uint64()
        _check(load().zset_server_submit(self._handle, set_id, n, ctypes.byref(t)),
               "zset_server_submit")
        return int(t.value)

    def wait(self, ticket: int) -> dict:
        r = ServerResult()
        _check(load().zset_server_wait(self._handle, ticket, ctypes.byref(r)), "zset_server_wait")
        return r.as_dict()

    def rows_of(self, set_id: int, result: dict):
        """The query's rows: an int32 view (rows, d) into the arena."""
        d = self.d[set_id]
        off, rows = int(result["out_offset"]), int(result["rows"])
        return self.arena[off:off + rows * d].view(rows, d)

    def release(self, ticket: int) -> None:
        _check(load().zset_server_release(self._handle, ticket), "zset_server_release")

    def stats(self) -> dict:
        a, c, m, t = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
        _check(load().zset_server_stats(self._handle, ctypes.byref(a), ctypes.byref(c),
                                        ctypes.byref(m), ctypes.byref(t)), "zset_server_stats")
        return {"admitted": int(a.value), "completed": int(c.value),
                "max_inflight": int(m.value), "launch_us": float(t.value)}

    def free(self) -> None:
        if self._handle is not None and self._handle.value:
            load().zset_server_free(self._handle)
        self._handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
