"""CPU oracle for Z(n; g_1..g_d) -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links or
calls it, and it shares no code with the HIP path.

The arithmetic lives in ``zset_oracle.c`` (plain C, built with gcc into
``liboracle.so`` next to it); this module only marshals numpy arrays through
ctypes.

Definition followed (paper, Section 1): Z(n; g) = {a in N^d : sum a_i g_i = n},
rows of d uint32 values, strictly ascending in lexicographic order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zset_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EOVERFLOW, ENOMEM, ECAPACITY = 0, -1, -2, -3, -4

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_lib_handle = None


def build(force: bool = False) -> str:
    """Compile zset_oracle.c with gcc into liboracle.so (idempotent)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _lib_handle
    if _lib_handle is None:
        # ZSET_ORACLE_LIB names another build of zset_oracle.c (the sanitizer
        # build of the CPU tests).
        lib = ctypes.CDLL(os.environ.get("ZSET_ORACLE_LIB") or build())
        lib.oracle_count.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, _u64p]
        lib.oracle_count_table.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, _u64p]
        lib.oracle_enumerate.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, _u32p,
                                         ctypes.c_uint64, _u64p]
        lib.oracle_enumerate_a1.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int,
                                            ctypes.c_uint64, ctypes.c_uint64, _u32p,
                                            ctypes.c_uint64, _u64p]
        lib.oracle_unrank.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int, _u64p,
                                      ctypes.c_uint64, _u32p]
        lib.oracle_memo.argtypes = [_u32p, ctypes.c_int, ctypes.c_uint64, _u64p, _u32p,
                                    ctypes.c_uint64]
        lib.oracle_memo_dynamic.argtypes = [_u32p, ctypes.c_int, ctypes.c_uint64, _u64p, _u32p,
                                            ctypes.c_uint64]
        lib.oracle_fnv1a64.argtypes = [ctypes.c_char_p, ctypes.c_uint64]
        lib.oracle_fnv1a64.restype = ctypes.c_uint64
        lib.oracle_checksum.argtypes = [_u32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64]
        lib.oracle_checksum.restype = ctypes.c_uint64
        lib.oracle_enumerate_a1_threads.argtypes = [
            ctypes.c_uint64, _u32p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, _u64p,
            _u32p, ctypes.c_uint64, ctypes.c_int, _u64p]
        _lib_handle = lib
    return _lib_handle


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _gens(gens) -> np.ndarray:
    g = np.ascontiguousarray(np.asarray(gens, dtype=np.uint32).reshape(-1))
    return g


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_u32p)


def _p64(a: np.ndarray):
    return a.ctypes.data_as(_u64p)


def count(n: int, gens) -> int:
    """|Z(n; g)| from the generating-function coefficient (coin recurrence)."""
    g = _gens(gens)
    out = np.zeros(1, dtype=np.uint64)
    st = _lib().oracle_count(n, _p32(g), len(g), _p64(out))
    if st == EOVERFLOW:
        raise OverflowError("|Z(n)| >= 2^64 - 1")
    if st != OK:
        raise OracleError(st, "oracle_count")
    return int(out[0])


def count_table(n: int, gens) -> np.ndarray:
    """(d+1, n+1) uint64: row j holds |Z(x; g_{j+1}..g_d)|, saturated at 2^64-1."""
    g = _gens(gens)
    t = np.empty((len(g) + 1, n + 1), dtype=np.uint64)
    st = _lib().oracle_count_table(n, _p32(g), len(g), _p64(t))
    if st != OK:
        raise OracleError(st, "oracle_count_table")
    return t


def enumerate_rows(n: int, gens, a1_lo: int = 0, a1_hi: int | None = None) -> np.ndarray:
    """Rows of Z(n; g) (optionally only those with a_1 in [a1_lo, a1_hi)), ascending,
    as an (rows, d) uint32 array."""
    g = _gens(gens)
    d = len(g)
    hi = (1 << 64) - 1 if a1_hi is None else a1_hi
    got = np.zeros(1, dtype=np.uint64)
    lib = _lib()
    st = lib.oracle_enumerate_a1(n, _p32(g), d, a1_lo, hi, None, 0, _p64(got))
    if st not in (OK, ECAPACITY):
        raise OracleError(st, "oracle_enumerate_a1")
    rows = int(got[0])
    out = np.empty((rows, d), dtype=np.uint32)
    st = lib.oracle_enumerate_a1(n, _p32(g), d, a1_lo, hi,
                                 _p32(out) if rows else None, rows, _p64(got))
    if st != OK:
        raise OracleError(st, "oracle_enumerate_a1")
    return out


def enumerate_rows_threads(n: int, gens, a1_lo: int, a1_hi: int, nthreads: int,
                           table: np.ndarray | None = None, out: np.ndarray | None = None):
    """Threaded form of enumerate_rows over a_1 in [a1_lo, a1_hi); returns (out, rows)."""
    g = _gens(gens)
    d = len(g)
    if table is None:
        table = count_table(n, g)
    row1 = np.ascontiguousarray(table[1])
    hi = min(a1_hi, n // int(g[0]) + 1)
    lo = min(a1_lo, hi)
    total = int(sum(int(row1[n - a * int(g[0])]) for a in range(lo, hi)))
    if out is None:
        out = np.empty((max(total, 1), d), dtype=np.uint32)
    got = np.zeros(1, dtype=np.uint64)
    st = _lib().oracle_enumerate_a1_threads(n, _p32(g), d, lo, hi, _p64(row1), _p32(out),
                                            out.shape[0], nthreads, _p64(got))
    if st != OK:
        raise OracleError(st, "oracle_enumerate_a1_threads")
    return out, int(got[0])


def unrank(n: int, gens, r: int, table: np.ndarray | None = None) -> np.ndarray:
    """The row at ascending rank r."""
    g = _gens(gens)
    if table is None:
        table = count_table(n, g)
    table = np.ascontiguousarray(table)
    row = np.empty(len(g), dtype=np.uint32)
    st = _lib().oracle_unrank(n, _p32(g), len(g), _p64(table), r, _p32(row))
    if st != OK:
        raise OracleError(st, "oracle_unrank")
    return row


def memo(h, top: int):
    """(off[top+1] uint64, rows[R, k] uint32): Z(p; h) ascending for p < top."""
    hh = _gens(h)
    k = len(hh)
    off = np.empty(top + 1, dtype=np.uint64)
    lib = _lib()
    st = lib.oracle_memo(_p32(hh), k, top, _p64(off), None, 0)
    if st != OK:
        raise OracleError(st, "oracle_memo (sizing)")
    total = int(off[top])
    rows = np.empty((max(total, 1), k), dtype=np.uint32)
    st = lib.oracle_memo(_p32(hh), k, top, _p64(off), _p32(rows), total)
    if st != OK:
        raise OracleError(st, "oracle_memo")
    return off, rows[:total]


def memo_dynamic(h, top: int, timed: bool = False):
    """The same (off, rows) built serially by the paper's dynamic recurrence
    (oracle_memo_dynamic).  With timed=True also returns the seconds of the
    building call alone (the sizing call and the allocation are not timed)."""
    import time
    hh = _gens(h)
    k = len(hh)
    off = np.empty(top + 1, dtype=np.uint64)
    lib = _lib()
    st = lib.oracle_memo_dynamic(_p32(hh), k, top, _p64(off), None, 0)
    if st != OK:
        raise OracleError(st, "oracle_memo_dynamic (sizing)")
    total = int(off[top])
    rows = np.empty((max(total, 1), k), dtype=np.uint32)
    rows.fill(0)
    t = time.perf_counter()
    st = lib.oracle_memo_dynamic(_p32(hh), k, top, _p64(off), _p32(rows), total)
    dt = time.perf_counter() - t
    if st != OK:
        raise OracleError(st, "oracle_memo_dynamic")
    return (off, rows[:total], dt) if timed else (off, rows[:total])


def fnv1a64(data: bytes) -> int:
    return int(_lib().oracle_fnv1a64(data, len(data)))


def checksum(rows: np.ndarray, rank0: int = 0) -> int:
    """Sum over rows of FNV1a64(LE64(rank) || LE32 coords), modulo 2^64."""
    r = np.ascontiguousarray(rows, dtype=np.uint32)
    d = r.shape[1] if r.ndim == 2 else 1
    n = r.shape[0]
    return int(_lib().oracle_checksum(_p32(r) if n else None, n, d, rank0))
