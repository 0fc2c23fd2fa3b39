"""Host-side checks of libzset.so that need no GPU: it loads, exports every
symbol include/zset.h declares, its host helpers pass their self-test, and
argument errors come back as status codes before any device call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2407_20474_amd import inputs
from paper_2407_20474_amd import zset

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "zset.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zset_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = zset.load()
    declared = header_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(zset.SYMBOLS) == declared


def test_host_selftest():
    zset.selftest_host()


def test_strerror_texts():
    texts = {s: zset.strerror(s) for s in (0, -1, -2, -3, -4, -5)}
    assert len(set(texts.values())) == 6
    assert zset.strerror(-99) == "unknown status"


def _count_status(n, gens, d=None):
    lib = zset.load()
    g = np.ascontiguousarray(np.asarray(gens, dtype=np.uint32))
    out = ctypes.c_uint64(0)
    d = len(g) if d is None else d
    ptr = g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if len(g) else None
    return lib.zset_count(n, ptr, d, ctypes.byref(out))


@pytest.mark.parametrize("n,gens,d", [
    (10, [3, 0, 5], None),          # a zero generator: Z would be infinite
    (10, [], 0),                    # d < 1
    (10, [1] * 33, None),           # d > 32
    (1 << 31, [3, 5], None),        # n beyond the supported range
    (10, None, 2),                  # NULL generators
])
def test_invalid_arguments_are_rejected_before_the_device(n, gens, d):
    if gens is None:
        lib = zset.load()
        out = ctypes.c_uint64(0)
        st = lib.zset_count(n, None, d, ctypes.byref(out))
    else:
        st = _count_status(n, gens, d)
    assert st == zset.EINVAL
    assert zset.last_error()


def test_enumerate_ex_option_checks():
    lib = zset.load()
    g = np.array([3, 5, 7], dtype=np.uint32)
    gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))

    def run(**kw):
        o = zset.Opts()
        lib.zset_default_opts(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return lib.zset_enumerate_ex(20, gp, 3, None, 0, ctypes.byref(o), None, None, None, None)

    assert run(k=3) == zset.EINVAL          # k must be <= d - 1
    assert run(k=-2) == zset.EINVAL
    assert run(order=2) == zset.EINVAL
    assert run(rows_per_tile=100) == zset.EINVAL   # not a multiple of 128
    assert run(claim_pct=101) == zset.EINVAL
    assert run(claim_pct=-2) == zset.EINVAL
    assert run() == zset.EINVAL              # out is NULL and rows are wanted


def test_enumerate_async_checks_before_the_device():
    lib = zset.load()
    g = np.array([3, 5, 7], dtype=np.uint32)
    gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))

    def run(result=None, **kw):
        o = zset.Opts()
        lib.zset_default_opts(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return lib.zset_enumerate_async(20, gp, 3, None, 0, ctypes.byref(o), result, None)

    assert run(k=3) == zset.EINVAL
    assert run(order=2) == zset.EINVAL
    assert run(rows_per_tile=100) == zset.EINVAL
    assert run() == zset.EINVAL                      # out is NULL and rows are wanted
    assert run(count_only=1) == zset.EINVAL          # result is NULL
    assert "result" in zset.last_error()
    assert lib.zset_enumerate_async(20, None, 3, None, 0, None, None, None) == zset.EINVAL


def test_memo_build_argument_checks():
    lib = zset.load()
    h = np.array([4, 9], dtype=np.uint32)
    hp = h.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    handle = ctypes.c_void_p()
    assert lib.zset_memo_build(hp, 0, 10, None, ctypes.byref(handle)) == zset.EINVAL
    assert lib.zset_memo_build(hp, 2, 0, None, ctypes.byref(handle)) == zset.EINVAL
    assert lib.zset_memo_build(hp, 2, 10, None, None) == zset.EINVAL
    assert lib.zset_memo_read(None, None, None, None, None, None) == zset.EINVAL


def test_default_opts():
    lib = zset.load()
    o = zset.Opts()
    o.k, o.order, o.rows_per_tile, o.count_only = 5, 1, 256, 1
    lib.zset_default_opts(ctypes.byref(o))
    o.claim_pct = 7
    lib.zset_default_opts(ctypes.byref(o))
    assert (o.k, o.order, o.rows_per_tile, o.count_only, o.claim_pct) == (-1, 0, 0, 0, -1)
    assert o.stream is None


# --------------------------------------------------------------------------
# Seeded inputs and the stored workloads
# --------------------------------------------------------------------------

def test_draw_gens_is_seeded_distinct_and_coprime():
    for seed in range(20):
        g = inputs.draw_gens(seed, 6, 10, 100)
        assert g == inputs.draw_gens(seed, 6, 10, 100)
        assert len(set(g)) == 6 and g == sorted(g)
        assert all(10 <= x <= 100 for x in g)
        assert math.gcd(*g) == 1


def test_stored_workloads_match_the_oracle():
    w = inputs.load_workloads()
    assert w["plain"]["rows"] == oracle.count(w["plain"]["n"], w["plain"]["gens"]) == 81205
    for item in w["large"]:
        g, n = item["gens"], item["n"]
        assert g == inputs.draw_gens(item["seed"], 6, 10, 100)
        ways = oracle.count_table(n, g)[0]
        assert int(ways[n]) == item["rows"] >= 200_000_000
        assert (ways[:n] < 200_000_000).all()   # n is the smallest such element
    for item in w["sweep"]:
        g, n = item["gens"], item["n"]
        assert g == inputs.draw_gens(item["seed"], len(g), 10, 200)
        assert oracle.count(n, g) == item["rows"]
        assert 1e8 <= item["rows"] <= 1e9


def test_server_argument_checks():
    lib = zset.load()
    handle = ctypes.c_void_p()
    assert lib.zset_server_create(None, ctypes.byref(handle)) == zset.EINVAL
    o = zset.ServerOpts()
    lib.zset_server_default_opts(ctypes.byref(o))
    assert o.slots == 8 and not o.arena and o.arena_bytes == 0
    assert lib.zset_server_create(ctypes.byref(o), ctypes.byref(handle)) == zset.EINVAL  # no arena
    o.slots = 65
    assert lib.zset_server_create(ctypes.byref(o), ctypes.byref(handle)) == zset.EINVAL
    t = ctypes.c_uint64()
    assert lib.zset_server_submit(None, 0, 10, ctypes.byref(t)) == zset.EINVAL
    assert lib.zset_server_wait(None, 1, None) == zset.EINVAL
    assert lib.zset_server_release(None, 1) == zset.EINVAL
    g = np.array([3, 5], dtype=np.uint32)
    sid = ctypes.c_int()
    assert lib.zset_server_add_set(None, g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 2, 10,
                                   -1, ctypes.byref(sid)) == zset.EINVAL
    lib.zset_server_free(None)


def test_autotune_table_is_well_formed():
    from paper_2407_20474_amd import autotune
    import json
    t = json.load(open(autotune.TUNING_JSON))["buckets"]
    for d in range(3, 10):
        for dec in autotune.DECADES:
            e = t[f"d={d},dec={dec}"]
            assert 0 <= e["k"] <= d - 1 and e["rows_per_tile"] % 128 == 0 and e["rows_per_s"] > 0
    assert autotune.bucket_key(5, 3e8) == "d=5,dec=8"
    assert autotune.bucket_key(4, 7) == "d=4,dec=3"       # below the first decade
    assert autotune.bucket_key(4, 5e12) == "d=4,dec=8"    # above the last
    assert autotune.choose(6, 2e8) == (t["d=6,dec=8"]["k"], t["d=6,dec=8"]["rows_per_tile"])
    assert autotune.choose(12, 1000) is None              # no bucket
