"""zset_enumerate_async through the C ABI: the same rows, counts and checksums
as the oracle (bit-exact) when several calls are queued before one wait, on one
stream or two, interleaved with synchronous calls, with scratch buffers that
must grow between queued calls, with errors found on the device, and on the
forms that run to completion inside the call.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2407_20474_amd import zset

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rows_of(out, r, d):
    return out[:r].cpu().numpy().view(np.uint32).reshape(r, d)


def pinned_result():
    return torch.full((3,), -99, dtype=torch.int64).pin_memory()


def assert_same(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.nonzero((got != want).any(axis=1))[0]
        i = int(bad[0])
        raise AssertionError(f"{what}: {len(bad)} rows differ, first at {i}: "
                             f"got {got[i].tolist()} want {want[i].tolist()}")


# (n, g, k): the first ones take the three-launch form (k = 1 or 2, n + 1 <=
# 16384); the last ones run to completion inside the call (k = 0, k = 3, a
# count table beyond LDS).
QUEUED = [(2000, [7, 11, 13, 17], 2), (1500, [5, 9, 23], 1), (16383, [90, 97, 120, 131], 2),
          (0, [3, 5], 1), (7, [3, 5, 11], 2), (3000, [6, 10, 14, 21], 2)]
IN_CALL = [(900, [4, 7, 9], 0), (700, [5, 6, 7, 8, 9], 3), (20000, [900, 1200, 2500], 2)]


def test_queued_calls_on_one_stream_match_the_oracle():
    cases = QUEUED + IN_CALL
    wants = [oracle.enumerate_rows(n, g) for n, g, _ in cases]
    # Largest case first would size every buffer at once; smallest first
    # makes later queued calls grow the library's scratch.
    order = sorted(range(len(cases)), key=lambda i: len(wants[i]))
    outs, results = {}, {}
    s = torch.cuda.Stream()
    for i in order:
        n, g, k = cases[i]
        outs[i] = torch.full((max(len(wants[i]), 1), len(g)), -1, dtype=torch.int32,
                             device="cuda")
        results[i] = pinned_result()
    torch.cuda.synchronize()
    for i in order:
        n, g, k = cases[i]
        say(f"  queued n={n} g={g} k={k}")
        zset.enumerate_async(n, g, outs[i], results[i], k=k, stream=s)
    s.synchronize()
    for i in order:
        n, g, k = cases[i]
        rows, csum = zset.async_outcome(results[i])
        assert rows == len(wants[i]) and csum == 0, (n, g, k)
        assert_same(rows_of(outs[i], rows, len(g)), wants[i], f"async n={n} g={g} k={k}")


def test_queued_descending_and_count_only():
    n, g = 5000, [7, 11, 13, 17, 19]
    want = oracle.enumerate_rows(n, g)
    out = torch.empty((len(want), len(g)), dtype=torch.int32, device="cuda")
    res = [pinned_result() for _ in range(4)]
    torch.cuda.synchronize()
    for k in (1, 2):
        zset.enumerate_async(n, g, out if k == 2 else None, res[k - 1], k=k, order=1,
                             count_only=k == 1)
    zset.enumerate_async(n, g, None, res[2], k=2, count_only=True)
    torch.cuda.synchronize()
    assert_same(rows_of(out, len(want), len(g)), np.ascontiguousarray(want[::-1]),
                "async descending")
    want_sum = oracle.checksum(want)
    assert zset.async_outcome(res[0]) == (len(want), want_sum)   # count-only, order ignored
    assert zset.async_outcome(res[1]) == (len(want), 0)
    assert zset.async_outcome(res[2]) == (len(want), want_sum)


def test_two_streams_and_synchronous_calls_between():
    a = (4000, [9, 13, 29, 31])
    b = (2500, [4, 6, 15, 35, 77])
    wa, wb = oracle.enumerate_rows(*a), oracle.enumerate_rows(*b)
    oa = torch.empty((len(wa), 4), dtype=torch.int32, device="cuda")
    ob = torch.empty((len(wb), 5), dtype=torch.int32, device="cuda")
    ra, rb = pinned_result(), pinned_result()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    zset.enumerate_async(*a, oa, ra, k=2, stream=s1)
    # Another stream: the call waits for the first one before reusing scratch.
    zset.enumerate_async(*b, ob, rb, k=2, stream=s2)
    # Synchronous calls in between wait for both as well.
    assert zset.count(*a) == len(wa)
    sync = zset.enumerate_ex(*b, k=1)
    assert_same(rows_of(sync.out, sync.rows, 5), wb, "synchronous call after queued ones")
    s1.synchronize()
    s2.synchronize()
    assert zset.async_outcome(ra) == (len(wa), 0)
    assert zset.async_outcome(rb) == (len(wb), 0)
    assert_same(rows_of(oa, len(wa), 4), wa, "stream 1")
    assert_same(rows_of(ob, len(wb), 5), wb, "stream 2")


def test_device_errors_are_reported_in_result():
    n, g = 3000, [7, 11, 13, 17]
    rows = oracle.count(n, g)
    out = torch.full((rows - 1, 4), 5, dtype=torch.int32, device="cuda")
    res = pinned_result()
    torch.cuda.synchronize()
    zset.enumerate_async(n, g, out, res, k=2)   # one row short: checked on the device
    ok = pinned_result()
    out2 = torch.empty((rows, 4), dtype=torch.int32, device="cuda")
    zset.enumerate_async(n, g, out2, ok, k=2)   # the next call is unaffected
    torch.cuda.synchronize()
    st, got_rows, _ = res.tolist()
    assert st == zset.ECAPACITY and got_rows == rows
    assert bool((out == 5).all()), "a call that reported ECAPACITY wrote rows"
    with pytest.raises(zset.ZsetError):
        zset.async_outcome(res)
    assert zset.async_outcome(ok) == (rows, 0)
    assert_same(rows_of(out2, rows, 4), oracle.enumerate_rows(n, g), "call after an error")
    # The in-call form reports the same way (and returns the status too).
    res3 = pinned_result()
    small = torch.empty((3, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(zset.ZsetError):
        zset.enumerate_async(900, [4, 7, 9], small, res3, k=0)
    assert res3[0].item() == zset.ECAPACITY


def test_argument_checks_need_pinned_result():
    out = torch.empty((100, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        zset.enumerate_async(20, [3, 5, 7], out, torch.zeros(3, dtype=torch.int64))
    lib = zset.load()
    g = np.array([3, 5, 7], dtype=np.uint32)
    plain = np.zeros(3, dtype=np.uint64)   # pageable host memory
    st = lib.zset_enumerate_async(20, g.ctypes.data_as(zset._u32p), 3, out.data_ptr(), 100, None,
                                  plain.ctypes.data, None)
    assert st == zset.EINVAL and "pinned" in zset.last_error()
    dev = torch.zeros(3, dtype=torch.int64, device="cuda")
    st = lib.zset_enumerate_async(20, g.ctypes.data_as(zset._u32p), 3, out.data_ptr(), 100, None,
                                  dev.data_ptr(), None)
    assert st == zset.EINVAL


def test_write_events_time_the_write_pass():
    n, g = 10130, [13, 34, 37, 54, 65, 83]
    rows = zset.count(n, g)
    out = torch.empty((rows, 6), dtype=torch.int32, device="cuda")
    res = pinned_result()
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    zset.enumerate_async(n, g, out, res, k=2, write_events=ev)
    torch.cuda.synchronize()
    assert zset.async_outcome(res) == (rows, 0)
    ms = ev[0].elapsed_time(ev[1])
    assert 0.1 < ms < 100.0, ms
    # Sampled rows against the oracle's unranking.
    rng = np.random.default_rng(11)
    idx = np.concatenate([[0, rows - 1], rng.integers(0, rows, 200)])
    host = out[torch.as_tensor(idx, device="cuda")].cpu().numpy().view(np.uint32)
    table = oracle.count_table(n, g)
    for j, r in enumerate(idx.tolist()):
        assert host[j].tolist() == oracle.unrank(n, g, r, table).tolist(), r
