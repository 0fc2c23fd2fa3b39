"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work: every comparison is bit-exact.  Small cases span several slices
and a ragged last slice (rows_per_tile = 128); the full-size case is the
large single enumeration in the launch configuration the benchmark times.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2407_20474_amd import inputs
from paper_2407_20474_amd import zset

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bounded_queries(seed, count, max_rows=300_000, **kw):
    """Random small queries whose |Z(n)| (from the oracle) stays below max_rows."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n, g = inputs.random_small_query(rng, **kw)
        if oracle.count(n, g) <= max_rows:
            out.append((n, g))
    return out


def gpu_rows(n, g, **kw):
    say(f"  enumerate_ex n={n} g={list(g)} {kw}")
    r = zset.enumerate_ex(n, g, **kw)
    if r.rows == 0:
        return np.zeros((0, len(g)), np.uint32), r
    host = r.out[: r.rows].cpu().numpy().view(np.uint32).reshape(r.rows, len(g))
    return host, r


def assert_same(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.nonzero((got != want).any(axis=1))[0]
        i = int(bad[0])
        raise AssertionError(f"{what}: {len(bad)} rows differ, first at {i}: "
                             f"got {got[i].tolist()} want {want[i].tolist()}")


# --------------------------------------------------------------------------
# Counting pass
# --------------------------------------------------------------------------

def test_count_table_matches_oracle(monkeypatch):
    rng = np.random.default_rng(11)
    cases = [(2000, [7, 11, 13, 17]), (10130, [13, 34, 37, 54, 65, 83]), (0, [5]),
             # the last two rows in closed form: gcd > 1, g > n, beyond LDS, and
             # h_2 / gcd >= 2^16 (scanned from row d instead)
             (9000, [6, 4]), (5, [7, 9]), (100000, [11, 2, 70000]), (200000, [3, 70001]),
             (16383, [1, 65537, 65536]),
             (3000, [1, 1, 2]), (500, [600, 7, 3]), (16383, [5, 9, 4]), (16384, [5, 9, 4]),
             (20000, [3, 5, 7]), (77847, [14, 99, 135, 161, 163]),
             # residue classes walked by one thread (<= 32 entries), one run per
             # lane, several passes, LDS bank strides of 32 and 64, saturation
             (5000, [300, 170, 41]), (16383, [2000, 513, 511, 9]), (16000, [32, 64, 1, 3]),
             (300, [1] * 20 + [3]), (12000, [1, 1, 1, 1, 1, 1, 1])]
    for _ in range(20):
        cases.append(inputs.random_small_query(rng, nmax=3000))
    for n, g in cases:
        say(f"count_table n={n} g={g}")
        t = zset.count_table(n, g).cpu().numpy().view(np.uint64)
        want = oracle.count_table(n, g)
        assert np.array_equal(t, want), (n, g)
        if int(want[0, n]) == (1 << 64) - 1:  # saturated: |Z(n)| >= 2^64 - 1
            with pytest.raises(zset.ZsetError) as e:
                zset.count(n, g)
            assert e.value.status == zset.EOVERFLOW
        else:
            assert zset.count(n, g) == int(want[0, n])
    # Every row scanned from row d (no closed-form rows), LDS and row forms.
    monkeypatch.setenv("ZSET_COUNT_LAST", "0")
    for n, g in cases[:12]:
        say(f"count_table scanned n={n} g={g}")
        t = zset.count_table(n, g).cpu().numpy().view(np.uint64)
        assert np.array_equal(t, oracle.count_table(n, g)), (n, g)


def test_count_overflow_is_reported():
    say("count overflow: 32 generators equal to 1, n = 100000")
    with pytest.raises(zset.ZsetError) as e:
        zset.count(100000, [1] * 32)
    assert e.value.status == zset.EOVERFLOW


# --------------------------------------------------------------------------
# Enumeration: small and medium cases, every memo dimension
# --------------------------------------------------------------------------

def test_plain_config_every_k_and_slice_size():
    w = inputs.load_workloads()["plain"]
    n, g = w["n"], w["gens"]
    want = oracle.enumerate_rows(n, g)
    assert len(want) == 81205
    for k in range(len(g)):
        for rpt in (128, 256, 1280, 0):
            got, r = gpu_rows(n, g, k=k, rows_per_tile=rpt)
            assert r.stats["k"] == k
            assert_same(got, want, f"plain k={k} rows_per_tile={rpt}")


def test_plain_entry_point():
    say("zset_enumerate (plain entry point) on (7, 11, 13, 17), n = 2000")
    out = zset.enumerate(2000, [7, 11, 13, 17])
    got = out.cpu().numpy().view(np.uint32)
    assert_same(got, oracle.enumerate_rows(2000, [7, 11, 13, 17]), "zset_enumerate")


def test_random_small_queries_every_k():
    for n, g in bounded_queries(12, 60, dmax=6, gmax=30, nmax=800):
        want = oracle.enumerate_rows(n, g)
        for k in range(len(g)):
            got, _ = gpu_rows(n, g, k=k, rows_per_tile=128)
            assert_same(got, want, f"n={n} g={g} k={k}")


@pytest.mark.parametrize("n,g", [
    (0, [5]), (0, [3, 7, 9]), (35, [5]), (36, [5]),        # n = 0 and d = 1
    (101, [4, 6, 10]),                                       # gcd does not divide n: empty
    (7 * 11 - 7 - 11, [7, 11]),                              # Frobenius number: empty
    (5000, [7, 11]), (40, [50, 60, 3]),                      # d = 2; generators above n
    (60, [1, 1, 1, 1]), (200, [2, 2, 3, 3, 5]),             # repeated generators
    (1000, [17, 5, 11, 3]),                                  # unsorted
    (400, [3, 5, 7, 11, 13, 17]),                            # k = d - 1: one segment
])
def test_edge_cases(n, g):
    want = oracle.enumerate_rows(n, g)
    for k in range(len(g)):
        got, r = gpu_rows(n, g, k=k, rows_per_tile=128)
        assert r.rows == len(want)
        assert_same(got, want, f"edge n={n} g={g} k={k}")


def test_medium_cases_default_slices():
    for n, g in [(5000, [13, 37, 38, 40]), (1000, [13, 37, 38, 40, 41, 42, 43]),
                 (700, [10, 12, 14, 16, 19]), (20000, [3, 5, 7])]:
        want = oracle.enumerate_rows(n, g)
        for k in range(len(g)):
            got, _ = gpu_rows(n, g, k=k)
            assert_same(got, want, f"medium n={n} g={g} k={k}")


@pytest.mark.parametrize("pair", ["0", "1"])
def test_pair_lanes_forced_on_and_off(pair, monkeypatch):
    # The write pass's lanes over (a_{U-2}, a_{U-1}) pairs (U >= 2) or over
    # a_{U-1} alone give the same bytes; the automatic choice takes pairs
    # only when a_{U-1} never fills a wavefront, so both forms are forced here
    # on small, medium, unsorted and repeated-generator cases, every k, short
    # and default slices, and count-only.
    monkeypatch.setenv("ZSET_PAIR", pair)
    cases = list(bounded_queries(31, 25, dmax=7, gmax=40, nmax=900))
    cases += [(7824 // 4, [31, 63, 87, 123, 132, 136, 157, 170, 187]),
              (1000, [13, 37, 38, 40, 41, 42, 43]), (5000, [13, 37, 38, 40]),
              (60, [1, 1, 1, 1, 1]), (3000, [170, 61, 44, 97, 5])]
    for n, g in cases:
        want = oracle.enumerate_rows(n, g)
        for k in range(1, len(g)):
            for T in (128, 0):
                got, r = gpu_rows(n, g, k=k, rows_per_tile=T)
                assert_same(got, want, f"pair={pair} n={n} g={g} k={k} T={T}")
            got, r = gpu_rows(n, g, k=k, order=1)
            assert_same(got, np.ascontiguousarray(want[::-1]), f"pair={pair} desc n={n} k={k}")
            c = zset.enumerate_ex(n, g, k=k, count_only=True)
            assert c.rows == len(want) and c.checksum == oracle.checksum(want), (pair, n, g, k)


def test_partial_memo_every_k(monkeypatch):
    # A memo covering only p < top <= n (Alg 3.2's Else branch): rows whose
    # memo remainder is >= top are unranked from the count table by the write
    # pass, the rest copied from the memo.  top = 1, n / 3 and n at every k,
    # short and default slices, ascending and descending, count-only, and
    # pair lanes forced on and off.
    cases = [(2000, [7, 11, 13, 17]), (1000, [13, 37, 38, 40, 41, 42, 43]), (400, [3, 5, 7, 11]),
             (60, [1, 1, 1, 1]), (700, [10, 12, 14, 16, 19])]
    cases += list(bounded_queries(51, 12, dmax=6, gmax=30, nmax=800))
    for pair in ("0", "1"):
        monkeypatch.setenv("ZSET_PAIR", pair)
        for n, g in cases:
            want = oracle.enumerate_rows(n, g)
            for k in range(1, len(g)):
                for top in sorted({1, max(1, n // 3), n}):
                    for T in (128, 0):
                        got, r = gpu_rows(n, g, k=k, rows_per_tile=T, memo_top=top)
                        assert_same(got, want, f"partial pair={pair} n={n} g={g} k={k} top={top} T={T}")
                    got, r = gpu_rows(n, g, k=k, order=1, memo_top=top)
                    assert_same(got, np.ascontiguousarray(want[::-1]), f"partial desc n={n} k={k} top={top}")
                    c = zset.enumerate_ex(n, g, k=k, count_only=True, memo_top=top)
                    assert c.rows == len(want) and c.checksum == oracle.checksum(want), (n, g, k, top)


def test_partial_memo_handle():
    # A memo handle whose top is <= n is accepted and treated as partial.
    n, g = 3000, [13, 37, 38, 40, 41]
    want = oracle.enumerate_rows(n, g)
    for k in (1, 2, 3):
        for top in (1, n // 2, n, n + 1):
            m = zset.Memo(g[len(g) - k:], top)
            got, r = gpu_rows(n, g, memo=m, rows_per_tile=256)
            assert_same(got, want, f"partial handle k={k} top={top}")
            m.free()


def test_partial_memo_full_size():
    # The large workload with its k = 2 memo capped at n / 2.
    w = inputs.load_workloads()["large"][0]
    n, g, k, rows = w["n"], w["gens"], w["k"], w["rows"]
    table = oracle.count_table(n, g)
    want = np.empty((rows, len(g)), dtype=np.uint32)
    _, got_rows = oracle.enumerate_rows_threads(n, g, 0, n // g[0] + 1, min(16, os.cpu_count() or 1),
                                                table=table, out=want)
    want_dev = torch.from_numpy(want.view(np.int32)).to("cuda")
    out = torch.full((rows, len(g)), -1, dtype=torch.int32, device="cuda")
    r = zset.enumerate_ex(n, g, out=out, k=k, memo_top=n // 2)
    assert r.rows == rows
    assert torch.equal(out, want_dev), "large partial memo"
    del out, want_dev
    torch.cuda.empty_cache()


def wide_queries(seed, count, max_rows=200_000):
    """Queries with d in [17, 32]: rows wider than 16 words use the 64-row
    staging ring, which stages each 64-row chunk in two halves."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        d = int(rng.integers(17, 33))
        g = [int(x) for x in rng.integers(5, 70, size=d)]
        n = int(rng.integers(40, 160))
        c = oracle.count(n, g)
        if 300 <= c <= max_rows:
            out.append((n, g))
    return out


def test_wide_rows_every_k():
    rng = np.random.default_rng(17)
    for n, g in wide_queries(1700, 8):
        want = oracle.enumerate_rows(n, g)
        d = len(g)
        for k in sorted({0, 1, 2, int(rng.integers(3, d))}):
            for T in (128, 0):
                got, r = gpu_rows(n, g, k=k, rows_per_tile=T)
                assert_same(got, want, f"wide n={n} d={d} k={k} T={T}")
            c = zset.enumerate_ex(n, g, k=k, count_only=True)
            assert c.rows == len(want) and c.checksum == oracle.checksum(want)


def test_claimed_slices_every_share():
    """Slices claimed at run time (any share, any chunking) give the dealt rows.
    3.6e6 rows over 28452 slices of 128 rows: far more than 16 slices per
    resident workgroup, so claiming is in use; the last slice is ragged."""
    n, g = 400, [2, 3, 5, 7, 11, 13]
    want = oracle.enumerate_rows(n, g)
    want_sum = oracle.checksum(want)
    cases = [(2, 128, p) for p in (0, 1, 25, 60, 100)] + [(0, 128, 100), (1, 384, 25),
                                                          (3, 128, 100), (2, 1152, 50)]
    for k, rpt, pct in cases:
        got, r = gpu_rows(n, g, k=k, rows_per_tile=rpt, claim_pct=pct)
        assert_same(got, want, f"claimed k={k} rows_per_tile={rpt} claim_pct={pct}")
        c = zset.enumerate_ex(n, g, k=k, rows_per_tile=rpt, claim_pct=pct, count_only=True)
        assert c.rows == len(want) and c.checksum == want_sum, (k, rpt, pct)


def test_write_pass_at_the_device_lds_limit():
    """Queries whose write pass, as first sized, asked for exactly the device's
    160 KiB of dynamic LDS (which the kernel's static shared variables do not
    leave): the sizing keeps a reserve for them, and the rows match."""
    for n, g, k in [(33722, [34, 65, 137], 2), (5937, [99, 101, 104, 141], 3),
                    (1688, [51, 64, 70, 88, 89, 90, 116, 118], 5)]:
        want = oracle.enumerate_rows(n, g)
        for kk in (-1, k):
            got, r = gpu_rows(n, g, k=kk)
            assert_same(got, want, f"lds limit n={n} g={g} k={kk}")


def test_descending_order_is_the_reversal():
    # The write pass stores rank r at row |Z| - 1 - r (each staged block
    # written in reverse): every k, short and default slices, pair lanes on
    # and off, d = 1 and empty sets.
    cases = [(2000, [7, 11, 13, 17]), (1000, [13, 37, 38, 40, 41, 42, 43]), (123, [41]),
             (101, [4, 6, 10]), (0, [3, 7, 9])]
    cases += list(bounded_queries(41, 10, dmax=6, gmax=30, nmax=800))
    for n, g in cases:
        want = np.ascontiguousarray(oracle.enumerate_rows(n, g)[::-1])
        for k in range(len(g)):
            for T in (128, 0):
                got, r = gpu_rows(n, g, k=k, order=1, rows_per_tile=T)
                assert_same(got, want, f"descending n={n} g={g} k={k} T={T}")


def test_count_only_checksum():
    cases = [(2000, [7, 11, 13, 17]), (5000, [13, 37, 38, 40]), (0, [4, 6]), (35, [5])]
    cases += bounded_queries(13, 10, dmax=5, gmax=20, nmax=200)
    for n, g in cases:
        rows = oracle.enumerate_rows(n, g)
        want = oracle.checksum(rows)
        for k in range(len(g)):
            for rpt in (128, 0):
                say(f"count_only n={n} g={g} k={k} rows_per_tile={rpt}")
                r = zset.enumerate_ex(n, g, k=k, rows_per_tile=rpt, count_only=True)
                assert r.rows == len(rows)
                assert r.checksum == want, (n, g, k, rpt)


# --------------------------------------------------------------------------
# Memo build (the dynamic recurrence) and memo handles
# --------------------------------------------------------------------------

@pytest.mark.parametrize("path", ["lds", "global", "window"])
def test_memo_build_matches_oracle(path, monkeypatch):
    monkeypatch.setenv("ZSET_MEMO_PATH", path)
    for h, top in [([3, 5], 200), ([72, 75], 3000), ([4, 6, 9], 300), ([7], 100),
                   ([2, 2], 50), ([9, 4, 6], 400), ([13, 37, 38], 2000), ([1], 10),
                   ([5, 3, 2, 7], 150)]:
        say(f"memo_build h={h} top={top} path={path}")
        m = zset.Memo(h, top)
        off, rows = m.read()
        want_off, want_rows = oracle.memo(h, top)
        assert np.array_equal(off, want_off), (h, top)
        assert np.array_equal(rows, want_rows), (h, top)
        m.free()


def test_windowed_memo_in_the_single_path(monkeypatch):
    """Memos built with a ring of recent lists in LDS, rows streamed to global
    memory, inside full enumerations (every k) against the oracle."""
    monkeypatch.setenv("ZSET_MEMO_PATH", "window")
    for n, g in [(2000, [7, 11, 13, 17]), (400, [2, 3, 5, 7, 11, 13]), (3000, [38, 40, 5, 9])]:
        want = oracle.enumerate_rows(n, g)
        for k in range(1, len(g)):
            got, r = gpu_rows(n, g, k=k, rows_per_tile=256)
            assert_same(got, want, f"window memo n={n} g={g} k={k}")


@pytest.mark.parametrize("path", ["default", "chain"])
def test_two_coordinate_memo_in_the_single_path(path, monkeypatch):
    """k = 2 memos of the single path: the closed form (default) and the
    recurrence (forced), inside full enumerations against the oracle; also
    generators with a common factor and a first generator larger than the
    second."""
    if path == "chain":
        monkeypatch.setenv("ZSET_MEMO_PATH", "chain")
    for n, g in [(2000, [7, 11, 13, 17]), (1500, [13, 34, 37, 54, 65, 83]),
                 (900, [5, 9, 6, 10]), (700, [3, 4, 12, 8]), (400, [2, 3, 1, 1]),
                 (3000, [38, 40, 45, 36]), (30000, [1000, 1500, 7, 11])]:
        # The last case's memo (5.8e6 rows) exceeds what the early build holds.
        want = oracle.enumerate_rows(n, g)
        got, r = gpu_rows(n, g, k=2, rows_per_tile=256)
        assert_same(got, want, f"k=2 memo ({path}) n={n} g={g}")


def test_memo_lists_of_the_table1_groups():
    """The FactorizationsUpToElement lists of the paper's Table 1 memo groups
    (generators the first d of 13, 37, 38, 40..45; memo of the trailing k up to
    the group's largest element), as zset_memo_build returns them, against the
    oracle's lists (one plain enumeration per element)."""
    gens = (13, 37, 38, 40, 41, 42, 43, 44, 45)
    for d, k, elem in [(3, 1, 300000), (4, 2, 15000), (5, 2, 10000), (5, 3, 5000),
                       (6, 3, 5000), (6, 4, 3000), (7, 4, 2000), (9, 5, 1500)]:
        h = list(gens[:d][d - k:])
        say(f"table 1 memo d={d} k={k} h={h} top={elem + 1}")
        m = zset.Memo(h, elem + 1)
        off, rows = m.read()
        m.free()
        want_off, want_rows = oracle.memo(h, elem + 1)
        assert np.array_equal(off, want_off), (d, k)
        assert np.array_equal(rows, want_rows), (d, k)


def test_memo_handle_gives_the_same_rows():
    n, g = 2000, [7, 11, 13, 17]
    want = oracle.enumerate_rows(n, g)
    for k in (1, 2, 3):
        for top in (n + 1, n + 500):
            say(f"memo handle k={k} top={top}")
            m = zset.Memo(g[len(g) - k:], top)
            got, r = gpu_rows(n, g, memo=m, rows_per_tile=256)
            assert r.stats["k"] == k and r.stats["memo_us"] == 0
            assert_same(got, want, f"memo handle k={k} top={top}")
            m.free()


# --------------------------------------------------------------------------
# Errors reported on the GPU side
# --------------------------------------------------------------------------

def test_errors():
    g = [7, 11, 13, 17]
    say("ECAPACITY: out holds one row too few")
    out = torch.empty((81204, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(zset.ZsetError) as e:
        zset.enumerate_ex(2000, g, out=out)
    assert e.value.status == zset.ECAPACITY
    say("EINVAL: memo generators differ from the trailing generators")
    m = zset.Memo([13, 16], 3000)
    with pytest.raises(zset.ZsetError) as e:
        zset.enumerate_ex(2000, g, memo=m)
    assert e.value.status == zset.EINVAL
    m.free()
    say("a memo whose top does not exceed n is a partial memo")
    m = zset.Memo([13, 17], 2000)
    got = zset.enumerate_ex(2000, g, memo=m)
    assert_same(got.out[:got.rows].cpu().numpy().view(np.uint32),
                oracle.enumerate_rows(2000, g), "partial memo handle")
    m.free()
    say("EINVAL: out is host memory")
    host = np.zeros(81205 * 4, dtype=np.int32)
    import ctypes
    lib = zset.load()
    gg = np.asarray(g, dtype=np.uint32)
    st = lib.zset_enumerate(2000, gg.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 4,
                            host.ctypes.data)
    assert st == zset.EINVAL
    assert not host.any()


def test_fixed_k_path_matches_the_readback_path(monkeypatch):
    """k = 1 or 2 fixed by the caller with automatic slices: every launch is
    enqueued at once and the device sizes the slices from |Z(n)|.  Its bytes,
    checksums and error statuses equal the path that reads |Z(n)| back first
    (ZSET_FIXED_K_READBACK=1), and the oracle's rows."""
    cases = [(2000, [7, 11, 13, 17]), (1000, [13, 37, 38, 40, 41, 42, 43]), (60, [1, 1, 1, 1]),
             (3, [5, 7, 9]), (700, [10, 12, 14, 16, 19]), (0, [4, 6]),
             (16383, [40, 50, 61, 77]), (3000, [6, 10, 14, 21]), (50, [3, 100, 5, 7]),
             (16384, [90, 97, 120, 131])]
    cases += list(bounded_queries(73, 6, dmax=6, gmax=30, nmax=800))
    for n, g in cases:
        want = oracle.enumerate_rows(n, g)
        for k in (1, 2):
            if k > len(g) - 1:
                continue
            for order in (0, 1):
                monkeypatch.delenv("ZSET_FIXED_K_READBACK", raising=False)
                # No stats structure: the call records no timing events.
                got, r = gpu_rows(n, g, k=k, order=order, stats=order == 1)
                ref = want if order == 0 else np.ascontiguousarray(want[::-1])
                assert_same(got, ref, f"fixed k={k} order={order} n={n} g={g}")
                # The same call with the setup launches split (count table,
                # class ends, memo, plan and leaf layout each on its own).
                monkeypatch.setenv("ZSET_FIXED_K_SPLIT", "1")
                got3, r3 = gpu_rows(n, g, k=k, order=order)
                monkeypatch.delenv("ZSET_FIXED_K_SPLIT")
                assert_same(got3, got, f"split setup k={k} order={order} n={n} g={g}")
                monkeypatch.setenv("ZSET_FIXED_K_READBACK", "1")
                got2, r2 = gpu_rows(n, g, k=k, order=order)
                assert_same(got2, got, f"readback path k={k} order={order} n={n} g={g}")
                assert r.rows == r2.rows == r3.rows == len(want)
            monkeypatch.delenv("ZSET_FIXED_K_READBACK", raising=False)
            for st in (True, False):
                c = zset.enumerate_ex(n, g, k=k, count_only=True, stats=st)
                assert c.rows == len(want) and c.checksum == oracle.checksum(want), (n, g, k)
    monkeypatch.delenv("ZSET_FIXED_K_READBACK", raising=False)
    g = [7, 11, 13, 17]
    for k in (1, 2):
        say(f"fixed k={k}: ECAPACITY with one row too few, nothing written")
        out = torch.full((81204, 4), -1, dtype=torch.int32, device="cuda")
        with pytest.raises(zset.ZsetError) as e:
            zset.enumerate_ex(2000, g, out=out, k=k)
        assert e.value.status == zset.ECAPACITY
        assert bool((out == -1).all())
        out = torch.empty((81205, 4), dtype=torch.int32, device="cuda")
        r = zset.enumerate_ex(2000, g, out=out, k=k)  # the same buffers, exactly enough rows
        assert_same(out.cpu().numpy().view(np.uint32), oracle.enumerate_rows(2000, g),
                    f"fixed k={k} after a refused call")
    say("fixed k=1: EOVERFLOW for 32 generators equal to 1, n = 100000")
    with pytest.raises(zset.ZsetError) as e:
        zset.enumerate_ex(100000, [1] * 32, k=1, count_only=True)
    assert e.value.status == zset.EOVERFLOW
    out = torch.full((16, 32), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(zset.ZsetError) as e:
        zset.enumerate_ex(100000, [1] * 32, out=out, k=1)
    assert e.value.status == zset.EOVERFLOW
    assert bool((out == -1).all())


def test_alloc_fault_is_reported(monkeypatch):
    say("ENOMEM: ZSET_FAULT=alloc on a memo build")
    monkeypatch.setenv("ZSET_FAULT", "alloc")
    with pytest.raises(zset.ZsetError) as e:
        zset.Memo([7, 9], 500)
    assert e.value.status == zset.ENOMEM


# --------------------------------------------------------------------------
# Full size: the large single enumeration, as the benchmark runs it
# --------------------------------------------------------------------------

def test_large_config_full_size_bit_exact():
    w = inputs.load_workloads()["large"][0]
    n, g, k = w["n"], w["gens"], w["k"]
    rows = w["rows"]
    say(f"large: n={n} g={g} k={k} rows={rows}: oracle (threads)")
    table = oracle.count_table(n, g)
    want = np.empty((rows, len(g)), dtype=np.uint32)
    nthreads = min(16, os.cpu_count() or 1)
    _, got_rows = oracle.enumerate_rows_threads(n, g, 0, n // g[0] + 1, nthreads,
                                                table=table, out=want)
    assert got_rows == rows
    say("large: GPU enumerate (default slices, k=2)")
    out = torch.empty((rows, len(g)), dtype=torch.int32, device="cuda")
    r = zset.enumerate_ex(n, g, out=out, k=k)
    assert r.rows == rows
    chunk = 20_000_000
    for s in range(0, rows, chunk):
        e = min(rows, s + chunk)
        got = out[s:e].cpu().numpy().view(np.uint32)
        assert_same(got, want[s:e], f"large rows [{s}, {e})")
    say("large: descending order, same launch configuration")
    want_dev = torch.from_numpy(want.view(np.int32)).to("cuda").flip(0)
    out.fill_(-1)
    r = zset.enumerate_ex(n, g, out=out, k=k, order=1)
    assert r.rows == rows
    assert torch.equal(out, want_dev), "large descending"
    del want_dev
    say("large: count-only checksum")
    want_sum = oracle.checksum(want)
    for pct in (-1, 0, 100):
        c = zset.enumerate_ex(n, g, k=k, count_only=True, claim_pct=pct)
        assert c.rows == rows
        assert c.checksum == want_sum, pct
    del out
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# Memo-dimension sweep at full size: d = 5, 7, 9, |Z| ~ 3.16e8, k = 0..3
# --------------------------------------------------------------------------

@pytest.mark.parametrize("idx", [0, 1, 2])
def test_sweep_config_full_size(idx):
    w = inputs.load_workloads()["sweep"][idx]
    n, g, rows = w["n"], w["gens"], w["rows"]
    d = len(g)
    say(f"sweep d={d}: n={n} g={g} rows={rows}: oracle (threads)")
    table = oracle.count_table(n, g)
    want = np.empty((rows, d), dtype=np.uint32)
    nthreads = min(16, os.cpu_count() or 1)
    _, got_rows = oracle.enumerate_rows_threads(n, g, 0, n // g[0] + 1, nthreads,
                                                table=table, out=want)
    assert got_rows == rows
    want_sum = oracle.checksum(want)
    # The oracle's rows go to the device once; every memo dimension is then
    # materialised at the size and launch configuration the sweep bench uses
    # and compared row for row there (the count-only pass is compared through
    # its checksum).
    want_dev = torch.from_numpy(want.view(np.int32)).to("cuda")
    out = torch.empty((rows, d), dtype=torch.int32, device="cuda")
    for k in w["ks"]:
        say(f"sweep d={d}: count-only k={k}")
        c = zset.enumerate_ex(n, g, k=k, count_only=True)
        assert c.rows == rows and c.checksum == want_sum, (d, k)
        say(f"sweep d={d}: materialise k={k}")
        out.fill_(-1)
        r = zset.enumerate_ex(n, g, out=out, k=k)
        assert r.rows == rows and r.stats["k"] == k
        if not torch.equal(out, want_dev):
            bad = torch.nonzero((out != want_dev).any(dim=1))[:, 0]
            i = int(bad[0])
            raise AssertionError(f"sweep d={d} k={k}: {bad.numel()} rows differ, first at {i}: "
                                 f"got {out[i].tolist()} want {want_dev[i].tolist()}")
    del out, want, want_dev
    torch.cuda.empty_cache()
