"""The request loop (zset_server_*, through the C ABI): every query served in
a mix of concurrent queries gives exactly the bytes zset_enumerate_ex writes
for it alone, and the oracle's rows on a sample.  Integer work: bit-exact."""
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


# (generators, n_max, requested k): memo dimensions auto, 0, 1, 2 and d = 1, 2.
SETS = [([7, 11, 13, 17], 3000, -1), ([13, 34, 37, 54, 65, 83], 1500, -1),
        ([5, 9], 5000, -1), ([11], 400, -1), ([6, 10, 15], 900, 0),
        ([9, 4, 6, 7], 700, 1), ([3, 5, 7, 11, 13], 300, 2), ([12, 18, 30], 500, -1)]


def alone(n, g, k):
    r = zset.enumerate_ex(n, g, k=k)
    if r.rows == 0:
        return np.zeros((0, len(g)), np.uint32)
    return r.out[: r.rows].cpu().numpy().view(np.uint32).reshape(r.rows, len(g))


@pytest.mark.parametrize("slots,dispatchers", [(8, 2), (5, 3), (4, 1)])
def test_served_mix_matches_each_query_alone(slots, dispatchers):
    rng = np.random.default_rng(77 + slots)
    arena = torch.empty(6_000_000, dtype=torch.int32, device="cuda")  # 24 MB: admission waits
    srv = zset.Server(arena, slots=slots, dispatchers=dispatchers)
    ids = []
    for g, n_max, k in SETS:
        sid = srv.add_set(g, n_max, k)
        info = srv.set_info(sid)
        say(f"set {sid}: g={g} n_max={n_max} k={info['k']} memo_rows={info['memo_rows']}")
        if k >= 0:
            assert info["k"] == k
        ids.append(sid)
    queries = []
    for _ in range(400):
        s = int(rng.integers(0, len(SETS)))
        n = int(rng.integers(0, SETS[s][1] + 1))
        queries.append((s, n))
    queries += [(0, 0), (0, 3000), (3, 0), (3, 11), (3, 12), (4, 1), (2, 5000)]
    say(f"submitting {len(queries)} queries at once")
    tickets = [srv.submit(ids[s], n) for s, n in queries]
    checked = 0
    for (s, n), t in zip(queries, tickets):
        res = srv.wait(t)
        g, _, _ = SETS[s]
        k = srv.set_info(ids[s])["k"]
        assert res["rows"] == srv.count(ids[s], n) == oracle.count(n, g)
        got = srv.rows_of(ids[s], res).cpu().numpy().view(np.uint32) if res["rows"] else \
            np.zeros((0, len(g)), np.uint32)
        want = alone(n, g, k)
        assert got.shape == want.shape and np.array_equal(got, want), (s, n, k)
        if checked < 60:
            assert np.array_equal(got, oracle.enumerate_rows(n, g)), (s, n)
            checked += 1
        assert res["submit_us"] <= res["admit_us"] <= res["done_us"]
        srv.release(t)
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == len(queries)
    assert st["max_inflight"] > 1  # queries overlapped on the device
    srv.free()


def test_served_slice_plans_alone_and_shared():
    """Queries from one row to millions of rows, each served alone (the whole
    device) and then all at once (a share of it): small ones plan their own
    slices inside the write pass, large ones run the slice planner and claim
    slices; every result equals zset_enumerate_ex's bytes."""
    arena = torch.empty(160_000_000, dtype=torch.int32, device="cuda")  # 640 MB
    srv = zset.Server(arena, slots=8)
    g = [13, 34, 37, 54, 65, 83]
    sid = srv.add_set(g, 5600, -1)
    k = srv.set_info(sid)["k"]
    ns = [0, 13, 200, 700, 1500, 2400, 3300, 4200, 5000, 5600, 4700, 3900, 2900, 1800, 900]
    rows = [srv.count(sid, n) for n in ns]
    say(f"k={k} rows {rows}")
    assert max(rows) > 4_000_000 and min(rows) <= 1
    want = {n: zset.enumerate_ex(n, g, k=k).out for n in ns}
    def check(mode, n, t):
        res = srv.wait(t)
        assert res["rows"] == srv.count(sid, n)
        if res["rows"]:
            got = srv.rows_of(sid, res)
            assert torch.equal(got, want[n][: res["rows"]]), (mode, n)
        srv.release(t)  # in arrival order: the arena (smaller than the sum) frees up

    for n in ns:
        check("alone", n, srv.submit(sid, n))
    say("alone: every query equal")
    for n, t in [(n, srv.submit(sid, n)) for n in ns]:
        check("shared", n, t)
    say("shared: every query equal")
    srv.free()


def test_served_capped_memos():
    """Resident memos capped by bytes (a partial memo, Alg 3.2's Else branch):
    queries below and above the memo's top, served in a mix, give the rows
    zset_enumerate_ex writes alone with the same capped memo, and the oracle's."""
    arena = torch.empty(8_000_000, dtype=torch.int32, device="cuda")
    srv = zset.Server(arena, slots=6, memo_bytes=4096)
    sets = [([7, 11, 13, 17], 3000, 2), ([13, 34, 37, 54, 65, 83], 1500, 3),
            ([3, 5, 7, 11, 13], 300, 3), ([9, 4, 6, 7], 700, 1), ([12, 18, 30], 500, -1)]
    ids, tops = [], []
    for g, n_max, k in sets:
        sid = srv.add_set(g, n_max, k)
        info = srv.set_info(sid)
        say(f"capped set {sid}: g={g} n_max={n_max} {info}")
        h = g[len(g) - info["k"]:]
        assert 1 <= info["memo_top"] <= n_max + 1
        assert info["memo_rows"] == sum(oracle.count(p, h) for p in range(info["memo_top"]))
        if info["memo_top"] <= n_max:  # capped: the next element's memo would not fit
            assert info["memo_rows"] * 4 <= 4096 * (info["k"] + 1)
        ids.append(sid)
        tops.append(info["memo_top"])
    assert min(t - 1 - s[1] for t, s in zip(tops, sets)) < 0  # at least one memo is capped
    rng = np.random.default_rng(91)
    queries = []
    for i, (g, n_max, k) in enumerate(sets):
        for n in {0, 1, tops[i] - 1, tops[i], min(n_max, tops[i] + 1), n_max}:
            if 0 <= n <= n_max:
                queries.append((i, n))
        queries += [(i, int(rng.integers(0, n_max + 1))) for _ in range(12)]
    rng.shuffle(queries)
    tickets = [srv.submit(ids[i], n) for i, n in queries]
    for (i, n), t in zip(queries, tickets):
        res = srv.wait(t)
        g = sets[i][0]
        info = srv.set_info(ids[i])
        want = oracle.enumerate_rows(n, g)
        assert res["rows"] == len(want)
        got = srv.rows_of(ids[i], res).cpu().numpy().view(np.uint32) if res["rows"] else \
            np.zeros((0, len(g)), np.uint32)
        assert np.array_equal(got, want), (i, n, info)
        if res["rows"]:
            alone_rows = zset.enumerate_ex(n, g, k=info["k"], memo_top=info["memo_top"])
            assert torch.equal(srv.rows_of(ids[i], res), alone_rows.out[: res["rows"]]), (i, n)
        srv.release(t)
    srv.free()


def test_server_errors():
    arena = torch.empty(1 << 16, dtype=torch.int32, device="cuda")
    srv = zset.Server(arena, slots=2)
    sid = srv.add_set([7, 11, 13, 17], 2000)
    with pytest.raises(zset.ZsetError) as e:
        srv.submit(sid, 2001)  # beyond n_max
    assert e.value.status == zset.EINVAL
    with pytest.raises(zset.ZsetError) as e:
        srv.submit(sid + 1, 10)  # no such set
    assert e.value.status == zset.EINVAL
    with pytest.raises(zset.ZsetError) as e:
        srv.submit(sid, 2000)  # 81205 rows x 4 words exceed the 65536-word arena
    assert e.value.status == zset.ECAPACITY
    with pytest.raises(zset.ZsetError) as e:
        srv.wait(12345)
    assert e.value.status == zset.EINVAL
    t = srv.submit(sid, 500)
    srv.wait(t)
    srv.release(t)
    with pytest.raises(zset.ZsetError) as e:
        srv.release(t)
    assert e.value.status == zset.EINVAL
    with pytest.raises(zset.ZsetError) as e:
        srv.add_set([3, 0], 10)
    assert e.value.status == zset.EINVAL
    # Queued queries that can never be admitted end with EINVAL when the server stops.
    t1 = srv.submit(sid, 900)
    srv.wait(t1)  # holds its rows: the next queries wait for room
    pending = [srv.submit(sid, 1000) for _ in range(3)]
    srv.release(t1)
    for t in pending:
        srv.wait(t)
        srv.release(t)
    srv.free()
