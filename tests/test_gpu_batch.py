"""Parity of the batched path (zset_batch_*, through the C ABI) with the CPU
oracle and with the single-query path.

Integer work: every comparison is bit-exact.  A batch must give every query
exactly the bytes the query gives alone (zset_enumerate_ex) and the oracle's
rows; the full 4096-query workload is checked by properties that pin the
whole set at any size (row count equal to |Z(n)|, every row in Z(n), rows
strictly increasing) plus sampled queries compared row for row.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2407_20474_amd import inputs
from paper_2407_20474_amd import zset

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="batched path switched off: its first GPU run stopped responding "
                            "and the cause is not identified; zset_batch_create returns "
                            "ZSET_EDEVICE"),
]

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_same(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.nonzero((got != want).any(axis=1))[0]
        i = int(bad[0])
        raise AssertionError(f"{what}: {len(bad)} rows differ, first at {i}: "
                             f"got {got[i].tolist()} want {want[i].tolist()}")


def small_queries(seed, count, max_rows=100_000, **kw):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n, g = inputs.random_small_query(rng, **kw)
        if oracle.count(n, g) <= max_rows:
            out.append((n, g))
    return out


EDGE = [(0, [5]), (10, [5]), (11, [5]), (0, [3, 4, 5]), (1, [3, 4, 5]), (5, [2, 4]),
        (7, [2, 4]), (400, [3, 5, 7, 11, 13, 17]), (1000, [1000, 999]), (999, [1000, 1]),
        (37, [37, 37, 37]), (1, [1] * 12), (60, [1] * 4), (123, [7])]


def host_rows(b, out, q):
    r, d = int(b.rows[q]), int(b.d[q])
    if r == 0:
        return np.zeros((0, d), np.uint32)
    return b.rows_of(out, q).cpu().numpy().view(np.uint32).reshape(r, d)


def check_against_oracle(b, out, queries, what):
    for q, (n, g) in enumerate(queries):
        want = oracle.enumerate_rows(n, g)
        assert int(b.rows[q]) == len(want), (what, q, n, g)
        assert_same(host_rows(b, out, q), want, f"{what} query {q} n={n} g={g} k={b.k[q]}")


def test_batch_small_queries_auto_k():
    queries = EDGE + small_queries(101, 250)
    say(f"batch of {len(queries)} small queries, automatic k")
    b = zset.Batch(queries, rows_per_tile=[128] * len(queries))
    r = b.run()
    check_against_oracle(b, r.out, queries, "auto-k")
    assert (b.offsets % 4 == 0).all()
    b.free()


def test_batch_small_queries_every_k():
    rng = np.random.default_rng(202)
    queries = EDGE + small_queries(203, 200)
    ks = [int(rng.integers(0, len(g))) for _, g in queries]
    say(f"batch of {len(queries)} small queries, forced k")
    b = zset.Batch(queries, k=ks, rows_per_tile=[128] * len(queries))
    assert [int(x) for x in b.k] == [k if len(g) > 1 and oracle.count(n, g) > 0 else 0
                                     for k, (n, g) in zip(ks, queries)]
    r = b.run()
    check_against_oracle(b, r.out, queries, "forced-k")
    b.free()


def test_batch_count_only_checksums():
    queries = EDGE + small_queries(303, 150)
    say(f"count-only batch of {len(queries)} queries")
    b = zset.Batch(queries, count_only=True, rows_per_tile=[128] * len(queries))
    r = b.run()
    for q, (n, g) in enumerate(queries):
        want = oracle.enumerate_rows(n, g)
        assert int(b.rows[q]) == len(want)
        assert int(r.checksums[q]) == oracle.checksum(want), (q, n, g)
    b.free()


def test_batch_graph_replays_and_eager_agree():
    queries = small_queries(404, 120, max_rows=50_000)
    say("graph replays vs eager run")
    b = zset.Batch(queries, use_graph=True)
    out = b.alloc()
    b.run(out)
    first = out.clone()
    for i in range(3):
        out.fill_(-1 if i % 2 else 7)
        torch.cuda.synchronize()
        junk = torch.arange(1 << 20, device="cuda").sum()  # eager work between replays
        b.run(out)
        torch.cuda.synchronize()
        assert int(junk) >= 0
        for q in range(len(queries)):
            assert torch.equal(b.rows_of(out, q), b.rows_of(first, q)), (i, q)
    # A different output buffer: the graph is captured again.
    out2 = b.alloc()
    b.run(out2)
    for q in range(len(queries)):
        assert torch.equal(b.rows_of(out2, q), b.rows_of(first, q))
    e = zset.Batch(queries, use_graph=False)
    r = e.run()
    assert r.stats["write_us"] > 0
    for q in range(len(queries)):
        assert torch.equal(e.rows_of(r.out, q), b.rows_of(first, q))
    check_against_oracle(b, first, queries, "graph")
    b.free()
    e.free()


def test_batch_matches_single_query_path():
    """Each query's bytes in the batch equal its bytes when enumerated alone."""
    allq = inputs.load_batch_queries()
    rng = np.random.default_rng(505)
    pick = sorted(set(rng.choice(len(allq), size=60, replace=False).tolist()))
    queries = [(allq[i][0], allq[i][1]) for i in pick]
    say(f"batch vs single path on {len(queries)} queries of the batched workload")
    b = zset.Batch(queries)
    r = b.run()
    for q, (n, g) in enumerate(queries):
        alone = zset.enumerate_ex(n, g, k=int(b.k[q]))
        assert alone.rows == int(b.rows[q]) == allq[pick[q]][2]
        if alone.rows:
            assert torch.equal(b.rows_of(r.out, q), alone.out.reshape(-1, len(g))[: alone.rows]), q
    b.free()


def test_batch_errors():
    queries = [(100, [3, 5, 7]), (50, [2, 9])]
    with pytest.raises(zset.ZsetError) as e:
        zset.Batch(queries, k=[3, 0])  # k > d - 1
    assert e.value.status == zset.EINVAL
    with pytest.raises(zset.ZsetError) as e:
        zset.Batch([(100, [3, 0, 7])])
    assert e.value.status == zset.EINVAL
    with pytest.raises(zset.ZsetError) as e:
        zset.Batch(queries, rows_per_tile=[100, 0])
    assert e.value.status == zset.EINVAL
    b = zset.Batch(queries)
    small = torch.empty(max(b.total_words - 4, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(zset.ZsetError) as e:
        b.run(small)
    assert e.value.status == zset.ECAPACITY
    big = torch.empty(b.total_words + 8, dtype=torch.int32, device="cuda")
    with pytest.raises(zset.ZsetError) as e:
        b.run(big[1:])  # 4-byte aligned only
    assert e.value.status == zset.EINVAL
    with pytest.raises(zset.ZsetError) as e:
        b.run(torch.empty(b.total_words, dtype=torch.int32))  # host memory
    assert e.value.status == zset.EINVAL
    b.free()


def rows_are_zset(rows_i32, n, g):
    """On the GPU: every row has sum a_i g_i = n and the rows strictly increase."""
    a = rows_i32.to(torch.int64)
    gv = torch.tensor(g, dtype=torch.int64, device=a.device)
    if not bool(((a * gv).sum(dim=1) == n).all()):
        return False
    if a.shape[0] < 2:
        return True
    diff = a[1:] - a[:-1]
    nz = diff != 0
    if not bool(nz.any(dim=1).all()):
        return False
    first = nz.to(torch.int8).argmax(dim=1, keepdim=True)
    return bool((diff.gather(1, first) > 0).all())


def test_batched_workload_full_size():
    """The 4096-query batched workload in the configuration the benchmark runs."""
    allq = inputs.load_batch_queries()
    queries = [(n, g) for n, g, _ in allq]
    say(f"full batched workload: {len(queries)} queries, planning")
    b = zset.Batch(queries)
    say(f"  total words {b.total_words} ({b.total_words * 4 / 1e9:.1f} GB), running")
    r = b.run()
    assert [int(x) for x in b.rows] == [rows for _, _, rows in allq]
    say("  invariants per query")
    for q, (n, g) in enumerate(queries):
        if int(b.rows[q]):
            assert rows_are_zset(b.rows_of(r.out, q), n, g), (q, n, g, int(b.k[q]))
    rng = np.random.default_rng(606)
    largest = np.argsort([rows for _, _, rows in allq])[-6:].tolist()
    sample = sorted(set(largest + rng.choice(len(queries), size=40, replace=False).tolist()))
    say(f"  {len(sample)} sampled queries against the oracle")
    for q in sample:
        n, g = queries[q]
        want = oracle.enumerate_rows(n, g)
        assert_same(host_rows(b, r.out, q), want, f"batch query {q} n={n} g={g} k={b.k[q]}")
    t = b.times()
    assert (t[b.rows > 0] > 0).all()
    del r
    b.free()
    torch.cuda.empty_cache()
