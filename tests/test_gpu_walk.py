"""The table-free walk (zset_enumerate_walk, through the C ABI): rows equal the
oracle's (ascending; reversed for descending order) and zset_enumerate_ex's,
also at elements near 2^31 where the count table would take gigabytes.
Integer work: bit-exact."""
import sys

import numpy as np
import pytest

import oracle
from paper_2407_20474_amd import inputs, zset

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def walk(n, g, order, rows):
    """The walk's rows, into a buffer of exactly max(rows, 1) rows."""
    out = torch.empty(max(rows, 1) * len(g), dtype=torch.int32, device="cuda")
    got = zset.enumerate_walk(n, g, out, order=order)
    return out[: got * len(g)].cpu().numpy().view(np.uint32).reshape(got, len(g))


@pytest.mark.parametrize("seed", range(12))
def test_walk_matches_oracle_small(seed):
    rng = np.random.default_rng(1000 + seed)
    while True:  # unsorted, possibly repeated generators; at most 300k rows
        n, g = inputs.random_small_query(rng)
        if oracle.count(n, g) <= 300_000:
            break
    want = oracle.enumerate_rows(n, g)
    say(f"seed {seed}: n={n} g={list(g)} rows={len(want)}")
    assert np.array_equal(walk(n, g, 0, len(want)), want)
    assert np.array_equal(walk(n, g, 1, len(want)), want[::-1])


@pytest.mark.parametrize("d", [2, 3, 9, 17, 32])
def test_walk_row_widths(d):
    """Rows of 2 to 32 words: each lane stages 16 rows (d = 2) down to one
    (d >= 17) per round, and the wavefront's writes cross lanes' row runs."""
    rng = np.random.default_rng(77 + d)
    cases = 0
    while cases < 3:
        g = [int(x) for x in rng.integers(2, 40 if d <= 9 else 90, size=d)]
        n = int(rng.integers(10, 400 if d <= 9 else 160))
        c = oracle.count(n, g)
        if c == 0 or c > 200_000:
            continue
        want = oracle.enumerate_rows(n, g)
        say(f"d={d}: n={n} g={g} rows={c}")
        assert np.array_equal(walk(n, g, 0, c), want)
        assert np.array_equal(walk(n, g, 1, c), want[::-1])
        cases += 1


def test_walk_matches_count_table_path():
    g = [13, 34, 37, 54, 65, 83]
    for n in (0, 12, 13, 700, 2400):
        r = zset.enumerate_ex(n, g)
        assert r.rows == oracle.count(n, g)
        for order in (0, 1):
            e = zset.enumerate_ex(n, g, order=order)
            want = e.out[: e.rows].cpu().numpy().view(np.uint32).reshape(e.rows, len(g))
            assert np.array_equal(walk(n, g, order, r.rows), want), (n, order)
        say(f"n={n}: {r.rows} rows equal")


def test_walk_at_large_elements():
    # Z(c n; c g) = Z(n; g): scaling every generator and the element by c
    # changes no coordinate.  At c = 200003 the element is 4.8e8 (a count
    # table of 3.4e9 entries); the rows must be those of the small problem.
    g = [13, 34, 37, 54, 65, 83]
    c = 200003
    base = oracle.enumerate_rows(2400, g)
    got = walk(2400 * c, [c * x for x in g], 0, len(base))
    assert np.array_equal(got, base)
    # An element c n + 1 has no factorization over multiples of c.
    assert walk(2400 * c + 1, [c * x for x in g], 0, 1).shape == (0, 6)
    # Generators of gcd 1 and elements above 1e9 (count tables of 4e10 and
    # 8e9 entries), against the oracle's own walk, which keeps no table.
    for g2, coef in (([100000007, 100000037, 100000039, 100000049], [3, 5, 7, 2]),
                     ([2000000, 3000000, 7000000, 11000000, 13000001], [100, 50, 30, 20, 40])):
        n = sum(a * b for a, b in zip(g2, coef))
        want = oracle.enumerate_rows(n, g2)
        say(f"n={n} g={g2}: {len(want)} rows")
        assert len(want) >= 1
        assert np.array_equal(walk(n, g2, 0, len(want)), want)
        assert np.array_equal(walk(n, g2, 1, len(want)), want[::-1])


def test_walk_edges_and_errors():
    assert walk(12, [4], 0, 1).tolist() == [[3]]
    assert walk(13, [4], 0, 1).shape == (0, 1)
    assert walk(0, [3, 5, 7], 0, 1).tolist() == [[0, 0, 0]]
    assert walk(1, [3, 5, 7], 0, 1).shape == (0, 3)
    out = torch.empty(3 * 2, dtype=torch.int32, device="cuda")
    with pytest.raises(zset.ZsetError):  # 4 rows do not fit in 2
        zset.enumerate_walk(30, [5, 6, 10], out)
    # 2^29 first-coordinate values (no prefix refinement fits): one prefix.
    assert walk(1 << 29, [1, 1 << 28], 0, 3).tolist() == [[0, 2], [1 << 28, 1], [1 << 29, 0]]
    with pytest.raises(zset.ZsetError):
        zset.enumerate_walk(10, [3, 5], out, order=2)
