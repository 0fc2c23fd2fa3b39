"""The allocation-free entry point (zset_enumerate_noalloc, through the C ABI)
against zset_enumerate_ex: the same rows (bit-exact, compared on the device)
and the same count-only checksum, on consecutive calls that share the
library's scratch array -- a large query, then smaller ones -- and the
refusal of a query whose scratch exceeds the array."""
import sys

import numpy as np
import pytest

from paper_2407_20474_amd import inputs
from paper_2407_20474_amd import zset

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same_as_ex(n, g, k, order=0, rows_per_tile=0):
    d = len(g)
    rows = zset.count(n, g)
    want = torch.empty((max(rows, 1), d), dtype=torch.int32, device="cuda")
    got = torch.full((max(rows, 1), d), -7, dtype=torch.int32, device="cuda")
    a = zset.enumerate_ex(n, g, out=want, k=k, order=order, rows_per_tile=rows_per_tile)
    b = zset.enumerate_noalloc(n, g, out=got, k=k, order=order, rows_per_tile=rows_per_tile)
    assert a.rows == b.rows == rows, (n, g, k)
    assert torch.equal(got[:rows], want[:rows]), (n, g, k, order)
    ca = zset.enumerate_ex(n, g, k=k, count_only=True)
    cb = zset.enumerate_noalloc(n, g, k=k, count_only=True)
    assert ca.rows == cb.rows == rows and ca.checksum == cb.checksum, (n, g, k)
    del want, got


def test_noalloc_large_then_smaller_queries():
    w = inputs.load_workloads()["large"][0]
    say(f"noalloc: large n={w['n']} g={w['gens']} k={w['k']}")
    same_as_ex(w["n"], w["gens"], w["k"])
    p = inputs.load_workloads()["plain"]
    for k in range(len(p["gens"])):
        say(f"noalloc: plain n={p['n']} g={p['gens']} k={k}")
        same_as_ex(p["n"], p["gens"], k, rows_per_tile=128)
    say("noalloc: descending, d = 1, empty set, n = 0")
    same_as_ex(p["n"], p["gens"], 2, order=1)
    for n, g, k in [(123, [41], 0), (7, [2, 4], 1), (0, [3, 4, 5], 2), (400, [9, 5, 7, 3, 11], 3),
                    (3000, [1, 1, 2], 2), (2000, [13, 37, 38, 40, 41], 4)]:
        same_as_ex(n, g, k)
    torch.cuda.empty_cache()


def test_noalloc_refuses_a_query_beyond_its_scratch():
    # Count table alone: 4 rows x (n + 1) x 8 bytes > 64 MiB.
    n, g = 3_000_000, [1000, 1500, 2500]
    rows = zset.count(n, g)
    out = torch.full((rows, 3), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(zset.ZsetError) as e:
        zset.enumerate_noalloc(n, g, out=out)
    assert e.value.status == zset.ENOMEM
    assert "scratch" in str(e.value)
    assert int((out != -7).sum()) == 0
    # The array still serves the next call.
    same_as_ex(2000, [7, 11, 13, 17], 2)
    # No partial memo here (memo_top <= n).
    with pytest.raises(zset.ZsetError) as e:
        zset.enumerate_noalloc(2000, [7, 11, 13, 17], out=out, k=2, memo_top=100)
    assert e.value.status == zset.EINVAL
