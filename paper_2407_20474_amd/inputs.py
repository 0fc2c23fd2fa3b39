"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
runs.  Only random draws live here -- none of the enumeration's arithmetic.

Generators: `numpy.random.default_rng(seed).choice(range(lo, hi + 1), d,
replace=False)`, redrawn on the same stream until their gcd is 1, then sorted
ascending (as the workloads of the paper's Table 1 are).  The element n of each
stored workload (the smallest n whose |Z(n)| reaches a row target) is fixed in
tests/golden/workloads.json, written by tests/golden/make_workloads.py.
"""
from __future__ import annotations

import json
import math
import os
from functools import reduce

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORKLOADS = os.path.join(ROOT, "tests", "golden", "workloads.json")


def draw_gens(seed: int, d: int, lo: int, hi: int, sort: bool = True) -> list[int]:
    rng = np.random.default_rng(seed)
    while True:
        g = rng.choice(np.arange(lo, hi + 1), size=d, replace=False)
        if reduce(math.gcd, (int(x) for x in g)) == 1:
            break
    g = [int(x) for x in g]
    return sorted(g) if sort else g


def random_small_query(rng: np.random.Generator, dmax: int = 6, gmax: int = 40,
                       nmax: int = 400):
    """A small query with unsorted, possibly repeated generators (parity tests)."""
    d = int(rng.integers(1, dmax + 1))
    g = [int(x) for x in rng.integers(1, gmax + 1, size=d)]
    n = int(rng.integers(0, nmax + 1))
    return n, g


def load_workloads() -> dict:
    with open(WORKLOADS) as f:
        return json.load(f)


def draw_query_specs(seed: int, count: int, dlo: int = 3, dhi: int = 8, glo: int = 5,
                     ghi: int = 150, log_lo: float = 2.0, log_hi: float = 7.0):
    """Random (generators, row target) pairs of a batch of independent queries:
    d uniform in [dlo, dhi], distinct generators uniform in [glo, ghi] with gcd 1
    (redrawn on the same stream), sorted ascending, and a row target
    ceil(10^u) with u uniform in [log_lo, log_hi] (log-uniform sizes).  Each
    query's n -- the smallest element whose |Z(n)| reaches the target -- is
    fixed by tests/golden/make_workloads.py."""
    rng = np.random.default_rng(seed)
    specs = []
    pool = np.arange(glo, ghi + 1)
    for _ in range(count):
        d = int(rng.integers(dlo, dhi + 1))
        while True:
            g = rng.choice(pool, size=d, replace=False)
            if reduce(math.gcd, (int(x) for x in g)) == 1:
                break
        target = int(math.ceil(10.0 ** rng.uniform(log_lo, log_hi)))
        specs.append((sorted(int(x) for x in g), target))
    return specs


def draw_generator_sets(seed: int, count: int, dlo: int = 3, dhi: int = 8, glo: int = 5,
                        ghi: int = 150):
    """Generator sets of the served workload, drawn as the batched queries' are:
    d uniform in [dlo, dhi], distinct generators uniform in [glo, ghi] with gcd 1
    (redrawn on the same stream), sorted ascending."""
    rng = np.random.default_rng(seed)
    pool = np.arange(glo, ghi + 1)
    sets = []
    for _ in range(count):
        d = int(rng.integers(dlo, dhi + 1))
        while True:
            g = rng.choice(pool, size=d, replace=False)
            if reduce(math.gcd, (int(x) for x in g)) == 1:
                break
        sets.append(sorted(int(x) for x in g))
    return sets


def draw_served_stream(seed: int, count: int, nsets: int, log_lo: float = 1.0,
                       log_hi: float = 8.0):
    """(set index, row target) pairs of a served query stream: the set uniform
    over nsets, the target ceil(10^u) with u uniform in [log_lo, log_hi]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = int(rng.integers(0, nsets))
        out.append((s, int(math.ceil(10.0 ** rng.uniform(log_lo, log_hi)))))
    return out


def poisson_arrivals(seed: int, count: int, rate: float):
    """Arrival times (seconds from 0) of a Poisson stream of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def load_query_file(path: str):
    """Rows 'n rows g_1 ... g_d' of a stored query list -> [(n, gens, rows)]."""
    out = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x) for x in line.split()]
            out.append((v[0], v[2:], v[1]))
    return out


BATCH_QUERIES = os.path.join(ROOT, "tests", "golden", "batch_queries.txt")


def load_batch_queries():
    """The 4096-query batched workload: [(n, gens, rows)]."""
    return load_query_file(BATCH_QUERIES)
