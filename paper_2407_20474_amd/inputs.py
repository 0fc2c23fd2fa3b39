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
