"""Autotuner for the memo dimension k and the slice length of zset_enumerate_ex.

For each bucket (d, decade of |Z(n)|) it draws seeded sample queries the way
the batched workload does (distinct generators in [5, 150] with gcd 1, sorted,
n the smallest element whose |Z(n)| reaches a target inside the decade), times
the whole call (count table, memo recurrence, slice plan, write pass) for
every memo dimension k and two slice lengths, and keeps the fastest pair.
The result is cached as JSON; `choose(d, rows)` reads it back.

    python -m paper_2407_20474_amd.autotune --out tuning.json

Every measurement goes through the library (one GPU); nothing here computes
rows itself.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import zset

TUNING_JSON = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
DECADES = (3, 4, 5, 6, 7, 8)


def bucket_key(d: int, rows: int) -> str:
    dec = int(math.floor(math.log10(max(rows, 1))))
    dec = min(max(dec, DECADES[0]), DECADES[-1])
    return f"d={d},dec={dec}"


def smallest_n(gens, target: int) -> int:
    """The smallest n with |Z(n)| >= target, from the running maximum of the
    count table's first row (computed by the library on the GPU)."""
    import torch
    d = len(gens)
    n_hi = int(1.3 * (target * math.factorial(d - 1) * math.prod(gens)) ** (1.0 / (d - 1))) + max(gens)
    while True:
        run = torch.cummax(zset.count_table(n_hi, gens)[0], dim=0).values
        if int(run[-1]) >= target:
            return int(torch.searchsorted(run, torch.tensor([target], device=run.device))[0])
        n_hi = int(n_hi * 1.5)


def memo_rows(n, gens):
    """Rows of the memo each k would build: sum over p <= n of |Z(p; g_{d-k+1..d})|
    (row sums of the library's count table)."""
    t = zset.count_table(n, gens)
    d = len(gens)
    return {k: int(t[d - k].sum()) for k in range(1, d)}


def time_call(n, gens, out, k, rows_per_tile, reps=2):
    ts = []
    for _ in range(reps + 1):
        t = time.perf_counter()
        zset.enumerate_ex(n, gens, out=out, k=k, rows_per_tile=rows_per_tile)
        ts.append(time.perf_counter() - t)
    return float(np.median(ts[1:]))


def tune(dims=range(3, 10), decades=DECADES, samples=2, seed=11, log=print):
    import torch
    rng = np.random.default_rng(seed)
    pool = np.arange(5, 151)
    table = {}
    out = None
    for d in dims:
        for dec in decades:
            votes = {}
            for _ in range(samples):
                while True:
                    g = sorted(int(x) for x in rng.choice(pool, size=d, replace=False))
                    if math.gcd(*g) == 1:
                        break
                target = int(10 ** rng.uniform(dec, dec + 1 if dec < 8 else dec + 0.3))
                n = smallest_n(g, target)
                rows = zset.count(n, g)
                need = rows * d
                if out is None or out.numel() < need:
                    out = torch.empty(max(need, 1 << 20), dtype=torch.int32, device="cuda")
                best = None
                sizes = memo_rows(n, g)
                for k in range(d - 1, -1, -1):
                    if k >= 1 and not 0 <= sizes[k] <= max(rows, 1 << 20):
                        continue  # a memo larger than the output
                    fastest = None
                    for T in ((0, 2048) if rows >= 10 ** 6 else (0,)):
                        try:
                            dt = time_call(n, g, out, k, T)
                        except zset.ZsetError:
                            continue
                        fastest = dt if fastest is None else min(fastest, dt)
                        if best is None or dt < best[0]:
                            best = (dt, k, T)
                    if best is not None and fastest is not None and fastest > 10 * best[0]:
                        break  # smaller k only visits more leaves per row
                if best is None:
                    continue
                key = (best[1], best[2])
                votes[key] = votes.get(key, 0.0) + rows / best[0]
                log(f"d={d} dec={dec} g={g} n={n} rows={rows}: best k={best[1]} "
                    f"rows_per_tile={best[2]} {rows / best[0]:.3e} rows/s")
            if not votes:
                continue
            (k, T), rate = max(votes.items(), key=lambda kv: kv[1])
            table[f"d={d},dec={dec}"] = {"k": k, "rows_per_tile": T,
                                         "rows_per_s": rate / samples}
    return table


def save(table, path=TUNING_JSON):
    with open(path, "w") as f:
        json.dump({"device": _device_name(), "buckets": table}, f, indent=1, sort_keys=True)


def _device_name():
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


_cache = None


def choose(d: int, rows: int, path=TUNING_JSON):
    """(k, rows_per_tile) of the bucket, or None when no table is cached."""
    global _cache
    if _cache is None:
        if not os.path.exists(path):
            return None
        with open(path) as f:
            _cache = json.load(f)["buckets"]
    e = _cache.get(bucket_key(d, rows))
    if e is None or e["k"] > d - 1:
        return None
    return e["k"], e["rows_per_tile"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TUNING_JSON)
    ap.add_argument("--samples", type=int, default=2)
    ap.add_argument("--dmin", type=int, default=3)
    ap.add_argument("--dmax", type=int, default=9)
    args = ap.parse_args()
    table = tune(range(args.dmin, args.dmax + 1), samples=args.samples,
                 log=lambda s: print(s, flush=True))
    save(table, args.out)
    print(f"wrote {args.out}: {len(table)} buckets", flush=True)


if __name__ == "__main__":
    sys.exit(main())
