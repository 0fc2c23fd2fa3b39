"""Writes tests/golden/workloads.json: the concrete synthetic workloads.

Generators come from paper_2407_20474_amd.inputs.draw_gens; each n is the
smallest element whose |Z(n)| reaches the row target, found with the CPU
oracle's count table (oracle/ only -- nothing here touches the HIP path).

  plain      (7, 11, 13, 17), n = 2000, k = 0
  large      d = 6, g distinct in [10, 100], gcd 1, sorted; seeds 0, 1, 2;
             |Z(n)| >= 2e8; k = 2
  sweep      d = 5, 7, 9 (seed = d), g distinct in [10, 200], gcd 1, sorted;
             |Z(n)| >= 10^8 * sqrt(10) (log-midpoint of [1e8, 1e9]); k = 0..3

and tests/golden/batch_queries.txt: the batched workload, 4096 independent
queries (seed 4) with d uniform in {3..8}, distinct generators in [5, 150]
with gcd 1, sorted, and |Z(n)| log-uniform in [1e2, 1e7] (inputs.draw_query_specs).
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2407_20474_amd.inputs import BATCH_QUERIES, draw_gens, draw_query_specs  # noqa: E402


def smallest_n(g, target, nmax):
    ways = oracle.count_table(nmax, g)[0]
    hit = np.nonzero(ways >= np.uint64(target))[0]
    if len(hit) == 0:
        raise ValueError(f"no n <= {nmax} reaches {target} for {g}")
    n = int(hit[0])
    return n, int(ways[n])


def smallest_n_grow(g, target):
    """smallest_n with the table bound doubled until the target is reached."""
    nmax = 256
    while True:
        try:
            return smallest_n(g, target, nmax)
        except ValueError:
            nmax *= 2


def write_batch():
    specs = draw_query_specs(4, 4096)
    lines = ["# n rows g_1 ... g_d  (seed 4: d in {3..8}, g in [5, 150], |Z| log-uniform "
             "in [1e2, 1e7])"]
    for g, target in specs:
        n, rows = smallest_n_grow(g, target)
        lines.append(" ".join(str(v) for v in [n, rows] + g))
    with open(BATCH_QUERIES, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    out = {"plain": {"gens": [7, 11, 13, 17], "n": 2000, "k": 0,
                     "rows": oracle.count(2000, [7, 11, 13, 17])}}
    out["large"] = []
    for seed in (0, 1, 2):
        g = draw_gens(seed, 6, 10, 100)
        n, rows = smallest_n(g, 200_000_000, 40_000)
        out["large"].append({"seed": seed, "gens": g, "n": n, "k": 2, "rows": rows})
    out["sweep"] = []
    target = int(math.ceil(1e8 * math.sqrt(10)))
    for d, nmax in ((5, 400_000), (7, 40_000), (9, 20_000)):
        g = draw_gens(d, d, 10, 200)
        n, rows = smallest_n(g, target, nmax)
        out["sweep"].append({"seed": d, "gens": g, "n": n, "ks": [0, 1, 2, 3], "rows": rows})
    with open(os.path.join(HERE, "workloads.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))
    write_batch()


if __name__ == "__main__":
    main()
