"""Benchmark: factorizations/s of one large enumeration of Z(n; g) on one GPU.

A step is one pass of the whole path over the workload with the output
buffer already resident in HBM: count table, memo build (k = 2: the library
builds two-coordinate memos in closed form, element-parallel, which gives the
same lists as the recurrence of Lemma 2.3; the recurrence itself is timed
beside the step and reported as stages_us.memo_recurrence_us), slice plan, and
the write pass that stores every uint32 row.  The timed steps are queued
calls (zset_enumerate_async: each enqueues the whole path and returns, the
host waits once after the last); the write pass is timed by HIP events that
the call records around it, in a second run of the same queued steps.
`--sync-steps` times synchronous calls instead, and the line also reports
their per-step time.  Prints one JSON line.

The default workload is the large single enumeration: d = 6 generators drawn
distinct in [10, 100] with gcd 1 (seed 0), n the smallest element with
|Z(n)| >= 2e8, memo dimension k = 2.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0     # MI355X HBM3E peak, GB/s
COUNTERS = os.path.join(ROOT, "profiles", "write_pass_large_d6_k2_counters.md")
ALU_COUNTERS = os.path.join(ROOT, "profiles", "count_only_alu.md")
WRITE_SRC = os.path.join(ROOT, "paper_2407_20474_amd", "csrc", "enumerate.hip")


def profile_field(path, key):
    """A `key: value` field of a committed counter summary, or None when the
    write kernel's source changed since those counters were taken."""
    import hashlib
    try:
        text = open(path).read()
        src = hashlib.sha256(open(WRITE_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.split(":", 1)[0].strip() in ("kernel_source_sha256", key):
            k, val = line.split(":", 1)
            fields[k.strip()] = val.strip().strip("`")
    if fields.get("kernel_source_sha256") != src or key not in fields:
        return None
    return fields[key]


def measured_traffic():
    """HBM bytes per write-pass launch from the committed counter summary."""
    v = profile_field(COUNTERS, "traffic_bytes_per_launch")
    return int(v) if v is not None else None
ALU_PEAK_OPS = 256 * 64 * 2.4e9   # 32-bit integer lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "plain", "sweep", "batch", "memo", "serve", "walk"])
    ap.add_argument("--sweep-d", type=int, default=5, choices=[5, 7, 9],
                    help="dimension of the memo-dimension sweep workload")
    ap.add_argument("--seed", type=int, default=0, help="large workload seed (0, 1 or 2)")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--rows-per-tile", type=int, default=0)
    ap.add_argument("--count-only", action="store_true")
    ap.add_argument("--sync-steps", action="store_true",
                    help="time synchronous calls (zset_enumerate_ex, a host wait per step) "
                         "instead of queued ones (zset_enumerate_async)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=float, default=2.5e8)
    ap.add_argument("--serve-queries", type=int, default=10000,
                    help="queries per arrival rate of the served workload")
    ap.add_argument("--slots", type=int, default=16, help="server slots (batched and served)")
    ap.add_argument("--memo-bytes", type=int, default=0,
                    help="served: memo budget per resident set (0: the library's 32 MiB); "
                         "larger memos are capped (partial memos)")
    ap.add_argument("--dispatchers", type=int, default=1, help="server dispatcher threads")
    ap.add_argument("--kmode", default="server", choices=["server", "tuned"],
                    help="memo dimension of the resident sets of the batched and served "
                         "workloads: the server's rule or the autotuner's table (the plain "
                         "path always takes the autotuner's choice per query)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(n, g, sample_rows):
    """The CPU oracle (threaded over a_1) on the rows with a_1 < A, the smallest
    prefix of a_1 values holding >= sample_rows rows."""
    import numpy as np

    import oracle
    table = oracle.count_table(n, g)
    row1 = table[1]
    acc, a1 = 0, 0
    while a1 * g[0] <= n and acc < sample_rows:
        acc += int(row1[n - a1 * g[0]])
        a1 += 1
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(int(threads), 64))
    out = np.empty((acc, len(g)), dtype=np.uint32)
    out[::max(1, acc // 1024)] = 0   # touch pages before timing
    out.fill(0)
    t = time.perf_counter()
    _, rows = oracle.enumerate_rows_threads(n, g, 0, a1, threads, table=table, out=out)
    dt = time.perf_counter() - t
    return {"value": rows / dt, "unit": "factorizations/s", "cores": threads, "kind": "oracle",
            "sample": f"rows with a_1 < {a1} ({rows} of the workload's rows), "
                      f"threaded C oracle, {dt:.2f} s"}


def batch_cpu_baseline(queries, sample_rows):
    """The CPU oracle (threaded over a_1 within each query) on the first queries
    of the batch whose rows add up to >= sample_rows."""
    import numpy as np

    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(int(threads), 64))
    picked, acc = [], 0
    for n, g, rows in queries:
        if acc >= sample_rows:
            break
        picked.append((n, g, rows))
        acc += rows
    bufs = [np.zeros((max(rows, 1), len(g)), dtype=np.uint32) for _, g, rows in picked]
    tables = [oracle.count_table(n, g) for n, g, _ in picked]
    t = time.perf_counter()
    done = 0
    for (n, g, rows), buf, table in zip(picked, bufs, tables):
        _, r = oracle.enumerate_rows_threads(n, g, 0, n // g[0] + 1, threads, table=table,
                                             out=buf)
        done += r
    dt = time.perf_counter() - t
    return {"value": done / dt, "unit": "factorizations/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {len(picked)} queries of the batch ({done} rows), threaded C "
                      f"oracle per query, {dt:.2f} s"}


def k_chooser(args):
    """Memo dimension of a resident set (the served path)."""
    from paper_2407_20474_amd import zset
    if args.kmode == "tuned":
        return lambda n, g: zset.tuned(n, g)[0]
    return lambda n, g: -1


def plain_k(n, g):
    """Memo dimension of one zset_enumerate_ex call: the autotuner's choice,
    timed over whole calls (memo recurrence included)."""
    from paper_2407_20474_amd import zset
    return zset.tuned(n, g)[0]


def run_batch(args):
    """The batched workload (4096 independent queries) through the request
    loop: at plan time every query's generator set is made resident up to its
    own n (count table, memo, leaf layout); a step submits all 4096 queries at
    once and waits for every one (slice plans and write passes on the server's
    slots, outputs side by side in one arena).  The plain path is one
    zset_enumerate_ex call per query, one at a time, every stage included."""
    import numpy as np
    import torch

    from paper_2407_20474_amd import inputs, zset

    allq = inputs.load_batch_queries()
    rows = sum(r for _, _, r in allq)
    bytes_written = sum(r * len(g) * 4 for _, g, r in allq)
    words = sum((r * len(g) + 3) // 4 * 4 for _, g, r in allq)
    arena = torch.empty(words + 4, dtype=torch.int32, device="cuda")
    srv = zset.Server(arena, slots=args.slots, dispatchers=args.dispatchers)
    kq = k_chooser(args)
    t = time.perf_counter()
    ks = []
    for i, (n, g, r) in enumerate(allq):
        sid = srv.add_set(g, n, k=kq(n, g))
        assert srv.count(sid, n) == r, "count disagrees with the stored workload"
        ks.append(srv.set_info(sid)["k"])
        if (i + 1) % 1024 == 0:
            print(f"# batch plan {i + 1}/{len(allq)}", file=sys.stderr, flush=True)
    create_s = time.perf_counter() - t
    print(f"# batch planned in {create_s:.2f} s: {len(allq)} queries, {rows} rows, "
          f"{bytes_written / 1e9:.1f} GB", file=sys.stderr, flush=True)

    def step():
        tickets = [srv.submit(i, n) for i, (n, _, _) in enumerate(allq)]
        res = [srv.wait(tk) for tk in tickets]
        return tickets, res

    for i in range(args.warmup):
        tickets, _ = step()
        for tk in tickets:
            srv.release(tk)
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        tickets, res = step()
        if i < args.steps - 1:
            for tk in tickets:
                srv.release(tk)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = rows / (dt / args.steps)
    start = min(r["submit_us"] for r in res)
    done = np.array([r["done_us"] - start for r in res])
    # Bit-exact against the plain path on a sample of queries (bytes on the device).
    rng = np.random.default_rng(4)
    sample = sorted(set(rng.choice(len(allq), size=32, replace=False).tolist()
                        + np.argsort([r for _, _, r in allq])[-4:].tolist()))
    for q in sample:
        n, g, r = allq[q]
        if r == 0:
            continue
        alone = zset.enumerate_ex(n, g, k=plain_k(n, g))
        assert torch.equal(srv.rows_of(q, res[q]), alone.out[:r]), q
    for tk in tickets:
        srv.release(tk)
    # The plain path: one zset_enumerate_ex call per query, into the arena.
    pks = [plain_k(n, g) for n, g, _ in allq]
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for q, (n, g, r) in enumerate(allq):
        zset.enumerate_ex(n, g, out=arena, k=pks[q])
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - tp
    plain_value = rows / plain_s
    print(f"# plain path: {plain_s:.2f} s for {len(allq)} calls", file=sys.stderr, flush=True)
    st = srv.stats()
    srv.free()
    if queued:
        stages["write_us_queued"] = round(write_us, 2)
        stages["ms_per_step_write_events"] = round(ms_events, 4)
        stages["ms_per_step_synchronous"] = round(ms_sync, 4)
    line = {
        "metric": "Z(n) factorizations/s emitted (bit-exact)",
        "value": value,
        "unit": "factorizations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": (f"batch: {len(allq)} queries (d in 3..8, g in [5, 150], |Z| log-uniform "
                         f"in [1e2, 1e7]), {rows} rows, {bytes_written / 1e9:.1f} GB; each step "
                         f"submits every query to the request loop ({args.slots} slots) and "
                         f"waits for all"),
            "queries": len(allq), "rows": rows,
            "k_histogram": {int(k): ks.count(k) for k in sorted(set(ks))},
        },
        "batch": {
            "plain_value": plain_value, "plain_s": plain_s, "speedup_vs_plain": value / plain_value,
            "p50_done_us": float(np.percentile(done, 50)),
            "p99_done_us": float(np.percentile(done, 99)),
            "create_s": create_s, "max_inflight": st["max_inflight"],
            "dispatcher_launch_us_per_query": round(st["launch_us"] / max(st["admitted"], 1), 2),
            "checked_against_plain": len(sample),
        },
        "step_hbm_write_frac": round(bytes_written / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = batch_cpu_baseline(allq, args.cpu_sample_rows / 10)
    print(json.dumps(line), flush=True)


# The table-free walk's workloads: elements above 1e9, where the count table
# of the main path would take tens of gigabytes.
#  - "scaled": the large workload's generators and an element scaled by
#    c = 200003 (Z(c n; c g) = Z(n; g)), n = 8000 c: 6.2e7 rows.
#  - "coprime": generators of gcd 1 near 1e6..1.3e7, n = 1,300,000,040.
WALK_CASES = [
    ("scaled", 8000 * 200003, [200003 * x for x in (13, 34, 37, 54, 65, 83)]),
    ("coprime", 1300000040, [2000000, 3000000, 7000000, 11000000, 13000001]),
]


def run_walk(args):
    """zset_enumerate_walk on elements above 1e9 (no count table): rows/s per
    case, checked against the oracle's walk on a sample of first coordinates
    (the whole output for the coprime case), with the count-table bytes the
    main path would need for the same query."""
    import numpy as np
    import torch

    import oracle
    from paper_2407_20474_amd import zset

    cases = []
    for name, n, g in WALK_CASES:
        d = len(g)
        t = time.perf_counter()
        a1_hi = 10 if name == "scaled" else None
        sample = oracle.enumerate_rows(n, g, 0, a1_hi)  # rows with a_1 < a1_hi (all if None)
        cpu_s = time.perf_counter() - t
        # Rows in all: the scaled case's count is that of the small problem.
        rows = oracle.count(n // 200003, [x // 200003 for x in g]) if name == "scaled" else len(sample)
        out = torch.empty(max(rows, 1) * d, dtype=torch.int32, device="cuda")
        for _ in range(args.warmup):
            zset.enumerate_walk(n, g, out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t = time.perf_counter()
            got = zset.enumerate_walk(n, g, out)
            ts.append(time.perf_counter() - t)
        assert got == rows
        view = out[: len(sample) * d].view(len(sample), d).cpu().numpy().view(np.uint32)
        assert np.array_equal(view, sample), name
        sec = float(np.median(ts))
        cases.append({"case": name, "n": n, "gens": g, "rows": rows, "ms": round(sec * 1e3, 3),
                      "rows_per_s": rows / sec,
                      "count_table_bytes_avoided": (d + 1) * (n + 1) * 8,
                      "checked_rows": len(sample),
                      "oracle_rows_per_s": len(sample) / cpu_s if cpu_s > 0 else None})
        print(f"# walk {name}: {rows} rows in {sec * 1e3:.2f} ms", file=sys.stderr, flush=True)
    main = cases[0]
    line = {
        "metric": "Z(n) factorizations/s emitted (bit-exact), table-free walk",
        "value": main["rows_per_s"], "unit": "factorizations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "walk: elements above 1e9 without the count table (value: the "
                               "scaled case)"},
        "walk": cases,
    }
    print(json.dumps(line), flush=True)


# The paper's Table 1 groups: (d, memo dimension, largest element), generators
# the first d of (13, 37, 38, 40, ..., 45), memo of the trailing k generators
# populated up to the largest element of the group; with the paper's own CPU
# and GPU memo population times (microseconds, Ryzen 3900X / RTX 3080).
TABLE1_GENS = (13, 37, 38, 40, 41, 42, 43, 44, 45)
TABLE1_GROUPS = [(3, 1, 300000, 452, 9205), (4, 2, 15000, 3073, 33543),
                 (5, 2, 10000, 1624, 33645), (5, 3, 5000, 7951, 28841),
                 (6, 3, 5000, 7341, 26576), (6, 4, 3000, 45837, 26152),
                 (7, 4, 2000, 55714, 26664), (8, 4, 2000, 46092, 28807),
                 (9, 4, 1500, 49328, 26591), (9, 5, 1500, 22711, 18628)]


def run_memo(args):
    """Memo population, CPU vs GPU (the paper's Section 4.1 crossover): the
    serial dynamic recurrence on one host core (the oracle's CPU form of it)
    against zset_memo_build on the GPU (device time between events on the
    call's stream, and the call's wall time), for the Table 1 groups and for a
    sweep of `top` at fixed generators.  The GPU lists are compared with the
    CPU lists for every case."""
    import numpy as np
    import torch

    import oracle
    from paper_2407_20474_amd import zset

    def gpu_time(h, top, reps=5):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        m = zset.Memo(h, top)  # warm-up (first use of the path)
        m.free()
        dev, wall = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ev0.record()
            m = zset.Memo(h, top)
            ev1.record()
            torch.cuda.synchronize()
            wall.append((time.perf_counter() - t) * 1e6)
            dev.append(ev0.elapsed_time(ev1) * 1e3)
            if _ < reps - 1:
                m.free()
        return m, float(np.median(dev)), float(np.median(wall))

    def cpu_time(h, top, reps=3):
        best, res = None, None
        for _ in range(reps):
            off, rows, dt = oracle.memo_dynamic(h, top, timed=True)
            if best is None or dt < best:
                best, res = dt, (off, rows)
        return res, best * 1e6

    def case(h, top, paper=None):
        (off, rows), cpu_us = cpu_time(h, top)
        m, gpu_dev_us, gpu_wall_us = gpu_time(h, top)
        goff, grows = m.read()
        m.free()
        assert np.array_equal(goff, off) and np.array_equal(grows, rows), (h, top)
        r = {"h": list(h), "top": top, "memo_rows": int(off[top]),
             "memo_bytes": int(off[top]) * len(h) * 4, "cpu_us": round(cpu_us, 1),
             "gpu_us": round(gpu_dev_us, 1), "gpu_wall_us": round(gpu_wall_us, 1),
             "gpu_faster": gpu_dev_us < cpu_us}
        if paper:
            r["paper_cpu_us"], r["paper_gpu_us"] = paper
        print(f"# memo h={h} top={top}: rows {r['memo_rows']}, cpu {r['cpu_us']} us, "
              f"gpu {r['gpu_us']} us (wall {r['gpu_wall_us']} us)", file=sys.stderr, flush=True)
        return r

    groups = []
    for d, k, elem, pc, pg in TABLE1_GROUPS:
        h = list(TABLE1_GENS[:d][d - k:])
        r = case(h, elem + 1, (pc, pg))
        r["d"], r["k"], r["element"] = d, k, elem
        groups.append(r)
    sweep_h = [40, 41, 42, 43]
    sweep = [case(sweep_h, top) for top in (50, 100, 200, 400, 800, 1600, 3200, 6400)]
    cross = next((r for r in sweep if r["gpu_faster"]), None)
    total_rows = sum(r["memo_rows"] for r in groups)
    gpu_total_us = sum(r["gpu_us"] for r in groups)
    line = {
        "metric": "memo rows/s populated by the GPU dynamic recurrence (zset_memo_build)",
        "value": total_rows / (gpu_total_us * 1e-6),
        "unit": "memo rows/s",
        "n_gpus": 1, "steps": 5, "warmup": 1, "ms_per_step": gpu_total_us / 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "memo: the paper's Table 1 memo groups (generators the first d of "
                               "13, 37, 38, 40..45; memo of the trailing k up to the group's "
                               "largest element) and a top sweep at h = (40, 41, 42, 43)"},
        "table1": groups,
        "top_sweep": sweep,
        "crossover": ({"h": sweep_h, "top": cross["top"], "memo_rows": cross["memo_rows"]}
                      if cross else None),
        "cpu_baseline": {"value": total_rows / (sum(r["cpu_us"] for r in groups) * 1e-6),
                         "unit": "memo rows/s", "cores": 1, "kind": "oracle",
                         "sample": "the Table 1 memo groups, serial dynamic recurrence, best of 3"},
    }
    print(json.dumps(line), flush=True)


def run_serve(args):
    """Served queries: 64 resident generator sets (drawn as the batched queries'
    are, seed 5), a stream of queries (set uniform, |Z(n)| target log-uniform in
    [1e1, 1e8], n the smallest element reaching it), Poisson arrivals at 0.5, 1
    and 2 times the plain path's saturation rate, into a 64 GiB output arena.
    The plain path is one zset_enumerate_ex call per query, one at a time: its
    service times are measured on the same stream, and its latencies at each
    rate follow from them (first come, first served, one query at a time)."""
    import math
    import threading

    import numpy as np
    import torch

    from paper_2407_20474_amd import inputs, zset

    nq = args.serve_queries
    sets = inputs.draw_generator_sets(5, 64)
    stream = inputs.draw_served_stream(5, nq, len(sets))
    top = 10 ** 8
    # n for each target: the smallest n whose |Z(n)| reaches it, from the
    # running maximum of the count table's first row.
    ns = [None] * nq
    n_need = [0] * len(sets)
    by_set = {}
    for i, (s, t) in enumerate(stream):
        by_set.setdefault(s, []).append((i, t))
    t_setup = time.perf_counter()
    for s, g in enumerate(sets):
        d = len(g)
        n_hi = int(1.3 * (top * math.factorial(d - 1) * math.prod(g)) ** (1.0 / (d - 1))) + max(g)
        while True:
            c0 = zset.count_table(n_hi, g)[0]
            run = torch.cummax(c0, dim=0).values
            if int(run[-1]) >= top:
                break
            n_hi = int(n_hi * 1.5)
        targets = torch.tensor([t for _, t in by_set.get(s, [])], dtype=torch.int64, device="cuda")
        if targets.numel():
            idx = torch.searchsorted(run, targets).tolist()
            for (i, _), n in zip(by_set[s], idx):
                ns[i] = int(n)
                n_need[s] = max(n_need[s], int(n))
        del c0, run
    arena = torch.empty((64 << 30) // 4, dtype=torch.int32, device="cuda")
    srv = zset.Server(arena, slots=args.slots, dispatchers=args.dispatchers,
                      memo_bytes=args.memo_bytes)
    kq = k_chooser(args)
    ks, capped = [], 0
    for s, g in enumerate(sets):
        srv.add_set(g, max(n_need[s], 1), k=kq(max(n_need[s], 1), g))
        info = srv.set_info(s)
        ks.append(info["k"])
        capped += info["memo_top"] <= info["n_max"]
    queries = [(s, ns[i]) for i, (s, _) in enumerate(stream)]
    rows = [srv.count(s, n) for s, n in queries]
    total_rows = sum(rows)
    setup_s = time.perf_counter() - t_setup
    print(f"# serve: {len(sets)} sets resident in {setup_s:.1f} s, {nq} queries, "
          f"{total_rows} rows", file=sys.stderr, flush=True)

    # Plain path: service times, one query at a time.
    service = np.zeros(nq)
    pks = [plain_k(n, sets[s]) for s, n in queries]
    for i, (s, n) in enumerate(queries):
        t = time.perf_counter()
        zset.enumerate_ex(n, sets[s], out=arena, k=pks[i])
        service[i] = time.perf_counter() - t
        if (i + 1) % 2000 == 0:
            print(f"# plain {i + 1}/{nq}", file=sys.stderr, flush=True)
    mu_plain = nq / service.sum()
    plain_rows_s = total_rows / service.sum()

    def plain_latency(arrive):
        end, lat = 0.0, np.zeros(nq)
        for i in range(nq):
            start = max(arrive[i], end)
            end = start + service[i]
            lat[i] = end - arrive[i]
        return lat

    results = {}
    for mult in (0.5, 1.0, 2.0, None):
        # None: every query arrives at time 0 (the server's saturation throughput).
        lam = mult * mu_plain if mult else float("inf")
        arrive = (inputs.poisson_arrivals(50 + int(mult * 10), nq, lam) if mult
                  else np.zeros(nq))
        tickets = [None] * nq
        got = [None] * nq
        ready = threading.Semaphore(0)

        def submitter():
            t0 = time.perf_counter()
            for i, (s, n) in enumerate(queries):
                dt = arrive[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(s, n)
                ready.release()

        th = threading.Thread(target=submitter)
        th.start()
        for i in range(nq):
            ready.acquire()
            got[i] = srv.wait(tickets[i])
            srv.release(tickets[i])
            if (i + 1) % 2000 == 0:
                print(f"# served x{mult or 'sat'} {i + 1}/{nq}", file=sys.stderr, flush=True)
        th.join()
        lat = np.array([r["done_us"] - r["submit_us"] for r in got])
        span = (max(r["done_us"] for r in got) - min(r["submit_us"] for r in got)) * 1e-6
        pl = plain_latency(arrive) * 1e6
        key = f"x{mult}" if mult else "saturation"
        results[key] = {
            "rate_qps": round(lam, 1) if mult else None,
            "p50_us": round(float(np.percentile(lat, 50)), 1),
            "p99_us": round(float(np.percentile(lat, 99)), 1),
            "rows_per_s": total_rows / span, "span_s": round(span, 3),
            "plain_p50_us": round(float(np.percentile(pl, 50)), 1),
            "plain_p99_us": round(float(np.percentile(pl, 99)), 1)}
        print(f"# served {key}: {results[key]}", file=sys.stderr, flush=True)
    # Verification (untimed): a sample of the queries -- every nq / 32-th and
    # the four largest -- is served again, and each query's rows are compared
    # byte for byte with what zset_enumerate_ex writes for it alone.
    sample = sorted(set(range(0, nq, max(1, nq // 32))) |
                    set(int(i) for i in np.argsort(rows)[-4:]))
    scratch = torch.empty(max(rows[i] for i in sample) * 8 + 4, dtype=torch.int32, device="cuda")
    checked_rows = 0
    for i in sample:
        s, n = queries[i]
        t = srv.submit(s, n)
        r = srv.wait(t)
        want = zset.enumerate_ex(n, sets[s], out=scratch, k=pks[i], out_rows_cap=rows[i])
        got = srv.rows_of(s, r)
        assert want.rows == rows[i] == got.shape[0], (i, s, n)
        if rows[i]:
            assert torch.equal(got.reshape(-1), scratch[:rows[i] * len(sets[s])]), (i, s, n)
        checked_rows += rows[i]
        srv.release(t)
    del scratch
    print(f"# serve: {len(sample)} sampled queries ({checked_rows} rows) equal "
          f"zset_enumerate_ex byte for byte", file=sys.stderr, flush=True)
    st = srv.stats()
    srv.free()
    best = results["saturation"]
    line = {
        "metric": "served Z(n) factorizations/s (bit-exact) with p50/p99 latency",
        "value": best["rows_per_s"],
        "unit": "factorizations/s",
        "n_gpus": 1, "steps": nq, "warmup": 0,
        "ms_per_step": best["span_s"] * 1e3 / nq,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": (f"serve: {len(sets)} resident generator sets (d in 3..8, g in "
                                f"[5, 150]), {nq} queries with |Z| log-uniform in [1e1, 1e8] "
                                f"({total_rows} rows), Poisson arrivals at 0.5/1/2 x the plain "
                                f"path's saturation rate and all at once (value: the last), "
                                f"64 GiB output arena, {args.slots} slots"),
                   "k_histogram": {int(k): ks.count(k) for k in sorted(set(ks))},
                   "memo_bytes": args.memo_bytes or (32 << 20), "capped_memos": capped},
        "serve": {"plain_qps": mu_plain, "plain_rows_per_s": plain_rows_s,
                  "verified": {"queries": len(sample), "rows": checked_rows,
                               "against": "zset_enumerate_ex, byte for byte"},
                  "speedup_vs_plain": best["rows_per_s"] / plain_rows_s,
                  "rates": results, "max_inflight": st["max_inflight"],
                  "setup_s": round(setup_s, 2)},
    }
    print(json.dumps(line), flush=True)


def run_sweep(args):
    """The memo-dimension sweep: d = 5, 7, 9 (the stored workloads, |Z| ~ 3.16e8
    each) and k = 0..3, each materialised and in count-only mode: memo build
    time, memo bytes, rows/s of the whole call (median of the timed calls) and
    of the write pass, and the count-only checksum."""
    import numpy as np
    import torch

    from paper_2407_20474_amd import inputs, zset

    table = []
    for item in inputs.load_workloads()["sweep"]:
        n, g, rows = item["n"], item["gens"], item["rows"]
        d = len(g)
        out = torch.empty((rows, d), dtype=torch.int32, device="cuda")
        for k in item["ks"]:
            rec = {"d": d, "k": k, "n": n, "rows": rows}
            for co in (False, True):
                stats, wall = [], []
                for i in range(args.warmup + args.steps):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    r = zset.enumerate_ex(n, g, out=None if co else out, k=k, count_only=co)
                    dt = time.perf_counter() - t
                    if i >= args.warmup:
                        stats.append(r.stats)
                        wall.append(dt)
                med = float(np.median(wall))
                wus = float(np.median([x["write_us"] for x in stats]))
                key = "count_only" if co else "materialise"
                rec[key] = {"rows_per_s": rows / med, "ms": round(med * 1e3, 3),
                            "write_us": round(wus, 1),
                            "memo_us": round(float(np.median([x["memo_us"] for x in stats])), 1),
                            "count_us": round(float(np.median([x["count_us"] for x in stats])), 1)}
                if co:
                    rec[key]["checksum"] = f"{r.checksum:016x}"
                else:
                    rec[key]["write_gbs"] = round(rows * d * 4 / (wus * 1e-6) / 1e9, 1)
                    rec["memo_rows"] = stats[-1]["memo_rows"]
                    rec["memo_bytes"] = stats[-1]["memo_bytes"]
                    rec["rows_per_tile"] = stats[-1]["rows_per_tile"]
            print(f"# sweep d={d} k={k}: {rec}", file=sys.stderr, flush=True)
            table.append(rec)
        del out
        torch.cuda.empty_cache()
    best = max(table, key=lambda r: r["materialise"]["rows_per_s"])
    line = {
        "metric": "Z(n) factorizations/s emitted (bit-exact), memo-dimension sweep",
        "value": best["materialise"]["rows_per_s"], "unit": "factorizations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": best["materialise"]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "sweep: d = 5, 7, 9 (generators in [10, 200], |Z| ~ 3.16e8 each), "
                               "k = 0..3, materialised and count-only (value: the best)"},
        "sweep": table,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.workload in ("batch", "serve"):
        # One hardware queue per server slot (HIP maps streams onto
        # GPU_MAX_HW_QUEUES queues, 4 by default, which caps how many queries
        # run at once); it must be set before the runtime starts.
        # An inherited smaller value is raised.
        want = min(32, max(4, args.slots))
        have = os.environ.get("GPU_MAX_HW_QUEUES", "")
        if not have.isdigit() or int(have) < want:
            os.environ["GPU_MAX_HW_QUEUES"] = str(want)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the enumeration shards by rank ranges with no "
              "communication, and this build runs on a single MI355X (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "memo":
        run_memo(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "walk":
        run_walk(args)
        return
    if args.workload == "sweep" and args.k is None:
        run_sweep(args)
        return

    import torch

    from paper_2407_20474_amd import inputs, zset

    w = inputs.load_workloads()
    if args.workload == "large":
        item = w["large"][args.seed]
        n, g, k = item["n"], item["gens"], item["k"]
    elif args.workload == "sweep":
        item = next(x for x in w["sweep"] if len(x["gens"]) == args.sweep_d)
        n, g, k = item["n"], item["gens"], 2
    else:
        item = w["plain"]
        n, g, k = item["n"], item["gens"], item["k"]
    if args.k is not None:
        k = args.k
    d = len(g)
    rows = zset.count(n, g)
    assert rows == item["rows"], "count disagrees with the stored workload"
    out = None
    if not args.count_only:
        out = torch.empty((rows, d), dtype=torch.int32, device="cuda")

    def step():
        return zset.enumerate_ex(n, g, out=out, k=k, rows_per_tile=args.rows_per_tile,
                                 count_only=args.count_only)

    # Queued steps (zset_enumerate_async): each call enqueues the whole path
    # (count table and memo, slice plan and memo layout, write pass, outcome
    # word) and returns; the host waits once after the last one.  Only the
    # three-launch form queues (k = 1 or 2, default slices, n + 1 <= 16384);
    # other workloads time synchronous calls.
    queued = (not args.sync_steps and args.rows_per_tile == 0 and k in (1, 2)
              and n + 1 <= 16384)
    results = torch.zeros((max(args.steps, args.warmup, 1), 4), dtype=torch.int64).pin_memory()
    wev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]

    def queue(i, events=None):
        zset.enumerate_async(n, g, out, results[i], k=k, count_only=args.count_only,
                             write_events=events)

    def outcomes():
        # Every queued step's outcome: |Z(n)| rows (and the checksum when
        # count-only) or the error it found.
        got = {zset.async_outcome(results[i]) for i in range(args.steps)}
        assert len(got) == 1 and next(iter(got))[0] == rows, got
        results.fill_(-1)

    for i in range(args.warmup):
        step()
        if queued:
            queue(i)
            torch.cuda.synchronize()
            zset.async_outcome(results[i])
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        if queued:
            queue(i)
        else:
            stats.append(step().stats)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = rows / (dt / args.steps)
    if queued:
        outcomes()
        # The write pass's duration: the same queued steps again, each with a
        # pair of HIP events around its write pass (recorded on the call's
        # stream by the library).  Event markers between launches idle the
        # device for a few microseconds each, so the steps above carry none.
        t1 = time.perf_counter()
        for i in range(args.steps):
            queue(i, wev[i])
        torch.cuda.synchronize()
        ms_events = (time.perf_counter() - t1) * 1e3 / args.steps
        outcomes()
        write_list = [a.elapsed_time(b) * 1e3 for a, b in wev]
        # The per-stage times come from synchronous calls (timing events
        # inside the call, a host wait per call).
        t1 = time.perf_counter()
        for _ in range(args.steps):
            stats.append(step().stats)
        torch.cuda.synchronize()
        ms_sync = (time.perf_counter() - t1) * 1e3 / args.steps

    def avg(key):
        return sum(s[key] for s in stats) / len(stats)

    write_us = sum(write_list) / len(write_list) if queued else avg("write_us")
    bytes_written = rows * d * 4
    stages = {key: round(avg(key), 2) for key in
              ("count_us", "memo_us", "plan_us", "write_us", "total_us")}
    if k == 2:
        # The library builds two-coordinate memos in closed form; the paper's
        # recurrence (Lemma 2.3 in elementwise batches) is timed here beside
        # the step, on the same call, as its memo stage.
        os.environ["ZSET_MEMO_PATH"] = "chain"
        step()  # warm-up: the first call on this path sets up its side stream's launches
        rec = [step().stats["memo_us"] for _ in range(3)]
        del os.environ["ZSET_MEMO_PATH"]
        stages["memo_recurrence_us"] = round(sum(rec) / len(rec), 2)
    ceiling = None
    if out is not None:
        # Measured store ceiling: the library's store-only kernels (16-byte
        # non-temporal stores, the write pass's store form; the fastest of
        # three launch shapes) over the same buffer.
        us = zset.store_ceiling(out, reps=5)
        ceiling = round(out.numel() * 4 / (us * 1e-6) / 1e9, 1)
    if args.count_only:
        # Count-only is integer-ALU bound: FNV-1a over 8 + 4d bytes per row,
        # 6 lane-ops per byte as compiled for gfx950 (byte extraction, xor,
        # shift, v_mad_u64_u32, v_mul_lo_u32, v_add3_u32: h x (2^40 + 0x1b3)).
        # The committed counters give the issued VALU fraction (row generation
        # included) for the large workload.
        ops = rows * (8 + 4 * d) * 6
        roof = {"bound": "alu", "achieved": round(ops / (write_us * 1e-6) / 1e12, 3),
                "peak": ALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                "frac": round((ops / (write_us * 1e-6)) / ALU_PEAK_OPS, 4), "traffic": None,
                "kernel": "k_write (count-only)", "algorithmic_ops_per_launch": ops}
        if args.workload == "large" and args.seed == 0:
            v = profile_field(ALU_COUNTERS, "valu_issue_frac_large")
            roof["valu_issue_frac_counted"] = float(v) if v is not None else None
    else:
        achieved = bytes_written / (write_us * 1e-6) / 1e9
        traffic = measured_traffic() if args.workload == "large" and args.seed == 0 else None
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": "k_write (write pass)",
                "algorithmic_bytes_per_launch": bytes_written}
    if queued:
        stages["write_us_queued"] = round(write_us, 2)
        stages["ms_per_step_write_events"] = round(ms_events, 4)
        stages["ms_per_step_synchronous"] = round(ms_sync, 4)
    line = {
        "metric": "Z(n) factorizations/s emitted (bit-exact)",
        "value": value,
        "unit": "factorizations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: Z(n={n}; g={tuple(g)}), d={d}, k={k}, "
                         f"|Z|={rows} rows of {d} uint32 ({bytes_written / 1e9:.2f} GB)"
                         + (", count-only" if args.count_only else "")),
            "rows": rows, "n": n, "gens": g, "k": k,
            "rows_per_tile": stats[-1]["rows_per_tile"], "tiles": stats[-1]["tiles"],
        },
        "stages_us": stages,
        "step_hbm_write_frac": round(bytes_written / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "store_ceiling_gbs": ceiling,
        "roofline": roof,
    }
    if args.calibrate:
        # A plain copy kernel of known size: 1 GiB read + 1 GiB written (an
        # elementwise kernel, so that it shows in the kernel counters).
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda").fill_(7)
        dst = torch.empty_like(src)
        torch.mul(src, 1, out=dst)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = src.numel() * 4
        del src, dst
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, g, args.cpu_sample_rows)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
