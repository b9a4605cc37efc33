#!/usr/bin/env python3
"""Benchmark: s-line graphs of non-uniform hypergraphs on one GPU.

Default workload (the largest one): the large skewed hypergraph at full
size, n = 5,000,000 vertices, m = 10,000,000 hyperedges, sizes
min(rint(LogNormal(1.5, 1)), 10,000), vertices drawn with weight ~
rank^-1.5 (seeded, synthetic), thresholds S = {8, 16} in one ensemble
pass. Its output (about 10^12 edges) is larger than device memory, so the
path is the streamed one: one step is one row range, of warmup + steps
ranges of equal 2-path work that together cover every row once, taken
through the whole path (pruning, work estimate, row-block plans, counting,
emit in chunks handed to a consumer) on inputs already resident in HBM.

Prints ONE JSON line. `value` is 2-paths traversed per second over the
timed steps; edges/s and the per-step latency percentiles ride along. The
`roofline` entry is for the dominant kernel, timed with HIP events on its
own stream inside the library, against the algorithmic bytes of the work it
does (4 B per 2-path read; 12 B per edge written for an emit pass);
`cpu_baseline` times the brute-force CPU oracle on a bounded row sample.
Other workloads (--workload): power_law (the whole output in memory),
dual, batched, served, components, preprocess.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

S_SET = [1, 2, 4, 8]
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2201_11326_amd", "csrc", "slg_kernels.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "heavy_tier_power_law_traffic.md")
METRIC = "2-paths traversed/sec + s-line edges/sec at 1 GPU; p50/p99 query latency"


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


DENSE_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "dense_tier_large_skewed_traffic.md")
DENSE_SQ_PROFILE = os.path.join(ROOT, "profiles", "dense_tier_large_skewed_sq_counters.md")
# count-store limit of the large skewed bench (GiB): half of it is the dense
# store, and a larger one cuts fewer row blocks (32 per range of 8.6e12
# 2-paths at 160 against 156 at 32; 7.26 against 7.58 s per range)
LARGE_STORE_GIB = 160.0


def measured_traffic(kernel: str, profile: str = TRAFFIC_PROFILE, work_per_launch: float = None):
    """HBM bytes per launch of `kernel` from the committed PMC summary, if it
    was taken on the current kernel source; else None. Where the summary
    states the 2-paths of its launches (a probe whose launches are smaller
    than the bench's), the bytes are scaled to `work_per_launch` 2-paths."""
    try:
        text = open(profile).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if not m_hash or m_hash.group(1) != kernel_source_hash():
        return None
    for block in text.split("kernel: ")[1:]:
        name = block.split("\n", 1)[0].strip()
        m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", block)
        if name == kernel and m_bytes:
            m_work = re.search(r"dense_two_paths_per_launch:\s*([0-9.eE+]+)", block)
            if m_work and work_per_launch:
                return float(m_bytes.group(1)) * work_per_launch / float(m_work.group(1))
            return float(m_bytes.group(1))
    return None


SQ_PROFILE = os.path.join(ROOT, "profiles", "heavy_tier_power_law_sq_counters.md")


def measured_sq(kernel: str, profile: str = None):
    """(waiting share of wave cycles, LDS bank-conflict rate) of `kernel` from
    the committed SQ-counter summary, if taken on the current kernel source."""
    try:
        text = open(profile or SQ_PROFILE).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if not m_hash or m_hash.group(1) != kernel_source_hash():
        return None
    for block in text.split("kernel: ")[1:]:
        if block.split("\n", 1)[0].strip() != kernel:
            continue
        w = re.search(r"SQ_WAIT_ANY / SQ_WAVE_CYCLES\):\s*([0-9.]+)", block)
        c = re.search(r"SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE\):\s*([0-9.]+)", block)
        if w and c:
            return {"waiting_share": float(w.group(1)), "lds_bank_conflict_rate": float(c.group(1))}
    return None


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def host_cpu() -> dict:
    """The host CPU as lscpu reports it (model, sockets x physical cores per
    socket, threads per core) plus the CPUs this process may use."""
    info = {"model": "unknown", "sockets": None, "cores_per_socket": None, "threads_per_core": None}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
                "Thread(s) per core": "threads_per_core"}
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                v = v.strip()
                info[keys[k.strip()]] = int(v) if v.isdigit() else v
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    if isinstance(info["sockets"], int) and isinstance(info["cores_per_socket"], int):
        info["physical_cores"] = info["sockets"] * info["cores_per_socket"]
    try:
        info["usable_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        info["usable_cpus"] = os.cpu_count()
    return info


# The paper's own CPU figures for this path (Section VI), quoted beside the
# oracle timing as context: they were measured on another machine and on
# datasets that are not available here, so they are not a target.
PAPER_CPU_CONTEXT = {
    "speedup": "5-31x for the hashmap-based algorithm (Algorithm 2) over the set-intersection "
               "heuristic (Algorithm 1), s = 8, cyclic partitioning, no relabelling (Web, LiveJournal)",
    "stage_times": "LiveJournal s-overlap stage 313.864 s (Algorithm 1) vs 12.085 s (Algorithm 2), 26x",
    "hardware": "2 x Intel Xeon Gold 6230 (20 cores per socket, 2.1 GHz, 28 MB L3), 188 GB RAM; "
                "C++17 with oneTBB 2020.3, GCC 10.2 -Ofast -march=native; thread count per table not stated",
}


def oracle_threads() -> int:
    """Threads the oracle may use: the usable CPUs, capped by OMP_NUM_THREADS."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return max(1, min(usable, int(os.environ.get("OMP_NUM_THREADS", "16") or 16)))


def heavy_roofline(stats, stages, profiled: bool = True):
    """The heavy tier's two kernels, each against the HBM roofline with the
    algorithmic bytes of the work it does: the counting pass reads one
    4-byte partner id per heavy 2-path; the emit pass writes 12 bytes
    (i, j, w) per heavy edge. The count store that carries the overlaps from
    one to the other is this implementation's own traffic, reported apart as
    overhead, never as algorithmic bytes. Returns the slower kernel's entry,
    with the other's under "other_heavy_kernel". `profiled`: the committed
    traffic and SQ summaries (taken on the power-law instance) apply."""
    store = stats.get("stored_ranks", 0) > 0
    kernels = {
        "count_heavy": ("heavy_kernel<false, false, true>" if store else "heavy_kernel<false, false, false>",
                        4 * stats["heavy_two_paths"],
                        {"count_store_written": 4 * stats["stored_ranks"]} if store else {}),
        "emit_heavy": ("heavy_store_emit_kernel<4, false>" if store else "heavy_kernel<true, false, false>",
                       12 * stats["heavy_edges"],
                       {"count_store_read": 4 * stats["stored_ranks"]} if store
                       else {"two_paths_walked_again": 4 * stats["heavy_two_paths"]}),
    }
    lines = {}
    for stage, (kname, algo_bytes, overhead) in kernels.items():
        launches, ms = stages.get(stage, (0, 0.0))
        avg_s = ms / 1e3 / max(launches, 1)
        achieved = algo_bytes / avg_s / 1e9 if avg_s > 0 else None
        lines[stage] = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": (achieved / PEAK_HBM_GBS) if achieved else None,
                        "traffic": measured_traffic(kname) if profiled else None, "kernel": f"{kname} ({stage})",
                        "avg_launch_ms": avg_s * 1e3, "algorithmic_bytes_per_launch": algo_bytes,
                        "overhead_bytes_per_launch": overhead,
                        "sq_counters": measured_sq(kname) if profiled else None}
    dominant = max(lines, key=lambda k: lines[k]["avg_launch_ms"])
    roofline = dict(lines[dominant])
    roofline["other_heavy_kernel"] = lines["emit_heavy" if dominant == "count_heavy" else "count_heavy"]
    return roofline


def cpu_baseline(inc, seconds: float, s_set=None, size_min=None, seed: int = 7):
    """Oracle on a random row sample sized to about `seconds` of CPU time.
    Rate = 2-paths of the sampled rows (the work the two-hop traversal does
    for them at the smallest s) / oracle wall time for every s of the set."""
    import numpy as np

    import oracle
    s_set = list(S_SET if s_set is None else s_set)
    size_min = s_set[0] if size_min is None else size_min
    threads = oracle_threads()
    rng = np.random.default_rng(seed)
    probe = np.sort(rng.choice(inc.m, size=4 * threads, replace=False))
    t0 = time.perf_counter()
    for s in s_set:
        oracle.line_graph_rows(inc, s, probe, size_min=size_min, threads=threads)
    per_row = (time.perf_counter() - t0) / probe.size
    nrows = int(max(threads, min(inc.m, seconds / max(per_row, 1e-9))))
    rows = np.sort(rng.choice(inc.m, size=nrows, replace=False))
    t0 = time.perf_counter()
    for s in s_set:
        oracle.line_graph_rows(inc, s, rows, size_min=size_min, threads=threads)
    dt = time.perf_counter() - t0
    work = int(oracle.row_two_paths(inc, size_min, rows, threads=threads).sum())
    return {"value": work / dt, "unit": "2-paths/s", "cores": threads, "kind": "oracle",
            "sample": f"{nrows} random rows (seed {seed}) of the same hypergraph, all of S={s_set}, "
                      f"{work} 2-paths, {dt:.2f} s wall", "host": host_cpu(),
            "paper": PAPER_CPU_CONTEXT}


def batched_cpu_baseline(members, seconds: float, seed: int = 7):
    """Oracle on whole member graphs, taken in a seeded random order until
    about `seconds` of CPU time; rate = their 2-paths / oracle wall time."""
    import numpy as np

    import oracle
    threads = oracle_threads()
    order = np.random.default_rng(seed).permutation(len(members))
    work, dt, used = 0, 0.0, 0
    for g in order:
        inc, s = members[g].inc, members[g].s
        t0 = time.perf_counter()
        oracle.line_graph(inc, s, threads=threads)
        dt += time.perf_counter() - t0
        work += oracle.two_paths(inc, s)
        used += 1
        if dt >= seconds:
            break
    return {"value": work / dt, "unit": "2-paths/s", "cores": threads, "kind": "oracle",
            "sample": f"{used} of {len(members)} member graphs (seeded order {seed}), each at its own s, "
                      f"{work} 2-paths, {dt:.2f} s wall", "host": host_cpu(),
            "paper": PAPER_CPU_CONTEXT}


def served_cpu_baseline(pool, reqs, seconds: float, seed: int = 7):
    """Oracle on whole queries of the served stream on its small members (the
    full-size power-law members would take the brute-force oracle minutes per
    query), taken in a seeded random order until about `seconds` of CPU time
    (each query: every s of its set over the whole graph); rate = their
    2-paths / oracle wall time."""
    import numpy as np

    import oracle
    threads = oracle_threads()
    order = np.random.default_rng(seed).permutation(len(reqs))
    work, dt, used = 0, 0.0, 0
    for r in order:
        q = reqs[int(r)]
        inc = pool[q.graph]
        if inc.m > 20_000:
            continue
        t0 = time.perf_counter()
        for s in q.s:
            oracle.line_graph(inc, s, size_min=q.s[0], threads=threads)
        dt += time.perf_counter() - t0
        work += oracle.two_paths(inc, q.s[0])
        used += 1
        if dt >= seconds:
            break
    return {"value": work / dt, "unit": "2-paths/s", "cores": threads, "kind": "oracle",
            "sample": f"{used} of {len(reqs)} requests (seeded order {seed}) on the large-skewed-generator "
                      f"members, every s of each set over the whole graph, {work} 2-paths, {dt:.2f} s wall", "host": host_cpu(), "paper": PAPER_CPU_CONTEXT}


def bench_batched(args) -> int:
    """256 hypergraphs of uneven size, each with its own s. Compares, in
    aggregate 2-paths/s over the same member set: (a) per-instance one-shot
    calls of the plain path, one graph after another; (b) building the batch
    from scratch every step (disjoint union, one plan, one emit); (c) replays
    of the captured HIP graph of the whole batched device path. `value` is
    (c), the batched form; (a) and (b) ride along."""
    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg
    from paper_2201_11326_amd import autotune

    t_gen = time.perf_counter()
    members = hg.batched_family()
    t_gen = time.perf_counter() - t_gen
    ctx = slg.Context(0)
    graphs = [ctx.register_incidence(mb.inc) for mb in members]
    svals = [mb.s for mb in members]
    torch.cuda.synchronize()
    note = lambda msg: print(f"[bench batched] {msg}", file=sys.stderr, flush=True)
    note(f"generated and registered {len(graphs)} graphs in {t_gen:.1f} s")

    tuning, tune_times = (0, 0, 0), {}
    if not args.no_tune:
        tuning, tune_times = autotune.tune_batch(ctx, graphs, svals, use_cache=False)
        note(f"tuned: {tuning}")

    def per_instance():
        outs = [ctx.line_graph(g, [s]) for g, s in zip(graphs, svals)]
        torch.cuda.synchronize()
        return outs

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        lat = []
        for _ in range(steps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t)
        return lat

    # (a) per-instance launches of the plain path
    outs = per_instance()
    work = sum(o[0].two_paths for o in outs)
    edges = sum(o[0].num_edges for o in outs)
    del outs
    lat_a = timed(per_instance, args.steps, args.warmup)
    note("per-instance timed")

    # (b) batch built from scratch each step
    def create_step():
        b = ctx.batch(graphs, svals)
        torch.cuda.synchronize()
        b.destroy()
    lat_b = timed(create_step, args.steps, args.warmup)
    note("batch create timed")

    # (c) HIP-graph replay of the whole batched device path
    b = ctx.batch(graphs, svals)
    info = b.info()
    assert info["two_paths"] == work and info["edges"] == edges, (info, work, edges)
    lat_c = timed(lambda: b.run(use_graph=True), args.steps, args.warmup)
    lat_e = timed(lambda: b.run(use_graph=False), args.steps, args.warmup)
    ctx.reset_timing()
    ctx.set_timing(True)
    for _ in range(args.steps):
        b.run(use_graph=False)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    stages = ctx.timing()
    note("replays timed")

    # parity spot check of a few members against the oracle (untimed)
    import numpy as np

    import oracle
    rng = np.random.default_rng(3)
    checked = []
    for gi in rng.choice(len(members), size=4, replace=False):
        res = b.result(int(gi))
        ref = oracle.line_graph(members[gi].inc, members[gi].s)
        got = (res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), res.w.cpu().numpy())
        ok = (np.array_equal(got[0], ref.row_ptr) and np.array_equal(got[1], ref.j)
              and np.array_equal(got[2], ref.w))
        if not ok:
            print(f"batched parity FAILED on member {gi}", file=sys.stderr)
            return 1
        checked.append(int(gi))
    b.destroy()

    total = lambda lat: sum(lat)
    rate = lambda lat: work * len(lat) / total(lat)
    ms_c = 1e3 * total(lat_c) / len(lat_c)
    nnz = sum(mb.inc.nnz for mb in members)
    rows = sum(mb.inc.m for mb in members)
    nv = sum(mb.inc.n for mb in members)
    step_bytes = 4 * work + 8 * nnz + 8 * (rows + nv) + 12 * edges + 8 * (rows + 1)
    achieved = step_bytes / (ms_c / 1e3) / 1e9
    cpu = None if args.no_cpu_baseline else batched_cpu_baseline(members, args.cpu_seconds)
    line = {
        "metric": METRIC, "value": rate(lat_c), "unit": "2-paths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_c, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batched: 256 hypergraphs, m log-uniform [1e3, 2e5], n=2m, "
                               "|e|~min(Zipf(2.1), 1000), own s ~ U{1..8}",
                   "graphs": len(members), "rows": rows, "nnz": nnz, "seed": hg.BASE_SEED + 4,
                   "tuning": {"light_max": tuning[0], "slot_work": tuning[1], "heavy_grid": tuning[2]},
                   "parallelism": "single GPU"},
        "two_paths_per_step": work, "edges_per_step": edges,
        "edges_per_s": edges * len(lat_c) / total(lat_c),
        "p50_ms": 1e3 * percentile(lat_c, 0.5), "p99_ms": 1e3 * percentile(lat_c, 0.99),
        "per_instance": {"value": rate(lat_a), "ms_per_step": 1e3 * total(lat_a) / len(lat_a),
                         "p50_ms": 1e3 * percentile(lat_a, 0.5), "p99_ms": 1e3 * percentile(lat_a, 0.99)},
        "batch_create": {"value": rate(lat_b), "ms_per_step": 1e3 * total(lat_b) / len(lat_b),
                         "p50_ms": 1e3 * percentile(lat_b, 0.5), "p99_ms": 1e3 * percentile(lat_b, 0.99)},
        "eager_replay": {"value": rate(lat_e), "ms_per_step": 1e3 * total(lat_e) / len(lat_e)},
        "speedup_vs_per_instance": rate(lat_c) / rate(lat_a),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "whole batched step (HIP-graph replay)", "avg_launch_ms": ms_c,
                     "algorithmic_bytes_per_launch": step_bytes},
        "stage_ms_per_step": {k: v[1] / args.steps for k, v in stages.items()},
        "tune_ms": {str(k): 1e3 * v for k, v in tune_times.items()},
        "parity_checked_members": checked, "cpu_baseline": cpu, "generate_s": t_gen,
    }
    print(json.dumps(line), flush=True)
    for g in graphs:
        g.release()
    ctx.close()
    return 0


def bench_served(args) -> int:
    """Request loop over a device-resident pool (64 large-skewed-generator
    graphs + 4 power-law-generator graphs) answering s-set queries drawn from
    {1,2,3,4,5,8}. Three runs over the same request list: (a) per-instance
    plain calls one after another (service times; FIFO latency under the
    Poisson arrivals derived from them); (b) the server fed at the Poisson
    arrival times (p50/p99 latency, achieved rate); (c) the server given every
    request at once (capacity). `value` is (c) in 2-paths/s."""
    import threading

    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg

    note = lambda msg: print(f"[bench served] {msg}", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    pool = hg.served_pool()
    reqs = hg.served_requests(len(pool), args.requests, rate=args.rate)
    t_gen = time.perf_counter() - t_gen
    ctx = slg.Context(0)
    graphs = [ctx.register_incidence(x) for x in pool]
    torch.cuda.synchronize()
    note(f"pool of {len(pool)} graphs, {len(reqs)} requests generated in {t_gen:.1f} s")

    # (a) per-instance plain calls, arrival order, back to back
    for q in reqs[:32]:
        outs = ctx.line_graph(graphs[q.graph], q.s)
        torch.cuda.synchronize()
        del outs
    service, work_of, bytes_of = [], [], []
    for q in reqs:
        t = time.perf_counter()
        outs = ctx.line_graph(graphs[q.graph], q.s)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t)
        work_of.append(outs[0].two_paths)
        x = pool[q.graph]
        # the scope table's algorithmic bytes of one query: 4 B per 2-path,
        # 8 B per incidence (both CSRs), 8 B per pointer, 12 B per edge,
        # 8 B per row_ptr entry of every threshold
        bytes_of.append(4 * outs[0].two_paths + 8 * x.nnz + 8 * (x.m + x.n)
                        + sum(12 * o.num_edges for o in outs) + 8 * (x.m + 1) * len(q.s))
        del outs
    work = sum(work_of)
    algo_bytes = sum(bytes_of)
    finish, lat_a = 0.0, []
    for q, sv in zip(reqs, service):  # one FIFO server, same arrivals
        finish = max(q.arrival, finish) + sv
        lat_a.append(finish - q.arrival)
    note(f"per-instance: {1e3 * sum(service):.1f} ms of service for {len(reqs)} requests")

    def serve(paced: bool):
        srv = ctx.server(workers=args.workers, mem_budget_bytes=int(args.budget_gb * (1 << 30)))
        done = []

        def collect():
            for _ in range(len(reqs)):
                r = srv.next(timeout_ms=120_000, keep=False)
                done.append((time.perf_counter(), r))
                if r is None:  # nothing ended for two minutes: give up
                    break
        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for q in reqs:
            if paced:
                dt = t0 + q.arrival - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            srv.submit(graphs[q.graph], q.s)
        th.join()
        stats = srv.stats()
        srv.close()
        bad = [r for _, r in done if r is None or not r.ok]
        if bad:
            raise RuntimeError(f"{len(bad)} served queries failed: {bad[0] and bad[0].message}")
        if len(done) != len(reqs):
            raise RuntimeError(f"only {len(done)} of {len(reqs)} served queries ended")
        span = max(t for t, _ in done) - t0
        return span, [r.latency_ms for _, r in done], sum(r.two_paths for _, r in done), stats

    span_b, lat_b, work_b, stats_b = serve(paced=True)
    note(f"paced run: {span_b:.2f} s")
    span_c, lat_c, work_c, stats_c = serve(paced=False)
    note(f"burst run: {span_c:.2f} s")
    assert work_b == work and work_c == work, (work, work_b, work_c)

    # untimed parity spot check: a mix through the server against the same
    # queries alone, and against the oracle where the graph is small
    import numpy as np

    import oracle
    rng = np.random.default_rng(9)
    pick = [reqs[int(i)] for i in rng.choice(len(reqs), size=16, replace=False)]
    srv = ctx.server(workers=args.workers)
    tick = {srv.submit(graphs[q.graph], q.s): q for q in pick}
    checked = 0
    for _ in pick:
        r = srv.next(timeout_ms=300_000)
        q = tick[r.ticket]
        alone = ctx.line_graph(graphs[q.graph], q.s)
        for a, b in zip(r.outs, alone):
            for f in ("row_ptr", "col", "w"):
                if not torch.equal(getattr(a, f), getattr(b, f)):
                    print(f"served parity FAILED: graph {q.graph} s={q.s} {f}", file=sys.stderr)
                    return 1
            if pool[q.graph].m <= 10_000:
                ref = oracle.line_graph(pool[q.graph], a.s)
                if not (np.array_equal(a.row_ptr.cpu().numpy(), ref.row_ptr)
                        and np.array_equal(a.col.cpu().numpy(), ref.j)
                        and np.array_equal(a.w.cpu().numpy(), ref.w)):
                    print(f"served oracle parity FAILED: graph {q.graph} s={a.s}", file=sys.stderr)
                    return 1
        checked += 1
        del r, alone
    srv.close()

    pct = lambda xs, q: percentile(xs, q)
    achieved = algo_bytes / span_c / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "kernel": "every kernel of the served run given all requests at once (burst)",
                "algorithmic_bytes": algo_bytes, "span_s": span_c}
    cpu = None if args.no_cpu_baseline else served_cpu_baseline(pool, reqs, args.cpu_seconds)
    line = {
        "metric": METRIC, "value": work / span_c, "unit": "2-paths/s", "n_gpus": 1, "steps": 1,
        "warmup": 32, "ms_per_step": 1e3 * span_c, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"served: {len(pool)} resident graphs (64 large-skewed-generator, m log-uniform "
                               f"[1e3, 1e4], n=m/2; 4 power-law-generator at full size, n=1e6, m=5e5), {len(reqs)} "
                               f"Poisson requests at {args.rate:g}/s, s-sets of 1-6 from {{1,2,3,4,5,8}}",
                   "workers": args.workers, "budget_gb": args.budget_gb, "seed": hg.BASE_SEED + 5,
                   "parallelism": "single GPU"},
        "two_paths_total": work,
        "p50_ms": pct(lat_b, 0.5), "p99_ms": pct(lat_b, 0.99),
        "paced": {"rate_2paths_per_s": work / span_b, "span_s": span_b, "p50_ms": pct(lat_b, 0.5),
                  "p99_ms": pct(lat_b, 0.99), "yields": stats_b.get("yields"),
                  "peak_bytes": stats_b.get("bytes_peak")},
        "burst": {"rate_2paths_per_s": work / span_c, "span_s": span_c, "p50_ms": pct(lat_c, 0.5),
                  "p99_ms": pct(lat_c, 0.99), "peak_bytes": stats_c.get("bytes_peak")},
        "per_instance": {"rate_2paths_per_s": work / sum(service), "service_s": sum(service),
                         "service_p50_ms": 1e3 * pct(service, 0.5), "service_p99_ms": 1e3 * pct(service, 0.99),
                         "fifo_p50_ms": 1e3 * pct(lat_a, 0.5), "fifo_p99_ms": 1e3 * pct(lat_a, 0.99)},
        "speedup_vs_per_instance": (work / span_c) / (work / sum(service)),
        "parity_checked_requests": checked, "generate_s": t_gen, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    for g in graphs:
        g.release()
    ctx.close()
    return 0


def components_cpu_baseline(inc, seconds: float, seed: int = 7):
    """The oracle's s-connected components (breadth-first search over an
    edge list) on its own L_1 edges of a seeded random row sample, grown
    fourfold until the search takes a second (or a quarter of `seconds`);
    rate = edges searched per second."""
    import numpy as np

    import oracle
    threads = oracle_threads()
    rng = np.random.default_rng(seed)
    nrows, dt, ne = 1000, 0.0, 0
    while True:
        rows = np.sort(rng.choice(inc.m, size=min(nrows, inc.m), replace=False))
        sub = oracle.line_graph_rows(inc, 1, rows, threads=threads)
        ends_i = np.repeat(sub.rows, np.diff(sub.ptr)).astype(np.int32)
        t0 = time.perf_counter()
        oracle.components(inc, 1, ends_i, sub.j)
        dt = time.perf_counter() - t0
        ne = int(sub.j.size)
        if dt >= min(seconds / 4, 1.0) or nrows >= inc.m:  # the oracle's construction costs ten times more
            break
        nrows *= 4
    return {"value": ne / dt, "unit": "s-line edges/s (components)", "cores": 1, "kind": "oracle",
            "sample": f"the oracle's L_1 edges of {rows.size} random rows (seed {seed}): {ne} edges, "
                      f"breadth-first search {dt:.2f} s wall (single thread)", "host": host_cpu()}


def bench_components(args) -> int:
    """s-connected components, ID squeezing and the symmetric CSR (the
    framework's stages after construction, Section IV) on the power-law
    instance's L_s for every s of S = {1,2,4,8}. value = s-line edges consumed
    per second by the component search; the squeeze and symmetric-CSR rates
    ride along. Inputs (the emitted L_s) are on the device before timing
    starts."""
    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg

    inc = hg.power_law()
    ctx = slg.Context(0)
    g = ctx.register_incidence(inc)
    outs = ctx.line_graph(g, S_SET)
    torch.cuda.synchronize()
    edges = [lg.num_edges for lg in outs]
    res = {}
    for _ in range(args.warmup):
        for lg in outs:
            ctx.components(g, lg.s, lg)
            ctx.squeeze(inc.m, lg)
            sym = ctx.symmetrize(lg)
            del sym
    torch.cuda.synchronize()
    t_cc = t_sq = t_sym = 0.0
    counts = {}
    for _ in range(args.steps):
        for lg in outs:
            t0 = time.perf_counter()
            _, nc = ctx.components(g, lg.s, lg)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, nk = ctx.squeeze(inc.m, lg)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            sym = ctx.symmetrize(lg)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            del sym
            t_cc += t1 - t0
            t_sq += t2 - t1
            t_sym += t3 - t2
            counts[lg.s] = {"components": nc, "squeezed": nk}
    total = sum(edges) * args.steps
    # the union-find: 8 B read per edge (its two ends), 4 B written per row
    # at the start and 4 B read + 4 B written per row at the end; the label
    # reads of the finds depend on the trees and are not counted. Timed on the
    # host around each call (three launches and a count read back), so the
    # fraction is a lower bound for the kernels.
    cc_bytes = (8 * sum(edges) + 12 * inc.m * len(edges)) * args.steps
    cc_gbs = cc_bytes / t_cc / 1e9
    roofline = {"bound": "hbm", "achieved": cc_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": cc_gbs / PEAK_HBM_GBS, "traffic": None,
                "kernel": "cc_init_kernel + cc_hook_kernel + cc_finish_kernel (components, host-timed)",
                "algorithmic_bytes_per_call": cc_bytes / (args.steps * len(edges))}
    cpu = None if args.no_cpu_baseline else components_cpu_baseline(inc, args.cpu_seconds)
    line = {
        "metric": METRIC, "value": total / t_cc, "unit": "s-line edges/s (components)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_cc / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "s-connected components, ID squeezing and symmetric CSR of the power-law "
                               "instance's L_s, "
                               "S={1,2,4,8}", "s": S_SET, "edges": edges, "parallelism": "single GPU"},
        "squeeze_edges_per_s": total / t_sq, "squeeze_ms_per_step": 1e3 * t_sq / args.steps,
        "symmetric_edges_per_s": total / t_sym, "symmetric_ms_per_step": 1e3 * t_sym / args.steps,
        "per_s": counts, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    del outs
    g.release()
    ctx.close()
    return 0


def ascending_incidence(inc):
    """The hypergraph relabelled by ascending size, built by the oracle (for
    the CPU baseline of the preprocessing line)."""
    import hypergen as hg
    import oracle
    he_ptr, he_idx, v_ptr, v_idx = oracle.select(inc, oracle.relabel_order(inc))
    return hg.Incidence(inc.m, inc.n, he_ptr, he_idx, v_ptr, v_idx)


def bench_preprocess(args) -> int:
    """The framework's optional preprocessing (Section IV, Stages 1-2) on the
    power-law instance: relabel-by-degree (ascending, descending) and the
    simplification to toplexes, and what relabelling does to the ensemble
    construction S = {1,2,4,8} on the GPU (the paper relabels to balance CPU
    threads). value = 2-paths/s of the construction on the ascending
    relabelling; the original order's rate rides along."""
    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg

    inc = hg.power_law()
    ctx = slg.Context(0)
    g = ctx.register_incidence(inc)
    torch.cuda.synchronize()

    def timed(fn, reps):
        ts = []
        out = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2] * 1e3, out

    stage_times = {}

    def construction(graph, name):
        for _ in range(args.warmup):
            outs = ctx.line_graph(graph, S_SET)
            del outs
        ctx.reset_timing()
        ctx.set_timing(True)
        ms, outs = timed(lambda: ctx.line_graph(graph, S_SET), args.steps)
        ctx.set_timing(False)
        stage_times[name] = ctx.timing()
        two_paths = outs[0].two_paths
        del outs
        return ms, two_paths

    res = {}
    res["original_ms"], W = construction(g, "original")
    for desc in (False, True):
        name = "descending" if desc else "ascending"
        timed(lambda: ctx.relabel(g, desc), args.warmup)
        rl_ms, (sub, _) = timed(lambda: ctx.relabel(g, desc), args.steps)
        res[f"relabel_{name}_ms"] = rl_ms
        res[f"{name}_ms"], _ = construction(sub, name)
        if not desc:  # the roofline of the line's construction (ascending order)
            p = ctx.plan(sub, S_SET)
            asc_stats = p.stats()
            p.destroy()
        sub.release()
    l1 = ctx.line_graph(g, [1])[0]
    timed(lambda: ctx.simplify(g, l1), args.warmup)
    sim_ms, (simple, ids) = timed(lambda: ctx.simplify(g, l1), args.steps)
    res["simplify_ms"] = sim_ms
    res["toplexes"] = int(ids.numel())
    simple.release()
    del l1
    line = {
        "metric": METRIC, "value": W / (res["ascending_ms"] * 1e-3), "unit": "2-paths/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ascending_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "relabel-by-degree and toplex simplification of the power-law hypergraph "
                               "n=1e6 m=5e5; ensemble S={1,2,4,8} on each order", "s": S_SET,
                   "parallelism": "single GPU"},
        "original_two_paths_per_s": W / (res["original_ms"] * 1e-3), "stages_ms": res,
        "roofline": heavy_roofline(asc_stats, stage_times["ascending"], profiled=False),
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(ascending_incidence(inc), args.cpu_seconds),
    }
    print(json.dumps(line), flush=True)
    g.release()
    ctx.close()
    return 0


def bench_large_skewed(args) -> int:
    """The large skewed workload at full size: n = 5e6 vertices, m = 1e7
    hyperedges, |e| = min(rint(LogNormal(1.5, 1)), 1e4), vertex weight ~
    rank^-1.5, ensemble S = {8, 16}. Its output (about 1e12 edges) exceeds
    device memory, so it is streamed (slg_line_graph_stream_rows): one step
    is one of warmup + steps row ranges of equal 2-path work at s = 8, which
    together cover every row once, taken through the whole path (pruning,
    work estimate, row-block plans, counting, emit in chunks of <= 8 GiB by default).
    The consumer counts each chunk's edges (--digest: digests each chunk on
    the device). value = 2-paths of the timed ranges / their wall time."""
    import numpy as np
    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg

    S = [8, 16]
    note = lambda msg: print(f"[bench large_skewed] {msg}", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    inc = hg.large_skewed()
    t_gen = time.perf_counter() - t_gen
    note(f"generated in {t_gen:.1f} s: nnz {inc.nnz}")
    ctx = slg.Context(0)
    if args.dense_ratio is not None:
        ctx.set_dense(args.dense_ratio, 0)
    ctx.set_count_store(int(args.store_gib * (1 << 30)))
    g = ctx.register_incidence(inc)
    prefix = ctx.work_prefix(g, S[0])  # untimed: the ranges' cuts
    W = int(prefix[-1])
    B = args.steps + args.warmup
    cuts = [0] + [int(np.searchsorted(prefix, W * b // B, side="left")) for b in range(1, B)] + [inc.m]
    chunk = int(args.chunk_gib * (1 << 30))
    edges = [0] * len(S)
    chunks = [0]

    def on_chunk(k, s, r0, r1, e0, row_ptr, row, col, w):
        if args.digest:
            ctx.digest(row, col, w)
        edges[k] += int(col.numel())
        chunks[0] += 1
        return False

    def step(b):
        ctx.line_graph_stream(g, S, chunk, on_chunk, rows=(cuts[b], cuts[b + 1]))
        torch.cuda.synchronize()

    for b in range(args.warmup):
        step(b)
        note(f"warmup range {b + 1}/{args.warmup} done")
    edges[:] = [0] * len(S)
    chunks[0] = 0
    ctx.reset_timing()
    ctx.set_timing(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(args.warmup, B):
        ts = time.perf_counter()
        step(b)
        lat.append(time.perf_counter() - ts)
        note(f"range {b + 1 - args.warmup}/{args.steps}: {1e3 * lat[-1]:.0f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    stages = ctx.timing()
    work = ctx.work()
    timed_two_paths = int(prefix[cuts[B]] - prefix[cuts[args.warmup]])
    assert work["two_paths"] == timed_two_paths, (work, timed_two_paths)
    assert sum(edges) == work["edges"], (edges, work)
    ms_per_step = 1e3 * elapsed / args.steps
    # the dominant kernel: the dense tier's counting pass, 4 B read per
    # 2-path of its slots (algorithmic bytes, the scope table's unit)
    launches, count_ms = stages.get("count_dense", (0, 0.0))
    dense_bytes = 4 * work["dense_two_paths"]
    achieved = dense_bytes / (count_ms / 1e3) / 1e9 if count_ms > 0 else None
    emit_launches, emit_ms = stages.get("emit_dense", (0, 0.0))
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": measured_traffic("dense_kernel<false>", DENSE_TRAFFIC_PROFILE,
                                                                                     work["dense_two_paths"] / max(launches, 1)),
                "kernel": "dense_kernel<false> (count_dense)", "launches": launches,
                "avg_launch_ms": count_ms / max(launches, 1),
                "algorithmic_bytes_per_launch": dense_bytes / max(launches, 1),
                "overhead_bytes_per_launch": {"dense_store_written": 4 * work["dense_stored"] / max(launches, 1)},
                "sq_counters": measured_sq("dense_kernel<false>", DENSE_SQ_PROFILE),
                "note": "window-major order serves most of the 2-paths' bytes from L2, so the algorithmic "
                        "bytes can exceed what HBM delivers; `traffic` is the measured HBM bytes per launch",
                "emit": {"kernel": "heavy_store_emit_kernel<4, true> (emit_dense)",
                         "launches": emit_launches, "ms": emit_ms,
                         "algorithmic_bytes": 12 * work["dense_edges"],
                         "achieved_gbs": 12 * work["dense_edges"] / (emit_ms / 1e3) / 1e9 if emit_ms > 0 else None}}
    edges_total = sum(edges)
    nrows_timed = cuts[B] - cuts[args.warmup]
    step_bytes = (4 * timed_two_paths + 12 * edges_total
                  + args.steps * (8 * inc.nnz + 8 * (inc.m + inc.n)) + 8 * (nrows_timed + args.steps) * len(S))
    cpu = None if args.no_cpu_baseline else cpu_baseline(inc, args.cpu_seconds, S, size_min=S[0])
    line = {
        "metric": METRIC, "value": timed_two_paths / elapsed, "unit": "2-paths/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "large skewed hypergraph n=5e6 m=1e7 |e|=min(rint(LogNormal(1.5,1)),1e4) "
                               f"vertex weight~rank^-1.5, ensemble S={{8,16}}, streamed in chunks of <= {args.chunk_gib:g} GiB; "
                               f"one step = one of {B} row ranges of equal 2-path work (all of them: every row once)",
                   "n": inc.n, "m": inc.m, "nnz": inc.nnz, "s": S, "seed": hg.BASE_SEED + 3,
                   "ranges": B, "consumer": "on-device digest per chunk" if args.digest else "edge count per chunk",
                   "dense_ratio": args.dense_ratio, "count_store_gib": args.store_gib,
                   "parallelism": "single GPU"},
        "two_paths_per_step": timed_two_paths / args.steps, "two_paths_whole_graph": W,
        "edges_timed": edges, "edges_per_s": edges_total / elapsed,
        "p50_ms": 1e3 * percentile(lat, 0.5), "p99_ms": 1e3 * percentile(lat, 0.99),
        "step_roofline_frac": (step_bytes / elapsed) / (PEAK_HBM_GBS * 1e9),
        "stage_ms_per_step": {k: v[1] / args.steps for k, v in stages.items()},
        "work_timed": work, "chunks_timed": chunks[0],
        "roofline": roofline, "cpu_baseline": cpu, "generate_s": t_gen,
    }
    print(json.dumps(line), flush=True)
    g.release()
    ctx.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("large_skewed", "power_law", "dual", "batched", "served", "components",
                                           "preprocess"),
                    default="large_skewed",
                    help="large_skewed (default): the largest workload, n=5e6 m=1e7, S={8,16}, streamed in "
                         "row ranges of equal work; power_law: n=1e6 m=5e5, S={1,2,4,8}, output in memory; "
                         "dual: the s-clique graph of the power-law hypergraph; batched: 256 small "
                         "hypergraphs, each with its own s, as one disjoint-union batch; served: a request "
                         "loop; components: components, squeezing and symmetric CSR of the power-law L_s; "
                         "preprocess: relabel-by-degree and toplexes of the power-law hypergraph")
    ap.add_argument("--dense-ratio", type=int, default=None,
                    help="large_skewed: the dense tier's 2-paths per eight candidate partners (default: the library's)")
    ap.add_argument("--store-gib", type=float, default=LARGE_STORE_GIB,
                    help="large_skewed: count-store limit of the context in GiB; half of it is the dense "
                         "store whose room cuts the row blocks (the library's default: 32)")
    ap.add_argument("--chunk-gib", type=float, default=8.0,
                    help="large_skewed: largest streamed chunk (all thresholds), GiB")
    ap.add_argument("--digest", action="store_true",
                    help="large_skewed: digest every streamed chunk on the device (default: count its edges)")
    ap.add_argument("--no-tune", action="store_true", help="batched: library-default plan shape")
    ap.add_argument("--requests", type=int, default=4000, help="served: number of requests")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: Poisson arrivals per second")
    ap.add_argument("--workers", type=int, default=8, help="served: queries in flight")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="served: device-memory budget")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the s-line graph path here runs on a single MI355X "
              "(rows would shard across GPUs with no exchange). Use --gpus 1.",
              file=sys.stderr)
        return 2

    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "components":
        return bench_components(args)
    if args.workload == "preprocess":
        return bench_preprocess(args)
    if args.workload == "large_skewed":
        return bench_large_skewed(args)
    if args.workload == "dual":
        return bench_power_law(args, dual=True)
    return bench_power_law(args)


def bench_power_law(args, dual: bool = False) -> int:
    """The power-law workload (n = 1e6, m = 5e5, |e| ~ Zipf(2.1) on [2, 5000],
    vertex weight ~ rank^-0.8), ensemble S = {1, 2, 4, 8}, the whole output
    in device memory: one step is the whole path (pruning, 2-path work
    estimate, counting pass, prefix sums, output allocation, the emit pass
    writing every L_s as COO + CSR). With dual: the s-clique graph, i.e. the
    same path on the dual hypergraph (the CSRs swapped: vertices become
    hyperedges, Section II-A)."""
    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg

    t_gen = time.perf_counter()
    inc = hg.power_law()
    if dual:
        inc = inc.dual()
    t_gen = time.perf_counter() - t_gen
    ctx = slg.Context(0)
    g = ctx.register_incidence(inc)

    # shape of the plan (untimed): tier sizes for the roofline accounting
    p = ctx.plan(g, S_SET)
    stats = p.stats()
    edges = p.num_edges()
    two_paths = p.two_paths
    p.destroy()

    for _ in range(args.warmup):
        outs = ctx.line_graph(g, S_SET)
        del outs
    torch.cuda.synchronize()

    ctx.reset_timing()
    ctx.set_timing(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        outs = ctx.line_graph(g, S_SET)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        del outs
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    stages = ctx.timing()

    ms_per_step = 1e3 * elapsed / args.steps
    value = two_paths * args.steps / elapsed
    edges_total = sum(edges)

    roofline = heavy_roofline(stats, stages, profiled=not dual)  # the summaries are of the power-law instance
    # whole-step algorithmic bytes: 4 B per 2-path, 8 B per incidence (both
    # CSRs), 8 B per row/vertex pointer, 12 B per edge, 8 B per row_ptr entry
    step_bytes = (4 * two_paths + 8 * inc.nnz + 8 * (inc.m + inc.n) + 12 * edges_total
                  + 8 * (inc.m + 1) * len(S_SET))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inc, args.cpu_seconds)

    line = {
        "metric": METRIC, "value": value, "unit": "2-paths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": ("s-clique graph (s-line graph of the dual) of " if dual else "")
                               + "power-law hypergraph n=1e6 m=5e5 |e|~Zipf(2.1)[2,5000] "
                               "vertex weight~rank^-0.8, ensemble S={1,2,4,8}",
                   "n": inc.n, "m": inc.m, "nnz": inc.nnz, "s": S_SET, "seed": hg.BASE_SEED + 2,
                   "parallelism": "single GPU"},
        "two_paths_per_step": two_paths, "edges_per_step": edges, "edges_per_s": edges_total * args.steps / elapsed,
        "p50_ms": 1e3 * percentile(lat, 0.5), "p99_ms": 1e3 * percentile(lat, 0.99),
        "step_roofline_frac": (step_bytes / (ms_per_step / 1e3)) / (PEAK_HBM_GBS * 1e9),
        "stage_ms_per_step": {k: v[1] / args.steps for k, v in stages.items()},
        "roofline": roofline, "cpu_baseline": cpu,
        "plan": stats, "generate_s": t_gen,
    }
    print(json.dumps(line), flush=True)
    g.release()
    ctx.close()
    return 0




if __name__ == "__main__":
    sys.exit(main())
