#!/usr/bin/env python3
"""Benchmark: s-line graph ensemble of the power-law hypergraph on one GPU.

Workload: n = 1,000,000 vertices, m = 500,000 hyperedges, sizes Zipf(2.1)
on [2, 5000], vertices drawn with weight ~ rank^-0.8 (seeded, synthetic),
thresholds S = {1, 2, 4, 8} computed in one ensemble pass. One step is the
whole path on inputs already resident in HBM: pruning, 2-path work
estimate, counting pass, prefix sums, output allocation and the emit pass
that writes every L_s as COO + CSR.

Prints ONE JSON line. `value` is 2-paths traversed per second over the
timed steps; edges/s and the per-step latency percentiles ride along. The
`roofline` entry is for the dominant kernel (the heavy-tier emit pass),
timed with HIP events on its own stream inside the library; `cpu_baseline`
times the brute-force CPU oracle on a bounded row sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

S_SET = [1, 2, 4, 8]
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2201_11326_amd", "csrc", "slg_kernels.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "heavy_emit_power_law_traffic.md")
METRIC = "2-paths traversed/sec + s-line edges/sec at 1 GPU; p50/p99 query latency"


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the heavy emit kernel from the committed PMC
    summary, if it was taken on the current kernel source; else None."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_hash and m_bytes) or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(inc, seconds: float, seed: int = 7):
    """Oracle on a random row sample sized to about `seconds` of CPU time.
    Rate = 2-paths of the sampled rows (the work the two-hop traversal does
    for them) / oracle wall time for every s of the ensemble."""
    import numpy as np

    import oracle
    threads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16)))
    rng = np.random.default_rng(seed)
    probe = np.sort(rng.choice(inc.m, size=4 * threads, replace=False))
    t0 = time.perf_counter()
    for s in S_SET:
        oracle.line_graph_rows(inc, s, probe, threads=threads)
    per_row = (time.perf_counter() - t0) / probe.size
    nrows = int(max(threads, min(inc.m, seconds / max(per_row, 1e-9))))
    rows = np.sort(rng.choice(inc.m, size=nrows, replace=False))
    t0 = time.perf_counter()
    for s in S_SET:
        oracle.line_graph_rows(inc, s, rows, threads=threads)
    dt = time.perf_counter() - t0
    work = int(oracle.row_two_paths(inc, S_SET[0], rows, threads=threads).sum())
    return {"value": work / dt, "unit": "2-paths/s", "cores": threads, "kind": "oracle",
            "sample": f"{nrows} random rows (seed {seed}) of the same hypergraph, all of S={S_SET}, "
                      f"{work} 2-paths, {dt:.2f} s wall"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the s-line graph path here runs on a single MI355X "
              "(rows would shard across GPUs with no exchange; see DESIGN.md). Use --gpus 1.",
              file=sys.stderr)
        return 2

    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    t_gen = time.perf_counter()
    inc = hg.power_law()
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

    launches, ms = stages.get("emit_heavy", (0, 0.0))
    avg_s = ms / 1e3 / max(launches, 1)
    algo_bytes = 4 * stats["heavy_two_paths"] + 12 * stats["heavy_edges"]
    achieved = algo_bytes / avg_s / 1e9 if avg_s > 0 else None
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": (achieved / PEAK_HBM_GBS) if achieved else None, "traffic": traffic,
                "kernel": "heavy_kernel<EMIT=true> (emit_heavy)", "avg_launch_ms": avg_s * 1e3,
                "algorithmic_bytes_per_launch": algo_bytes}
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
        "config": {"workload": "power-law hypergraph n=1e6 m=5e5 |e|~Zipf(2.1)[2,5000] "
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
