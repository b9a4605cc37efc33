"""Measurement helpers around rocprofv3 (no part of the compute path).

  python -m paper_2201_11326_amd.profiling probe
      The power-law ensemble twice, preceded by a plain 1 GiB device copy
      whose HBM traffic is known; run it under `rocprofv3 --pmc FETCH_SIZE`
      and again under `--pmc WRITE_SIZE`.
  python -m paper_2201_11326_amd.profiling probe_large
      The same calibration copy, then one row range of the large skewed
      workload at full size (range 5 of 25 ranges of equal 2-path work, the
      first one a default bench run times), S = {8, 16}, streamed, with the
      bench's count-store limit (160 GiB).
  python -m paper_2201_11326_amd.profiling stats DB [--match NAME]
      Per-kernel launch count / total / average / min / max duration from a
      rocprofv3 --kernel-trace database.
  python -m paper_2201_11326_amd.profiling sq SQ1_DB SQ2_DB
      Waiting share and LDS bank-conflict rate of each heavy-tier kernel from
      two SQ counter runs of the probe (SQ_PASS1, then SQ_PASS2).
  python -m paper_2201_11326_amd.profiling traffic FETCH_DB WRITE_DB
      HBM bytes per launch of each heavy-tier kernel, scaled by what the same
      counters read for the calibration copy (1 GiB read + 1 GiB written).
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SRC = os.path.join(HERE, "csrc", "slg_kernels.hip")
COPY_BYTES = 1 << 30


def short_name(kname: str) -> str:
    k = kname.replace("void ", "").replace("slg::(anonymous namespace)::", "")
    return k.split("(")[0]


def probe() -> None:
    sys.path.insert(0, ROOT)
    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg
    x = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)  # calibration: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    del x, y
    inc = hg.power_law()
    ctx = slg.Context(0)
    g = ctx.register_incidence(inc)
    for _ in range(2):
        outs = ctx.line_graph(g, [1, 2, 4, 8])
        torch.cuda.synchronize()
        del outs
    print("probe done", flush=True)


def probe_large() -> None:
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import hypergen as hg
    import paper_2201_11326_amd as slg
    x = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)  # calibration: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    del x, y
    inc = hg.large_skewed()
    ctx = slg.Context(0)
    ctx.set_count_store(160 << 30)  # the large skewed bench's count-store limit
    g = ctx.register_incidence(inc)
    prefix = ctx.work_prefix(g, 8)
    W, B, b = int(prefix[-1]), 25, 5
    r0 = int(np.searchsorted(prefix, W * b // B, side="left"))
    r1 = int(np.searchsorted(prefix, W * (b + 1) // B, side="left"))
    edges = [0]

    def on_chunk(k, s, c0, c1, e0, row_ptr, row, col, w):
        edges[0] += int(col.numel())
        return False

    ctx.reset_timing()
    ctx.line_graph_stream(g, [8, 16], 2 << 30, on_chunk, rows=(r0, r1))
    torch.cuda.synchronize()
    print(f"probe done: rows [{r0}, {r1}), {edges[0]} edges, work {ctx.work()}", flush=True)


def kernel_rows(db: str):
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(kernels)")]
    name_col = "name" if "name" in cols else "kernel_name"
    return [(short_name(n), (e - s) / 1e6) for n, s, e in
            con.execute(f"select {name_col}, start, end from kernels")]


def stats(db: str, match: str = "") -> str:
    agg = collections.OrderedDict()
    for name, ms in kernel_rows(db):
        if match and match not in name:
            continue
        a = agg.setdefault(name, [0, 0.0, float("inf"), 0.0])
        a[0] += 1
        a[1] += ms
        a[2] = min(a[2], ms)
        a[3] = max(a[3], ms)
    total = sum(v[1] for v in agg.values()) or 1.0
    out = [f"{'kernel':44s} {'calls':>6s} {'total_ms':>10s} {'avg_ms':>9s} {'min_ms':>9s} {'max_ms':>9s} {'pct':>6s}"]
    for name, (c, t, lo, hi) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"{name[:44]:44s} {c:6d} {t:10.3f} {t / c:9.3f} {lo:9.3f} {hi:9.3f} {100 * t / total:6.1f}")
    return "\n".join(out)


def counter_per_kernel(db: str, counter: str):
    con = sqlite3.connect(db)
    per = collections.defaultdict(list)
    for kname, cname, val in con.execute(
            "select kernel_name, counter_name, value from counters_collection"):
        if cname == counter:
            per[short_name(kname)].append(val)
    return per


HEAVY_KERNELS = ("heavy_kernel<false, false, true>", "heavy_kernel<false, false, false>",
                 "heavy_store_emit_kernel<4, false>", "heavy_kernel<true, false, false>")
DENSE_KERNELS = ("dense_kernel<false>", "heavy_store_emit_kernel<4, true>", "dense_kernel<true>")
WORKLOADS = {  # probe -> (title, kernels)
    "power_law": ("the heavy-tier kernels (power-law ensemble S={1,2,4,8})", HEAVY_KERNELS),
    "large_skewed": ("the dense-tier kernels (large skewed workload at full size, one row range, S={8,16})",
                     DENSE_KERNELS),
}


def traffic(fetch_db: str, write_db: str, workload: str = "power_law") -> str:
    """HBM bytes per launch of every heavy-tier kernel found in the two runs
    (the counting pass, with or without the count store, and the emit pass,
    from the store or by walking the 2-paths again)."""
    f = counter_per_kernel(fetch_db, "FETCH_SIZE")
    w = counter_per_kernel(write_db, "WRITE_SIZE")
    copy = [k for k in f if "copy" in k.lower() or "elementwise" in k.lower()]
    # the calibration copy is the largest-traffic copy-like kernel
    ck = max(copy, key=lambda k: max(f[k])) if copy else None
    fetch_factor = COPY_BYTES / (max(f[ck]) * 1024) if ck else 1.0
    write_factor = COPY_BYTES / (max(w.get(ck, [0])) * 1024) if ck and w.get(ck) else 1.0
    with open(KERNEL_SRC, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    title, kernels = WORKLOADS[workload]
    lines = [
        f"# HBM traffic of {title}",
        "",
        f"kernel_source_sha256: {sha}",
        f"calibration kernel: {ck} (1 GiB read + 1 GiB written)",
        f"calibration FETCH_SIZE KiB: {max(f[ck]) if ck else None}; factor {fetch_factor:.4f}",
        f"calibration WRITE_SIZE KiB: {max(w[ck]) if ck and w.get(ck) else None}; factor {write_factor:.4f}",
    ]
    for name in kernels:
        fe, we = f.get(name, []), w.get(name, [])
        if not fe or not we:
            continue
        fetch_b = fetch_factor * 1024 * sum(fe) / len(fe)
        write_b = write_factor * 1024 * sum(we) / len(we)
        lines += [
            "",
            f"kernel: {name}",
            f"launches measured: {len(fe)} (FETCH_SIZE), {len(we)} (WRITE_SIZE)",
            f"FETCH_SIZE KiB per launch (raw): {sum(fe) / len(fe):.1f}",
            f"WRITE_SIZE KiB per launch (raw): {sum(we) / len(we):.1f}",
            f"hbm_fetch_bytes_per_launch: {fetch_b:.6e}",
            f"hbm_write_bytes_per_launch: {write_b:.6e}",
            f"hbm_bytes_per_launch: {fetch_b + write_b:.6e}",
        ]
    return "\n".join(lines)


SQ_PASS1 = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_INSTS_VALU",
            "SQ_INSTS_LDS", "SQ_INSTS_SALU")
SQ_PASS2 = ("SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VMEM",
            "SQ_INSTS_VMEM_WR", "SQ_WAIT_INST_LDS", "SQ_INSTS_BRANCH")


def sq(db1: str, db2: str, workload: str = "power_law") -> str:
    """Per heavy-tier kernel: the share of wave cycles spent waiting and the
    LDS bank-conflict rate (conflict cycles / LDS-active cycles), from one
    run per counter pass (SQ_PASS1, SQ_PASS2)."""
    per = {}
    for db, names in ((db1, SQ_PASS1), (db2, SQ_PASS2)):
        for name in names:
            for k, vals in counter_per_kernel(db, name).items():
                per.setdefault(k, {})[name] = sum(vals) / len(vals)
    title, kernels = WORKLOADS[workload]
    lines = [f"# SQ counters of {title}", ""]
    for k in kernels:
        c = per.get(k)
        if not c:
            continue
        wait = c.get("SQ_WAIT_ANY", 0) / max(c.get("SQ_WAVE_CYCLES", 0), 1)
        conflict = c.get("SQ_LDS_BANK_CONFLICT", 0) / max(c.get("SQ_LDS_IDX_ACTIVE", 0), 1)
        lines += [f"kernel: {k}",
                  f"waiting share of wave cycles (SQ_WAIT_ANY / SQ_WAVE_CYCLES): {wait:.3f}",
                  f"LDS bank-conflict rate (SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE): {conflict:.3f}"]
        lines += [f"  {n}: {c[n]:.4g}" for n in SQ_PASS1 + SQ_PASS2 if n in c]
        lines.append("")
    return "\n".join(lines)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("probe")
    sub.add_parser("probe_large")
    a = sub.add_parser("stats")
    a.add_argument("db")
    a.add_argument("--match", default="")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_db")
    b.add_argument("write_db")
    b.add_argument("--workload", choices=sorted(WORKLOADS), default="power_law")
    c = sub.add_parser("sq")
    c.add_argument("db1")
    c.add_argument("db2")
    c.add_argument("--workload", choices=sorted(WORKLOADS), default="power_law")
    args = ap.parse_args(argv)
    if args.cmd == "probe":
        probe()
    elif args.cmd == "probe_large":
        probe_large()
    elif args.cmd == "stats":
        print(stats(args.db, args.match))
    elif args.cmd == "sq":
        print(sq(args.db1, args.db2, args.workload))
    else:
        print(traffic(args.fetch_db, args.write_db, args.workload))
    return 0


if __name__ == "__main__":
    sys.exit(main())
