#!/usr/bin/env python3
"""Writes the oracle's digests that pin the GPU path on whole workloads.

Test infrastructure: calls only ``oracle/`` (and ``hypergen/`` for the seeded
inputs, which hold none of the method's arithmetic). Each digest is the
oracle's (number of edges, sum of overlaps, sum mod 2^64 of
SplitMix64(i * 2^32 + j) xor w) of a set of edges of L_s (Section II-B:
pairs i < j of E_s with |e_i n e_j| >= s, weighted by the overlap). Digests
are order-free and add over disjoint parts, so the GPU's output can be
compared with them block by block on the device.

The ensemble's thresholds are one oracle pass at the smallest s, filtered
by w >= s_k: the overlap does not depend on s, and w >= s_k already forces
both hyperedges into E_{s_k}.

    python tests/golden/make_digests.py power_law      [--threads N]
    python tests/golden/make_digests.py batched        [--threads N]
    python tests/golden/make_digests.py large_skewed   [--threads N]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import hypergen as hg  # noqa: E402
import oracle  # noqa: E402

POWER_LAW_S = (1, 2, 4, 8)
POWER_LAW_BLOCK = 5000
LARGE_SKEWED_S = 16


def _block_digests(inc, s_list, r0, r1, threads):
    rows = np.arange(r0, r1, dtype=np.int64)
    ref = oracle.line_graph_rows(inc, s_list[0], rows, size_min=s_list[0], threads=threads)
    i = np.repeat(rows.astype(np.int32), np.diff(ref.ptr))
    out = []
    for s in s_list:
        keep = ref.w >= s
        out.append(oracle.digest(i[keep], ref.j[keep], ref.w[keep]))
    return out


def power_law(threads):
    inc = hg.power_law()
    path = os.path.join(HERE, "power_law_block_digests.txt")
    t0 = time.time()
    lines = ["# Oracle digests of every L_s of the power-law workload, by blocks of rows.",
             "# Input: hypergen.power_law() (n=1e6, m=5e5, |e|~Zipf(2.1) on [2,5000], vertex weight ~ rank^-0.8,",
             f"#   seed {hg.BASE_SEED + 2}); nnz {inc.nnz}.",
             "# Written by tests/golden/make_digests.py power_law (calls only oracle/).",
             f"# two_paths {' '.join(f'{s}:{oracle.two_paths(inc, s)}' for s in POWER_LAW_S)}",
             "# columns: s row_begin row_end edges sum_w hash(hex)"]
    for r0 in range(0, inc.m, POWER_LAW_BLOCK):
        r1 = min(inc.m, r0 + POWER_LAW_BLOCK)
        for s, (e, sw, h) in zip(POWER_LAW_S, _block_digests(inc, POWER_LAW_S, r0, r1, threads)):
            lines.append(f"{s} {r0} {r1} {e} {sw} {h:016x}")
        print(f"power_law rows {r1}/{inc.m} {time.time() - t0:.0f}s", flush=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def batched(threads):
    fam = hg.batched_family()
    path = os.path.join(HERE, "batched_member_digests.txt")
    t0 = time.time()
    lines = ["# Oracle digests of L_s of every member of the batched family, each at its own s.",
             f"# Input: hypergen.batched_family() (256 graphs, seed {hg.BASE_SEED + 4}).",
             "# Written by tests/golden/make_digests.py batched (calls only oracle/).",
             "# columns: graph m s two_paths edges sum_w hash(hex)"]
    for g, mem in enumerate(fam):
        (e, sw, h), = _block_digests(mem.inc, [mem.s], 0, mem.inc.m, threads)
        lines.append(f"{g} {mem.inc.m} {mem.s} {oracle.two_paths(mem.inc, mem.s)} {e} {sw} {h:016x}")
        if g % 16 == 15:
            print(f"batched {g + 1}/256 {time.time() - t0:.0f}s", flush=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def large_skewed_sample(inc, count=160, seed=11):
    """Rows of E_16 to check: the first and last ones, the ones at the edges
    of every window of 2^15 consecutive E_16 rows, and a seeded random set."""
    kept = np.nonzero(inc.sizes() >= LARGE_SKEWED_S)[0]
    win = 1 << 15
    edges = []
    for b in range(win, kept.size, win):
        edges += [b - 1, b]
    pick = list(range(4)) + list(range(kept.size - 4, kept.size)) + edges
    rng = np.random.default_rng(seed)
    rest = rng.choice(kept.size, size=max(0, count - len(set(pick))), replace=False)
    return np.unique(kept[np.asarray(sorted(set(pick) | set(rest.tolist())))])


def large_skewed(threads):
    t0 = time.time()
    inc = hg.large_skewed()
    print(f"generated in {time.time() - t0:.0f}s", flush=True)
    rows = large_skewed_sample(inc)
    ref = oracle.line_graph_rows(inc, LARGE_SKEWED_S, rows, threads=threads)
    path = os.path.join(HERE, "large_skewed_s16_rows.txt")
    lines = ["# Oracle rows of L_16 of the large skewed workload (sampled rows; the whole graph has",
             "#   about 3e10 edges).",
             "# Input: hypergen.large_skewed() (n=5e6, m=1e7, |e|=min(rint(LogNormal(1.5,1)),1e4),",
             f"#   vertex weight ~ rank^-1.5, seed {hg.BASE_SEED + 3}); nnz {inc.nnz}.",
             "# Written by tests/golden/make_digests.py large_skewed (calls only oracle/).",
             f"# two_paths 8:{oracle.two_paths(inc, 8)} 16:{oracle.two_paths(inc, 16)}",
             "# columns: s row edges sum_w hash(hex)   (the row's edges (row, j, w), j > row)"]
    for t, i in enumerate(ref.rows):
        j, w = ref.row(t)
        e, sw, h = oracle.digest(np.full(j.size, i, np.int64), j, w)
        lines.append(f"{LARGE_SKEWED_S} {int(i)} {e} {sw} {h:016x}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"large_skewed {len(ref.rows)} rows in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=("power_law", "batched", "large_skewed"))
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    {"power_law": power_law, "batched": batched, "large_skewed": large_skewed}[a.which](a.threads)
