"""Whole-workload parity with the oracle through committed digests.

tests/golden/*.txt are written by tests/golden/make_digests.py, which calls
only the oracle. A digest is (edges, sum of overlaps, sum mod 2^64 of
SplitMix64(i * 2^32 + j) xor w) of a set of edges; it is order-free and adds
over disjoint parts, so the device's output is compared block by block
without copying it out:
  * the power-law workload: every edge of every L_s of S = {1, 2, 4, 8}, by
    blocks of 5,000 rows (with the library's own tier choice and with the
    dense tier forced);
  * the batched family: every member's L_s at its own s, after the batch is
    built and after a replay of its captured HIP graph;
  * the large skewed workload at full size (n = 5e6, m = 1e7), L_16 streamed
    in row blocks: sampled rows (both ends of E_16, both sides of every
    window boundary, random rows) and the 2-path count.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import hypergen as hg
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read(name):
    """(rows of ints / hex, header dict of 'two_paths' entries)."""
    rows, head = [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("# two_paths"):
                head = {int(a): int(b) for a, b in (t.split(":") for t in line.split()[2:])}
            elif line.strip() and not line.startswith("#"):
                parts = line.split()
                rows.append([int(x) for x in parts[:-1]] + [int(parts[-1], 16)])
    return rows, head


def _ctx(dense=None):
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    if dense is not None:
        c.set_dense(*dense)
    return c


@pytest.mark.parametrize("dense", [None, (8, 1)], ids=["own_tiers", "dense_forced"])
def test_power_law_every_edge_by_block_digest(dense):
    rows, two_paths = _read("power_law_block_digests.txt")
    S = [1, 2, 4, 8]
    inc = hg.power_law()
    ctx = _ctx(dense)
    g = ctx.register_incidence(inc)
    p = ctx.plan(g, S)
    st = p.stats()
    p.destroy()
    # the library's own rule mixes tiers in one plan: the rows with at least
    # half a 2-path per candidate on the dense tier, the other heavy rows on
    # the bitmap tier
    assert st["dense_slots"] > 0 and (dense is not None or st["heavy_slots"] > 0), st
    outs = ctx.line_graph(g, S)
    assert outs[0].two_paths == two_paths[1] == oracle.two_paths(inc, 1)
    rp = {lg.s: lg.row_ptr.cpu().numpy() for lg in outs}
    by_s = {lg.s: lg for lg in outs}
    totals = {s: 0 for s in S}
    for s, r0, r1, e, sw, h in rows:
        lg, p = by_s[s], rp[s]
        a, b = int(p[r0]), int(p[r1])
        got = ctx.digest(lg.row[a:b], lg.col[a:b], lg.w[a:b])
        assert got == (e, sw, h), (s, r0, r1, got, (e, sw, h))
        totals[s] += e
    for lg in outs:
        assert lg.num_edges == totals[lg.s]
    del outs
    g.release()
    ctx.close()


def test_batched_family_every_member_digest():
    import torch
    rows, _ = _read("batched_member_digests.txt")
    fam = hg.batched_family()
    assert len(rows) == len(fam)
    ctx = _ctx()
    graphs = [ctx.register_incidence(mem.inc) for mem in fam]
    b = ctx.batch(graphs, [mem.s for mem in fam])

    def check(tag):
        for gi, m, s, two_paths, e, sw, h in rows:
            assert fam[gi].inc.m == m and fam[gi].s == s
            res = b.result(gi)
            got = ctx.digest(res.row, res.col, res.w)
            assert got == (e, sw, h), (tag, gi, got, (e, sw, h))

    check("created")
    assert b.info()["two_paths"] == sum(r[3] for r in rows)
    b.run(use_graph=True)
    torch.cuda.synchronize()
    check("replayed")
    b.destroy()
    for g in graphs:
        g.release()
    ctx.close()


def test_large_skewed_full_size_s16_streamed_rows():
    import torch
    rows, two_paths = _read("large_skewed_s16_rows.txt")
    want = {r[1]: tuple(r[2:]) for r in rows}
    inc = hg.large_skewed()
    print(f"large skewed: m={inc.m} nnz={inc.nnz}; streaming L_16", flush=True)
    assert two_paths[16] == oracle.two_paths(inc, 16)
    ctx = _ctx()
    g = ctx.register_incidence(inc)
    sample = np.array(sorted(want), dtype=np.int64)
    got = {}
    edges = [0]
    bad = []

    def fn(k, s, r0, r1, e0, rp, ri, rj, rw):
        edges[0] += int(rj.numel())
        if rj.numel() and not (bool((rw >= s).all()) and bool((rj > ri).all())):
            bad.append((r0, r1))
        lo, hi = np.searchsorted(sample, [r0, r1])
        if hi > lo:
            crp = rp.cpu().numpy()
            for i in sample[lo:hi]:
                a, b = int(crp[i - r0]), int(crp[i - r0 + 1])
                got[int(i)] = ctx.digest(ri[a:b], rj[a:b], rw[a:b])
        return False

    ctx.reset_timing()
    ctx.line_graph_stream(g, [16], 2 << 30, fn)
    torch.cuda.synchronize()
    work = ctx.work()
    print(f"streamed: {edges[0]} edges, {work}", flush=True)
    assert not bad
    assert work["two_paths"] == two_paths[16] and work["edges"] == edges[0]
    assert work["dense_two_paths"] > 0
    assert sorted(got) == sorted(want)
    for i, d in want.items():
        assert got[i] == d, (i, got[i], d)
    g.release()
    ctx.close()
