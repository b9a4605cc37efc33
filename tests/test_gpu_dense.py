"""The dense tier (direct counters over windows of E_s positions) through the
C ABI: against the oracle where the whole graph can be checked, against the
other tiers bit for bit where it spans several windows, and with a store too
small for its survivors (those slots walk their 2-paths again)."""
from __future__ import annotations

import numpy as np
import pytest

import hypergen as hg
import oracle
from gpu_util import assert_matches_oracle, assert_well_formed, planted

pytestmark = pytest.mark.gpu

WINDOW = 1 << 14  # E_s positions per dense slot


def _ctx(dense, store_limit=32 << 30, store_min=0):
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    c.set_count_store(store_limit, store_min)
    c.set_dense(*dense)
    return c


@pytest.fixture(scope="module")
def skewed():
    # the large-skewed generator's laws at m = 3e5: |E_8| = 90,526 rows, so
    # rows span up to six windows; W_8 = 2.3e10 2-paths
    return hg.large_skewed(n=150_000, m=300_000)


def test_dense_forced_small_graph_matches_oracle():
    """Rows sharing vertex 0 (every other row), all on the dense tier."""
    inc = planted(6000, 20000, [([0], 2, 0), ([1, 2], 3, 1)], 3, seed=17)
    ctx = _ctx((8, 1))
    g = ctx.register_incidence(inc)
    p = ctx.plan(g, [1, 2, 3])
    st = p.stats()
    assert st["dense_slots"] > 0 and st["dense_store_full"] == 0, st
    p.destroy()
    outs = [o.cpu() for o in ctx.line_graph(g, [1, 2, 3])]
    for lg in outs:
        assert_matches_oracle(inc, lg, lg.s, "dense forced")
        assert_well_formed(inc, lg, lg.s)
    assert outs[0].two_paths == oracle.two_paths(inc, 1)
    g.release()
    ctx.close()


def test_dense_store_overflow_matches_oracle():
    """A dense store with room for about a third of the survivors: the slots
    that find it full write their edges by walking their 2-paths again."""
    inc = planted(6000, 20000, [([0], 2, 0), ([1, 2], 3, 1)], 3, seed=18)
    probe = _ctx((8, 1), store_min=1 << 62)  # heavy and light stores off, the dense one on
    g = probe.register_incidence(inc)
    p = probe.plan(g, [1, 2])
    st = p.stats()
    p.destroy()
    g.release()
    probe.close()
    assert st["dense_slots"] > 0 and st["dense_stored"] > 30, st
    limit = 12 * st["dense_slots"] + 16 + 4 * (st["dense_stored"] // 3)
    ctx = _ctx((8, 1), store_limit=limit, store_min=1 << 62)
    g = ctx.register_incidence(inc)
    p = ctx.plan(g, [1, 2])
    assert p.stats()["dense_store_full"] == 1
    p.destroy()
    for lg in [o.cpu() for o in ctx.line_graph(g, [1, 2])]:
        assert_matches_oracle(inc, lg, lg.s, "dense store full")
    g.release()
    ctx.close()


def test_dense_windows_equal_other_tiers_and_oracle_rows(skewed):
    """Several windows per row, ensemble S = {8, 16}: the dense tier (default
    rule) and the bitmap tier (dense off) give identical arrays; sampled rows
    (both ends of every window boundary, the longest rows, random rows)
    equal the oracle; W_8 equals the closed form."""
    import torch
    inc = skewed
    S = [8, 16]
    dense, plain = _ctx((4, 0)), _ctx((0, 0))
    gd, gp = dense.register_incidence(inc), plain.register_incidence(inc)
    p = dense.plan(gd, S)
    st = p.stats()
    p.destroy()
    assert st["dense_slots"] > 0 and st["dense_two_paths"] > st["two_paths"] // 2, st
    a = dense.line_graph(gd, S)
    b = plain.line_graph(gp, S)
    for x, y in zip(a, b):
        for f in ("row_ptr", "row", "col", "w"):
            assert torch.equal(getattr(x, f), getattr(y, f)), (x.s, f)
    assert a[0].two_paths == oracle.two_paths(inc, 8)
    # rows at the window boundaries of E_8 (positions 16383/16384, 32767/32768)
    kept = np.nonzero(inc.sizes() >= 8)[0]
    edges = [WINDOW - 2, WINDOW - 1, WINDOW, 2 * WINDOW - 1, 2 * WINDOW, 2 * WINDOW + 1]
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([kept[[e for e in edges if e < kept.size]], kept[:4],
                                     rng.choice(kept, 24, replace=False)]))
    for lg in a:
        rp = lg.row_ptr.cpu().numpy()
        ref = oracle.line_graph_rows(inc, lg.s, rows, size_min=8)
        for t, i in enumerate(ref.rows):
            rj, rw = ref.row(t)
            lo, hi = int(rp[i]), int(rp[i + 1])
            assert np.array_equal(lg.col[lo:hi].cpu().numpy(), rj), (lg.s, int(i))
            assert np.array_equal(lg.w[lo:hi].cpu().numpy(), rw), (lg.s, int(i))
        assert int(lg.row_ptr[-1]) == lg.num_edges
        assert bool((lg.col > lg.row).all()) and bool((lg.w >= lg.s).all())
    del a, b
    gd.release()
    gp.release()
    dense.close()
    plain.close()


def test_dense_stream_chunks_equal_one_shot(skewed):
    """Streamed in chunks (dense slots split across chunks), the edges equal
    the one-shot result's, in order."""
    import torch
    inc = skewed
    ctx = _ctx((4, 0))
    g = ctx.register_incidence(inc)
    whole = ctx.line_graph(g, [16])[0]
    got = []

    def fn(k, s, r0, r1, e0, rp, ri, rj, rw):
        assert int(whole.row_ptr[r0]) == e0
        got.append((e0, rj.clone(), rw.clone()))
        return False

    ctx.line_graph_stream(g, [16], 32 << 20, fn)
    assert len(got) > 2
    col = torch.cat([c for _, c, _ in got])
    w = torch.cat([x for _, _, x in got])
    assert torch.equal(col, whole.col) and torch.equal(w, whole.w)
    g.release()
    ctx.close()


def _collect(ctx, g, S, chunk, rows=None):
    """Every streamed chunk, copied out, per threshold: (rows, edges)."""
    import torch
    got = {s: [] for s in S}

    def fn(k, s, r0, r1, e0, rp, ri, rj, rw):
        got[s].append((r0, r1, e0, rp.cpu(), ri.cpu(), rj.cpu(), rw.cpu()))
        return False

    ctx.line_graph_stream(g, S, chunk, fn, rows=rows)
    torch.cuda.synchronize()
    return got


@pytest.mark.parametrize("dense", [(4, 0), (0, 0)])
def test_stream_in_small_row_blocks_equals_one_shot(dense):
    """A count-store limit of 4 MiB cuts the rows into many blocks, each
    planned, counted and emitted on its own; the chunks reassemble to the
    one-shot result (edge offsets, row pointers and every edge)."""
    import torch
    inc = hg.large_skewed(n=20_000, m=40_000)
    S = [2, 3, 5]
    whole_ctx = _ctx(dense)
    gw = whole_ctx.register_incidence(inc)
    whole = [o.cpu() for o in whole_ctx.line_graph(gw, S)]
    gw.release()
    whole_ctx.close()
    ctx = _ctx(dense, store_limit=4 << 20)
    g = ctx.register_incidence(inc)
    ctx.reset_timing()
    got = _collect(ctx, g, S, 1 << 20)
    work = ctx.work()
    assert work["blocks"] > 4, work
    for lg in whole:
        parts = got[lg.s]
        assert parts[0][0] == 0 and parts[-1][1] == inc.m
        col = torch.cat([p[5] for p in parts])
        w = torch.cat([p[6] for p in parts])
        row = torch.cat([p[4] for p in parts])
        assert torch.equal(col, lg.col) and torch.equal(w, lg.w) and torch.equal(row, lg.row), lg.s
        for r0, r1, e0, rp, _, _, _ in parts:
            assert int(lg.row_ptr[r0]) == e0
            assert torch.equal(rp + e0, lg.row_ptr[r0:r1 + 1])
    assert work["two_paths"] == oracle.two_paths(inc, 2)
    g.release()
    ctx.close()


def test_stream_row_ranges_and_work_prefix():
    """Disjoint row ranges of equal work (from the work prefix) together give
    the whole L_s; the prefix equals the oracle's per-row 2-paths."""
    import torch
    inc = hg.random_small(77, 4000, 900, 30, 1.2, kmin=0)
    ctx = _ctx((4, 0))
    g = ctx.register_incidence(inc)
    pre = ctx.work_prefix(g, 2)
    per_row = oracle.row_two_paths(inc, 2, np.arange(inc.m))
    assert np.array_equal(np.diff(pre), per_row) and pre[0] == 0
    cuts = [0] + [int(np.searchsorted(pre, pre[-1] * b // 3)) for b in (1, 2)] + [inc.m]
    ref = oracle.line_graph(inc, 2)
    cols, ws = [], []
    for b in range(3):
        got = _collect(ctx, g, [2], 1 << 16, rows=(cuts[b], cuts[b + 1]))[2]
        e_base = int(ref.row_ptr[cuts[b]])
        for r0, r1, e0, rp, ri, rj, rw in got:
            assert int(ref.row_ptr[r0]) - e_base == e0
            cols.append(rj)
            ws.append(rw)
    assert np.array_equal(torch.cat(cols).numpy(), ref.j) and np.array_equal(torch.cat(ws).numpy(), ref.w)
    g.release()
    ctx.close()
