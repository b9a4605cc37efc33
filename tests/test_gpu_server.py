"""The served form: queries of several sizes and s-sets submitted to the
request loop, with several in flight at once and, in one test, a memory
budget tight enough that queries wait for each other. Every result must be
identical, element by element, to the same query run alone and to the
oracle."""
from __future__ import annotations

import threading

import numpy as np
import pytest

import hypergen as hg
import oracle
from gpu_util import assert_matches_oracle

pytestmark = pytest.mark.gpu

S_CHOICES = (1, 2, 3, 4, 5, 8)


@pytest.fixture(scope="module")
def ctx():
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    yield c
    c.close()


def pool():
    """Uneven members: skewed (lognormal sizes, Zipf vertex weights), power-law
    and uniform small hypergraphs."""
    out = [hg.large_skewed(n=600, m=1200, seed=11), hg.large_skewed(n=2000, m=4000, seed=12),
           hg.power_law(n=6000, m=3000, seed=13), hg.tiny_uniform(),
           hg.random_small(14, m=500, n=300, kmax=30, exponent=1.2)]
    return out


def queries(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        g = int(rng.integers(0, 5))
        k = int(rng.integers(1, 4))
        s = sorted(rng.choice(S_CHOICES, size=k, replace=False).tolist())
        out.append((g, [int(x) for x in s]))
    return out


def host(outs):
    return [o.cpu() for o in outs]


def same(a, b, what):
    for x, y in zip(a, b):
        for f in ("row_ptr", "row", "col", "w"):
            np.testing.assert_array_equal(getattr(x, f).numpy(), getattr(y, f).numpy(), err_msg=f"{what} {f}")


def test_served_results_equal_alone_and_oracle(ctx):
    incs = pool()
    graphs = [ctx.register_incidence(inc) for inc in incs]
    qs = queries(48, seed=5)
    alone = {}
    for g, s in qs:  # the same query alone, one at a time
        alone.setdefault((g, tuple(s)), host(ctx.line_graph(graphs[g], s)))
    srv = ctx.server(workers=4)
    tickets = {srv.submit(graphs[g], s): (g, s) for g, s in qs}
    seen = set()
    for _ in range(len(qs)):
        r = srv.next(timeout_ms=60_000)
        assert r is not None and r.ok, (r and r.message)
        g, s = tickets[r.ticket]
        assert r.s == s and r.attempts == 1
        got = host(r.outs)
        same(got, alone[(g, tuple(s))], f"ticket {r.ticket} graph {g} s={s}")
        seen.add(r.ticket)
        del r
    assert seen == set(tickets)
    st = srv.stats()
    assert st["completed"] == len(qs) and st["failed"] == 0 and st["queued"] == 0
    srv.close()
    for (g, s), outs in alone.items():  # and alone == oracle
        for lg in outs:
            assert_matches_oracle(incs[g], lg, lg.s, what=f"graph {g}")
    for gr in graphs:
        gr.release()


def test_budget_bounds_memory_and_results_stay_exact(ctx):
    incs = pool()
    graphs = [ctx.register_incidence(inc) for inc in incs]
    qs = queries(40, seed=6)
    # each query's own peak need, measured alone on an unlimited server
    need = {}
    probe = ctx.server(workers=1)
    for g, s in set((g, tuple(s)) for g, s in qs):
        t = probe.submit(graphs[g], list(s))
        r = probe.wait(t, timeout_ms=60_000)
        assert r.ok
        del r
        need[(g, s)] = probe.stats()["bytes_peak"]
        probe.close()
        probe = ctx.server(workers=1)
    probe.close()
    budget = int(max(need.values()) * 1.25)
    srv = ctx.server(workers=4, mem_budget_bytes=budget)
    lock = threading.Lock()
    tickets = {}

    def submit(part):
        for g, s in part:
            t = srv.submit(graphs[g], s)
            with lock:
                tickets[t] = (g, s)

    th = [threading.Thread(target=submit, args=(qs[i::2],)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for _ in range(len(qs)):
        r = srv.next(timeout_ms=120_000)
        assert r is not None and r.ok, (r and r.message)
        g, s = tickets[r.ticket]
        got = host(r.outs)
        del r  # give the memory back at once
        for lg in got:
            assert_matches_oracle(incs[g], lg, lg.s, what=f"graph {g}")
    st = srv.stats()
    assert st["completed"] == len(qs) and st["failed"] == 0
    assert 0 < st["bytes_peak"] <= budget, (st, budget)
    assert st["bytes_used"] == 0 and st["bytes_in_results"] == 0
    srv.close()
    for gr in graphs:
        gr.release()


def test_query_larger_than_budget_fails_alone(ctx):
    import paper_2201_11326_amd as slg
    inc = hg.power_law(n=6000, m=3000, seed=13)
    g = ctx.register_incidence(inc)
    srv = ctx.server(workers=2, mem_budget_bytes=4096)
    t_big = srv.submit(g, [1])
    r = srv.wait(t_big, timeout_ms=60_000)
    assert r.status == slg.SLG_ERR_OUT_OF_MEMORY and r.outs is None and "budget" in r.message
    srv.close()
    # the next server is unaffected
    srv = ctx.server(workers=2)
    r = srv.wait(srv.submit(g, [2, 4]), timeout_ms=60_000)
    assert r.ok
    for lg in host(r.outs):
        assert_matches_oracle(inc, lg, lg.s)
    del r
    srv.close()
    g.release()


def test_unknown_ticket_and_shutdown_with_queued_queries(ctx):
    import paper_2201_11326_amd as slg
    inc = hg.random_small(21, m=400, n=200, kmax=25, exponent=1.1)
    g = ctx.register_incidence(inc)
    srv = ctx.server(workers=1)
    with pytest.raises(slg.SlgError):
        srv.wait(987654, timeout_ms=0)
    tickets = [srv.submit(g, [1, 3]) for _ in range(12)]
    first = srv.wait(tickets[0], timeout_ms=60_000)
    assert first.ok
    ref = host(first.outs)
    for lg in ref:
        assert_matches_oracle(inc, lg, lg.s)
    del first
    srv.close()  # cancels what is still queued, frees what nobody took
    g.release()
    with pytest.raises(slg.SlgError):
        slg.Server(ctx, workers=0)


def test_two_stream_plan_equals_one_stream_plan(ctx):
    """A plan with at least 2^28 2-paths runs its light counting pass on the
    context's second stream; a server's slots run everything on one stream.
    The power-law workload (n=1e6, m=5e5, S = {1, 2, 4, 8}; 2.4e9 2-paths)
    through both must give identical arrays."""
    import torch
    inc = hg.power_law()
    g = ctx.register_incidence(inc)
    forked = ctx.line_graph(g, [1, 2, 4, 8])
    assert forked[0].two_paths >= 1 << 28
    srv = ctx.server(workers=1)
    srv.submit(g, [1, 2, 4, 8])
    r = srv.next(timeout_ms=120_000)
    assert r is not None and r.ok, (r and r.message)
    for a, b in zip(forked, r.outs):
        assert a.s == b.s and a.num_edges == b.num_edges
        for f in ("row_ptr", "row", "col", "w"):
            assert torch.equal(getattr(a, f), getattr(b, f)), f"s={a.s} {f}"
    del r, forked
    srv.close()
    g.release()


def test_full_served_pool_mix_equals_alone():
    """The served workload's own pool (64 large-skewed-generator graphs and
    4 power-law-generator graphs at full size, n = 1e6, m = 5e5) with a
    seeded sample of its request stream, 8 queries in flight under a 64 GiB
    budget: every result equals the same query run alone, array for array.
    The sample holds every power-law member at least once."""
    import torch

    import paper_2201_11326_amd as slg
    pool = hg.served_pool()
    reqs = hg.served_requests(len(pool), 400, seed=hg.BASE_SEED + 7)
    rng = np.random.default_rng(21)
    pick = [reqs[int(i)] for i in rng.choice(len(reqs), size=28, replace=False)]
    big = [r for r in reqs if r.graph >= 64]
    for gidx in range(64, len(pool)):  # each full-size member once, at s >= 2 (its L_1 alone is 24 GB)
        cand = [r for r in big if r.graph == gidx and r.s[0] >= 2]
        q = cand[0] if cand else hg.Request(0.0, gidx, [2, 4])
        pick.append(q)
    ctx = slg.Context(0)
    graphs = [ctx.register_incidence(x) for x in pool]
    srv = ctx.server(workers=8, mem_budget_bytes=64 << 30)
    tick = {srv.submit(graphs[q.graph], q.s): q for q in pick}
    done = 0
    for _ in pick:
        r = srv.next(timeout_ms=300_000)
        assert r is not None and r.ok, (r and r.message)
        q = tick[r.ticket]
        alone = ctx.line_graph(graphs[q.graph], q.s)
        for a, b in zip(r.outs, alone):
            assert a.s == b.s
            for f in ("row_ptr", "row", "col", "w"):
                assert torch.equal(getattr(a, f), getattr(b, f)), (q.graph, q.s, f)
        done += 1
        del r, alone
    assert done == len(pick)
    stats = srv.stats()
    srv.close()
    assert stats["bytes_peak"] <= 64 << 30, stats
    for g in graphs:
        g.release()
    ctx.close()
