"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact integer comparisons: row pointers, i, j and overlap of every edge.
"""
import numpy as np
import pytest

import hypergen as hg
import oracle
from gpu_util import (assert_matches_oracle, assert_rows_match_oracle, assert_well_formed, planted,
                      run_gpu)
from helpers import load_toy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["store", "rewalk", "dense", "dense_rewalk"])
def ctx(request):
    """Every parity case runs four times: with the count store (the emit
    pass reads the heavy overlaps kept by the counting pass) and without it
    (the emit pass walks the 2-paths again), each with the library's own
    tier choice and with every heavy row that has at least one 2-path per
    candidate partner forced onto the dense tier."""
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    if request.param.endswith("rewalk"):
        c.set_count_store(0)
    else:  # the stores on every graph with heavy or dense slots, however small
        c.set_count_store(32 << 30, 0)
    if request.param.startswith("dense"):
        c.set_dense(8, 1)
    c.store_mode = "rewalk" if request.param.endswith("rewalk") else "store"
    c.dense_mode = request.param.startswith("dense")
    yield c
    c.close()


def test_library_is_native(ctx):
    import paper_2201_11326_amd as slg
    assert slg.version().startswith("slg")


def test_toy_example_each_s_and_ensemble(ctx):
    inc, keep, lines, _ = load_toy()
    for s in (1, 2, 3, 4):
        (lg,) = run_gpu(ctx, inc, [s])
        got = list(zip(lg.row.tolist(), lg.col.tolist(), lg.w.tolist()))
        assert got == lines.get(s, []), f"L_{s}"
        assert_matches_oracle(inc, lg, s, "toy")
    outs = run_gpu(ctx, inc, [1, 2, 3, 4])
    for lg in outs:
        assert_matches_oracle(inc, lg, lg.s, "toy ensemble")
    assert outs[0].two_paths == 9  # sum_v C(d(v), 2) for the example


def test_toy_dual_is_s_clique(ctx):
    inc, _, _, dual = load_toy()
    (lg,) = run_gpu(ctx, inc.dual(), [1])
    pairs = {(i, j): w for i, j, w in zip(lg.row.tolist(), lg.col.tolist(), lg.w.tolist())}
    for (i, j, w) in dual[1]:
        assert pairs[(i, j)] == w  # adj(b, c) = 3
    assert_matches_oracle(inc.dual(), lg, 1, "dual")


@pytest.mark.parametrize("seed,m,n,kmax,expo,s_list", [
    (121, 3000, 800, 25, 0.8, [1, 2, 3]),    # vertices of very uneven degree
    (122, 2000, 300, 40, 1.5, [2, 5]),       # a few hub vertices in most hyperedges
    (123, 5000, 1500, 8, None, [1]),         # uniform members
])
def test_dual_is_s_clique_full(ctx, seed, m, n, kmax, expo, s_list):
    """The s-clique graph (the s-line graph of the dual H*, Section II-A and
    Section III): the same library with the two CSRs swapped, compared with
    the oracle on the dual element by element."""
    dual = hg.random_small(seed, m, n, kmax, expo).dual()
    outs = run_gpu(ctx, dual, s_list)
    for lg in outs:
        assert_matches_oracle(dual, lg, lg.s, f"dual seed {seed}")
        assert_well_formed(dual, lg, lg.s)
    assert outs[0].two_paths == oracle.two_paths(dual, s_list[0])


def test_dual_of_power_law_shape_full(ctx):
    """The dual of a power-law-shaped hypergraph (|e| ~ Zipf(2.1), vertex
    weight ~ rank^-0.8, the power-law workload's laws at m = 6,000): its
    hyperedges are the vertex lists, so a few are very large."""
    dual = hg.power_law(seed=11340, n=3000, m=6000).dual()
    outs = run_gpu(ctx, dual, [1, 2, 4])
    for lg in outs:
        assert_matches_oracle(dual, lg, lg.s, "power-law dual")
    assert outs[0].two_paths == oracle.two_paths(dual, 1)


def test_tiny_uniform_full(ctx):
    inc = hg.tiny_uniform()
    for s in (1, 2, 3, 4):
        (lg,) = run_gpu(ctx, inc, [s])
        assert_matches_oracle(inc, lg, s, "tiny")
        assert lg.two_paths == oracle.two_paths(inc, s)
    outs = run_gpu(ctx, inc, [1, 2, 3, 4])
    for lg in outs:
        assert_matches_oracle(inc, lg, lg.s, "tiny ensemble")


@pytest.mark.parametrize("seed,m,n,kmax,expo,s_list", [
    (101, 3000, 400, 30, 0.8, [1]),
    (102, 3000, 200, 40, 1.5, [2]),
    (103, 2500, 150, 60, 1.5, [1, 2, 3, 5, 8]),
    (104, 4000, 5000, 12, None, [1, 2]),
    (105, 2000, 60, 25, 0.8, [3, 4]),
    (106, 1500, 1000, 6, 1.5, [1, 3]),
])
def test_random_skewed_full(ctx, seed, m, n, kmax, expo, s_list):
    inc = hg.random_small(seed, m, n, kmax, expo)  # includes empty hyperedges
    outs = run_gpu(ctx, inc, s_list)
    for lg in outs:
        assert_matches_oracle(inc, lg, lg.s, f"seed {seed}")
        assert_well_formed(inc, lg, lg.s)
    assert outs[0].two_paths == oracle.two_paths(inc, s_list[0])


def _rows_in_order(inc, order):
    """The same hypergraph with hyperedge k holding the old row order[k]."""
    sizes = np.diff(inc.he_ptr)[order]
    he_ptr = np.zeros(inc.m + 1, np.int64)
    np.cumsum(sizes, out=he_ptr[1:])
    src = np.repeat(inc.he_ptr[order] - he_ptr[:-1], sizes) + np.arange(he_ptr[-1])
    return hg.from_csr(inc.m, inc.n, he_ptr, inc.he_idx[src])


@pytest.mark.parametrize("direction", ["ascending", "descending"])
def test_rows_sorted_by_size_full(ctx, direction):
    # runs of large rows side by side (up to 600 members: several planning
    # pieces per row), as in an input relabelled by degree
    inc = hg.random_small(111, 1500, 3000, 600, 0.8)
    sizes = np.diff(inc.he_ptr)
    order = np.argsort(sizes if direction == "ascending" else -sizes, kind="stable")
    inc = _rows_in_order(inc, order)
    outs = run_gpu(ctx, inc, [1, 2, 40])
    for lg in outs:
        assert_matches_oracle(inc, lg, lg.s, direction)
    assert outs[0].two_paths == oracle.two_paths(inc, 1)


def test_heavy_rank_windows_full(ctx):
    # half of the rows share vertex 0: partner sets of several thousand per
    # row, more than one LDS rank window per slot
    inc = planted(12000, 40000, [([0], 2, 0), ([1, 2], 6, 0)], 3, seed=7)
    outs = run_gpu(ctx, inc, [1, 2, 3])
    for lg in outs:
        assert_matches_oracle(inc, lg, lg.s, "windows")


def test_heavy_range_split_sampled(ctx):
    # rows span more hyperedge ids than one slot's bitmap covers
    m = 300_000
    inc = planted(m, 1_000_000, [([0], 300, 0), ([1], 900, 0)], 2, seed=8)
    outs = run_gpu(ctx, inc, [1, 2])
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([np.arange(0, m, 300)[:400], rng.integers(0, m, 150), [m - 1]]))
    for lg in outs:
        assert_well_formed(inc, lg, lg.s)
        assert_rows_match_oracle(inc, lg, lg.s, rows, "range split")


def test_heavy_work_split_sampled(ctx):
    # 20 shared vertices in 4,000 rows: w_i up to 8e4 2-paths, split by work
    m = 200_000
    inc = planted(m, 500_000, [(list(range(20)), 50, 0)], 2, seed=9)
    outs = run_gpu(ctx, inc, [1, 20])
    rows = np.concatenate([np.arange(0, m, 50)[:600], [1, 2, 3, m - 2, m - 1]])
    for lg in outs:
        assert_well_formed(inc, lg, lg.s)
        assert_rows_match_oracle(inc, lg, lg.s, np.unique(rows), "work split")
    assert outs[1].num_edges == 4000 * 3999 // 2  # the planted clique, overlap 20


@pytest.mark.parametrize("tune", [(0, 1 << 24, 0), (256, 1 << 24, 8), (0, 1024, 0)])
def test_heavy_repeat_list_and_windows_under_tuning(ctx, tune):
    # slot_work 2^24 leaves each heavy row in one slot (split by id range
    # only): a shared 30-vertex core makes > 8,192 repeated 2-paths per slot
    # (the repeat list overflows) over > 8,192 partners (several rank
    # windows); 20 random members over 300 vertices give the first rows
    # ~8,800 distinct partners and ~7,200 repeats (the list serves the
    # counting windows, the emit pass re-walks)
    core = planted(9000, 3000, [(list(range(30)), 1, 0)], 5, seed=31)
    spread = hg.random_small(32, m=12000, n=300, kmax=20, kmin=20)
    ctx.set_tuning(*tune)
    try:
        for inc, s_list, what in ((core, [1, 30, 31], "core"), (spread, [1, 2, 3], "spread")):
            outs = run_gpu(ctx, inc, s_list)
            rows = np.unique(np.concatenate([np.arange(0, 48), np.arange(0, inc.m, inc.m // 40),
                                             [inc.m - 2, inc.m - 1]]))
            for lg in outs:
                assert_well_formed(inc, lg, lg.s)
                assert_rows_match_oracle(inc, lg, lg.s, rows, f"{what} tune={tune}")
                if what == "core" and lg.s == 30:
                    assert lg.num_edges == 9000 * 8999 // 2  # the core alone gives overlap >= 30
    finally:
        ctx.set_tuning()


def test_edge_cases(ctx):
    empty = hg.from_rows([], n=0)
    (lg,) = run_gpu(ctx, empty, [1])
    assert lg.num_edges == 0 and lg.row_ptr.tolist() == [0]
    hollow = hg.from_rows([[], [], []], n=5)
    (lg,) = run_gpu(ctx, hollow, [1])
    assert lg.num_edges == 0 and lg.row_ptr.tolist() == [0, 0, 0, 0]
    inc = hg.tiny_uniform()
    (lg,) = run_gpu(ctx, inc, [int(inc.sizes().max()) + 1])
    assert lg.num_edges == 0
    dup = hg.from_rows([[0, 1, 2], [3, 4], [0, 1, 2], [5], [0, 1, 2]], n=8)
    for lg in run_gpu(ctx, dup, [1, 3]):
        assert_matches_oracle(dup, lg, lg.s, "duplicates")
    single = hg.from_rows([[0, 1, 2, 3]], n=4)
    (lg,) = run_gpu(ctx, single, [1])
    assert lg.num_edges == 0


def test_two_uniform_graph(ctx):
    rng = np.random.default_rng(5)
    nv = 300
    pairs = set()
    while len(pairs) < 2000:
        a, b = sorted(rng.integers(0, nv, 2).tolist())
        if a != b:
            pairs.add((a, b))
    inc = hg.from_rows(sorted(pairs), n=nv)
    l1, l2 = run_gpu(ctx, inc, [1, 2])
    assert_matches_oracle(inc, l1, 1, "2-uniform")
    assert np.all(l1.w.numpy() == 1) and l2.num_edges == 0
    deg = np.diff(inc.v_ptr)
    assert l1.num_edges == int((deg * (deg - 1) // 2).sum())


def test_ensemble_equals_single_runs_and_is_deterministic(ctx):
    inc = hg.random_small(201, 5000, 300, 40, 1.5)
    ens = run_gpu(ctx, inc, [1, 2, 4, 8])
    again = run_gpu(ctx, inc, [1, 2, 4, 8])
    for a, b in zip(ens, again):
        assert np.array_equal(a.col.numpy(), b.col.numpy()) and np.array_equal(a.w.numpy(), b.w.numpy())
    for lg in ens:
        (single,) = run_gpu(ctx, inc, [lg.s])
        for f in ("row_ptr", "row", "col", "w"):
            assert np.array_equal(getattr(lg, f).numpy(), getattr(single, f).numpy()), f


def test_one_shot_result_matches_plan(ctx):
    inc = hg.random_small(202, 3000, 200, 30, 0.8)
    a = run_gpu(ctx, inc, [1, 3])
    b = run_gpu(ctx, inc, [1, 3], one_shot=True)
    for x, y in zip(a, b):
        for f in ("row_ptr", "row", "col", "w"):
            assert np.array_equal(getattr(x, f).numpy(), getattr(y, f).numpy()), f


def test_side_stream(ctx):
    import torch
    inc = hg.random_small(203, 2000, 100, 20, 1.5)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        outs = run_gpu(ctx, inc, [1, 2], stream=st)
    torch.cuda.synchronize()
    for lg in outs:
        assert_matches_oracle(inc, lg, lg.s, "side stream")


def test_power_law_config_ensemble_sampled(ctx):
    """The power-law workload (n=1e6, m=5e5) with S = {1, 2, 4, 8}."""
    import paper_2201_11326_amd as slg
    import torch
    inc = hg.power_law()
    g = ctx.register_incidence(inc)
    outs = ctx.line_graph(g, [1, 2, 4, 8])
    assert outs[0].two_paths == oracle.two_paths(inc, 1)
    # heaviest rows by 2-path work (at s = 1 nothing is pruned: the entry
    # of row i in vertex v's list has as many 2-paths as entries after it),
    # the largest hyperedges, the ends and a random sample
    rng = np.random.default_rng(1)
    deg = np.diff(inc.v_ptr)
    after = np.repeat(inc.v_ptr[1:], deg) - np.arange(inc.nnz) - 1
    work = np.bincount(inc.v_idx, weights=after, minlength=inc.m)
    big = np.concatenate([np.argsort(-work, kind="stable")[:24], np.argsort(-np.diff(inc.he_ptr))[:8]])
    rows = np.unique(np.concatenate([big, [0, 1, inc.m - 2, inc.m - 1], rng.integers(0, inc.m, 40)]))
    for lg in outs:
        # row-wise parity on the sampled rows
        rp = lg.row_ptr.cpu().numpy()
        ref = oracle.line_graph_rows(inc, lg.s, rows)
        for k, i in enumerate(ref.rows):
            a, b = int(rp[i]), int(rp[i + 1])
            rj, rw = ref.row(k)
            assert np.array_equal(lg.col[a:b].cpu().numpy(), rj), f"s={lg.s} row {i}"
            assert np.array_equal(lg.w[a:b].cpu().numpy(), rw), f"s={lg.s} row {i}"
        # properties at full size, checked on the device
        assert int(lg.row_ptr[-1]) == lg.num_edges
        assert bool((lg.row_ptr[1:] >= lg.row_ptr[:-1]).all())
        assert bool((lg.col > lg.row).all()) and bool((lg.w >= lg.s).all())
    # single-s run equals the ensemble's member
    (s8,) = ctx.line_graph(g, [8])
    assert torch.equal(s8.col, outs[3].col) and torch.equal(s8.w, outs[3].w)
    assert torch.equal(s8.row_ptr, outs[3].row_ptr)
    del outs
    g.release()


def test_errors(ctx):
    import paper_2201_11326_amd as slg
    inc = hg.tiny_uniform()
    g = ctx.register_incidence(inc)
    for bad in ([], [0], [2, 2], [3, 1], list(range(1, 18))):
        with pytest.raises(slg.SlgError) as e:
            ctx.line_graph(g, bad)
        assert e.value.status == slg.SLG_ERR_INVALID_ARG
    g.release()


def test_validate_rejects_malformed(ctx):
    import paper_2201_11326_amd as slg
    import torch
    inc = hg.random_small(301, 300, 50, 8, None, kmin=2)
    ok = ctx.register_incidence(inc, validate=True)
    ok.release()
    dev = torch.device("cuda", 0)
    T = lambda a, dt: torch.as_tensor(np.asarray(a), dtype=dt, device=dev)

    def reg(he_ptr, he_idx, v_ptr, v_idx):
        return ctx.register(inc.m, inc.n, T(he_ptr, torch.int64), T(he_idx, torch.int32),
                            T(v_ptr, torch.int64), T(v_idx, torch.int32), validate=True)

    unsorted = inc.he_idx.copy()
    unsorted[0], unsorted[1] = unsorted[1], unsorted[0]
    out_of_range = inc.he_idx.copy()
    out_of_range[5] = inc.n + 3
    bad_ptr = inc.he_ptr.copy()
    bad_ptr[-1] -= 1
    v_bad = inc.v_idx.copy()
    nz = np.nonzero(np.diff(inc.v_ptr) > 0)[0][0]
    v_bad[inc.v_ptr[nz]] = (v_bad[inc.v_ptr[nz]] + 1) % inc.m  # breaks the transpose
    cases = [(inc.he_ptr, unsorted, inc.v_ptr, inc.v_idx),
             (inc.he_ptr, out_of_range, inc.v_ptr, inc.v_idx),
             (bad_ptr, inc.he_idx, inc.v_ptr, inc.v_idx)]
    for c in cases:
        with pytest.raises(slg.SlgError) as e:
            reg(*c)
        assert e.value.status == slg.SLG_ERR_INVALID_GRAPH
    # a vertex CSR that is not the transpose: caught with VALIDATE, and by
    # the planner even without it
    srt = v_bad.copy()
    for v in range(inc.n):
        a, b = inc.v_ptr[v], inc.v_ptr[v + 1]
        srt[a:b] = np.sort(srt[a:b])
    if np.all(np.diff(srt[inc.v_ptr[nz]:inc.v_ptr[nz + 1]]) > 0):
        with pytest.raises(slg.SlgError) as e:
            reg(inc.he_ptr, inc.he_idx, inc.v_ptr, srt)
        assert e.value.status == slg.SLG_ERR_INVALID_GRAPH
        g = ctx.register(inc.m, inc.n, T(inc.he_ptr, torch.int64), T(inc.he_idx, torch.int32),
                         T(inc.v_ptr, torch.int64), T(srt, torch.int32), validate=False)
        with pytest.raises(slg.SlgError) as e:
            ctx.line_graph(g, [1])
        assert e.value.status == slg.SLG_ERR_INVALID_GRAPH
        g.release()


def test_wide_rows_full(ctx):
    # one hyperedge with 70,000 members: its overlaps need 32-bit counters
    rng = np.random.default_rng(11)
    rows = [list(range(70_000))]
    rows += [sorted(set(rng.integers(0, 100_000, 6).tolist())) for _ in range(1500)]
    rows += [list(range(0, 70_000, 2)), list(range(1, 70_000, 3))]
    inc = hg.from_rows(rows, n=100_000)
    for lg in run_gpu(ctx, inc, [1, 2, 3, 20_000]):
        assert_matches_oracle(inc, lg, lg.s, "wide")


def _stream_collect(ctx, g, s_list, chunk_bytes):
    got = {k: [] for k in range(len(s_list))}

    def fn(k, s, r0, r1, e0, rp, ri, rj, rw):
        got[k].append((r0, r1, e0, rp.cpu().numpy(), ri.cpu().numpy(), rj.cpu().numpy(), rw.cpu().numpy()))
        return False

    ctx.line_graph_stream(g, s_list, chunk_bytes, fn)
    return got


@pytest.mark.parametrize("chunk_bytes", [128 << 10, 1 << 20, 16 << 20])
def test_stream_chunks_reassemble_to_oracle(ctx, chunk_bytes):
    inc = hg.random_small(401, 3000, 250, 30, 1.5)
    g = ctx.register_incidence(inc)
    s_list = [1, 2, 5]
    got = _stream_collect(ctx, g, s_list, chunk_bytes)
    nchunks = len(got[0])
    for c in range(nchunks):  # every chunk's output, all thresholds, fits the budget
        used = sum(12 * len(got[k][c][5]) + 8 * (got[k][c][1] - got[k][c][0] + 1) for k in got)
        assert used <= chunk_bytes
        assert len({(got[k][c][0], got[k][c][1]) for k in got}) == 1  # same rows for every s
    for k, s in enumerate(s_list):
        chunks = got[k]
        assert chunks[0][0] == 0 and chunks[-1][1] == inc.m
        rp = [0]
        for (r0, r1, e0, crp, ci, cj, cw) in chunks:
            assert crp[0] == 0 and r0 == len(rp) - 1 and e0 == rp[-1]
            rp.extend((e0 + crp[1:]).tolist())
        ref = oracle.line_graph(inc, s)
        assert np.array_equal(np.array(rp), ref.row_ptr)
        assert np.array_equal(np.concatenate([c[4] for c in chunks]), ref.i)
        assert np.array_equal(np.concatenate([c[5] for c in chunks]), ref.j)
        assert np.array_equal(np.concatenate([c[6] for c in chunks]), ref.w)
    if chunk_bytes == 128 << 10:
        assert nchunks > 10
    g.release()


def test_stream_cancel_and_budget_errors(ctx):
    import paper_2201_11326_amd as slg
    inc = hg.random_small(402, 2000, 200, 25, 1.5)
    g = ctx.register_incidence(inc)
    calls = []
    with pytest.raises(slg.SlgError) as e:
        ctx.line_graph_stream(g, [1], 1 << 20, lambda *a: calls.append(1) or True)
    assert e.value.status == slg.SLG_ERR_CANCELLED and len(calls) == 1
    with pytest.raises(slg.SlgError) as e:
        ctx.line_graph_stream(g, [1], 16, lambda *a: False)
    assert e.value.status == slg.SLG_ERR_OUT_OF_MEMORY
    g.release()


def test_stream_large_skewed_shape_sampled(ctx):
    """The large skewed hypergraph's shape (lognormal sizes, vertex weight
    rank^-1.5) scaled to m = 2e5, s = 16, streamed in chunks."""
    inc = hg.large_skewed(n=100_000, m=200_000)
    g = ctx.register_incidence(inc)
    seen = {}
    total = [0]

    def fn(k, s, r0, r1, e0, rp, ri, rj, rw):
        total[0] += int(rj.numel())
        crp = rp.cpu().numpy()
        for i in sample:
            if r0 <= i < r1:
                a, b = int(crp[i - r0]), int(crp[i - r0 + 1])
                seen[i] = (rj[a:b].cpu().numpy(), rw[a:b].cpu().numpy())
        assert bool((rw >= s).all()) and bool((rj > ri).all())
        return False

    sizes = inc.sizes()
    kept = np.nonzero(sizes >= 16)[0]
    rng = np.random.default_rng(3)
    sample = set(kept[:5].tolist()) | set(rng.choice(kept, 40, replace=False).tolist())
    ctx.line_graph_stream(g, [16], 64 << 20, fn)
    ref = oracle.line_graph_rows(inc, 16, sorted(sample))
    for t, i in enumerate(ref.rows):
        rj, rw = ref.row(t)
        assert np.array_equal(seen[int(i)][0], rj) and np.array_equal(seen[int(i)][1], rw)
    p = ctx.plan(g, [16])
    assert total[0] == p.num_edges()[0] and p.two_paths == oracle.two_paths(inc, 16)
    p.destroy()
    g.release()


def test_batch_matches_per_graph_oracle_and_replays(ctx):
    import torch
    fam = hg.batched_family(count=12, m_lo=200, m_hi=3000)
    graphs = [ctx.register_incidence(mem.inc) for mem in fam]
    s_list = [mem.s for mem in fam]
    b = ctx.batch(graphs, s_list)
    ref = [oracle.line_graph(mem.inc, mem.s) for mem in fam]

    def check(tag):
        for gidx, mem in enumerate(fam):
            lg = b.result(gidx).cpu()
            r = ref[gidx]
            for got, want, f in ((lg.row_ptr, r.row_ptr, "row_ptr"), (lg.row, r.i, "i"), (lg.col, r.j, "j"),
                                 (lg.w, r.w, "w")):
                assert np.array_equal(got.numpy(), want), f"{tag} graph {gidx} {f}"

    check("create")
    assert b.info()["two_paths"] == sum(oracle.two_paths(m.inc, m.s) for m in fam)
    b.run(use_graph=False)
    torch.cuda.synchronize()
    check("eager")
    for rep in range(3):  # graph replays with eager work and syncs between
        junk = torch.randint(0, 100, (1 << 20,), device="cuda").sum()
        b.run(use_graph=True)
        torch.cuda.synchronize()
        check(f"replay {rep}")
        del junk
    b.destroy()
    for g in graphs:
        g.release()


def test_batch_tuning_variants_agree(ctx):
    fam = hg.batched_family(count=6, m_lo=2000, m_hi=20000)
    graphs = [ctx.register_incidence(mem.inc) for mem in fam]
    s_list = [mem.s for mem in fam]
    outs = []
    for tune in ((0, 0, 0), (512, 4096, 64), (2048, 16384, 0)):
        ctx.set_tuning(*tune)
        b = ctx.batch(graphs, s_list)
        outs.append([b.result(g).cpu() for g in range(len(fam))])
        b.destroy()
    ctx.set_tuning()
    for g in range(len(fam)):
        for o in outs[1:]:
            for f in ("row_ptr", "row", "col", "w"):
                assert np.array_equal(getattr(outs[0][g], f).numpy(), getattr(o[g], f).numpy())
        rows = np.linspace(0, fam[g].inc.m - 1, 25).astype(np.int64)
        ref = oracle.line_graph_rows(fam[g].inc, s_list[g], rows)
        rp = outs[0][g].row_ptr.numpy()
        for t, i in enumerate(ref.rows):
            rj, rw = ref.row(t)
            assert np.array_equal(outs[0][g].col.numpy()[rp[i]:rp[i + 1]], rj)
            assert np.array_equal(outs[0][g].w.numpy()[rp[i]:rp[i + 1]], rw)
    for gr in graphs:
        gr.release()


def test_count_store_engages_when_asked(ctx):
    # every row holds vertex 0, so rows have heavy slots (or, with the dense
    # tier forced, at least one 2-path per candidate partner: dense slots);
    # with the store on, the counting pass keeps one entry per distinct
    # heavy partner (s_min = 1: the heavy edges of L_1), with it off none
    inc = planted(6000, 20000, [([0], 1, 0)], 3, seed=17)
    g = ctx.register_incidence(inc)
    p = ctx.plan(g, [1])
    st = p.stats()
    if ctx.dense_mode:  # the same rows on the dense tier: its store keeps the survivors of s_min
        assert st["dense_slots"] > 0 and st["dense_edges"] > 0
        want = st["dense_edges"] if ctx.store_mode == "store" else 0
        assert st["dense_stored"] == want and st["dense_store_full"] == 0
    else:
        assert st["heavy_slots"] > 0 and st["heavy_edges"] > 0
        want = st["heavy_edges"] if ctx.store_mode == "store" else 0
        assert st["stored_ranks"] == want
    p.destroy()
    g.release()
