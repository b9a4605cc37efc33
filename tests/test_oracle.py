"""Pins for the CPU oracle: facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself, chosen so
that a plausible slip (dropped term, wrong threshold, i <= j instead of
i < j, H H^T instead of H^T H, pruning the wrong side) fails at least one.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st

import hypergen as hg
import oracle
from helpers import (brute_force_sets, edges_of, load_toy, rows_of, load_toy_components, load_toy_symmetric,
                     load_toy_preprocess, with_subsets)


# --- the worked example of Section I (hand-enumerated fixture) -------------

def test_toy_line_graphs_match_fixture():
    inc, keep, lines, _ = load_toy()
    assert oracle.validate(inc) == 0
    for s in (1, 2, 3, 4):
        lg = oracle.line_graph(inc, s)
        assert edges_of(lg) == lines.get(s, []), f"L_{s}"
        # row_ptr covers all m rows and is consistent with the COO
        assert lg.row_ptr.shape == (inc.m + 1,)
        assert np.all(np.diff(lg.row_ptr) >= 0)
        # E_s membership printed by the paper (E_4 = {3}, 1-based)
        assert [i for i in range(inc.m) if inc.sizes()[i] >= s] == keep[s]


def test_toy_dual_adjacency():
    """adj(b, c) = 3 (Section II-A) is an edge weight of L_1 of the dual."""
    inc, _, _, dual = load_toy()
    lg = oracle.line_graph(inc.dual(), 1)
    pairs = lg.pairs()
    for (i, j, w) in dual[1]:
        assert pairs[(i, j)] == w


def test_toy_two_paths():
    inc, _, lines, _ = load_toy()
    # vertex degrees a..f = 2,3,3,2,2,1 -> 1+3+3+1+1+0 = 9
    assert oracle.two_paths(inc, 1) == 9
    assert sum(w for (_, _, w) in lines[1]) == 9
    # E_3 drops hyperedge 3, so e's degree falls to 1 -> 8
    assert oracle.two_paths(inc, 3) == 8
    assert oracle.two_paths(inc, 4) == 0


# --- L = H^T H (Section II-B) through an independent sparse product --------

def _hth(inc):
    rows = np.repeat(np.arange(inc.m), np.diff(inc.he_ptr))
    H = sp.csr_matrix((np.ones(inc.nnz, np.int64), (inc.he_idx.astype(np.int64), rows)),
                      shape=(inc.n, inc.m))  # n x m, b_ij = 1 iff v_i in e_j
    return (H.T @ H).toarray()


@pytest.mark.parametrize("seed,m,n,kmax,expo", [
    (1, 300, 120, 12, None),
    (2, 400, 60, 25, 0.8),
    (3, 250, 40, 30, 1.5),
    (4, 500, 1000, 8, None),
])
def test_weights_equal_HtH_offdiagonal(seed, m, n, kmax, expo):
    inc = hg.random_small(seed, m, n, kmax, expo)
    L = _hth(inc)
    sizes = inc.sizes()
    assert np.array_equal(np.diag(L), sizes)  # diagonal = |e_i|
    for s in (1, 2, 3, 5):
        lg = oracle.line_graph(inc, s)
        iu, ju = np.triu_indices(inc.m, k=1)
        keep = (L[iu, ju] >= s) & (sizes[iu] >= s) & (sizes[ju] >= s)
        exp = list(zip(iu[keep].tolist(), ju[keep].tolist(), L[iu, ju][keep].tolist()))
        assert edges_of(lg) == exp, f"s={s}"


@pytest.mark.parametrize("seed,m,n,kmax,expo", [
    (11, 300, 120, 12, None),
    (12, 400, 90, 25, 0.8),
    (13, 250, 300, 30, 1.5),
])
def test_dual_is_the_s_clique_graph_of_HHt(seed, m, n, kmax, expo):
    """The s-line graph of the dual H* is the s-clique graph over vertices
    (Section III, relation to the clique-expansion graph): two vertices are
    joined when they share at least s hyperedges, with weight (H H^T)[u, v];
    the diagonal of H H^T is the vertex degree D_V, and E_s of H* keeps the
    vertices of degree >= s. Checked against scipy's H H^T - D_V."""
    inc = hg.random_small(seed, m, n, kmax, expo)
    rows = np.repeat(np.arange(inc.m), np.diff(inc.he_ptr))
    H = sp.csr_matrix((np.ones(inc.nnz, np.int64), (inc.he_idx.astype(np.int64), rows)),
                      shape=(inc.n, inc.m))
    A = (H @ H.T).toarray()
    deg = np.diff(inc.v_ptr)
    assert np.array_equal(np.diag(A), deg)  # D_V
    A = A - np.diag(deg)  # the clique expansion's weighted adjacency
    for s in (1, 2, 3, 4):
        lg = oracle.line_graph(inc.dual(), s)
        iu, ju = np.triu_indices(inc.n, k=1)
        keep = (A[iu, ju] >= s) & (deg[iu] >= s) & (deg[ju] >= s)
        exp = list(zip(iu[keep].tolist(), ju[keep].tolist(), A[iu, ju][keep].tolist()))
        assert edges_of(lg) == exp, f"s={s}"


# --- closed form for the number of 2-paths --------------------------------

@pytest.mark.parametrize("seed,expo", [(5, None), (6, 0.8), (7, 1.5)])
def test_two_paths_closed_form(seed, expo):
    inc = hg.random_small(seed, 400, 150, 15, expo)
    sizes = inc.sizes()
    rows = np.repeat(np.arange(inc.m), sizes)
    for s in (1, 2, 4):
        kept = sizes[rows] >= s
        d = np.bincount(inc.he_idx[kept], minlength=inc.n).astype(np.int64)
        closed = int((d * (d - 1) // 2).sum())
        assert oracle.two_paths(inc, s) == closed
        # every 2-path lands on exactly one intersecting pair of E_s
        lg1 = oracle.line_graph(inc, 1, size_min=s)
        assert int(lg1.w.astype(np.int64).sum()) == closed
        per_row = oracle.row_two_paths(inc, s, np.arange(inc.m))
        assert int(per_row.sum()) == closed


# --- graphs are 2-uniform hypergraphs (Section I) -------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_two_uniform_is_textbook_line_graph(seed):
    rng = np.random.default_rng(seed)
    nv = 60
    all_pairs = list(itertools.combinations(range(nv), 2))
    pick = rng.choice(len(all_pairs), size=150, replace=False)
    graph_edges = [all_pairs[k] for k in sorted(pick)]
    inc = hg.from_rows(graph_edges, n=nv)
    lg = oracle.line_graph(inc, 1)
    exp = [(a, b, 1) for a, b in itertools.combinations(range(len(graph_edges)), 2)
           if set(graph_edges[a]) & set(graph_edges[b])]
    assert edges_of(lg) == exp
    deg = np.bincount(np.array(graph_edges).ravel(), minlength=nv)
    assert lg.num_edges == int((deg * (deg - 1) // 2).sum())
    assert oracle.line_graph(inc, 2).num_edges == 0


# --- invariants ----------------------------------------------------------

def test_nested_filtration_and_weight_bounds():
    inc = hg.random_small(11, 600, 80, 20, 0.8)
    sizes = inc.sizes()
    prev = None
    for s in range(1, 9):
        lg = oracle.line_graph(inc, s)
        pairs = lg.pairs()
        for (i, j), w in pairs.items():
            assert i < j
            assert s <= w <= min(sizes[i], sizes[j])
        if prev is not None:
            # L_{s} is contained in L_{s-1} with the same weights
            for k, w in pairs.items():
                assert prev[k] == w
            assert set(prev) - set(pairs) == {k for k, w in prev.items() if w < s}
        prev = pairs


def test_vertex_and_hyperedge_permutation():
    inc = hg.random_small(12, 300, 70, 15, 0.8)
    rng = np.random.default_rng(3)
    vperm = rng.permutation(inc.n)
    rows = rows_of(inc)
    inc_v = hg.from_rows([[int(vperm[v]) for v in r] for r in rows], n=inc.n)
    eperm = rng.permutation(inc.m)  # new id of old hyperedge k is eperm[k]
    new_rows = [None] * inc.m
    for k, r in enumerate(rows):
        new_rows[eperm[k]] = r
    inc_e = hg.from_rows(new_rows, n=inc.n)
    for s in (1, 2, 3):
        base = oracle.line_graph(inc, s).pairs()
        assert oracle.line_graph(inc_v, s).pairs() == base
        mapped = {(min(eperm[i], eperm[j]), max(eperm[i], eperm[j])): w for (i, j), w in base.items()}
        assert oracle.line_graph(inc_e, s).pairs() == mapped


def test_duplicate_hyperedges_are_distinct_and_joined():
    inc = hg.from_rows([[0, 1, 2], [3, 4], [0, 1, 2], [5]], n=6)
    assert edges_of(oracle.line_graph(inc, 3)) == [(0, 2, 3)]
    assert edges_of(oracle.line_graph(inc, 1)) == [(0, 2, 3)]


def test_disjoint_union_is_block_result():
    a = hg.random_small(21, 120, 40, 10, None)
    b = hg.random_small(22, 90, 30, 10, 1.5)
    rows = rows_of(a) + [[v + a.n for v in r] for r in rows_of(b)]
    u = hg.from_rows(rows, n=a.n + b.n)
    for s in (1, 2, 3):
        pa = oracle.line_graph(a, s).pairs()
        pb = oracle.line_graph(b, s).pairs()
        exp = dict(pa)
        exp.update({(i + a.m, j + a.m): w for (i, j), w in pb.items()})
        assert oracle.line_graph(u, s).pairs() == exp


def test_edge_cases():
    empty = hg.from_rows([], n=0)
    assert oracle.line_graph(empty, 1).num_edges == 0
    hollow = hg.from_rows([[], [], []], n=4)
    lg = oracle.line_graph(hollow, 1)
    assert lg.num_edges == 0 and list(lg.row_ptr) == [0, 0, 0, 0]
    inc = hg.tiny_uniform()
    assert oracle.line_graph(inc, int(inc.sizes().max()) + 1).num_edges == 0
    with pytest.raises(ValueError):
        oracle.line_graph(inc, 0)


def test_validate_rejects_malformed():
    inc = hg.from_rows([[0, 1, 2], [1, 3]], n=4)
    assert oracle.validate(inc) == 0
    bad = hg.Incidence(2, 4, inc.he_ptr.copy(), inc.he_idx.copy(), inc.v_ptr, inc.v_idx)
    bad.he_idx[1] = 0  # row 0 becomes [0, 0, 2]: not a set
    assert oracle.validate(bad) == 3
    bad2 = hg.Incidence(2, 4, inc.he_ptr.copy(), inc.he_idx.copy(), inc.v_ptr, inc.v_idx)
    bad2.he_idx[-1] = 9
    assert oracle.validate(bad2) == 2
    bad3 = hg.Incidence(2, 4, np.array([0, 4, 3]), inc.he_idx, inc.v_ptr, inc.v_idx)
    assert oracle.validate(bad3) == 1


def test_tiny_uniform_rows_against_sets():
    inc = hg.tiny_uniform()
    rows = rows_of(inc)
    for s in (1, 2, 3, 4):
        assert edges_of(oracle.line_graph(inc, s)) == brute_force_sets(rows, s)


@settings(max_examples=60, deadline=None)
@given(st.lists(st.sets(st.integers(0, 11), max_size=8), max_size=14), st.integers(1, 4))
def test_random_sets_brute_force(sets_, s):
    rows = [sorted(x) for x in sets_]
    inc = hg.from_rows(rows, n=12)
    assert edges_of(oracle.line_graph(inc, s)) == brute_force_sets(rows, s)


def test_sampled_rows_match_full_graph():
    inc = hg.random_small(31, 500, 100, 12, 0.8)
    full = oracle.line_graph(inc, 2)
    sample = [0, 7, 99, 250, 498, 499]
    r = oracle.line_graph_rows(inc, 2, sample)
    for k, i in enumerate(sample):
        j, w = r.row(k)
        a, b = full.row_ptr[i], full.row_ptr[i + 1]
        assert np.array_equal(j, full.j[a:b]) and np.array_equal(w, full.w[a:b])


# --- s-connected components and ID squeezing -------------------------------

def _canonical(labels):
    """Component labels as the smallest member id (-1 stays -1)."""
    labels = np.asarray(labels)
    out = np.full(labels.shape, -1, dtype=np.int64)
    first = {}
    for i, l in enumerate(labels):
        if l < 0:
            continue
        first.setdefault(int(l), i)
        out[i] = first[int(l)]
    return out


def test_components_and_squeeze_of_the_worked_example():
    inc, _, _, _ = load_toy()
    cc, sq = load_toy_components()
    for s, want in cc.items():
        lab, count = oracle.components(inc, s)
        assert lab.tolist() == want
        assert count == len({l for l in want if l >= 0})
        lg = oracle.line_graph(inc, s)
        lab2, count2 = oracle.components(inc, s, lg.i, lg.j)
        assert lab2.tolist() == want and count2 == count
        new_id, kept = oracle.squeeze(inc.m, lg.i, lg.j)
        assert new_id.tolist() == sq[s] and kept == sum(1 for x in sq[s] if x >= 0)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_components_match_scipy_on_the_thresholded_product(seed):
    from scipy.sparse.csgraph import connected_components
    inc = hg.random_small(seed + 40, m=70, n=30, kmax=9, exponent=1.0)
    H = sp.csr_matrix((np.ones(inc.nnz), inc.he_idx, inc.he_ptr), shape=(inc.m, inc.n))
    G = (H @ H.T).tocsr()  # (H^T H) in hyperedge x hyperedge orientation
    sizes = inc.sizes()
    for s in (1, 2, 3):
        keep = np.flatnonzero(sizes >= s)
        A = G[keep][:, keep].tolil()
        A.setdiag(0)
        A = (A.tocsr() >= s).astype(np.int8)
        _, comp = connected_components(A, directed=False)
        ref = np.full(inc.m, -1)
        for c in np.unique(comp):
            members = keep[comp == c]
            ref[members] = members.min()
        lab, count = oracle.components(inc, s)
        np.testing.assert_array_equal(lab, ref)
        assert count == len(np.unique(comp)) if keep.size else count == 0
        lg = oracle.line_graph(inc, s)
        lab2, _ = oracle.components(inc, s, lg.i, lg.j)
        np.testing.assert_array_equal(lab2, ref)


def test_components_refine_as_s_grows():
    inc = hg.random_small(77, m=120, n=40, kmax=12, exponent=1.1)
    prev = None
    for s in range(1, 6):
        lab, _ = oracle.components(inc, s)
        if prev is not None:
            kept = np.flatnonzero(lab >= 0)
            assert np.all(prev[kept] >= 0)  # E_{s+1} is inside E_s
            for a in kept:  # same component at s+1 => same component at s
                same = kept[lab[kept] == lab[a]]
                assert np.all(prev[same] == prev[a])
        prev = lab


def test_squeeze_is_the_order_preserving_rank_of_the_edge_ends():
    rng = np.random.default_rng(5)
    m = 50
    row = rng.integers(0, m, 40).astype(np.int32)
    col = rng.integers(0, m, 40).astype(np.int32)
    new_id, kept = oracle.squeeze(m, row, col)
    ends = sorted(set(row.tolist()) | set(col.tolist()))
    assert kept == len(ends)
    assert [int(new_id[e]) for e in ends] == list(range(kept))
    assert all(new_id[i] == -1 for i in range(m) if i not in set(ends))


# --- symmetric CSR (Stage 4) ----------------------------------------------

def _sym_rows(ptr, col, w):
    return [list(zip(col[ptr[r]:ptr[r + 1]].tolist(), w[ptr[r]:ptr[r + 1]].tolist()))
            for r in range(len(ptr) - 1)]


def test_symmetric_of_the_worked_example():
    inc, _, _, _ = load_toy()
    want = load_toy_symmetric()
    for s in (1, 2, 3, 4):
        lg = oracle.line_graph(inc, s)
        ptr, col, w = oracle.symmetric(inc.m, lg.i, lg.j, lg.w)
        assert _sym_rows(ptr, col, w) == want[s], f"s={s}"


@pytest.mark.parametrize("seed,m,n,kmax,expo", [(11, 300, 90, 14, 1.0), (12, 200, 400, 9, None)])
def test_symmetric_matches_scipy_thresholded_product(seed, m, n, kmax, expo):
    # off the diagonal, the thresholded H^T H on E_s is the symmetric
    # adjacency of L_s; scipy's CSR with sorted indices is its row form
    inc = hg.random_small(seed, m, n, kmax, expo)
    H = sp.csr_matrix((np.ones(inc.nnz, np.int64), inc.he_idx, inc.he_ptr), shape=(inc.m, inc.n))
    G = (H @ H.T).tocsr()
    sizes = inc.sizes()
    for s in (1, 2, 4):
        off = sizes < s
        A = G.tolil()
        A.setdiag(0)
        A = A.tocsr()
        A = sp.diags((~off).astype(np.int64)) @ A @ sp.diags((~off).astype(np.int64))
        A.data[A.data < s] = 0
        A.eliminate_zeros()
        A.sort_indices()
        lg = oracle.line_graph(inc, s)
        ptr, col, w = oracle.symmetric(inc.m, lg.i, lg.j, lg.w)
        np.testing.assert_array_equal(ptr, A.indptr)
        np.testing.assert_array_equal(col, A.indices)
        np.testing.assert_array_equal(w, A.data)


def test_symmetric_is_its_own_transpose_and_doubles_the_edges():
    inc = hg.random_small(13, 400, 150, 12, 0.9)
    lg = oracle.line_graph(inc, 2)
    ptr, col, w = oracle.symmetric(inc.m, lg.i, lg.j, lg.w)
    assert ptr[-1] == 2 * len(lg.j)
    rows = np.repeat(np.arange(inc.m), np.diff(ptr))
    fwd = set(zip(rows.tolist(), col.tolist(), w.tolist()))
    assert fwd == set(zip(col.tolist(), rows.tolist(), w.tolist()))
    assert all(np.all(np.diff(col[ptr[r]:ptr[r + 1]]) > 0) for r in range(inc.m))


# --- relabel-by-degree, selection, toplexes (Stages 1-2) --------------------

def _as_incidence(inc, arrays):
    he_ptr, he_idx, v_ptr, v_idx = arrays
    return hg.Incidence(len(he_ptr) - 1, inc.n, he_ptr, he_idx, v_ptr, v_idx)


def test_preprocessing_of_the_worked_example():
    inc, _, _, _ = load_toy()
    want = load_toy_preprocess()
    assert oracle.relabel_order(inc).tolist() == want["asc"]
    assert oracle.relabel_order(inc, descending=True).tolist() == want["desc"]
    assert oracle.toplexes(inc).tolist() == want["top"]
    lg = oracle.line_graph(inc, 1)
    assert oracle.toplexes_from_edges(inc, lg.i, lg.j, lg.w).tolist() == want["top"]


@pytest.mark.parametrize("seed,descending", [(21, False), (22, True), (23, False)])
def test_relabelled_line_graph_maps_back_to_the_original(seed, descending):
    inc = hg.random_small(seed, 300, 100, 14, 1.0)
    order = oracle.relabel_order(inc, descending)
    sizes = inc.sizes()[order]
    assert sorted(order.tolist()) == list(range(inc.m))
    assert np.all(np.diff(sizes) <= 0) if descending else np.all(np.diff(sizes) >= 0)
    sub = _as_incidence(inc, oracle.select(inc, order))
    # the vertex CSR is the exact transpose (an independent stable transpose)
    ptr_t, idx_t = hg.transpose_csr(sub.m, sub.n, sub.he_ptr, sub.he_idx)
    np.testing.assert_array_equal(sub.v_ptr, ptr_t)
    np.testing.assert_array_equal(sub.v_idx, idx_t)
    for s in (1, 2, 3):
        a = oracle.line_graph(sub, s)
        i, j = order[a.i], order[a.j]
        got = sorted(zip(np.minimum(i, j).tolist(), np.maximum(i, j).tolist(), a.w.tolist()))
        assert got == edges_of(oracle.line_graph(inc, s)), f"s={s}"


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_toplexes_brute_force_and_from_edges_agree(seed):
    inc = with_subsets(seed, 120, 40, 10, 60)
    top = oracle.toplexes(inc)
    lg = oracle.line_graph(inc, 1)
    np.testing.assert_array_equal(oracle.toplexes_from_edges(inc, lg.i, lg.j, lg.w), top)
    # no kept hyperedge inside another kept one; every dropped non-empty one
    # lies inside a kept one
    sets = [frozenset(inc.row(i).tolist()) for i in range(inc.m)]
    kept = set(top.tolist())
    for a in kept:
        assert not any(b != a and sets[a] <= sets[b] for b in kept)
    for a in range(inc.m):
        if a not in kept and sets[a]:
            assert any(sets[a] <= sets[b] for b in kept)


def test_select_of_a_subset():
    inc = hg.random_small(41, 200, 60, 9, None)
    order = np.array([150, 3, 77, 4, 199], dtype=np.int32)
    he_ptr, he_idx, v_ptr, v_idx = oracle.select(inc, order)
    for k, i in enumerate(order):
        assert he_idx[he_ptr[k]:he_ptr[k + 1]].tolist() == inc.row(int(i)).tolist()
    ptr_t, idx_t = hg.transpose_csr(len(order), inc.n, he_ptr, he_idx)
    np.testing.assert_array_equal(v_ptr, ptr_t)
    np.testing.assert_array_equal(v_idx, idx_t)


# --- edge-list digest ------------------------------------------------------

def test_splitmix64_matches_the_published_sequence():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
    want = [int(l, 16) for l in open(path) if l.strip() and not l.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    states = np.array([(k * gamma) % (1 << 64) for k in range(len(want))], dtype=np.uint64)
    got = [int(v) for v in oracle._splitmix64(states)]
    assert got == want


def test_digest_is_order_free_additive_and_sensitive():
    inc = hg.random_small(91, 300, 100, 12, 1.0)
    lg = oracle.line_graph(inc, 1)
    d = oracle.digest(lg.i, lg.j, lg.w)
    assert d[0] == len(lg.j) and d[1] == int(lg.w.sum())
    perm = np.random.default_rng(0).permutation(len(lg.j))
    assert oracle.digest(lg.i[perm], lg.j[perm], lg.w[perm]) == d
    cut = len(lg.j) // 3
    a = oracle.digest(lg.i[:cut], lg.j[:cut], lg.w[:cut])
    b = oracle.digest(lg.i[cut:], lg.j[cut:], lg.w[cut:])
    assert (a[0] + b[0], a[1] + b[1], (a[2] + b[2]) % (1 << 64)) == d
    w2 = lg.w.copy()
    w2[5] += 1
    assert oracle.digest(lg.i, lg.j, w2)[2] != d[2]
    j2 = lg.j.copy()
    j2[7] += 1
    assert oracle.digest(lg.i, j2, lg.w)[2] != d[2]
