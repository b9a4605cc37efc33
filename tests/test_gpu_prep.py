"""Relabel-by-degree, toplexes and selection on the device (Stages 1-2 of
the framework), through the C ABI, against the oracle bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

import hypergen as hg
import oracle
from helpers import load_toy, load_toy_preprocess, with_subsets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    yield c
    c.close()


def _arrays(g):
    return [t.cpu().numpy() for t in g._tensors]


def _check_select(ctx, inc, g, order, what):
    sub = ctx.select(g, __import__("torch").as_tensor(order, dtype=__import__("torch").int32))
    got = _arrays(sub)
    want = oracle.select(inc, order)
    for name, a, b in zip(("he_ptr", "he_idx", "v_ptr", "v_idx"), got, want):
        np.testing.assert_array_equal(a, b, err_msg=f"{what} {name}")
    return sub


def test_worked_example(ctx):
    inc, _, _, _ = load_toy()
    want = load_toy_preprocess()
    g = ctx.register_incidence(inc)
    assert ctx.relabel_order(g).cpu().tolist() == want["asc"]
    assert ctx.relabel_order(g, descending=True).cpu().tolist() == want["desc"]
    l1 = ctx.line_graph(g, [1])[0]
    assert ctx.toplexes(g, l1).cpu().tolist() == want["top"]
    simple, ids = ctx.simplify(g, l1)
    assert ids.cpu().tolist() == want["top"]
    _check_select(ctx, inc, g, np.asarray(want["top"], np.int32), "toy simplify")
    g.release()


@pytest.mark.parametrize("seed,m,n,kmax,expo", [(51, 3000, 400, 30, 0.8), (52, 20000, 5000, 12, 1.2)])
def test_relabel_matches_oracle_and_maps_back(ctx, seed, m, n, kmax, expo):
    inc = hg.random_small(seed, m, n, kmax, expo)
    g = ctx.register_incidence(inc)
    for desc in (False, True):
        order = ctx.relabel_order(g, desc).cpu().numpy()
        np.testing.assert_array_equal(order, oracle.relabel_order(inc, desc))
        sub = _check_select(ctx, inc, g, order, f"relabel desc={desc}")
        # the relabelled graph's L_s, mapped back, is the oracle's L_s
        for lg in ctx.line_graph(sub, [1, 3]):
            h = lg.cpu()
            i, j = order[h.row.numpy()], order[h.col.numpy()]
            a, b = np.minimum(i, j).astype(np.int64), np.maximum(i, j).astype(np.int64)
            idx = np.lexsort((b, a))
            ref = oracle.line_graph(inc, lg.s)
            np.testing.assert_array_equal(a[idx], ref.i)
            np.testing.assert_array_equal(b[idx], ref.j)
            np.testing.assert_array_equal(h.w.numpy()[idx], ref.w)
        sub.release()
    g.release()


@pytest.mark.parametrize("seed,m,n,kmax,extra", [(61, 400, 60, 12, 200), (62, 3000, 300, 20, 1500)])
def test_toplexes_and_simplification(ctx, seed, m, n, kmax, extra):
    inc = with_subsets(seed, m, n, kmax, extra)
    g = ctx.register_incidence(inc)
    l1 = ctx.line_graph(g, [1])[0]
    ref_l1 = oracle.line_graph(inc, 1)
    want = oracle.toplexes_from_edges(inc, ref_l1.i, ref_l1.j, ref_l1.w)
    if inc.m <= 600:
        np.testing.assert_array_equal(want, oracle.toplexes(inc))
    ids = ctx.toplexes(g, l1).cpu().numpy()
    np.testing.assert_array_equal(ids, want)
    sub = _check_select(ctx, inc, g, ids, "simplify")
    sub.release()
    g.release()


def test_power_law_relabel(ctx):
    inc = hg.power_law()
    g = ctx.register_incidence(inc)
    order = ctx.relabel_order(g).cpu().numpy()
    np.testing.assert_array_equal(order, oracle.relabel_order(inc))
    sub = _check_select(ctx, inc, g, order, "power law")
    sub.release()
    g.release()


def test_errors(ctx):
    import torch

    import paper_2201_11326_amd as slg
    inc = hg.random_small(71, 100, 50, 8, None)
    g = ctx.register_incidence(inc)
    for bad in ([0, 1, 1], [0, 100], [-1]):
        with pytest.raises(slg.SlgError) as ei:
            ctx.select(g, torch.as_tensor(bad, dtype=torch.int32))
        assert ei.value.status == slg.SLG_ERR_INVALID_ARG
    l1 = ctx.line_graph(g, [1])[0]
    l1.w.fill_(1000)  # overlaps above every size: not the edges of L_1
    if l1.num_edges:
        with pytest.raises(slg.SlgError):
            ctx.toplexes(g, l1)
    empty = ctx.select(g, torch.zeros(0, dtype=torch.int32))
    assert empty.m == 0 and int(empty._tensors[1].numel()) == 0
    assert ctx.line_graph(empty, [1])[0].num_edges == 0
    g.release()
