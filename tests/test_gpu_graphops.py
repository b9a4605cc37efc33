"""s-connected components, ID squeezing and the symmetric CSR on the
device, through the C ABI, against the oracle (bit for bit)."""
from __future__ import annotations

import numpy as np
import pytest

import hypergen as hg
import oracle
from gpu_util import planted
from helpers import load_toy, load_toy_components, load_toy_symmetric

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    yield c
    c.close()


def check(ctx, inc, s_list, what):
    """Device labels and ids against the oracle's, both computed from each
    side's own L_s (the edge lists themselves are compared first)."""
    g = ctx.register_incidence(inc)
    outs = ctx.line_graph(g, s_list)
    for lg in outs:
        ref_lg = oracle.line_graph(inc, lg.s)
        host = lg.cpu()
        np.testing.assert_array_equal(host.row.numpy(), ref_lg.i)
        np.testing.assert_array_equal(host.col.numpy(), ref_lg.j)
        labels, count = ctx.components(g, lg.s, lg)
        ref, ref_count = oracle.components(inc, lg.s, ref_lg.i, ref_lg.j)
        np.testing.assert_array_equal(labels.cpu().numpy(), ref, err_msg=f"{what} s={lg.s} labels")
        assert count == ref_count, (what, lg.s)
        sym_ptr, sym_col, sym_w = ctx.symmetrize(lg)
        ref_ptr, ref_col, ref_w = oracle.symmetric(inc.m, ref_lg.i, ref_lg.j, ref_lg.w)
        np.testing.assert_array_equal(sym_ptr.cpu().numpy(), ref_ptr, err_msg=f"{what} s={lg.s} sym_ptr")
        np.testing.assert_array_equal(sym_col.cpu().numpy(), ref_col, err_msg=f"{what} s={lg.s} sym_col")
        np.testing.assert_array_equal(sym_w.cpu().numpy(), ref_w, err_msg=f"{what} s={lg.s} sym_w")
        new_id, kept = ctx.squeeze(inc.m, lg)
        ref_id, ref_kept = oracle.squeeze(inc.m, ref_lg.i, ref_lg.j)
        np.testing.assert_array_equal(new_id.cpu().numpy(), ref_id, err_msg=f"{what} s={lg.s} squeeze")
        assert kept == ref_kept
        # in place: the edge list takes the new ids and stays sorted
        ctx.squeeze(inc.m, lg, remap=True)
        np.testing.assert_array_equal(lg.row.cpu().numpy(), ref_id[ref_lg.i])
        np.testing.assert_array_equal(lg.col.cpu().numpy(), ref_id[ref_lg.j])
    g.release()


def test_worked_example(ctx):
    inc, _, _, _ = load_toy()
    cc, sq = load_toy_components()
    g = ctx.register_incidence(inc)
    for s in (1, 2, 3, 4):
        lg = ctx.line_graph(g, [s])[0]
        labels, count = ctx.components(g, s, lg)
        assert labels.cpu().tolist() == cc[s]
        assert count == len({l for l in cc[s] if l >= 0})
        new_id, kept = ctx.squeeze(inc.m, lg)
        assert new_id.cpu().tolist() == sq[s]
        sym_ptr, sym_col, sym_w = ctx.symmetrize(lg)
        ptr, col, w = sym_ptr.cpu().numpy(), sym_col.cpu().numpy(), sym_w.cpu().numpy()
        rows = [list(zip(col[ptr[r]:ptr[r + 1]].tolist(), w[ptr[r]:ptr[r + 1]].tolist())) for r in range(inc.m)]
        assert rows == load_toy_symmetric()[s], f"s={s}"
    g.release()


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_random_graphs(ctx, seed):
    inc = hg.random_small(seed + 100, m=3000, n=2500, kmax=12, exponent=1.2, kmin=0)
    check(ctx, inc, [1, 2, 3, 5], f"random {seed}")


def test_many_small_components_and_a_giant(ctx):
    # blocks of rows sharing a private vertex give many components; one
    # vertex in every 7th row merges those rows into one giant component
    inc = planted(8000, 30000, [([0], 7, 3)], 2, seed=12)
    check(ctx, inc, [1, 2], "planted")


def test_power_law_thresholds(ctx):
    inc = hg.power_law(n=40_000, m=20_000, seed=21)
    check(ctx, inc, [2, 4, 8], "power law")


def test_errors(ctx):
    import torch

    import paper_2201_11326_amd as slg
    inc = hg.tiny_uniform()
    g = ctx.register_incidence(inc)
    lg = ctx.line_graph(g, [2])[0]
    with pytest.raises(slg.SlgError):  # an edge end outside E_3 (|e| = 2 rows exist)
        ctx.components(g, 30, lg)
    bad = slg.LineGraph(1, lg.row_ptr, torch.full((3,), inc.m + 5, dtype=torch.int32, device="cuda"),
                        torch.zeros(3, dtype=torch.int32, device="cuda"),
                        torch.ones(3, dtype=torch.int32, device="cuda"), 0)
    with pytest.raises(slg.SlgError):
        ctx.components(g, 1, bad)
    with pytest.raises(slg.SlgError):
        ctx.squeeze(inc.m, bad)
    g.release()
