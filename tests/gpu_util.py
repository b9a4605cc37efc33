"""Helpers for GPU tests: run the library, pull results to the host, compare
against the oracle element by element."""
from __future__ import annotations

import numpy as np

import hypergen as hg
import oracle


def planted(m: int, n: int, groups, extra: int, seed: int) -> hg.Incidence:
    """Rows hold `extra` uniform random vertices from [len(groups_vertices), n)
    plus, for every (vertices, step, offset) group, those vertices whenever
    row % step == offset. Input construction only."""
    rng = np.random.default_rng(seed)
    planted_v = sorted({v for vs, _, _ in groups for v in vs})
    lo = (max(planted_v) + 1) if planted_v else 0
    rows = []
    for r in range(m):
        members = set(rng.integers(lo, n, size=extra).tolist()) if extra else set()
        for vs, step, off in groups:
            if r % step == off:
                members.update(vs)
        rows.append(sorted(members))
    return hg.from_rows(rows, n=n)


def run_gpu(ctx, inc, s_list, stream=None, one_shot=False):
    g = ctx.register_incidence(inc)
    outs = (ctx.line_graph_result(g, s_list, stream) if one_shot
            else ctx.line_graph(g, s_list, stream))
    host = [o.cpu() for o in outs]
    g.release()
    return host


def assert_matches_oracle(inc, lg, s, what=""):
    """Whole-graph, element-by-element comparison with the oracle."""
    ref = oracle.line_graph(inc, s)
    np.testing.assert_array_equal(lg.row_ptr.numpy(), ref.row_ptr, err_msg=f"{what} s={s} row_ptr")
    np.testing.assert_array_equal(lg.col.numpy(), ref.j, err_msg=f"{what} s={s} col")
    np.testing.assert_array_equal(lg.w.numpy(), ref.w, err_msg=f"{what} s={s} w")
    np.testing.assert_array_equal(lg.row.numpy(), ref.i, err_msg=f"{what} s={s} row")


def assert_rows_match_oracle(inc, lg, s, rows, what="", threads=0):
    """Sampled rows: row i of the GPU result == oracle row i (all j > i)."""
    ref = oracle.line_graph_rows(inc, s, rows, threads=threads)
    rp = lg.row_ptr.numpy()
    col = lg.col.numpy()
    w = lg.w.numpy()
    for k, i in enumerate(ref.rows):
        a, b = int(rp[i]), int(rp[i + 1])
        rj, rw = ref.row(k)
        np.testing.assert_array_equal(col[a:b], rj, err_msg=f"{what} s={s} row {i} col")
        np.testing.assert_array_equal(w[a:b], rw, err_msg=f"{what} s={s} row {i} w")


def assert_well_formed(inc, lg, s):
    """Properties that hold at any size: sorted rows, i < j, weight bounds."""
    rp = lg.row_ptr.numpy()
    assert rp[0] == 0 and rp[-1] == lg.num_edges and np.all(np.diff(rp) >= 0)
    row = lg.row.numpy()
    col = lg.col.numpy()
    w = lg.w.numpy()
    np.testing.assert_array_equal(row, np.repeat(np.arange(inc.m, dtype=np.int32), np.diff(rp)))
    assert np.all(col > row)
    same = row[1:] == row[:-1]
    assert np.all(col[1:][same] > col[:-1][same])
    sizes = inc.sizes()
    assert np.all(w >= s)
    assert np.all(w <= np.minimum(sizes[row], sizes[col]))
