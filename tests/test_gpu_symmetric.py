"""Symmetric CSR of an edge list on the device (slg_symmetrize, the stable
radix sort behind it), through the C ABI, against the oracle bit for bit.
Inputs are seeded upper-triangle edge lists from hypergen, sized so that the
sort takes one, two and three digit passes."""
from __future__ import annotations

import numpy as np
import pytest

import hypergen as hg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    yield c
    c.close()


class _Edges:
    """The shape of a LineGraph, on the device, for an edge list."""

    def __init__(self, row_ptr, row, col, w):
        import torch
        self.row_ptr = torch.from_numpy(row_ptr).cuda()
        self.row = torch.from_numpy(row).cuda()
        self.col = torch.from_numpy(col).cuda()
        self.w = torch.from_numpy(w).cuda()
        self.num_edges = int(row.shape[0])


def _check(ctx, m, row_ptr, row, col, w, weights=True):
    got_ptr, got_col, got_w = ctx.symmetrize(_Edges(row_ptr, row, col, w), weights=weights)
    ref_ptr, ref_col, ref_w = oracle.symmetric(m, row, col, w)
    np.testing.assert_array_equal(got_ptr.cpu().numpy(), ref_ptr)
    np.testing.assert_array_equal(got_col.cpu().numpy(), ref_col)
    if weights:
        np.testing.assert_array_equal(got_w.cpu().numpy(), ref_w)
    else:
        assert got_w is None


@pytest.mark.parametrize("seed,m,count,expo", [
    (1, 2, 8, 0.0),             # two ids: one 1-bit pass
    (2, 200, 5000, 0.5),        # one 8-bit pass
    (3, 256, 20000, 1.2),       # keys fill exactly 8 bits
    (4, 257, 20000, 1.2),       # two passes of 5 bits
    (5, 65536, 400000, 1.0),    # two full 8-bit passes
    (6, 65537, 400000, 1.0),    # three passes
    (7, 300000, 4000000, 1.0),  # three passes, hub columns of ~7e4 entries, ragged last chunk
])
def test_matches_oracle(ctx, seed, m, count, expo):
    row_ptr, row, col, w = hg.random_upper_edges(seed, m, count, expo)
    _check(ctx, m, row_ptr, row, col, w)


def test_structure_only(ctx):
    row_ptr, row, col, w = hg.random_upper_edges(8, 5000, 100000, 1.0)
    _check(ctx, 5000, row_ptr, row, col, w, weights=False)


def test_empty_and_edgeless(ctx):
    for m in (0, 1, 7):
        row_ptr = np.zeros(m + 1, np.int64)
        e = np.zeros(0, np.int32)
        _check(ctx, m, row_ptr, e, e, e)


def test_rejects_what_is_not_an_upper_triangle(ctx):
    import paper_2201_11326_amd as slg
    row_ptr, row, col, w = hg.random_upper_edges(9, 1000, 20000, 1.0)
    bad = []
    r2, c2 = row.copy(), col.copy()
    r2[5], c2[5] = c2[5], r2[5]  # a lower-triangle entry
    bad.append((row_ptr, r2, c2))
    k = int(np.flatnonzero(np.diff(row) == 0)[0])
    c3 = col.copy()
    c3[k], c3[k + 1] = c3[k + 1], c3[k]  # a row out of order
    bad.append((row_ptr, row, c3))
    p4 = row_ptr.copy()
    p4[-1] += 1  # pointers that do not end at the edge count
    bad.append((p4, row, col))
    c5 = col.copy()
    c5[0] = 1000  # a column outside [0, m)
    bad.append((row_ptr, row, c5))
    for rp, r, c in bad:
        with pytest.raises(slg.SlgError) as ei:
            ctx.symmetrize(_Edges(rp, r, c, w))
        assert ei.value.status == slg.SLG_ERR_INVALID_ARG
    # the context stays usable
    _check(ctx, 1000, row_ptr, row, col, w)
