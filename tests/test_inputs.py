"""The seeded generators produce well-formed inputs of the stated shapes."""
import numpy as np
import pytest

import hypergen as hg


def _check_wellformed(inc):
    assert inc.he_ptr.dtype == np.int64 and inc.v_ptr.dtype == np.int64
    assert inc.he_idx.dtype == np.int32 and inc.v_idx.dtype == np.int32
    assert inc.he_ptr[0] == 0 and inc.he_ptr[-1] == inc.nnz
    assert inc.v_ptr[0] == 0 and inc.v_ptr[-1] == inc.nnz
    rows = np.repeat(np.arange(inc.m), np.diff(inc.he_ptr))
    # rows are strictly increasing sets of valid ids
    same = rows[1:] == rows[:-1]
    assert np.all(inc.he_idx[1:][same] > inc.he_idx[:-1][same])
    assert inc.nnz == 0 or (inc.he_idx.min() >= 0 and inc.he_idx.max() < inc.n)
    # the vertex CSR is the exact transpose, hyperedge ids ascending
    key_he = np.sort(rows.astype(np.int64) * inc.n + inc.he_idx)
    vcol = np.repeat(np.arange(inc.n), np.diff(inc.v_ptr))
    key_v = vcol.astype(np.int64) + inc.v_idx.astype(np.int64) * inc.n
    assert np.array_equal(np.sort(key_v), key_he)
    same_v = vcol[1:] == vcol[:-1]
    assert np.all(inc.v_idx[1:][same_v] > inc.v_idx[:-1][same_v])


def test_tiny_uniform_shape_and_determinism():
    a = hg.tiny_uniform()
    b = hg.tiny_uniform()
    _check_wellformed(a)
    assert a.m == 1000 and a.n == 2000
    sz = a.sizes()
    assert sz.min() >= 2 and sz.max() <= 20
    assert np.array_equal(a.he_idx, b.he_idx)
    c = hg.tiny_uniform(seed=99)
    assert not np.array_equal(a.he_idx[:200], c.he_idx[:200])


def test_random_small_wellformed():
    for seed in range(5):
        _check_wellformed(hg.random_small(seed, 200, 50, 12, 1.5 if seed % 2 else None))


def test_power_law_small_instance_shape():
    inc = hg.power_law(n=20000, m=10000)
    _check_wellformed(inc)
    sz = inc.sizes()
    assert sz.min() >= 2 and sz.max() <= 5000
    # skewed vertex degrees: the heaviest vertex far above the mean
    dv = np.diff(inc.v_ptr)
    assert dv.max() > 20 * dv.mean()


def test_batched_family_members():
    fam = hg.batched_family(count=6, m_hi=5000)
    for mem in fam:
        _check_wellformed(mem.inc)
        assert mem.inc.n == 2 * mem.inc.m
        assert 1 <= mem.s <= 8
        assert mem.inc.sizes().max() <= 1000


def test_toy_and_dual():
    inc = hg.toy_paper_example()
    _check_wellformed(inc)
    d = inc.dual()
    assert d.m == 6 and d.n == 4
    assert list(d.row(1)) == [0, 1, 2]  # vertex b lies in hyperedges 1, 2, 3 (1-based)


@pytest.mark.slow
def test_power_law_full_shape():
    inc = hg.power_law()
    assert inc.m == 500_000 and inc.n == 1_000_000
    _check_wellformed(inc)
