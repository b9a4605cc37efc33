"""Graph registration with SLG_COPY: the library's own device copies, from
host arrays or from device tensors the caller then reuses; results equal
the oracle's."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import hypergen as hg
import oracle
from gpu_util import assert_matches_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2201_11326_amd as slg
    c = slg.Context(0)
    yield c
    c.close()


def test_copy_from_host_arrays(ctx):
    inc = hg.random_small(81, 2000, 600, 25, 1.0)
    g = ctx.register_host(inc, validate=True)
    for lg in ctx.line_graph(g, [1, 3]):
        assert_matches_oracle(inc, lg.cpu(), lg.s, "host copy")
    g.release()


def test_copy_from_device_tensors_then_reused(ctx):
    import torch
    inc = hg.random_small(82, 1500, 400, 30, 1.2)
    dev = torch.device("cuda", 0)
    t = [torch.as_tensor(inc.he_ptr, dtype=torch.int64).to(dev), torch.as_tensor(inc.he_idx, dtype=torch.int32).to(dev),
         torch.as_tensor(inc.v_ptr, dtype=torch.int64).to(dev), torch.as_tensor(inc.v_idx, dtype=torch.int32).to(dev)]
    g = ctx.register(inc.m, inc.n, *t, copy=True)
    for x in t:  # the caller's arrays are free again
        x.fill_(-1)
    del t
    torch.cuda.synchronize()
    for lg in ctx.line_graph(g, [1, 2]):
        assert_matches_oracle(inc, lg.cpu(), lg.s, "device copy")
    g.release()


def test_copy_validate_rejects_and_flags_are_checked(ctx):
    import paper_2201_11326_amd as slg
    inc = hg.random_small(83, 200, 80, 10, None)
    bad = hg.Incidence(inc.m, inc.n, inc.he_ptr, inc.he_idx.copy(), inc.v_ptr, inc.v_idx)
    bad.he_idx[0] = inc.n + 5  # a vertex id out of range
    with pytest.raises(slg.SlgError) as ei:
        ctx.register_host(bad, validate=True)
    assert ei.value.status == slg.SLG_ERR_INVALID_GRAPH
    arrs = [np.ascontiguousarray(a) for a in (inc.he_ptr, inc.he_idx, inc.v_ptr, inc.v_idx)]
    c = slg.Incidence(inc.n, inc.m, inc.nnz, *[a.ctypes.data for a in arrs])
    h = ctypes.c_void_p()
    st = slg.lib().slg_graph_register(ctx.handle, ctypes.byref(c), 4, None, ctypes.byref(h))
    assert st == slg.SLG_ERR_INVALID_ARG and not h.value
    # the context still works
    g = ctx.register_host(inc)
    assert_matches_oracle(inc, ctx.line_graph(g, [1])[0].cpu(), 1, "after errors")
    g.release()
