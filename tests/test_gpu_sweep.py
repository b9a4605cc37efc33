"""A seeded sweep of random hypergraph shapes and s-sets through the C ABI,
with and without the count store and with the dense tier forced, each compared with the oracle element by
element (sizes from a single row to a few thousand, empty hyperedges,
ragged tiles)."""
from __future__ import annotations

import numpy as np
import pytest

import hypergen as hg
import oracle
from gpu_util import assert_matches_oracle, assert_well_formed, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def contexts():
    import paper_2201_11326_amd as slg
    store, rewalk, dense = slg.Context(0), slg.Context(0), slg.Context(0)
    store.set_count_store(32 << 30, 0)  # the store wherever there are heavy slots
    rewalk.set_count_store(0)
    dense.set_count_store(32 << 30, 0)
    dense.set_dense(8, 1)  # every heavy row with a 2-path per candidate on the dense tier
    yield {"store": store, "rewalk": rewalk, "dense": dense}
    store.close()
    rewalk.close()
    dense.close()


def _case(seed: int):
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(1, 3001))
    n = int(rng.integers(1, 2001))
    kmax = int(rng.integers(1, 61))
    expo = [None, 0.8, 1.5][seed % 3]
    s_list = sorted(set(int(x) for x in rng.integers(1, 9, size=int(rng.integers(1, 5)))))
    return hg.random_small(seed + 500, m, n, kmax, expo), s_list


@pytest.mark.parametrize("seed", range(48))
def test_random_shapes_both_modes(contexts, seed):
    inc, s_list = _case(seed)
    for mode, ctx in contexts.items():
        outs = run_gpu(ctx, inc, s_list)
        for lg in outs:
            assert_matches_oracle(inc, lg, lg.s, f"seed {seed} {mode}")
            assert_well_formed(inc, lg, lg.s)
        assert outs[0].two_paths == oracle.two_paths(inc, s_list[0])
