"""The on-device edge-list digest against the oracle's: whole emitted line
graphs, and the chunks of a streamed result summed (the digest is order
free and additive over disjoint parts)."""
from __future__ import annotations

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


@pytest.mark.parametrize("seed,m,n,kmax,expo", [(95, 3000, 500, 30, 1.0), (96, 20000, 5000, 12, 1.4)])
def test_digest_of_emitted_line_graphs(ctx, seed, m, n, kmax, expo):
    inc = hg.random_small(seed, m, n, kmax, expo)
    g = ctx.register_incidence(inc)
    for lg in ctx.line_graph(g, [1, 2, 5]):
        ref = oracle.line_graph(inc, lg.s)
        assert ctx.digest(lg.row, lg.col, lg.w) == oracle.digest(ref.i, ref.j, ref.w), lg.s
    g.release()


def test_streamed_chunk_digests_add_up(ctx):
    inc = hg.large_skewed(n=10_000, m=20_000)
    g = ctx.register_incidence(inc)
    S = [4, 6]
    acc = {s: [0, 0, 0] for s in S}
    chunks = {s: 0 for s in S}

    def on_chunk(k, s, r0, r1, e0, row_ptr, row, col, w):
        d = ctx.digest(row, col, w)
        acc[s] = [acc[s][0] + d[0], acc[s][1] + d[1], (acc[s][2] + d[2]) % (1 << 64)]
        chunks[s] += 1
        return False

    ctx.line_graph_stream(g, S, 32 << 20, on_chunk)
    for s in S:
        ref = oracle.line_graph(inc, s)
        assert tuple(acc[s]) == oracle.digest(ref.i, ref.j, ref.w), s
        assert chunks[s] > 1
    g.release()


def test_digest_of_nothing(ctx):
    import torch
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert ctx.digest(e, e, e) == (0, 0, 0)
