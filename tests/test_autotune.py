"""The batched form's autotuner: the host-side choice (the fastest candidate
is set on the context and cached per workload key; a second call takes the
cache without timing) with stand-ins for the batch, and on the GPU a tuning
run whose chosen plan shape gives the oracle's result."""
from __future__ import annotations

import json

import numpy as np
import pytest

from paper_2201_11326_amd import autotune


class _Batch:
    def __init__(self, ctx):
        self.ctx, self.tuning = ctx, ctx.tuning

    def info(self):
        return {"rows": 5000, "two_paths": 123456, "edges": 0}

    def destroy(self):
        self.ctx.destroyed += 1


class _Ctx:
    def __init__(self):
        self.tuning, self.destroyed, self.built = (0, 0, 0), 0, 0

    def set_tuning(self, *t):
        self.tuning = tuple(t)

    def batch(self, graphs, s):
        self.built += 1
        return _Batch(self)


def test_tune_batch_picks_fastest_and_caches(tmp_path, monkeypatch):
    seconds = {(0, 0, 0): 3.0, (512, 0, 0): 1.0, (1024, 8192, 256): 2.0}
    monkeypatch.setattr(autotune, "time_replays", lambda b, reps: seconds[b.tuning])
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    cache = tmp_path / "tuning.json"
    ctx = _Ctx()
    best, times = autotune.tune_batch(ctx, [], [], candidates=list(seconds), cache_path=str(cache))
    assert best == (512, 0, 0) and ctx.tuning == best and times == seconds
    assert ctx.built == 1 + len(seconds) and ctx.destroyed == ctx.built  # probe + one batch per candidate
    key = autotune.workload_key(5000, 123456)
    assert key == "gfx950/rows2^12/paths2^16"
    assert json.loads(cache.read_text())[key] == {"tuning": [512, 0, 0], "seconds": 1.0}
    # the cache answers the same workload without timing anything
    monkeypatch.setattr(autotune, "time_replays", lambda b, reps: pytest.fail("timed despite the cache"))
    ctx2 = _Ctx()
    best2, times2 = autotune.tune_batch(ctx2, [], [], candidates=list(seconds), cache_path=str(cache))
    assert best2 == best and ctx2.tuning == best and times2 == {best: 1.0} and ctx2.built == 1


def test_tune_batch_without_cache_and_unreadable_cache(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "time_replays", lambda b, reps: 1.0 + b.tuning[0])
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    ctx = _Ctx()
    best, _ = autotune.tune_batch(ctx, [], [], candidates=[(7, 0, 0), (0, 0, 0)], cache_path=str(bad))
    assert best == (0, 0, 0)  # an unreadable cache is ignored, then replaced
    assert json.loads(bad.read_text())
    ctx = _Ctx()
    best, _ = autotune.tune_batch(ctx, [], [], candidates=[(3, 0, 0), (5, 0, 0)], cache_path=str(bad),
                                  use_cache=False)
    assert best == (3, 0, 0) and ctx.built == 3


@pytest.mark.gpu
def test_tuned_batch_matches_oracle(tmp_path):
    import hypergen as hg
    import oracle
    import paper_2201_11326_amd as slg
    ctx = slg.Context(0)
    fam = hg.batched_family(count=8, m_lo=500, m_hi=4000)
    graphs = [ctx.register_incidence(mem.inc) for mem in fam]
    s_list = [mem.s for mem in fam]
    cands = [(0, 0, 0), (512, 4096, 64), (2048, 16384, 0)]
    best, times = autotune.tune_batch(ctx, graphs, s_list, candidates=cands, reps=2,
                                      cache_path=str(tmp_path / "t.json"))
    assert best in cands and set(times) == set(cands) and all(t > 0 for t in times.values())
    b = ctx.batch(graphs, s_list)  # built with the tuning left on the context
    for gidx, mem in enumerate(fam):
        lg = b.result(gidx).cpu()
        ref = oracle.line_graph(mem.inc, mem.s)
        assert np.array_equal(lg.row_ptr.numpy(), ref.row_ptr) and np.array_equal(lg.col.numpy(), ref.j)
        assert np.array_equal(lg.w.numpy(), ref.w) and np.array_equal(lg.row.numpy(), ref.i)
    b.destroy()
    for g in graphs:
        g.release()
    ctx.close()
