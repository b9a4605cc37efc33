"""Autotuner for the batched form: picks the plan shape (wavefront-sort
bound, heavy slot work, persistent heavy grid) by timing HIP-graph replays
of the batch, and caches the winner per GPU architecture and workload-size
bucket in a JSON file."""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, Optional, Sequence, Tuple

# (light_max, slot_work, heavy_grid); 0 = library default
DEFAULT_CANDIDATES: Tuple[Tuple[int, int, int], ...] = (
    (0, 0, 0),
    (512, 0, 0),
    (1024, 0, 0),
    (2048, 4096, 0),
    (2048, 16384, 0),
    (1024, 8192, 256),
)
CACHE = os.environ.get("SLG_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "slg_tuning.json"))


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def workload_key(rows: int, two_paths: int) -> str:
    b = lambda x: int(math.log2(max(x, 1)))
    return f"{_arch()}/rows2^{b(rows)}/paths2^{b(two_paths)}"


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: Dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_replays(batch, reps: int) -> float:
    """Median seconds of `reps` HIP-graph replays (after one warm replay)."""
    import torch
    batch.run(use_graph=True)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        batch.run(use_graph=True)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2]


def tune_batch(ctx, graphs: Sequence, s: Sequence[int], candidates: Optional[Iterable] = None,
               reps: int = 5, cache_path: str = CACHE, use_cache: bool = True):
    """Returns (best tuning tuple, {tuning: seconds}) and leaves the best
    tuning set on `ctx`."""
    probe = ctx.batch(graphs, s)
    info = probe.info()
    probe.destroy()
    key = workload_key(info["rows"], info["two_paths"])
    cache = _load(cache_path) if use_cache else {}
    if use_cache and key in cache:
        best = tuple(cache[key]["tuning"])
        ctx.set_tuning(*best)
        return best, {best: cache[key]["seconds"]}
    times = {}
    for cand in (candidates or DEFAULT_CANDIDATES):
        ctx.set_tuning(*cand)
        b = ctx.batch(graphs, s)
        times[tuple(cand)] = time_replays(b, reps)
        b.destroy()
    best = min(times, key=times.get)
    ctx.set_tuning(*best)
    if use_cache:
        cache[key] = {"tuning": list(best), "seconds": times[best]}
        _save(cache_path, cache)
    return best, times
