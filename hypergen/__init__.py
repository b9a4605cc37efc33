"""Seeded synthetic hypergraph generators.

This module builds *inputs* only: the incidence of a hypergraph H = (V, E)
held as both CSR orientations (Section II-A: the bipartite graph B(H) /
the n x m incidence matrix H, and the hyperedge->vertex adjacency used by
the two-hop traversal of Section III-B, the "ikj" form). It holds none of
the line-graph arithmetic, so both the CPU oracle and the GPU library can
read the same arrays.

Conventions (0-based; the paper's example is 1-based):
  * ``he_ptr`` int64[m+1], ``he_idx`` int32[nnz]: vertices of hyperedge i in
    ``he_idx[he_ptr[i]:he_ptr[i+1]]``, strictly increasing (each e_i is a set).
  * ``v_ptr`` int64[n+1], ``v_idx`` int32[nnz]: hyperedges containing vertex v,
    strictly increasing; it is the exact transpose of the hyperedge CSR.

Workload recipes (the paper's datasets are not available, so these seeded
shapes stand in for them):
  * ``tiny_uniform``    n=2,000, m=1,000, |e| ~ U{2..20}, members uniform.
  * ``power_law``       n=1e6, m=5e5, |e| ~ Zipf(2.1) on [2, 5000], vertex
                         weight ~ rank^-0.8.
  * ``large_skewed``    n=5e6, m=1e7, |e| = min(rint(LogNormal(1.5, 1.0)),
                         10000), vertex weight ~ rank^-1.5.
  * ``batched_family``  256 graphs, m log-uniform in [1e3, 2e5], n = 2m,
                         |e| = min(Zipf(2.1), 1000), members uniform, s ~ U{1..8}.
Weighted sampling without replacement is successive sampling: draw with
replacement from the weights and drop repeats until |e| distinct members
are held. A seeded permutation maps vertex rank to vertex id so heavy
vertices are spread over the id space.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 11326


@dataclasses.dataclass
class Incidence:
    """A hypergraph as both CSR orientations of its incidence matrix."""

    m: int
    n: int
    he_ptr: np.ndarray  # int64 [m+1]
    he_idx: np.ndarray  # int32 [nnz]
    v_ptr: np.ndarray  # int64 [n+1]
    v_idx: np.ndarray  # int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.he_idx.shape[0])

    def sizes(self) -> np.ndarray:
        return np.diff(self.he_ptr)

    def row(self, i: int) -> np.ndarray:
        return self.he_idx[self.he_ptr[i]:self.he_ptr[i + 1]]

    def dual(self) -> "Incidence":
        """The dual hypergraph H* (Section II-A): roles of V and E swapped."""
        return Incidence(self.n, self.m, self.v_ptr, self.v_idx, self.he_ptr, self.he_idx)


def transpose_csr(num_rows: int, num_cols: int, ptr: np.ndarray, idx: np.ndarray):
    """Column-major view of a 0/1 CSR: returns (ptr_t, idx_t), rows ascending.

    Input preparation only (the paper's H versus H^T adjacency); a stable
    counting sort by column keeps the row ids ascending inside each column.
    """
    ptr = np.asarray(ptr, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int32)
    nnz = idx.shape[0]
    rows = np.repeat(np.arange(num_rows, dtype=np.int32), np.diff(ptr))
    order = np.argsort(idx, kind="stable")
    idx_t = rows[order].astype(np.int32, copy=False)
    counts = np.bincount(idx, minlength=num_cols).astype(np.int64) if nnz else np.zeros(num_cols, np.int64)
    ptr_t = np.zeros(num_cols + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr_t[1:])
    return ptr_t, idx_t


def from_rows(rows: Sequence[Sequence[int]], n: Optional[int] = None) -> Incidence:
    """Build an Incidence from explicit member lists (each sorted and deduped)."""
    clean = [np.unique(np.asarray(r, dtype=np.int64)) for r in rows]
    m = len(clean)
    if n is None:
        n = int(max((int(r.max()) + 1 for r in clean if r.size), default=0))
    he_ptr = np.zeros(m + 1, dtype=np.int64)
    if m:
        np.cumsum([r.size for r in clean], out=he_ptr[1:])
    he_idx = (np.concatenate(clean) if m and he_ptr[-1] else np.zeros(0, np.int64)).astype(np.int32)
    v_ptr, v_idx = transpose_csr(m, n, he_ptr, he_idx)
    return Incidence(m, n, he_ptr, he_idx, v_ptr, v_idx)


def from_csr(m: int, n: int, he_ptr: np.ndarray, he_idx: np.ndarray) -> Incidence:
    v_ptr, v_idx = transpose_csr(m, n, he_ptr, he_idx)
    return Incidence(m, n, np.asarray(he_ptr, np.int64), np.asarray(he_idx, np.int32), v_ptr, v_idx)


def _successive_sample(rng: np.random.Generator, sizes: np.ndarray, n: int,
                       cdf: Optional[np.ndarray]) -> tuple:
    """Per row r, draw ``sizes[r]`` distinct members in [0, n).

    ``cdf`` is the cumulative vertex-rank weight (None = uniform). Each round
    draws, with replacement, exactly the deficit of every unfinished row and
    keeps the draws not already held, so a row never overshoots its size:
    the same law as drawing one at a time and dropping repeats.
    Returns (he_ptr, he_idx) with rows sorted.
    """
    m = sizes.shape[0]
    sizes = np.minimum(sizes.astype(np.int64), n)

    def draw(k: int) -> np.ndarray:
        if cdf is None:
            return rng.integers(0, n, size=k, dtype=np.int64)
        u = rng.random(k)
        return np.minimum(np.searchsorted(cdf, u * cdf[-1], side="right"), n - 1).astype(np.int64)

    need = sizes.copy()
    chunks = []
    held_def = np.zeros(0, dtype=np.int64)  # sorted keys row*n+v of unfinished rows
    rows_need = np.nonzero(need)[0]
    while rows_need.size:
        cnt = need[rows_need]
        row_of = np.repeat(rows_need.astype(np.int64), cnt)
        uniq = np.unique(row_of * n + draw(int(cnt.sum())))
        if held_def.size:
            uniq = uniq[~np.isin(uniq, held_def, assume_unique=True)]
        chunks.append(uniq)
        need -= np.bincount(uniq // n, minlength=m)
        still = need > 0
        hd = np.concatenate([held_def, uniq])
        hd = hd[still[hd // n]]
        hd.sort()
        held_def = hd
        rows_need = np.nonzero(still)[0]
    held = np.concatenate(chunks) if chunks else np.zeros(0, np.int64)
    held.sort()
    he_idx = (held % n).astype(np.int32)
    he_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=he_ptr[1:])
    return he_ptr, he_idx


def _rank_cdf(n: int, exponent: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-exponent)
    return np.cumsum(w)


def _relabel(rng: np.random.Generator, n: int, he_ptr: np.ndarray, he_idx: np.ndarray) -> np.ndarray:
    """Map vertex rank -> id by a seeded permutation; re-sort each row."""
    perm = rng.permutation(n).astype(np.int64)
    m = he_ptr.shape[0] - 1
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(he_ptr))
    key = rows * n + perm[he_idx.astype(np.int64)]
    key.sort()
    return (key % n).astype(np.int32)


def _truncated_zipf(rng: np.random.Generator, m: int, alpha: float, lo: int, hi: int) -> np.ndarray:
    k = np.arange(lo, hi + 1, dtype=np.float64)
    p = k ** (-alpha)
    p /= p.sum()
    return rng.choice(np.arange(lo, hi + 1), size=m, p=p).astype(np.int64)


def _build(rng, n, sizes, exponent: Optional[float]) -> Incidence:
    cdf = None if exponent is None else _rank_cdf(n, exponent)
    he_ptr, he_idx = _successive_sample(rng, sizes, n, cdf)
    if exponent is not None:
        he_idx = _relabel(rng, n, he_ptr, he_idx)
    return from_csr(sizes.shape[0], n, he_ptr, he_idx)


def tiny_uniform(seed: int = BASE_SEED + 1, n: int = 2000, m: int = 1000,
                 kmin: int = 2, kmax: int = 20) -> Incidence:
    rng = np.random.default_rng(seed)
    sizes = rng.integers(kmin, kmax + 1, size=m, dtype=np.int64)
    return _build(rng, n, sizes, None)


def power_law(seed: int = BASE_SEED + 2, n: int = 1_000_000, m: int = 500_000,
              alpha: float = 2.1, kmin: int = 2, kmax: int = 5000,
              vertex_exponent: float = 0.8) -> Incidence:
    rng = np.random.default_rng(seed)
    sizes = _truncated_zipf(rng, m, alpha, kmin, min(kmax, n))
    return _build(rng, n, sizes, vertex_exponent)


def large_skewed(seed: int = BASE_SEED + 3, n: int = 5_000_000, m: int = 10_000_000,
                 mu: float = 1.5, sigma: float = 1.0, kmax: int = 10_000,
                 vertex_exponent: float = 1.5) -> Incidence:
    rng = np.random.default_rng(seed)
    sizes = np.minimum(np.rint(rng.lognormal(mu, sigma, size=m)), kmax).astype(np.int64)
    return _build(rng, n, sizes, vertex_exponent)


@dataclasses.dataclass
class BatchMember:
    inc: Incidence
    s: int


def batched_family(seed: int = BASE_SEED + 4, count: int = 256, m_lo: int = 1000,
                   m_hi: int = 200_000, alpha: float = 2.1, kmax: int = 1000,
                   s_max: int = 8) -> List[BatchMember]:
    """Independent hypergraphs of uneven size, each with its own s."""
    ss = np.random.SeedSequence(seed)
    out = []
    for child in ss.spawn(count):
        rng = np.random.default_rng(child)
        m = int(math.floor(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        n = 2 * m
        sizes = np.minimum(rng.zipf(alpha, size=m), kmax).astype(np.int64)
        s = int(rng.integers(1, s_max + 1))
        out.append(BatchMember(_build(rng, n, sizes, None), s))
    return out


def served_pool(seed: int = BASE_SEED + 5, skewed: int = 64, power: int = 4,
                skewed_m: Tuple[int, int] = (1_000, 10_000),
                power_n: int = 1_000_000, power_m: int = 500_000) -> List[Incidence]:
    """Device-resident pool of the served workload: `skewed` graphs from the
    large-skewed generator (n = m/2, m log-uniform in skewed_m: whole-graph
    queries on the full-size shape are out of reach, each would emit about
    10^13 edges) followed by `power` graphs from the power-law generator at
    its full size (n = power_n, m = power_m), each from its own seed."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(skewed + power)
    out = []
    for t in range(skewed):
        rng = np.random.default_rng(kids[t])
        m = int(math.floor(math.exp(rng.uniform(math.log(skewed_m[0]), math.log(skewed_m[1])))))
        out.append(large_skewed(seed=int(rng.integers(1 << 62)), n=max(m // 2, 1), m=m))
    for t in range(power):
        rng = np.random.default_rng(kids[skewed + t])
        out.append(power_law(seed=int(rng.integers(1 << 62)), n=power_n, m=power_m))
    return out


@dataclasses.dataclass
class Request:
    arrival: float     # seconds from the start of the stream
    graph: int         # index into the pool
    s: List[int]       # increasing thresholds


def served_requests(pool_size: int, count: int, rate: float = 2000.0, seed: int = BASE_SEED + 6,
                    s_choices: Sequence[int] = (1, 2, 3, 4, 5, 8), max_set: int = 6) -> List[Request]:
    """Poisson arrivals at `rate` per second; each request names a pool
    graph uniformly and an s-set of 1..max_set distinct thresholds drawn
    from s_choices."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for a in t:
        g = int(rng.integers(0, pool_size))
        k = int(rng.integers(1, max_set + 1))
        s = sorted(int(x) for x in rng.choice(np.asarray(s_choices), size=k, replace=False))
        out.append(Request(float(a), g, s))
    return out


def random_small(seed: int, m: int, n: int, kmax: int, exponent: Optional[float] = None,
                 kmin: int = 0) -> Incidence:
    """Small hypergraphs for property tests (sizes may be 0 = empty hyperedge)."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(kmin, kmax + 1, size=m, dtype=np.int64)
    return _build(rng, n, sizes, exponent)


def toy_paper_example() -> Incidence:
    """The worked example of Section I: E = {1:{a,b,c}, 2:{b,c,d},
    3:{a,b,c,d,e}, 4:{e,f}}, relabelled 0-based (a..f -> 0..5, 1..4 -> 0..3)."""
    return from_rows([[0, 1, 2], [1, 2, 3], [0, 1, 2, 3, 4], [4, 5]], n=6)


def random_upper_edges(seed: int, m: int, count: int, exponent: float = 1.0, wmax: int = 50):
    """A seeded edge list shaped like the upper triangle of an s-line graph,
    for tests of the edge-list operations: about `count` distinct pairs i < j
    over m ids, the ends drawn with weight ~ rank^-exponent (a few hub ids,
    permuted over the id space), sorted by (i, j), with weights in
    [1, wmax]. Returns (row_ptr int64[m+1], row, col, w int32)."""
    rng = np.random.default_rng(seed)
    cdf = _rank_cdf(m, exponent)
    perm = rng.permutation(m)
    a = perm[np.searchsorted(cdf, rng.random(count) * cdf[-1], side="right").clip(0, m - 1)]
    b = perm[np.searchsorted(cdf, rng.random(count) * cdf[-1], side="right").clip(0, m - 1)]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo[lo < hi].astype(np.int64) * m + hi[lo < hi])
    row = (key // m).astype(np.int32)
    col = (key % m).astype(np.int32)
    w = rng.integers(1, wmax + 1, size=key.size).astype(np.int32)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(row, minlength=m), out=row_ptr[1:])
    return row_ptr, row, col, w


def stats(inc: Incidence) -> dict:
    sz = inc.sizes()
    dv = np.diff(inc.v_ptr)
    return {
        "m": inc.m, "n": inc.n, "nnz": inc.nnz,
        "max_edge": int(sz.max()) if sz.size else 0,
        "mean_edge": float(sz.mean()) if sz.size else 0.0,
        "max_vdeg": int(dv.max()) if dv.size else 0,
    }
