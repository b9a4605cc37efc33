"""CPU oracle for s-line graphs — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and
shares no code with it. The arithmetic lives in ``slg_oracle.c`` (plain C,
OpenMP over rows): for every pair of hyperedges (i, j), i < j, both in E_s,
it counts |e_i n e_j| by flagging the members of e_i and testing those of
e_j, and keeps the pair when the count is at least s (Section II-B: E_s,
s-incidence, L_s(H) = <E_s, F>, and L = H^T H). The multi-s ensemble
(Algorithm 3's output) is the same definition evaluated once per s.

All functions take a ``hypergen.Incidence`` and return numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slg_oracle.c")
_LIB = os.path.join(_HERE, "libslg_oracle.so")
_lib = None

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP); returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.slgo_validate.argtypes = [_i64, _i64, _p, _p]
        lib.slgo_validate.restype = ctypes.c_int
        lib.slgo_rows_count.argtypes = [_i64, _i64, _p, _p, _i64, _i64, _p, _i64, _p, ctypes.c_int]
        lib.slgo_rows_count.restype = ctypes.c_int
        lib.slgo_rows_emit.argtypes = [_i64, _i64, _p, _p, _i64, _i64, _p, _i64, _p, _p, _p,
                                       ctypes.c_int]
        lib.slgo_rows_emit.restype = ctypes.c_int
        lib.slgo_two_paths.argtypes = [_i64, _i64, _p, _p, _i64]
        lib.slgo_two_paths.restype = _i64
        lib.slgo_row_two_paths.argtypes = [_i64, _i64, _p, _p, _i64, _p, _i64, _p, ctypes.c_int]
        lib.slgo_row_two_paths.restype = ctypes.c_int
        lib.slgo_components_brute.argtypes = [_i64, _i64, _p, _p, _i64, _p]
        lib.slgo_components_brute.restype = _i64
        lib.slgo_components_edges.argtypes = [_i64, _p, _i64, _i64, _p, _p, _p]
        lib.slgo_components_edges.restype = _i64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _csr(inc):
    he_ptr = np.ascontiguousarray(inc.he_ptr, dtype=np.int64)
    he_idx = np.ascontiguousarray(inc.he_idx, dtype=np.int32)
    if he_idx.size == 0:
        he_idx = np.zeros(1, np.int32)  # a valid address for an empty array
    return he_ptr, he_idx


def validate(inc) -> int:
    """0 = valid; 1 bad pointers; 2 id out of range; 3 row not a sorted set."""
    he_ptr, he_idx = _csr(inc)
    return int(_load().slgo_validate(inc.m, inc.n, _ptr(he_ptr), _ptr(he_idx)))


class Rows:
    """Rows of an s-line graph: ``rows[r]`` owns ``j/w[ptr[r]:ptr[r+1]]``."""

    def __init__(self, rows, ptr, j, w):
        self.rows, self.ptr, self.j, self.w = rows, ptr, j, w

    def row(self, r: int):
        a, b = self.ptr[r], self.ptr[r + 1]
        return self.j[a:b], self.w[a:b]


def line_graph_rows(inc, s: int, rows: Optional[Sequence[int]] = None,
                    size_min: Optional[int] = None, threads: int = 0) -> Rows:
    """Rows ``rows`` (default: all) of L_s over E_{size_min} (default s)."""
    if s < 1:
        raise ValueError("s must be >= 1")
    size_min = s if size_min is None else int(size_min)
    lib = _load()
    he_ptr, he_idx = _csr(inc)
    rows_a = (np.arange(inc.m, dtype=np.int64) if rows is None
              else np.ascontiguousarray(rows, dtype=np.int64))
    nr = rows_a.shape[0]
    counts = np.zeros(max(nr, 1), np.int64)
    rp = rows_a if nr else np.zeros(1, np.int64)
    if lib.slgo_rows_count(inc.m, inc.n, _ptr(he_ptr), _ptr(he_idx), size_min, s,
                           _ptr(rp), nr, _ptr(counts), threads):
        raise MemoryError("oracle: allocation failed")
    ptr = np.zeros(nr + 1, np.int64)
    np.cumsum(counts[:nr], out=ptr[1:])
    total = int(ptr[-1])
    j = np.zeros(max(total, 1), np.int32)
    w = np.zeros(max(total, 1), np.int32)
    if lib.slgo_rows_emit(inc.m, inc.n, _ptr(he_ptr), _ptr(he_idx), size_min, s, _ptr(rp), nr,
                          _ptr(ptr), _ptr(j), _ptr(w), threads):
        raise RuntimeError("oracle: emit disagreed with count")
    return Rows(rows_a, ptr, j[:total], w[:total])


class LineGraph:
    """A whole s-line graph: CSR over all m rows plus the COO arrays."""

    def __init__(self, s, row_ptr, i, j, w):
        self.s, self.row_ptr, self.i, self.j, self.w = s, row_ptr, i, j, w

    @property
    def num_edges(self) -> int:
        return int(self.j.shape[0])

    def pairs(self) -> Dict[tuple, int]:
        return {(int(a), int(b)): int(c) for a, b, c in zip(self.i, self.j, self.w)}


def line_graph(inc, s: int, size_min: Optional[int] = None, threads: int = 0) -> LineGraph:
    """L_s(H) (Section II-B), sorted by (i, j), i < j, original ids."""
    r = line_graph_rows(inc, s, None, size_min, threads)
    i = np.repeat(np.arange(inc.m, dtype=np.int32), np.diff(r.ptr))
    return LineGraph(s, r.ptr, i, r.j, r.w)


def ensemble(inc, s_values: Sequence[int], threads: int = 0) -> List[LineGraph]:
    """One L_s per requested s (the outputs of the ensemble algorithm)."""
    return [line_graph(inc, int(s), threads=threads) for s in s_values]


def two_paths(inc, size_min: int) -> int:
    """Number of 2-paths (e_i, v, e_j), i < j, e_i, e_j in E_{size_min}."""
    he_ptr, he_idx = _csr(inc)
    return int(_load().slgo_two_paths(inc.m, inc.n, _ptr(he_ptr), _ptr(he_idx), size_min))


def row_two_paths(inc, size_min: int, rows: Sequence[int], threads: int = 0) -> np.ndarray:
    """Per sampled row i: the number of 2-paths (e_i, v, e_j) with j > i."""
    he_ptr, he_idx = _csr(inc)
    rows_a = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(max(rows_a.shape[0], 1), np.int64)
    rp = rows_a if rows_a.size else np.zeros(1, np.int64)
    if _load().slgo_row_two_paths(inc.m, inc.n, _ptr(he_ptr), _ptr(he_idx), size_min, _ptr(rp),
                                  rows_a.shape[0], _ptr(out), threads):
        raise MemoryError("oracle: allocation failed")
    return out[:rows_a.shape[0]]


def components(inc, s: int, row: Optional[np.ndarray] = None, col: Optional[np.ndarray] = None):
    """s-connected components (Section II-B): (labels int32[m], count). The
    label of e_i is the smallest id of its component, -1 when |e_i| < s.
    Without an edge list, s-incidence is tested by brute force for every
    pair met by the search (small inputs); with one (the edges of L_s), the
    search follows those edges."""
    he_ptr, he_idx = _csr(inc)
    label = np.empty(max(inc.m, 1), np.int32)
    lib = _load()
    if row is None:
        count = lib.slgo_components_brute(inc.m, inc.n, _ptr(he_ptr), _ptr(he_idx), int(s), _ptr(label))
    else:
        r = np.ascontiguousarray(row, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        if r.size == 0:
            r = c = np.zeros(1, np.int32)
        count = lib.slgo_components_edges(inc.m, _ptr(he_ptr), int(s), int(np.asarray(row).size), _ptr(r),
                                          _ptr(c), _ptr(label))
    if count == -1:
        raise MemoryError("oracle: allocation failed")
    if count == -2:
        raise ValueError("an edge names an id outside [0, m) or a hyperedge outside E_s")
    return label[: inc.m], int(count)


def squeeze(m: int, row: np.ndarray, col: np.ndarray):
    """ID squeezing (Stage 4 of the framework, Section IV): hyperedges that end at least one
    edge keep their order and are numbered 0, 1, ...; (new_id int32[m] with
    -1 for the others, number kept)."""
    present = np.zeros(m, dtype=bool)
    present[np.asarray(row, dtype=np.int64)] = True
    present[np.asarray(col, dtype=np.int64)] = True
    new_id = np.full(m, -1, dtype=np.int32)
    new_id[present] = np.arange(int(present.sum()), dtype=np.int32)
    return new_id, int(present.sum())


def symmetric(m: int, row: np.ndarray, col: np.ndarray, w: Optional[np.ndarray] = None):
    """Symmetric CSR of L_s (Stage 4 of the framework, Section IV; the
    adjacency of L_s is the symmetric matrix of Section II-B): every edge
    {i, j} appears in row i and in row j, each row in ascending order.
    Returns (ptr int64[m+1], col int32[2E], w int32[2E] or None)."""
    row = np.asarray(row, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    r = np.concatenate([row, col])
    c = np.concatenate([col, row])
    order = np.lexsort((c, r))  # by row, then column
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m)[:m], out=ptr[1:])
    ww = None
    if w is not None:
        w = np.asarray(w, dtype=np.int32)
        ww = np.concatenate([w, w])[order]
    return ptr, c[order].astype(np.int32), ww


def relabel_order(inc, descending: bool = False) -> np.ndarray:
    """Relabel-by-degree (Stage 1 of the framework, Section IV): hyperedge
    ids ordered by size, ascending or descending, equal sizes in id order;
    order[k] = the old id that becomes id k."""
    sizes = np.diff(np.asarray(inc.he_ptr, dtype=np.int64))
    return np.argsort(-sizes if descending else sizes, kind="stable").astype(np.int32)


def select(inc, order):
    """The sub-hypergraph of hyperedges order[0..count): hyperedge k is
    order[k], vertex ids unchanged. Returns (he_ptr, he_idx, v_ptr, v_idx)
    with every vertex list ascending."""
    he_ptr = np.asarray(inc.he_ptr, dtype=np.int64)
    he_idx = np.asarray(inc.he_idx, dtype=np.int32)
    order = np.asarray(order, dtype=np.int64)
    rows = [he_idx[he_ptr[i]:he_ptr[i + 1]] for i in order]
    new_ptr = np.zeros(order.size + 1, dtype=np.int64)
    np.cumsum([r.size for r in rows], out=new_ptr[1:])
    new_idx = np.concatenate(rows).astype(np.int32) if rows and new_ptr[-1] else np.zeros(0, np.int32)
    # the vertex lists: incidences (k, v) ordered by vertex, then by k
    k_of = np.repeat(np.arange(order.size, dtype=np.int64), np.diff(new_ptr))
    by_v = np.lexsort((k_of, new_idx))
    v_ptr = np.zeros(inc.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(new_idx, minlength=inc.n)[: inc.n], out=v_ptr[1:])
    return new_ptr, new_idx, v_ptr, k_of[by_v].astype(np.int32)


def toplexes(inc) -> np.ndarray:
    """Toplexes (Stage 2 of the framework, Section IV), by subset tests on
    every pair of hyperedges: e is kept unless some other hyperedge is a
    strict superset, or an identical set with a smaller id; empty
    hyperedges are not kept. Small inputs only."""
    sets = [frozenset(inc.row(i).tolist()) for i in range(inc.m)]
    keep = []
    for i, e in enumerate(sets):
        if not e:
            continue
        if any((j != i and e < f) or (j < i and e == f) for j, f in enumerate(sets)):
            continue
        keep.append(i)
    return np.asarray(keep, dtype=np.int32)


def toplexes_from_edges(inc, row, col, w) -> np.ndarray:
    """Toplexes from the edges of L_1: e_i lies inside e_j exactly when
    their overlap is |e_i| (same keep rule as toplexes())."""
    sizes = np.diff(np.asarray(inc.he_ptr, dtype=np.int64))
    drop = sizes == 0
    a = np.asarray(row, dtype=np.int64)
    b = np.asarray(col, dtype=np.int64)
    x = np.asarray(w, dtype=np.int64)
    sa, sb = sizes[a], sizes[b]
    drop[a[(x == sa) & ((sb > sa) | ((sb == sa) & (b < a)))]] = True
    drop[b[(x == sb) & ((sa > sb) | ((sa == sb) & (a < b)))]] = True
    return np.flatnonzero(~drop).astype(np.int32)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64's output function on uint64 inputs (the published mixer of
    Steele, Lea and Flood, with Vigna's constants), wrapping mod 2^64."""
    z = x + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def digest(i, j, w):
    """Order-independent digest of an edge list: (number of edges, sum of w,
    sum mod 2^64 of SplitMix64(i * 2^32 + j) xor w)."""
    i = np.asarray(i, dtype=np.int64).astype(np.uint64)
    j = np.asarray(j, dtype=np.int64).astype(np.uint64)
    w = np.asarray(w, dtype=np.int64).astype(np.uint64)
    with np.errstate(over="ignore"):
        h = _splitmix64((i << np.uint64(32)) | j) ^ w
        total = int(h.sum(dtype=np.uint64)) if h.size else 0
    return int(i.size), int(w.sum()) if w.size else 0, total % (1 << 64)
