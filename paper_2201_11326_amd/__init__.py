"""s-line graphs of non-uniform hypergraphs on AMD MI355X.

Thin Python binding over the C ABI of ``libslg.so`` (include/slg.h):
argument marshalling only. Every step of the computation runs in the
library's HIP kernels; torch supplies device memory and streams. If the
library has not been built this module raises on first use — there is no
CPU fallback.

    import paper_2201_11326_amd as slg
    ctx = slg.Context()
    g = ctx.register_incidence(inc)           # hypergen.Incidence -> device
    outs = ctx.line_graph(g, [1, 2, 4, 8])    # one L_s per threshold
    outs[0].row_ptr, outs[0].row, outs[0].col, outs[0].w   # torch tensors

    ctx.line_graph_stream(g, [8, 16], 2 << 30, fn)   # chunked, for outputs beyond memory
    ctx.batch([g1, g2, ...], [s1, s2, ...]).run()     # many graphs, one HIP-graph replay
    ctx.server(workers=8)                             # request loop (submit / wait / next)
    ctx.components(g, s, outs[k]); ctx.squeeze(m, outs[k]); ctx.symmetrize(outs[k])
    ctx.relabel(g); ctx.simplify(g, l1)               # relabel-by-degree; toplexes only
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import re
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libslg.so")
HEADER = os.path.join(ROOT, "include", "slg.h")

SLG_OK = 0
SLG_ERR_INVALID_ARG = 1
SLG_ERR_INVALID_GRAPH = 2
SLG_ERR_OUT_OF_MEMORY = 3
SLG_ERR_DEVICE = 4
SLG_ERR_OVERFLOW = 5
SLG_ERR_CANCELLED = 6
SLG_ERR_TIMEOUT = 7
SLG_MAX_S = 16
SLG_VALIDATE = 1
SLG_COPY = 2

_STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "INVALID_GRAPH", 3: "OUT_OF_MEMORY", 4: "DEVICE",
                 5: "OVERFLOW", 6: "CANCELLED", 7: "TIMEOUT"}

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


class SlgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"slg {_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Incidence(ctypes.Structure):
    _fields_ = [("num_vertices", _i64), ("num_hyperedges", _i64), ("nnz", _i64),
                ("he_ptr", _p), ("he_idx", _p), ("v_ptr", _p), ("v_idx", _p)]


_ALLOC_FN = ctypes.CFUNCTYPE(_p, _p, ctypes.c_size_t, _p)
_CHUNK_FN = ctypes.CFUNCTYPE(ctypes.c_int, _p, _i32, _i32, _i64, _i64, _i64, _i64, _p, _p, _p, _p, _p)
_FREE_FN = ctypes.CFUNCTYPE(None, _p, _p, _p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _FREE_FN), ("user", _p)]


class StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", _i64), ("milliseconds", ctypes.c_double)]


_lib = None


def header_symbols() -> List[str]:
    """Entry points declared in include/slg.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slg_[a-z_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load libslg.so (built by __graft_entry__.build() / build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2201_11326_amd.build` "
                           "or __graft_entry__.build(). There is no fallback path.")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "slg_version": (ctypes.c_char_p, []),
        "slg_context_create": (_i32, [ctypes.c_int, _u64, _p, ctypes.POINTER(_p)]),
        "slg_context_destroy": (_i32, [_p]),
        "slg_last_error": (ctypes.c_char_p, [_p]),
        "slg_graph_register": (_i32, [_p, ctypes.POINTER(Incidence), _u32, _p, ctypes.POINTER(_p)]),
        "slg_graph_release": (_i32, [_p]),
        "slg_plan_create": (_i32, [_p, _p, ctypes.POINTER(_i32), _i32, _p, ctypes.POINTER(_p)]),
        "slg_plan_info": (_i32, [_p, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
        "slg_plan_emit": (_i32, [_p, ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_p),
                                 ctypes.POINTER(_p), _p]),
        "slg_plan_destroy": (_i32, [_p]),
        "slg_plan_stats": (_i32, [_p, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i32)]),
        "slg_line_graph": (_i32, [_p, _p, ctypes.POINTER(_i32), _i32, _p, ctypes.POINTER(_p)]),
        "slg_line_graph_stream": (_i32, [_p, _p, ctypes.POINTER(_i32), _i32, _i64, _CHUNK_FN, _p, _p]),
        "slg_line_graph_stream_rows": (_i32, [_p, _p, ctypes.POINTER(_i32), _i32, _i64, _i64, _i64, _CHUNK_FN,
                                              _p, _p]),
        "slg_work_prefix": (_i32, [_p, _p, _i32, _p, _p]),
        "slg_batch_create": (_i32, [_p, ctypes.POINTER(_p), ctypes.POINTER(_i32), _i32, _p, ctypes.POINTER(_p)]),
        "slg_batch_run": (_i32, [_p, _i32, _p]),
        "slg_batch_info": (_i32, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
        "slg_batch_result": (_i32, [_p, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_p),
                                    ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_p)]),
        "slg_batch_destroy": (_i32, [_p]),
        "slg_context_set_tuning": (_i32, [_p, _i32, _i64, _i32]),
        "slg_context_set_dense": (_i32, [_p, _i32, _i32]),
        "slg_context_set_list_shortfall": (_i32, [_p, _i64]),
        "slg_context_set_timing": (_i32, [_p, ctypes.c_int]),
        "slg_context_get_timing": (_i32, [_p, ctypes.POINTER(StageTime), _i32, ctypes.POINTER(_i32)]),
        "slg_context_reset_timing": (_i32, [_p]),
        "slg_context_get_work": (_i32, [_p, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i32)]),
        "slg_result_info": (_i32, [_p, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
        "slg_result_coo": (_i32, [_p, _i32, ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_p)]),
        "slg_result_csr": (_i32, [_p, _i32, ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_p)]),
        "slg_result_free": (_i32, [_p]),
        "slg_components": (_i32, [_p, _p, _i32, _p, _p, _i64, _p, ctypes.POINTER(_i64), _p]),
        "slg_components_noalloc": (_i32, [_p, _p, _i32, _p, _p, _i64, _p, ctypes.POINTER(_i64), _p]),
        "slg_squeeze": (_i32, [_p, _i64, _p, _p, _i64, _i32, _p, ctypes.POINTER(_i64), _p]),
        "slg_symmetrize": (_i32, [_p, _i64, _p, _p, _p, _p, _i64, _p, _p, _p, _p]),
        "slg_relabel_order": (_i32, [_p, _p, _i32, _p, _p]),
        "slg_digest": (_i32, [_p, _p, _p, _p, _i64, ctypes.POINTER(_u64), _p]),
        "slg_context_set_count_store": (_i32, [_p, _i64, _i64]),
        "slg_toplexes": (_i32, [_p, _p, _p, _p, _p, _i64, _p, ctypes.POINTER(_i64), _p]),
        "slg_select": (_i32, [_p, _p, _p, _i64, _p, _p, _p, _p, ctypes.POINTER(_i64), _p]),
        "slg_server_create": (_i32, [_p, _i32, _u64, ctypes.POINTER(_p)]),
        "slg_server_submit": (_i32, [_p, _p, ctypes.POINTER(_i32), _i32, ctypes.POINTER(_u64)]),
        "slg_server_wait": (_i32, [_p, _u64, _i32, ctypes.POINTER(_p), ctypes.POINTER(RequestInfo)]),
        "slg_server_next": (_i32, [_p, _i32, ctypes.POINTER(_p), ctypes.POINTER(RequestInfo)]),
        "slg_server_stats": (_i32, [_p, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i32)]),
        "slg_server_destroy": (_i32, [_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def version() -> str:
    return lib().slg_version().decode()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _s_array(s: Sequence[int]):
    vals = [int(x) for x in s]
    return (_i32 * max(len(vals), 1))(*vals), len(vals)


class _DeviceView:
    """Zero-copy __cuda_array_interface__ view of library-owned device memory."""

    def __init__(self, ptr: int, n: int, typestr: str, owner):
        self._owner = owner
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr,
                                         "data": (int(ptr or 0), False), "version": 3, "strides": None}


class LineGraph:
    """One L_s: CSR ``row_ptr`` (int64, m+1) plus COO ``row``/``col``/``w`` (int32)."""

    def __init__(self, s: int, row_ptr, row, col, w, two_paths: int, owner=None):
        self.s, self.row_ptr, self.row, self.col, self.w = s, row_ptr, row, col, w
        self.two_paths = int(two_paths)
        self._owner = owner

    @property
    def num_edges(self) -> int:
        return int(self.col.shape[0])

    def cpu(self):
        return LineGraph(self.s, self.row_ptr.cpu(), None if self.row is None else self.row.cpu(),
                         self.col.cpu(), self.w.cpu(), self.two_paths)


class Graph:
    """A registered hypergraph; keeps its device CSR tensors alive."""

    def __init__(self, ctx: "Context", handle: int, tensors, m: int, n: int, nnz: int = 0):
        self.ctx, self.handle, self._tensors, self.m, self.n = ctx, handle, tensors, m, n
        self.nnz = nnz

    def release(self):
        if self.handle:
            lib().slg_graph_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Plan:
    """Counting pass done: edge counts known; emit() writes caller tensors."""

    def __init__(self, ctx: "Context", handle: int, s: List[int], m: int):
        self.ctx, self.handle, self.s, self.m = ctx, handle, s, m

    def info(self, k: int):
        e, w = _i64(), _i64()
        self.ctx._check(lib().slg_plan_info(self.handle, k, ctypes.byref(e), ctypes.byref(w)))
        return int(e.value), int(w.value)

    @property
    def two_paths(self) -> int:
        return self.info(0)[1]

    def num_edges(self) -> List[int]:
        return [self.info(k)[0] for k in range(len(self.s))]

    STAT_NAMES = ("slots", "tiny8", "light64", "light128", "light256", "light512", "light1024", "light2048",
                  "heavy_slots", "heavy_wide_slots", "two_paths", "heavy_two_paths", "bound_entries",
                  "heavy_edges", "stored_ranks", "dense_slots", "dense_two_paths", "dense_edges",
                  "dense_stored", "dense_store_full")

    def stats(self) -> dict:
        out = (_i64 * 32)()
        n = _i32()
        self.ctx._check(lib().slg_plan_stats(self.handle, out, 32, ctypes.byref(n)))
        return {name: int(out[t]) for t, name in enumerate(self.STAT_NAMES[: n.value])}

    def emit(self, row_ptr, row, col, w, stream=None):
        K = len(self.s)
        arr = lambda ts: (_p * K)(*[0 if t is None else t.data_ptr() for t in ts])
        rp, rw, cl, ww = arr(row_ptr), arr(row) if row is not None else None, arr(col), arr(w)
        self.ctx._check(lib().slg_plan_emit(self.handle, rp, rw, cl, ww, _stream_handle(stream)))

    def destroy(self):
        if self.handle:
            lib().slg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """Many hypergraphs, each with its own s, planned as one disjoint union."""

    def __init__(self, ctx: "Context", handle: int, graphs, s: List[int]):
        self.ctx, self.handle, self.graphs, self.s = ctx, handle, list(graphs), list(s)

    def run(self, use_graph: bool = True, stream=None):
        """Repeat the whole device path (HIP-graph replay when use_graph)."""
        self.ctx._check(lib().slg_batch_run(self.handle, 1 if use_graph else 0, _stream_handle(stream)))

    def info(self):
        e, w, r = _i64(), _i64(), _i64()
        self.ctx._check(lib().slg_batch_info(self.handle, ctypes.byref(e), ctypes.byref(w), ctypes.byref(r)))
        return {"edges": int(e.value), "two_paths": int(w.value), "rows": int(r.value)}

    def result(self, g: int) -> LineGraph:
        """Graph g's L_s as zero-copy views (row_ptr rebased to start at 0)."""
        import torch
        e0, ne = _i64(), _i64()
        rp, ri, rj, rw = _p(), _p(), _p(), _p()
        self.ctx._check(lib().slg_batch_result(self.handle, g, ctypes.byref(e0), ctypes.byref(ne),
                                               ctypes.byref(rp), ctypes.byref(ri), ctypes.byref(rj),
                                               ctypes.byref(rw)))
        dev = f"cuda:{self.ctx.device}"
        view = lambda ptr, n, ts: torch.as_tensor(_DeviceView(ptr, n, ts, self), device=dev)
        m = self.graphs[g].m
        n = int(ne.value)
        return LineGraph(self.s[g], view(rp.value, m + 1, "<i8") - int(e0.value), view(ri.value, n, "<i4"),
                         view(rj.value, n, "<i4"), view(rw.value, n, "<i4"), 0, owner=self)

    def destroy(self):
        if self.handle:
            lib().slg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0, mem_budget_bytes: int = 0, torch_allocator: bool = True):
        import torch
        self.device = device
        L = lib()
        self._alloc = None
        alloc_ptr = None
        if torch_allocator:
            def _a(user, nbytes, stream):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0)
                except Exception:
                    return None

            def _f(user, ptr, stream):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc = Allocator(_ALLOC_FN(_a), _FREE_FN(_f), None)
            alloc_ptr = ctypes.byref(self._alloc)
        h = _p()
        st = L.slg_context_create(device, mem_budget_bytes, alloc_ptr, ctypes.byref(h))
        if st != SLG_OK:
            raise SlgError(st, "slg_context_create failed")
        self.handle = h.value

    # -- batched form and tuning ---------------------------------------------
    def batch(self, graphs: Sequence[Graph], s: Sequence[int], stream=None) -> Batch:
        hs = (_p * len(graphs))(*[g.handle for g in graphs])
        arr = (_i32 * len(s))(*[int(x) for x in s])
        h = _p()
        self._check(lib().slg_batch_create(self.handle, hs, arr, len(graphs), _stream_handle(stream),
                                           ctypes.byref(h)))
        return Batch(self, h.value, graphs, [int(x) for x in s])

    def set_tuning(self, light_max: int = 0, slot_work: int = 0, heavy_grid: int = 0):
        self._check(lib().slg_context_set_tuning(self.handle, light_max, slot_work, heavy_grid))

    def set_dense(self, min_ratio: int = 4, min_range: int = 0):
        """The dense tier's rule: at least min_ratio 2-paths per eight candidate
        partners (0 turns it off) and at least min_range candidates (0 = its
        default); results are identical either way."""
        self._check(lib().slg_context_set_dense(self.handle, int(min_ratio), int(min_range)))

    def set_list_shortfall(self, entries: int):
        """Fault injection for error-path tests: later plans give their heavy
        descriptor lists `entries` fewer places than counted, so their
        appends are refused and the plan fails with SLG_ERR_DEVICE."""
        self._check(lib().slg_context_set_list_shortfall(self.handle, int(entries)))

    # -- measurement ---------------------------------------------------------
    def set_count_store(self, max_bytes: int, min_two_paths: int = 1 << 24):
        """Largest count store a plan may keep (0: the emit pass walks the
        2-paths again) and the fewest heavy 2-paths that make one worth it;
        results are identical either way."""
        self._check(lib().slg_context_set_count_store(self.handle, int(max_bytes), int(min_two_paths)))

    def set_timing(self, enable: bool = True):
        self._check(lib().slg_context_set_timing(self.handle, 1 if enable else 0))

    def timing(self) -> dict:
        """{stage: (launches, milliseconds)} summed since the last reset."""
        out = (StageTime * 32)()
        n = _i32()
        self._check(lib().slg_context_get_timing(self.handle, out, 32, ctypes.byref(n)))
        return {out[t].name.decode(): (int(out[t].launches), float(out[t].milliseconds))
                for t in range(n.value)}

    def reset_timing(self):
        """Clears the stage times and the work counters."""
        self._check(lib().slg_context_reset_timing(self.handle))

    WORK_NAMES = ("blocks", "two_paths", "heavy_two_paths", "dense_two_paths", "edges", "heavy_edges",
                  "dense_edges", "dense_slots", "dense_stored", "dense_store_full_blocks")

    def work(self) -> dict:
        """Work of the counting passes since the last reset_timing()."""
        out = (_i64 * 16)()
        n = _i32()
        self._check(lib().slg_context_get_work(self.handle, out, 16, ctypes.byref(n)))
        return {self.WORK_NAMES[t]: int(out[t]) for t in range(n.value)}

    def _check(self, status: int):
        if status != SLG_OK:
            msg = lib().slg_last_error(self.handle)
            raise SlgError(status, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "handle", None):
            lib().slg_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- graphs ------------------------------------------------------------
    def register(self, m: int, n: int, he_ptr, he_idx, v_ptr, v_idx, validate: bool = False,
                 stream=None, copy: bool = False) -> Graph:
        """Register device tensors (int64 ptrs, int32 ids) of both CSRs. With
        copy=True the library keeps its own copies (SLG_COPY) and the tensors
        may be reused at once."""
        inc = Incidence(n, m, int(he_idx.numel()), he_ptr.data_ptr(), he_idx.data_ptr(),
                        v_ptr.data_ptr(), v_idx.data_ptr())
        h = _p()
        flags = (SLG_VALIDATE if validate else 0) | (SLG_COPY if copy else 0)
        self._check(lib().slg_graph_register(self.handle, ctypes.byref(inc), flags,
                                             _stream_handle(stream), ctypes.byref(h)))
        return Graph(self, h.value, () if copy else (he_ptr, he_idx, v_ptr, v_idx), m, n, int(he_idx.numel()))

    def register_host(self, inc, validate: bool = False, stream=None) -> Graph:
        """Register a host hypergen.Incidence through SLG_COPY: the library
        copies the numpy arrays to the device itself."""
        import numpy as np
        arrs = [np.ascontiguousarray(inc.he_ptr, dtype=np.int64), np.ascontiguousarray(inc.he_idx, dtype=np.int32),
                np.ascontiguousarray(inc.v_ptr, dtype=np.int64), np.ascontiguousarray(inc.v_idx, dtype=np.int32)]
        ptrs = [a.ctypes.data if a.size else None for a in arrs]
        c = Incidence(inc.n, inc.m, int(arrs[1].size), *ptrs)
        h = _p()
        self._check(lib().slg_graph_register(self.handle, ctypes.byref(c),
                                             SLG_COPY | (SLG_VALIDATE if validate else 0),
                                             _stream_handle(stream), ctypes.byref(h)))
        return Graph(self, h.value, (), inc.m, inc.n, int(arrs[1].size))

    def register_incidence(self, inc, validate: bool = False, stream=None) -> Graph:
        """Copy a host hypergen.Incidence to the device and register it."""
        import torch
        dev = torch.device("cuda", self.device)
        t = lambda a, dt: torch.as_tensor(a, dtype=dt).to(dev)
        he_ptr = t(inc.he_ptr, torch.int64)
        he_idx = t(inc.he_idx if inc.nnz else [0], torch.int32)[: inc.nnz]
        v_ptr = t(inc.v_ptr, torch.int64)
        v_idx = t(inc.v_idx if inc.nnz else [0], torch.int32)[: inc.nnz]
        return self.register(inc.m, inc.n, he_ptr, he_idx, v_ptr, v_idx, validate, stream)

    # -- s-line graphs -------------------------------------------------------
    def plan(self, g: Graph, s: Sequence[int], stream=None) -> Plan:
        arr, k = _s_array(s)
        h = _p()
        self._check(lib().slg_plan_create(self.handle, g.handle, arr, k, _stream_handle(stream),
                                          ctypes.byref(h)))
        return Plan(self, h.value, [int(x) for x in s], g.m)

    def line_graph(self, g: Graph, s: Sequence[int], stream=None, coo: bool = True) -> List[LineGraph]:
        """L_s for every s (one counting pass for the whole set), into torch tensors."""
        import torch
        p = self.plan(g, s, stream)
        try:
            dev = torch.device("cuda", self.device)
            outs = []
            for k, sk in enumerate(p.s):
                e, wpaths = p.info(k)
                outs.append(LineGraph(sk, torch.empty(g.m + 1, dtype=torch.int64, device=dev),
                                      torch.empty(e, dtype=torch.int32, device=dev) if coo else None,
                                      torch.empty(e, dtype=torch.int32, device=dev),
                                      torch.empty(e, dtype=torch.int32, device=dev), wpaths))
            p.emit([o.row_ptr for o in outs], [o.row for o in outs] if coo else None,
                   [o.col for o in outs], [o.w for o in outs], stream)
        finally:
            p.destroy()
        return outs

    def line_graph_stream(self, g: Graph, s: Sequence[int], chunk_bytes: int, fn, stream=None,
                          rows: Optional[Sequence[int]] = None):
        """Chunked L_s: fn(k, s, row_begin, row_end, edge_begin, row_ptr, row, col, w) is called
        per chunk and threshold with torch views of library buffers; torch work inside fn runs
        on the library's consumer stream (it overlaps the next chunk's emit) and may use the
        views until it completes, not after fn's work is done. Return True to stop (SlgError
        CANCELLED). rows=(row_begin, row_end) streams only those rows."""
        import torch
        dev = f"cuda:{self.device}"
        errors = []

        def _cb(user, k, sk, r0, r1, e0, ne, rp, ri, rj, rw, st):
            try:
                view = lambda ptr, n, ts: torch.as_tensor(_DeviceView(ptr, n, ts, None), device=dev)
                # torch work inside fn goes to the consumer stream
                cm = torch.cuda.stream(torch.cuda.ExternalStream(st, device=dev)) if st else contextlib.nullcontext()
                with cm:
                    stop = fn(int(k), int(sk), int(r0), int(r1), int(e0), view(rp, r1 - r0 + 1, "<i8"),
                              view(ri, ne, "<i4"), view(rj, ne, "<i4"), view(rw, ne, "<i4"))
                return 1 if stop else 0
            except Exception as exc:  # surface Python errors after the call
                errors.append(exc)
                return 1

        cb = _CHUNK_FN(_cb)
        arr, kk = _s_array(s)
        if rows is None:
            st = lib().slg_line_graph_stream(self.handle, g.handle, arr, kk, int(chunk_bytes), cb, None,
                                             _stream_handle(stream))
        else:
            st = lib().slg_line_graph_stream_rows(self.handle, g.handle, arr, kk, int(rows[0]), int(rows[1]),
                                                  int(chunk_bytes), cb, None, _stream_handle(stream))
        if errors:
            raise errors[0]
        self._check(st)

    def work_prefix(self, g: Graph, s_min: int, stream=None):
        """Per-row 2-path work at s_min as an exclusive prefix (numpy int64[m+1])."""
        import numpy as np
        out = np.zeros(g.m + 1, dtype=np.int64)
        self._check(lib().slg_work_prefix(self.handle, g.handle, int(s_min), out.ctypes.data,
                                          _stream_handle(stream)))
        return out

    def line_graph_result(self, g: Graph, s: Sequence[int], stream=None) -> List[LineGraph]:
        """The one-shot ABI call (slg_line_graph): library-owned result buffers."""
        arr, k = _s_array(s)
        h = _p()
        self._check(lib().slg_line_graph(self.handle, g.handle, arr, k, _stream_handle(stream),
                                         ctypes.byref(h)))
        return _wrap_result(_Result(h.value), s, g.m, self.device)

    def components(self, g: Graph, s: int, lg: "LineGraph", stream=None):
        """s-connected components of L_s given its edges: (labels int32[m] on the
        device, smallest id of each component or -1 off E_s; number of components)."""
        import torch
        labels = torch.empty(max(g.m, 1), dtype=torch.int32, device=f"cuda:{self.device}")[: g.m]
        nc = _i64()
        row = _need_rows(lg)
        self._check(lib().slg_components(self.handle, g.handle, int(s), row.data_ptr(), lg.col.data_ptr(),
                                         int(lg.num_edges), labels.data_ptr(), ctypes.byref(nc),
                                         _stream_handle(stream)))
        return labels, int(nc.value)

    def components_noalloc(self, g: Graph, s: int, lg: "LineGraph", labels=None, stream=None):
        """components() through slg_components_noalloc: no device allocation
        inside the library (its fixed per-GPU array, at most 2^24
        hyperedges). `labels` (int32[m] on the device) may be given so that
        the call allocates nothing at all."""
        import torch
        if labels is None:
            labels = torch.empty(max(g.m, 1), dtype=torch.int32, device=f"cuda:{self.device}")[: g.m]
        nc = _i64()
        row = _need_rows(lg)
        self._check(lib().slg_components_noalloc(self.handle, g.handle, int(s), row.data_ptr(), lg.col.data_ptr(),
                                                 int(lg.num_edges), labels.data_ptr(), ctypes.byref(nc),
                                                 _stream_handle(stream)))
        return labels, int(nc.value)

    def squeeze(self, m: int, lg: "LineGraph", remap: bool = False, stream=None):
        """ID squeezing: (new_id int32[m], -1 for hyperedges without an edge;
        number kept). remap=True rewrites lg.row/lg.col in place."""
        import torch
        new_id = torch.empty(max(m, 1), dtype=torch.int32, device=f"cuda:{self.device}")[:m]
        nk = _i64()
        row = _need_rows(lg)
        self._check(lib().slg_squeeze(self.handle, int(m), row.data_ptr(), lg.col.data_ptr(), int(lg.num_edges),
                                      1 if remap else 0, new_id.data_ptr(), ctypes.byref(nk),
                                      _stream_handle(stream)))
        return new_id, int(nk.value)

    def symmetrize(self, lg: "LineGraph", weights: bool = True, stream=None):
        """Symmetric CSR of L_s from its upper triangle: (sym_ptr int64[m+1],
        sym_col int32[2E], sym_w int32[2E] or None) on the device; row r holds
        every partner of r, ascending."""
        import torch
        dev = f"cuda:{self.device}"
        m = int(lg.row_ptr.shape[0]) - 1
        e = int(lg.num_edges)
        row = _need_rows(lg)
        sym_ptr = torch.empty(m + 1, dtype=torch.int64, device=dev)
        sym_col = torch.empty(max(2 * e, 1), dtype=torch.int32, device=dev)[: 2 * e]
        sym_w = torch.empty(max(2 * e, 1), dtype=torch.int32, device=dev)[: 2 * e] if weights else None
        self._check(lib().slg_symmetrize(self.handle, m, lg.row_ptr.data_ptr(), row.data_ptr(), lg.col.data_ptr(),
                                         lg.w.data_ptr() if weights else None, e, sym_ptr.data_ptr(),
                                         sym_col.data_ptr(), sym_w.data_ptr() if weights else None,
                                         _stream_handle(stream)))
        return sym_ptr, sym_col, sym_w

    def digest(self, row, col, w, stream=None):
        """Order-independent digest of device edge arrays: (edges, sum of w,
        sum mod 2^64 of SplitMix64(i * 2^32 + j) xor w); digests of disjoint
        parts add up (chunks of a streamed result)."""
        out = (_u64 * 3)()
        n = int(col.numel())
        self._check(lib().slg_digest(self.handle, row.data_ptr() if n else None, col.data_ptr() if n else None,
                                     w.data_ptr() if n else None, n, out, _stream_handle(stream)))
        return int(out[0]), int(out[1]), int(out[2])

    # -- preprocessing (relabel-by-degree, toplexes) ------------------------
    def relabel_order(self, g: Graph, descending: bool = False, stream=None):
        """Hyperedge ids ordered by size: int32[m] on the device, order[k] =
        the old id that becomes id k (equal sizes keep their id order)."""
        import torch
        order = torch.empty(max(g.m, 1), dtype=torch.int32, device=f"cuda:{self.device}")[: g.m]
        self._check(lib().slg_relabel_order(self.handle, g.handle, 1 if descending else 0, order.data_ptr(),
                                            _stream_handle(stream)))
        return order

    def select(self, g: Graph, order, stream=None) -> Graph:
        """The sub-hypergraph of the hyperedges order[0..count), registered."""
        import torch
        dev = f"cuda:{self.device}"
        order = order.to(device=dev, dtype=torch.int32).contiguous()
        count = int(order.numel())
        nnz_cap = int(g.nnz)
        he_ptr = torch.empty(count + 1, dtype=torch.int64, device=dev)
        v_ptr = torch.empty(g.n + 1, dtype=torch.int64, device=dev)
        he_idx = torch.empty(max(nnz_cap, 1), dtype=torch.int32, device=dev)
        v_idx = torch.empty(max(nnz_cap, 1), dtype=torch.int32, device=dev)
        nz = _i64()
        self._check(lib().slg_select(self.handle, g.handle, order.data_ptr() if count else None, count,
                                     he_ptr.data_ptr(), he_idx.data_ptr(), v_ptr.data_ptr(), v_idx.data_ptr(),
                                     ctypes.byref(nz), _stream_handle(stream)))
        k = int(nz.value)
        return self.register(count, g.n, he_ptr, he_idx[:k], v_ptr, v_idx[:k], stream=stream)

    def relabel(self, g: Graph, descending: bool = False, stream=None):
        """Relabel-by-degree: (the relabelled graph, order) with old id =
        order[new id]."""
        order = self.relabel_order(g, descending, stream)
        return self.select(g, order, stream), order

    def toplexes(self, g: Graph, l1: "LineGraph", stream=None):
        """Toplex ids (ascending, int32 on the device) from the edges of L_1."""
        import torch
        ids = torch.empty(max(g.m, 1), dtype=torch.int32, device=f"cuda:{self.device}")
        cnt = _i64()
        row = _need_rows(l1)
        self._check(lib().slg_toplexes(self.handle, g.handle, row.data_ptr(), l1.col.data_ptr(), l1.w.data_ptr(),
                                       int(l1.num_edges), ids.data_ptr(), ctypes.byref(cnt), _stream_handle(stream)))
        return ids[: int(cnt.value)]

    def simplify(self, g: Graph, l1: "LineGraph", stream=None):
        """The simplification (toplexes only): (graph, toplex ids), hyperedge
        k of the graph being toplex ids[k]."""
        ids = self.toplexes(g, l1, stream)
        return self.select(g, ids, stream), ids

    def server(self, workers: int = 4, mem_budget_bytes: int = 0) -> "Server":
        """The served form (slg_server_*): a request loop over registered graphs."""
        return Server(self, workers, mem_budget_bytes)


def _need_rows(lg: "LineGraph"):
    if lg.row is None:
        raise ValueError("this call needs the COO rows of the line graph (line_graph(..., coo=True))")
    return lg.row


def _wrap_result(res: "_Result", s: Sequence[int], m: int, device: int) -> List[LineGraph]:
    """Zero-copy torch views of an slg_result, one LineGraph per threshold."""
    import torch

    def check(st):
        if st != SLG_OK:
            raise SlgError(st, "result query failed")
    outs = []
    for kk, sk in enumerate(s):
        e, wpaths = _i64(), _i64()
        check(lib().slg_result_info(res.handle, kk, ctypes.byref(e), ctypes.byref(wpaths)))
        ip, jp, wp, rp = _p(), _p(), _p(), _p()
        check(lib().slg_result_coo(res.handle, kk, ctypes.byref(ip), ctypes.byref(jp), ctypes.byref(wp)))
        check(lib().slg_result_csr(res.handle, kk, ctypes.byref(rp), None, None))
        view = lambda ptr, n, ts: torch.as_tensor(_DeviceView(ptr, n, ts, res), device=f"cuda:{device}")
        ne = int(e.value)
        outs.append(LineGraph(int(sk), view(rp.value, m + 1, "<i8"), view(ip.value, ne, "<i4"),
                              view(jp.value, ne, "<i4"), view(wp.value, ne, "<i4"), int(wpaths.value),
                              owner=res))
    return outs


class RequestInfo(ctypes.Structure):
    _fields_ = [("ticket", _u64), ("status", ctypes.c_int), ("attempts", _i32), ("queue_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("two_paths", _i64), ("message", ctypes.c_char * 192)]


class Served:
    """One finished query of a Server: its outcome, timings and (on success)
    one LineGraph per threshold. The outputs count against the server's
    memory budget until every reference to them is dropped."""

    def __init__(self, info: RequestInfo, s: List[int], graph: "Graph", outs):
        self.ticket = int(info.ticket)
        self.status = int(info.status)
        self.attempts = int(info.attempts)
        self.queue_ms = float(info.queue_ms)
        self.latency_ms = float(info.latency_ms)
        self.two_paths = int(info.two_paths)
        self.message = info.message.decode(errors="replace")
        self.s, self.graph, self.outs = s, graph, outs

    @property
    def ok(self) -> bool:
        return self.status == SLG_OK


class Server:
    SERVER_STAT_NAMES = ("submitted", "completed", "failed", "yields", "queued", "running", "bytes_used",
                         "bytes_peak", "bytes_in_results")

    def __init__(self, ctx: Context, workers: int = 4, mem_budget_bytes: int = 0):
        import threading
        self.ctx = ctx
        self._pending = {}  # ticket -> (graph, s)
        self._lock = threading.Lock()  # a query may end before submit has recorded it
        h = _p()
        ctx._check(lib().slg_server_create(ctx.handle, int(workers), int(mem_budget_bytes), ctypes.byref(h)))
        self.handle = h.value

    def submit(self, g: Graph, s: Sequence[int]) -> int:
        arr, k = _s_array(s)
        t = _u64()
        with self._lock:
            st = lib().slg_server_submit(self.handle, g.handle, arr, k, ctypes.byref(t))
            if st != SLG_OK:
                raise SlgError(st, "slg_server_submit refused the query")
            self._pending[int(t.value)] = (g, [int(x) for x in s])
        return int(t.value)

    def _finish(self, st: int, h, info: RequestInfo) -> Optional[Served]:
        if st == SLG_ERR_TIMEOUT:
            return None
        ticket = int(info.ticket)
        with self._lock:
            if ticket not in self._pending:
                raise SlgError(st, "unknown or retired ticket")
            g, s = self._pending.pop(ticket)
        outs = _wrap_result(_Result(h.value), s, g.m, self.ctx.device) if h.value else None
        return Served(info, s, g, outs)

    def wait(self, ticket: int, timeout_ms: int = -1) -> Optional[Served]:
        """The query's outcome once it has ended; None on timeout."""
        h, info = _p(), RequestInfo()
        st = lib().slg_server_wait(self.handle, int(ticket), int(timeout_ms), ctypes.byref(h), ctypes.byref(info))
        if st == SLG_ERR_INVALID_ARG and h.value is None and int(info.ticket) == 0:
            raise SlgError(st, f"unknown or retired ticket {ticket}")
        return self._finish(st, h, info)

    def next(self, timeout_ms: int = -1, keep: bool = True) -> Optional[Served]:
        """Whichever query ended first (completion order); None on timeout.
        keep=False frees the outputs at once (outcome and timings only)."""
        h, info = _p(), RequestInfo()
        st = lib().slg_server_next(self.handle, int(timeout_ms), ctypes.byref(h) if keep else None,
                                   ctypes.byref(info))
        return self._finish(st, h, info)

    def stats(self) -> dict:
        out = (_i64 * 16)()
        n = _i32()
        st = lib().slg_server_stats(self.handle, out, 16, ctypes.byref(n))
        if st != SLG_OK:
            raise SlgError(st, "slg_server_stats failed")
        return {self.SERVER_STAT_NAMES[t]: int(out[t]) for t in range(n.value)}

    def close(self):
        if getattr(self, "handle", None):
            lib().slg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Result:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        try:
            if self.handle:
                lib().slg_result_free(self.handle)
        except Exception:
            pass
