"""Python binding of libringo (argument marshalling only).

Every step of the conversion runs in the library's HIP kernels; PyTorch is
used for device memory and streams only.  There is no fallback: if the
library is missing, every entry point raises.

    g = to_graph(src, dst)              # src, dst: int64 tensors on the GPU
    gs = to_graph_batched(srcs, dsts)   # many tables, one batched call

A `Graph` exposes the converted graph (Section 2.4) as tensors that share
the library's device memory; the memory is released when the last of them
(and the Graph) is gone.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libringo.so")

RINGO_OK = 0
STATUS_EVICTED = 5
STATUS_PENDING = 6
STATUS_NAMES = {0: "RINGO_OK", 1: "RINGO_ERR_INVALID_ARG", 2: "RINGO_ERR_TOO_MANY_NODES",
                3: "RINGO_ERR_OUT_OF_MEMORY", 4: "RINGO_ERR_HIP", 5: "RINGO_ERR_EVICTED",
                6: "RINGO_ERR_PENDING"}

# Every symbol include/ringo.h declares.
EXPORTED_SYMBOLS = (
    "ringo_table_to_graph", "ringo_table_to_graph_batched", "ringo_graph_free",
    "ringo_status_string", "ringo_set_allocator", "ringo_tune_get", "ringo_tune_set",
    "ringo_version", "ringo_trace_enable", "ringo_trace_read",
    "ringo_server_create", "ringo_server_submit", "ringo_server_poll", "ringo_server_release",
    "ringo_server_stats", "ringo_server_destroy",
    "ringo_graph_to_edge_table", "ringo_graph_to_node_table", "ringo_pagerank",
    "ringo_table_to_graph_ex", "ringo_table_to_graph_batched_ex", "ringo_sort_keys",
    "ringo_table_to_graph_noalloc", "ringo_server_pin", "ringo_server_unpin", "ringo_server_batches",
    "ringo_release_cached",
)

NOALLOC_MAX_ROWS = 1 << 20


class RingoError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}" if what else STATUS_NAMES.get(status, str(status)))


class RawGraph(ctypes.Structure):
    """ringo_graph_t"""
    _fields_ = [
        ("num_rows", ctypes.c_int64),
        ("num_nodes", ctypes.c_int64),
        ("num_edges", ctypes.c_int64),
        ("node_ids", ctypes.c_void_p),
        ("out_offsets", ctypes.c_void_p),
        ("out_nbrs", ctypes.c_void_p),
        ("in_offsets", ctypes.c_void_p),
        ("in_nbrs", ctypes.c_void_p),
        ("_alloc", ctypes.c_void_p),
        ("kind", ctypes.c_int32),
        ("_reserved", ctypes.c_int32),
        ("out_eids", ctypes.c_void_p),
        ("in_eids", ctypes.c_void_p),
    ]


GRAPH_DIRECTED, GRAPH_UNDIRECTED, GRAPH_MULTI = 0, 1, 2


class TraceEntry(ctypes.Structure):
    """ringo_trace_entry_t"""
    _fields_ = [("kernel", ctypes.c_char_p), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("units", ctypes.c_int64)]


class Schedule(ctypes.Structure):
    """ringo_schedule_t"""
    _fields_ = [("digit_bits", ctypes.c_int32), ("items_per_thread", ctypes.c_int32),
                ("node_method", ctypes.c_int32)]


NODES_SORT = 0
NODES_HASH = 1


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libringo.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        p, i64 = ctypes.c_void_p, ctypes.c_int64
        L.ringo_table_to_graph.argtypes = [p, p, i64, ctypes.POINTER(RawGraph), p]
        L.ringo_table_to_graph.restype = ctypes.c_int
        L.ringo_table_to_graph_batched.argtypes = [ctypes.c_int32, p, p, p, ctypes.POINTER(RawGraph), p]
        L.ringo_table_to_graph_batched.restype = ctypes.c_int
        L.ringo_table_to_graph_ex.argtypes = [p, p, i64, ctypes.c_int32, ctypes.POINTER(RawGraph), p]
        L.ringo_table_to_graph_ex.restype = ctypes.c_int
        L.ringo_table_to_graph_batched_ex.argtypes = [ctypes.c_int32, p, p, p, ctypes.c_int32,
                                                      ctypes.POINTER(RawGraph), p]
        L.ringo_table_to_graph_batched_ex.restype = ctypes.c_int
        L.ringo_graph_free.argtypes = [ctypes.POINTER(RawGraph)]
        L.ringo_graph_free.restype = None
        L.ringo_status_string.argtypes = [ctypes.c_int]
        L.ringo_status_string.restype = ctypes.c_char_p
        L.ringo_set_allocator.argtypes = [p, p, p]
        L.ringo_set_allocator.restype = ctypes.c_int
        L.ringo_release_cached.argtypes = [ctypes.POINTER(ctypes.c_int64)]
        L.ringo_release_cached.restype = ctypes.c_int
        L.ringo_tune_get.argtypes = [i64, ctypes.POINTER(Schedule)]
        L.ringo_tune_get.restype = ctypes.c_int
        L.ringo_tune_set.argtypes = [i64, ctypes.POINTER(Schedule)]
        L.ringo_tune_set.restype = ctypes.c_int
        L.ringo_trace_enable.argtypes = [ctypes.c_int]
        L.ringo_trace_enable.restype = None
        L.ringo_trace_read.argtypes = [ctypes.POINTER(TraceEntry), ctypes.c_int]
        L.ringo_trace_read.restype = ctypes.c_int
        L.ringo_version.argtypes = []
        L.ringo_version.restype = ctypes.c_char_p
        L.ringo_graph_to_edge_table.argtypes = [ctypes.POINTER(RawGraph), p, p, p]
        L.ringo_graph_to_edge_table.restype = ctypes.c_int
        L.ringo_graph_to_node_table.argtypes = [ctypes.POINTER(RawGraph), p, p, p, p]
        L.ringo_graph_to_node_table.restype = ctypes.c_int
        L.ringo_pagerank.argtypes = [ctypes.POINTER(RawGraph), ctypes.c_double, ctypes.c_int32, p, p]
        L.ringo_pagerank.restype = ctypes.c_int
        L.ringo_sort_keys.argtypes = [p, p, i64, ctypes.c_int32, p]
        L.ringo_sort_keys.restype = ctypes.c_int
        L.ringo_table_to_graph_noalloc.argtypes = [p, p, i64, p, p, p, p, p, p, p]
        L.ringo_table_to_graph_noalloc.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != RINGO_OK:
        raise RingoError(rc, what)


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _column(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or t.dim() != 1:
        raise TypeError(f"{name} must be a 1-D int64 tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must live on the GPU")
    return t.contiguous()


# ------------------------------------------------------------- raw calls

def table_to_graph_raw(src_ptr: int, dst_ptr: int, num_rows: int, stream: int,
                       kind: int = GRAPH_DIRECTED) -> RawGraph:
    """ringo_table_to_graph(_ex) on raw device pointers; free with graph_free."""
    g = RawGraph()
    if kind == GRAPH_DIRECTED:
        rc = lib().ringo_table_to_graph(src_ptr, dst_ptr, num_rows, ctypes.byref(g), stream)
    else:
        rc = lib().ringo_table_to_graph_ex(src_ptr, dst_ptr, num_rows, kind, ctypes.byref(g), stream)
    _check(rc, "ringo_table_to_graph")
    return g


def table_to_graph_batched_raw(src_ptrs, dst_ptrs, num_rows, stream: int,
                               kind: int = GRAPH_DIRECTED) -> list[RawGraph]:
    k = len(num_rows)
    S = (ctypes.c_void_p * k)(*src_ptrs)
    D = (ctypes.c_void_p * k)(*dst_ptrs)
    N = (ctypes.c_int64 * k)(*num_rows)
    outs = (RawGraph * k)()
    if kind == GRAPH_DIRECTED:
        rc = lib().ringo_table_to_graph_batched(k, S, D, N, outs, stream)
    else:
        rc = lib().ringo_table_to_graph_batched_ex(k, S, D, N, kind, outs, stream)
    _check(rc, "ringo_table_to_graph_batched")
    return [outs[i] for i in range(k)]


def table_to_graph_noalloc_raw(src_ptr: int, dst_ptr: int, num_rows: int, node_ids_ptr: int,
                               out_offsets_ptr: int, out_nbrs_ptr: int, in_offsets_ptr: int,
                               in_nbrs_ptr: int, counts_ptr: int, stream: int) -> None:
    """ringo_table_to_graph_noalloc into caller-allocated worst-case device
    arrays (node_ids [2n], offsets [2n + 1], neighbours [n], counts [2])."""
    _check(lib().ringo_table_to_graph_noalloc(src_ptr, dst_ptr, num_rows, node_ids_ptr, out_offsets_ptr,
                                              out_nbrs_ptr, in_offsets_ptr, in_nbrs_ptr, counts_ptr, stream),
           "ringo_table_to_graph_noalloc")


def graph_to_edge_table_raw(g: RawGraph, src_ptr: int, dst_ptr: int, stream: int) -> None:
    """ringo_graph_to_edge_table into caller-allocated device arrays."""
    _check(lib().ringo_graph_to_edge_table(ctypes.byref(g), src_ptr, dst_ptr, stream),
           "ringo_graph_to_edge_table")


def graph_to_node_table_raw(g: RawGraph, ids_ptr: int, out_deg_ptr: int, in_deg_ptr: int,
                            stream: int) -> None:
    _check(lib().ringo_graph_to_node_table(ctypes.byref(g), ids_ptr, out_deg_ptr, in_deg_ptr, stream),
           "ringo_graph_to_node_table")


def pagerank_raw(g: RawGraph, damping: float, iterations: int, ranks_ptr: int, stream: int) -> None:
    _check(lib().ringo_pagerank(ctypes.byref(g), damping, iterations, ranks_ptr, stream), "ringo_pagerank")


def sort_keys_raw(in_ptr: int, out_ptr: int, n: int, bits: int, stream: int) -> None:
    _check(lib().ringo_sort_keys(in_ptr, out_ptr, n, bits, stream), "ringo_sort_keys")


def sort_keys(keys: torch.Tensor, bits: int = 64, stream=None) -> torch.Tensor:
    """Stable radix sort of int64 keys (as uint64 bit patterns) by their low
    min(64, d * ceil(bits / d)) bits, d being the schedule's digit width for
    that many keys (tune_get; 8 by default); returns a new tensor."""
    if not isinstance(keys, torch.Tensor) or keys.dtype != torch.int64 or keys.dim() != 1 or not keys.is_cuda:
        raise TypeError("keys must be a 1-D int64 tensor on the GPU")
    keys = keys.contiguous()
    out = torch.empty_like(keys)
    with torch.cuda.device(keys.device):
        sort_keys_raw(keys.data_ptr(), out.data_ptr(), keys.numel(), bits, _stream_handle(stream))
    return out


def graph_free(g: RawGraph) -> None:
    lib().ringo_graph_free(ctypes.byref(g))


def release_cached() -> int:
    """Returns the built-in allocator's idle cached blocks on the current
    device to the device; the bytes returned."""
    n = ctypes.c_int64(0)
    rc = lib().ringo_release_cached(ctypes.byref(n))
    if rc != 0:
        raise RingoError(rc, "ringo_release_cached")
    return n.value


def status_string(status: int) -> str:
    return lib().ringo_status_string(status).decode()


def version() -> str:
    return lib().ringo_version().decode()


def tune_get(num_rows: int) -> tuple[int, int, int]:
    """(digit_bits, items_per_thread, node_method) used for num_rows rows."""
    s = Schedule()
    _check(lib().ringo_tune_get(num_rows, ctypes.byref(s)), "ringo_tune_get")
    return s.digit_bits, s.items_per_thread, s.node_method


def tune_set(num_rows: int, digit_bits: int, items_per_thread: int, node_method: int | None = None) -> None:
    """Overrides the schedule of num_rows' size bucket; node_method None keeps
    the bucket's current method."""
    if node_method is None:
        node_method = tune_get(num_rows)[2]
    s = Schedule(digit_bits, items_per_thread, node_method)
    _check(lib().ringo_tune_set(num_rows, ctypes.byref(s)), "ringo_tune_set")


def set_node_method(node_method: int, min_rows: int = 0) -> None:
    """Sets the node-numbering method of every size bucket from min_rows up,
    keeping each bucket's tile shape."""
    for e in range(63):
        rows = 1 << e
        if rows < min_rows:
            continue
        d, it, _ = tune_get(rows)
        tune_set(rows, d, it, node_method)


def trace_enable(on: bool) -> None:
    lib().ringo_trace_enable(1 if on else 0)


def trace_read() -> dict:
    """Per-kernel launches, summed event time (ms), algorithmic bytes, units."""
    buf = (TraceEntry * 32)()
    n = lib().ringo_trace_read(buf, 32)
    if n < 0:
        raise RingoError(4, "ringo_trace_read")
    return {buf[i].kernel.decode(): {"launches": buf[i].launches, "ms": buf[i].total_ms, "bytes": buf[i].bytes,
                                     "units": buf[i].units} for i in range(n)}


# ----------------------------------------------------------- tensor views

class _Owner:
    """Keeps one library graph alive while any tensor view of it exists."""

    def __init__(self, raw: RawGraph):
        self.raw = raw

    def __del__(self):
        try:
            lib().ringo_graph_free(ctypes.byref(self.raw))
        except Exception:
            pass


class _DeviceArray:
    """__cuda_array_interface__ holder: torch.as_tensor keeps it (and the
    owner) referenced for as long as the tensor lives."""

    def __init__(self, ptr: int, n: int, typestr: str, owner: _Owner):
        self._owner = owner
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": None}


def _view(ptr, n: int, dtype: torch.dtype, owner: _Owner, device) -> torch.Tensor:
    if n == 0 or not ptr:
        return torch.empty(0, dtype=dtype, device=device)
    typestr = {torch.int64: "<i8", torch.int32: "<i4"}[dtype]
    return torch.as_tensor(_DeviceArray(int(ptr), n, typestr, owner), device=device)


@dataclass
class Graph:
    """The converted graph: node identifiers and CSR in both directions."""
    num_rows: int
    num_nodes: int
    num_edges: int
    node_ids: torch.Tensor     # int64 [V]
    out_offsets: torch.Tensor  # int64 [V+1]
    out_nbrs: torch.Tensor     # int32 [E]
    in_offsets: torch.Tensor   # int64 [V+1]
    in_nbrs: torch.Tensor      # int32 [E]
    kind: int = 0              # GRAPH_DIRECTED / GRAPH_UNDIRECTED / GRAPH_MULTI
    out_eids: torch.Tensor | None = None  # int32 [E] multigraph: row of each out-entry
    in_eids: torch.Tensor | None = None   # int32 [E] multigraph: row of each in-entry


def _graph_of(raw: RawGraph, owner, device) -> Graph:
    V, E = raw.num_nodes, raw.num_edges
    multi = raw.kind == GRAPH_MULTI
    return Graph(raw.num_rows, V, E,
                 _view(raw.node_ids, V, torch.int64, owner, device),
                 _view(raw.out_offsets, V + 1, torch.int64, owner, device),
                 _view(raw.out_nbrs, E, torch.int32, owner, device),
                 _view(raw.in_offsets, V + 1, torch.int64, owner, device),
                 _view(raw.in_nbrs, E, torch.int32, owner, device),
                 raw.kind,
                 _view(raw.out_eids, E, torch.int32, owner, device) if multi else None,
                 _view(raw.in_eids, E, torch.int32, owner, device) if multi else None)


def _wrap(raw: RawGraph, device) -> Graph:
    return _graph_of(raw, _Owner(raw), device)


def view_graph(raw: RawGraph, device) -> Graph:
    """Tensor views of a graph owned elsewhere (for example by the server);
    valid only while the owner keeps it."""
    return _graph_of(raw, None, device)


def to_graph(src: torch.Tensor, dst: torch.Tensor, stream=None, kind: int = GRAPH_DIRECTED) -> Graph:
    """Table-to-graph conversion of one edge table (src, dst columns);
    kind: GRAPH_DIRECTED (default), GRAPH_UNDIRECTED or GRAPH_MULTI."""
    src = _column(src, "src")
    dst = _column(dst, "dst")
    if src.numel() != dst.numel():
        raise ValueError("src and dst must have the same length")
    if src.device != dst.device:
        raise ValueError("src and dst must be on the same device")
    with torch.cuda.device(src.device):
        raw = table_to_graph_raw(src.data_ptr(), dst.data_ptr(), src.numel(), _stream_handle(stream), kind)
    return _wrap(raw, src.device)


def raw_of(g: Graph) -> RawGraph:
    """A RawGraph struct over the tensors of `g` (it owns nothing)."""
    r = RawGraph()
    r.num_rows, r.num_nodes, r.num_edges = g.num_rows, g.num_nodes, g.num_edges
    for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs", "out_eids", "in_eids"):
        t = getattr(g, f)
        setattr(r, f, t.data_ptr() if t is not None and t.numel() else None)
    r.kind = g.kind
    return r


def to_edge_table(g: Graph, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    """Graph-to-table conversion: the (src, dst) identifier columns of the
    graph's edges in ascending (src, dst) order."""
    dev = g.out_offsets.device
    src = torch.empty(g.num_edges, dtype=torch.int64, device=dev)
    dst = torch.empty(g.num_edges, dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        graph_to_edge_table_raw(raw_of(g), src.data_ptr(), dst.data_ptr(), _stream_handle(stream))
    return src, dst


def to_node_table(g: Graph, stream=None) -> tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """The node table: identifiers, out-degrees and in-degrees."""
    dev = g.out_offsets.device
    cols = [torch.empty(g.num_nodes, dtype=torch.int64, device=dev) for _ in range(3)]
    with torch.cuda.device(dev):
        graph_to_node_table_raw(raw_of(g), *(c.data_ptr() for c in cols), _stream_handle(stream))
    return tuple(cols)


def pagerank(g: Graph, damping: float = 0.85, iterations: int = 10, stream=None) -> torch.Tensor:
    """PageRank scores (fp64) of every node after `iterations` iterations."""
    dev = g.out_offsets.device
    ranks = torch.empty(g.num_nodes, dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        pagerank_raw(raw_of(g), damping, iterations, ranks.data_ptr(), _stream_handle(stream))
    return ranks


def to_graph_batched(srcs, dsts, stream=None, kind: int = GRAPH_DIRECTED) -> list[Graph]:
    """Batched conversion: one library call for all tables."""
    if len(srcs) != len(dsts):
        raise ValueError("srcs and dsts must have the same length")
    if len(srcs) == 0:
        return []
    srcs = [_column(s, "src") for s in srcs]
    dsts = [_column(d, "dst") for d in dsts]
    dev = srcs[0].device
    for s, d in zip(srcs, dsts):
        if s.numel() != d.numel():
            raise ValueError("src and dst must have the same length")
        if s.device != dev or d.device != dev:
            raise ValueError("all tables must be on the same device")
    with torch.cuda.device(dev):
        raws = table_to_graph_batched_raw([s.data_ptr() for s in srcs], [d.data_ptr() for d in dsts],
                                          [s.numel() for s in srcs], _stream_handle(stream), kind)
    return [_wrap(r, dev) for r in raws]
