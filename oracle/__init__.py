"""CPU oracle of the table-to-graph conversion -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  The product path (the C-ABI library and
its Python binding) never imports or calls it, and the two share no code.

`table_to_graph(src, dst)` returns the plain definition of the conversion
(Section 2.4, "Conversion of tables to graphs"): the sorted distinct node
identifiers, and CSR out- and in-adjacency over dense node positions with
each neighbour list strictly increasing.  See `oracle.cpp` for the steps and
the readings taken where the paper is silent.

`pagerank(g, damping, iterations)` is PageRank on a graph (Page, Brin,
Motwani & Winograd 1999), the consumer the paper runs on converted graphs
(ten iterations in Section 3), in fp64.

`graph_to_edge_table(g)` and `graph_to_node_table(g)` are the inverse
direction (Section 2.4, "Conversion of graphs to tables"): one output row per
edge (visiting the nodes in order, and each node's out-neighbours in order)
or per node (identifier, out-degree, in-degree).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC_PATH = os.path.join(_HERE, "oracle.cpp")
LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(source: str = SRC_PATH, out: str = LIB_PATH) -> str:
    """Compile the oracle with the host C++ compiler (no GPU code)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", out, source]
    subprocess.run(cmd, check=True)
    return out


@dataclass
class Graph:
    node_ids: np.ndarray     # int64 [V]
    out_offsets: np.ndarray  # int64 [V+1]
    out_nbrs: np.ndarray     # int32 [E]
    in_offsets: np.ndarray   # int64 [V+1]
    in_nbrs: np.ndarray      # int32 [E]

    @property
    def num_nodes(self) -> int:
        return int(self.node_ids.size)

    @property
    def num_edges(self) -> int:
        return int(self.out_nbrs.size)


class OracleError(RuntimeError):
    pass


_libs: dict[str, ctypes.CDLL] = {}
last_threads = 1  # host threads the last table_to_graph call used


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if path not in _libs:
        if not os.path.exists(path) and path == LIB_PATH:
            build()
        L = ctypes.CDLL(path)
        p = ctypes.c_void_p
        L.oracle_table_to_graph.argtypes = [p, p, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.oracle_table_to_graph.restype = ctypes.c_int
        L.oracle_table_to_graph_par.argtypes = L.oracle_table_to_graph.argtypes + [ctypes.POINTER(ctypes.c_int32)]
        L.oracle_table_to_graph_par.restype = ctypes.c_int
        L.oracle_copy.argtypes = [p, p, p, p, p, p]
        L.oracle_copy.restype = None
        L.oracle_free.argtypes = [p]
        L.oracle_free.restype = None
        L.oracle_table_to_graph_kind.argtypes = [p, p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.oracle_table_to_graph_kind.restype = ctypes.c_int
        L.oracle_copy_eids.argtypes = [p, p, p]
        L.oracle_copy_eids.restype = None
        _libs[path] = L
    return _libs[path]


def table_to_graph(src, dst, lib_path: str = LIB_PATH, all_cores: bool = False) -> Graph:
    """The directed conversion. all_cores: the same steps with a parallel sort
    on every host thread (for timing; the result is identical); the thread
    count used is then in the module's last_threads."""
    global last_threads
    src = np.ascontiguousarray(src, dtype=np.int64)
    dst = np.ascontiguousarray(dst, dtype=np.int64)
    if src.shape != dst.shape or src.ndim != 1:
        raise ValueError("src and dst must be 1-D arrays of equal length")
    L = load(lib_path)
    h = ctypes.c_void_p()
    V = ctypes.c_int64()
    E = ctypes.c_int64()
    if all_cores:
        t = ctypes.c_int32()
        rc = L.oracle_table_to_graph_par(src.ctypes.data, dst.ctypes.data, src.size, ctypes.byref(h),
                                         ctypes.byref(V), ctypes.byref(E), ctypes.byref(t))
        last_threads = t.value
    else:
        rc = L.oracle_table_to_graph(src.ctypes.data, dst.ctypes.data, src.size, ctypes.byref(h),
                                     ctypes.byref(V), ctypes.byref(E))
        last_threads = 1
    if rc != 0:
        raise OracleError({1: "invalid argument", 2: "too many nodes", 3: "out of memory"}.get(rc, str(rc)))
    try:
        g = Graph(np.empty(V.value, np.int64), np.empty(V.value + 1, np.int64), np.empty(E.value, np.int32),
                  np.empty(V.value + 1, np.int64), np.empty(E.value, np.int32))
        L.oracle_copy(h, g.node_ids.ctypes.data, g.out_offsets.ctypes.data, g.out_nbrs.ctypes.data,
                      g.in_offsets.ctypes.data, g.in_nbrs.ctypes.data)
    finally:
        L.oracle_free(h)
    return g


DIRECTED, UNDIRECTED, MULTIGRAPH = 0, 1, 2


@dataclass
class MultiGraph(Graph):
    out_eids: np.ndarray = None  # int32 [E] row index of each out-list entry
    in_eids: np.ndarray = None   # int32 [E] row index of each in-list entry


def table_to_graph_kind(src, dst, kind: int, lib_path: str = LIB_PATH) -> Graph:
    """The conversion for one graph kind: DIRECTED (as table_to_graph),
    UNDIRECTED (adjacency = distinct neighbours over both orientations; the
    in-arrays equal the out-arrays) or MULTIGRAPH (every row an edge, lists
    ordered by (neighbour, row), with the row index of every entry)."""
    src = np.ascontiguousarray(src, dtype=np.int64)
    dst = np.ascontiguousarray(dst, dtype=np.int64)
    if src.shape != dst.shape or src.ndim != 1:
        raise ValueError("src and dst must be 1-D arrays of equal length")
    L = load(lib_path)
    h = ctypes.c_void_p()
    V = ctypes.c_int64()
    E = ctypes.c_int64()
    rc = L.oracle_table_to_graph_kind(src.ctypes.data, dst.ctypes.data, src.size, kind, ctypes.byref(h),
                                      ctypes.byref(V), ctypes.byref(E))
    if rc != 0:
        raise OracleError({1: "invalid argument", 2: "too many nodes", 3: "out of memory"}.get(rc, str(rc)))
    try:
        arrays = (np.empty(V.value, np.int64), np.empty(V.value + 1, np.int64), np.empty(E.value, np.int32),
                  np.empty(V.value + 1, np.int64), np.empty(E.value, np.int32))
        g = MultiGraph(*arrays) if kind == MULTIGRAPH else Graph(*arrays)
        L.oracle_copy(h, g.node_ids.ctypes.data, g.out_offsets.ctypes.data, g.out_nbrs.ctypes.data,
                      g.in_offsets.ctypes.data, g.in_nbrs.ctypes.data)
        if kind == MULTIGRAPH:
            g.out_eids = np.empty(E.value, np.int32)
            g.in_eids = np.empty(E.value, np.int32)
            L.oracle_copy_eids(h, g.out_eids.ctypes.data, g.in_eids.ctypes.data)
    finally:
        L.oracle_free(h)
    return g


def graph_to_edge_table(g) -> tuple[np.ndarray, np.ndarray]:
    """Edge table of a graph (Section 2.4, "Conversion of graphs to tables"):
    for every node v in order and every out-neighbour w of v in order, the row
    (id of v, id of w).  `g` has numpy (or array-like) node_ids, out_offsets
    and out_nbrs."""
    ids = np.asarray(g.node_ids, dtype=np.int64)
    off = np.asarray(g.out_offsets, dtype=np.int64)
    nbr = np.asarray(g.out_nbrs, dtype=np.int64)
    V = ids.size
    src_idx = np.repeat(np.arange(V, dtype=np.int64), np.diff(off)) if V else np.zeros(0, np.int64)
    return ids[src_idx], ids[nbr]


def graph_to_node_table(g) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Node table of a graph: identifier, out-degree and in-degree per node."""
    ids = np.asarray(g.node_ids, dtype=np.int64)
    return (ids.copy(), np.diff(np.asarray(g.out_offsets, dtype=np.int64)),
            np.diff(np.asarray(g.in_offsets, dtype=np.int64)))


def graph_to_edge_table_loops(g) -> tuple[list, list]:
    """The same edge table written as two plain loops (small graphs only)."""
    src, dst = [], []
    for v in range(len(g.node_ids)):
        for i in range(int(g.out_offsets[v]), int(g.out_offsets[v + 1])):
            src.append(int(g.node_ids[v]))
            dst.append(int(g.node_ids[int(g.out_nbrs[i])]))
    return src, dst


def pagerank(g, damping: float = 0.85, iterations: int = 10) -> np.ndarray:
    """PageRank in fp64 (Page, Brin, Motwani & Winograd 1999), with the
    teleport and the rank of nodes without out-edges spread uniformly:
        r_0 = 1/V
        r_{t+1}[v] = (1-d)/V + d * (sum_{(u,v) in E} r_t[u]/outdeg(u) + D_t/V),
        D_t = sum of r_t[u] over u with outdeg(u) = 0.
    The edge sum walks the edge list (every (u, v) with u's out-neighbours)
    through numpy's bincount; no blocking, no reordering beyond that."""
    V = len(g.node_ids)
    if V == 0:
        return np.zeros(0)
    off = np.asarray(g.out_offsets, dtype=np.int64)
    nbr = np.asarray(g.out_nbrs, dtype=np.int64)
    outdeg = np.diff(off)
    src = np.repeat(np.arange(V, dtype=np.int64), outdeg)
    r = np.full(V, 1.0 / V)
    for _ in range(iterations):
        contrib = np.zeros(V)
        has = outdeg > 0
        contrib[has] = r[has] / outdeg[has]
        dangling = r[~has].sum()
        s = np.bincount(nbr, weights=contrib[src], minlength=V)
        r = (1.0 - damping) / V + damping * (s + dangling / V)
    return r


def pagerank_dense(g, damping: float = 0.85, iterations: int = 10) -> np.ndarray:
    """The same iteration as a dense V x V matrix power (small graphs): an
    independent route to pin `pagerank` against."""
    V = len(g.node_ids)
    off = np.asarray(g.out_offsets, dtype=np.int64)
    A = np.zeros((V, V))
    for u in range(V):
        for i in range(off[u], off[u + 1]):
            A[u, int(g.out_nbrs[i])] = 1.0
    deg = A.sum(axis=1)
    P = np.where(deg[:, None] > 0, A / np.maximum(deg, 1)[:, None], 1.0 / V)  # row-stochastic walk
    M = damping * P.T + (1.0 - damping) / V                                   # column-stochastic
    return np.linalg.matrix_power(M, iterations) @ np.full(V, 1.0 / V)
