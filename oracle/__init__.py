"""CPU oracle of the table-to-graph conversion -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  The product path (the C-ABI library and
its Python binding) never imports or calls it, and the two share no code.

`table_to_graph(src, dst)` returns the plain definition of the conversion
(Section 2.4, "Conversion of tables to graphs"): the sorted distinct node
identifiers, and CSR out- and in-adjacency over dense node positions with
each neighbour list strictly increasing.  See `oracle.cpp` for the steps and
the readings taken where the paper is silent.
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
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out, source]
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


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if path not in _libs:
        if not os.path.exists(path) and path == LIB_PATH:
            build()
        L = ctypes.CDLL(path)
        p = ctypes.c_void_p
        L.oracle_table_to_graph.argtypes = [p, p, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.oracle_table_to_graph.restype = ctypes.c_int
        L.oracle_copy.argtypes = [p, p, p, p, p, p]
        L.oracle_copy.restype = None
        L.oracle_free.argtypes = [p]
        L.oracle_free.restype = None
        _libs[path] = L
    return _libs[path]


def table_to_graph(src, dst, lib_path: str = LIB_PATH) -> Graph:
    src = np.ascontiguousarray(src, dtype=np.int64)
    dst = np.ascontiguousarray(dst, dtype=np.int64)
    if src.shape != dst.shape or src.ndim != 1:
        raise ValueError("src and dst must be 1-D arrays of equal length")
    L = load(lib_path)
    h = ctypes.c_void_p()
    V = ctypes.c_int64()
    E = ctypes.c_int64()
    rc = L.oracle_table_to_graph(src.ctypes.data, dst.ctypes.data, src.size, ctypes.byref(h),
                                 ctypes.byref(V), ctypes.byref(E))
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
