"""Seeded synthetic edge tables shaped like the paper's conversion workloads.

The paper times table-to-graph conversion on LiveJournal (4.8M nodes, 69M
edges) and Twitter2010 (42M nodes, 1.5B edges) (Section 3, Tables 2 and 5).
Neither dataset is available here; R-MAT tables of the same shape stand in
for them, with node indices hashed to random signed 64-bit identifiers.

This module draws input rows only.  It holds none of the conversion's
arithmetic and is the one piece shared by the GPU path's tests and the CPU
oracle's tests.  Every draw is counter-based SplitMix64, so the host and the
device generators produce identical rows.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
GEN_LIB_PATH = os.path.join(_HERE, "libringo_gen.so")

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

# stream purposes
TAG_SALT, TAG_SRC, TAG_DST, TAG_DUP, TAG_SHUF, TAG_RMAT, TAG_SIZE, TAG_KIND, TAG_ARRIVAL = range(1, 10)


def mix64(z: int) -> int:
    """SplitMix64 output finaliser (Steele, Lea & Flood, OOPSLA 2014)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def draw(stream: int, k: int) -> int:
    return mix64(stream + (k + 1) * GAMMA)


def stream(seed: int, table: int, tag: int) -> int:
    """Seed of the random stream for (config seed, table index, purpose)."""
    return mix64(mix64(mix64(seed) ^ (table & MASK64)) ^ ((tag * GAMMA) & MASK64))


def unit(stream_seed: int, k: int) -> float:
    """Uniform double in [0, 1) from the top 53 bits of a draw."""
    return (draw(stream_seed, k) >> 11) * (1.0 / (1 << 53))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(GEN_LIB_PATH):
            raise RuntimeError(f"generator library missing: {GEN_LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(GEN_LIB_PATH)
        i64, u64, p64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        L.ringo_gen_uniform.argtypes = [i64, i64, i64, ctypes.c_int, u64, u64, u64, u64, u64, ctypes.c_int, p64, p64]
        L.ringo_gen_uniform.restype = ctypes.c_int
        L.ringo_gen_rmat.argtypes = [i64, ctypes.c_int, u64, u64, ctypes.c_int, p64, p64]
        L.ringo_gen_rmat.restype = ctypes.c_int
        L.ringo_gen_rmat_device.argtypes = [i64, ctypes.c_int, u64, u64, p64, p64, p64]
        L.ringo_gen_rmat_device.restype = ctypes.c_int
        L.ringo_gen_uniform_device.argtypes = [i64, i64, u64, u64, u64, p64, p64, p64]
        L.ringo_gen_uniform_device.restype = ctypes.c_int
        L.ringo_gen_copy_device.argtypes = [p64, p64, i64, p64]
        L.ringo_gen_copy_device.restype = ctypes.c_int
        L.ringo_gen_mix64.argtypes = [u64]
        L.ringo_gen_mix64.restype = u64
        _lib = L
    return _lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


@dataclass(frozen=True)
class TableSpec:
    """Recipe of one synthetic edge table."""
    kind: str          # "uniform" or "rmat"
    n: int             # rows
    seed: int          # config seed
    table: int = 0     # table index inside the config
    pool: int = 0      # uniform: number of distinct identifiers drawn from
    ndup: int = 0      # uniform: injected exact duplicate rows
    shuffle: bool = False
    scale: int = 0     # rmat: levels (2^scale node slots)

    def streams(self):
        return {t: stream(self.seed, self.table, t) for t in
                (TAG_SALT, TAG_SRC, TAG_DST, TAG_DUP, TAG_SHUF, TAG_RMAT)}


def generate_host(spec: TableSpec, threads: int | None = None):
    """Rows of `spec` as two int64 numpy arrays (src, dst)."""
    n = int(spec.n)
    src = np.empty(n, dtype=np.int64)
    dst = np.empty(n, dtype=np.int64)
    if n == 0:
        return src, dst
    s = spec.streams()
    th = _threads() if threads is None else threads
    L = lib()
    if spec.kind == "uniform":
        rc = L.ringo_gen_uniform(n, spec.pool, spec.ndup, int(spec.shuffle), s[TAG_SALT], s[TAG_SRC],
                                 s[TAG_DST], s[TAG_DUP], s[TAG_SHUF], th,
                                 src.ctypes.data, dst.ctypes.data)
    elif spec.kind == "rmat":
        rc = L.ringo_gen_rmat(n, spec.scale, s[TAG_SALT], s[TAG_RMAT], th, src.ctypes.data, dst.ctypes.data)
    else:
        raise ValueError(spec.kind)
    if rc != 0:
        raise ValueError(f"generator rejected {spec}")
    return src, dst


def generate_device(spec: TableSpec, src_ptr: int, dst_ptr: int, stream_handle: int = 0):
    """Write the rows of `spec` into caller-owned device arrays (no injected
    duplicates or shuffle on the device)."""
    s = spec.streams()
    L = lib()
    if spec.kind == "rmat":
        rc = L.ringo_gen_rmat_device(spec.n, spec.scale, s[TAG_SALT], s[TAG_RMAT], src_ptr, dst_ptr, stream_handle)
    elif spec.kind == "uniform" and spec.ndup == 0 and not spec.shuffle:
        rc = L.ringo_gen_uniform_device(spec.n, spec.pool, s[TAG_SALT], s[TAG_SRC], s[TAG_DST], src_ptr, dst_ptr,
                                        stream_handle)
    else:
        raise ValueError(f"no device generator for {spec}")
    if rc != 0:
        raise RuntimeError(f"device generator failed ({rc}) for {spec}")


def copy_device(dst_ptr: int, src_ptr: int, nbytes: int, stream_handle: int = 0):
    """Plain streaming copy (bandwidth and counter calibration)."""
    if lib().ringo_gen_copy_device(dst_ptr, src_ptr, nbytes, stream_handle) != 0:
        raise RuntimeError("copy kernel rejected its arguments")


# ------------------------------------------------------------------ the workloads

def config1() -> TableSpec:
    """1,000,000 rows drawn uniformly from 100,000 identifiers, 1% exact
    duplicate rows injected, rows shuffled; self-loops occur naturally."""
    return TableSpec("uniform", 1_000_000, seed=1, pool=100_000, ndup=10_000, shuffle=True)


def config2() -> TableSpec:
    """R-MAT scale 22, 2^26 rows (edge factor 16): LiveJournal-shaped."""
    return TableSpec("rmat", 1 << 26, seed=2, scale=22)


def config3() -> TableSpec:
    """R-MAT scale 26, 1.5e9 rows: Twitter2010-shaped (24 GB of input)."""
    return TableSpec("rmat", 1_500_000_000, seed=3, scale=26)


def rmat_scale_for(n: int) -> int:
    return max(1, math.ceil(math.log2(max(n, 1) / 16))) if n > 16 else 1


def mixed_table(seed: int, i: int, lo: float, hi: float) -> TableSpec:
    """Table i of a mixed batch: n log-uniform in [lo, hi]; even i uniform
    (pool n/10, no injected duplicates), odd i R-MAT (scale ceil(log2(n/16)))."""
    u = unit(stream(seed, i, TAG_SIZE), 0)
    n = int(math.floor(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))
    if i % 2 == 0:
        return TableSpec("uniform", n, seed=seed, table=i, pool=max(1, n // 10))
    return TableSpec("rmat", n, seed=seed, table=i, scale=rmat_scale_for(n))


def config4(num_tables: int = 4096) -> list[TableSpec]:
    """4096 tables, rows log-uniform in [1e3, 2e6], half uniform, half R-MAT."""
    return [mixed_table(4, i, 1e3, 2e6) for i in range(num_tables)]


def config5_request(j: int) -> TableSpec:
    """Request j of the served stream: rows log-uniform in [1e4, 5e7], uniform
    or R-MAT with probability 1/2 each."""
    u = unit(stream(5, j, TAG_SIZE), 0)
    n = int(math.floor(math.exp(math.log(1e4) + u * (math.log(5e7) - math.log(1e4)))))
    if draw(stream(5, j, TAG_KIND), 0) >> 63:
        return TableSpec("rmat", n, seed=5, table=j, scale=rmat_scale_for(n))
    return TableSpec("uniform", n, seed=5, table=j, pool=max(1, n // 10))


def config5_arrivals(num: int, rate_per_s: float) -> np.ndarray:
    """Poisson arrival times (seconds) of `num` requests at `rate_per_s`."""
    s = stream(5, 0, TAG_ARRIVAL)
    gaps = [-math.log(1.0 - unit(s, k)) / rate_per_s for k in range(num)]
    return np.cumsum(np.array(gaps, dtype=np.float64))
