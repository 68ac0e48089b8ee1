"""Python driver of the served form (argument marshalling only).

The server itself (queue, workers, admission, eviction, latency) is the
library's C++ code behind ringo_server_*; this module wraps it and replays
request traces with Poisson arrivals to report p50/p99 latency and
throughput.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass

import numpy as np

from . import ringo


class ServerConfig(ctypes.Structure):
    """ringo_server_config_t"""
    _fields_ = [("budget_bytes", ctypes.c_int64), ("num_streams", ctypes.c_int32),
                ("max_batch_tables", ctypes.c_int32), ("max_batch_rows", ctypes.c_int64)]


class BatchTimes(ctypes.Structure):
    """ringo_server_batch_t"""
    _fields_ = [("first_request", ctypes.c_int64), ("rows", ctypes.c_int64), ("stream", ctypes.c_int32),
                ("tables", ctypes.c_int32), ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    """ringo_server_stats_t"""
    _fields_ = [(n, ctypes.c_int64) for n in
                ("submitted", "completed", "failed", "evicted", "queued", "batches", "max_concurrent_batches",
                 "rows_completed", "resident_bytes", "peak_reserved_bytes")]


_bound = False


def _lib():
    global _bound
    L = ringo.lib()
    if not _bound:
        p, i64 = ctypes.c_void_p, ctypes.c_int64
        L.ringo_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]
        L.ringo_server_create.restype = ctypes.c_int
        L.ringo_server_submit.argtypes = [p, p, p, i64, ctypes.POINTER(ctypes.c_int64)]
        L.ringo_server_submit.restype = ctypes.c_int
        L.ringo_server_poll.argtypes = [p, i64, ctypes.POINTER(ringo.RawGraph), ctypes.POINTER(ctypes.c_double)]
        L.ringo_server_poll.restype = ctypes.c_int
        L.ringo_server_release.argtypes = [p, i64]
        L.ringo_server_release.restype = ctypes.c_int
        L.ringo_server_pin.argtypes = [p, i64, ctypes.POINTER(ringo.RawGraph)]
        L.ringo_server_pin.restype = ctypes.c_int
        L.ringo_server_unpin.argtypes = [p, i64]
        L.ringo_server_unpin.restype = ctypes.c_int
        L.ringo_server_batches.argtypes = [p, ctypes.POINTER(BatchTimes), ctypes.c_int]
        L.ringo_server_batches.restype = ctypes.c_int
        L.ringo_server_stats.argtypes = [p, ctypes.POINTER(ServerStats)]
        L.ringo_server_stats.restype = ctypes.c_int
        L.ringo_server_destroy.argtypes = [p]
        L.ringo_server_destroy.restype = None
        _bound = True
    return L


class Server:
    """A running server on the current device."""

    def __init__(self, budget_bytes: int = 200 << 30, num_streams: int = 3, max_batch_tables: int = 16,
                 max_batch_rows: int = 8 << 20):
        self._cfg = ServerConfig(budget_bytes, num_streams, max_batch_tables, max_batch_rows)
        h = ctypes.c_void_p()
        rc = _lib().ringo_server_create(ctypes.byref(self._cfg), ctypes.byref(h))
        if rc != 0:
            raise ringo.RingoError(rc, "ringo_server_create")
        self._h = h
        self._inputs = {}  # keeps host arrays alive while requests are pending

    def submit(self, src: np.ndarray, dst: np.ndarray) -> int:
        if src.dtype != np.int64 or dst.dtype != np.int64 or src.shape != dst.shape or src.ndim != 1:
            raise TypeError("src and dst must be 1-D int64 arrays of equal length")
        src = np.ascontiguousarray(src)
        dst = np.ascontiguousarray(dst)
        rid = ctypes.c_int64()
        rc = _lib().ringo_server_submit(self._h, src.ctypes.data, dst.ctypes.data, src.size, ctypes.byref(rid))
        if rc != 0:
            raise ringo.RingoError(rc, "ringo_server_submit")
        self._inputs[rid.value] = (src, dst)
        return rid.value

    def poll(self, req_id: int):
        """(status, RawGraph view or None, latency seconds or None)"""
        g = ringo.RawGraph()
        lat = ctypes.c_double(-1.0)
        rc = _lib().ringo_server_poll(self._h, req_id, ctypes.byref(g), ctypes.byref(lat))
        if rc != ringo.STATUS_PENDING:
            self._inputs.pop(req_id, None)
        return rc, (g if rc == 0 else None), (lat.value if lat.value >= 0 else None)

    def wait(self, req_id: int, timeout_s: float = 120.0):
        t0 = time.perf_counter()
        while True:
            rc, g, lat = self.poll(req_id)
            if rc != ringo.STATUS_PENDING:
                return rc, g, lat
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"request {req_id} still pending after {timeout_s} s")
            time.sleep(0.0002)

    def pin(self, req_id: int):
        """(status, RawGraph view or None): the graph is not evicted until unpin."""
        g = ringo.RawGraph()
        rc = _lib().ringo_server_pin(self._h, req_id, ctypes.byref(g))
        return rc, (g if rc == 0 else None)

    def unpin(self, req_id: int) -> int:
        return _lib().ringo_server_unpin(self._h, req_id)

    def graph(self, req_id: int, device) -> ringo.Graph:
        """Tensor copies of a resident graph: the view is pinned while the
        copies are made on the current stream, and unpinned once that stream
        has finished them (the view stays owned by the server)."""
        import torch
        rc, g = self.pin(req_id)
        if rc != 0:
            raise ringo.RingoError(rc, "ringo_server_pin")
        try:
            out = ringo.view_graph(g, device)
            copy = ringo.Graph(out.num_rows, out.num_nodes, out.num_edges,
                               *(torch.clone(getattr(out, f)) for f in
                                 ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs")))
            torch.cuda.current_stream(device).synchronize()
        finally:
            self.unpin(req_id)
        return copy

    def batches(self, max_entries: int = 1 << 16) -> list[dict]:
        """Device start/end (ms since the server started) of finished batches."""
        buf = (BatchTimes * max_entries)()
        k = _lib().ringo_server_batches(self._h, buf, max_entries)
        if k < 0:
            raise ringo.RingoError(4, "ringo_server_batches")
        return [{f: getattr(buf[i], f) for f, _ in BatchTimes._fields_} for i in range(k)]

    def release(self, req_id: int) -> int:
        self._inputs.pop(req_id, None)
        return _lib().ringo_server_release(self._h, req_id)

    def stats(self) -> dict:
        s = ServerStats()
        _lib().ringo_server_stats(self._h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            _lib().ringo_server_destroy(self._h)
            self._h = None
            self._inputs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@dataclass
class TraceResult:
    latencies_s: np.ndarray  # measured requests, in submission order
    rows: int                # rows of the measured requests
    makespan_s: float        # first measured submission to last completion
    failed: int
    evicted: int
    stats: dict

    def summary(self) -> dict:
        lat = self.latencies_s
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
                "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
                "edges_per_s": self.rows / self.makespan_s if self.makespan_s > 0 else None,
                "requests": int(lat.size), "failed": self.failed, "evicted": self.evicted,
                "batches": self.stats.get("batches"),
                "max_concurrent_batches": self.stats.get("max_concurrent_batches")}


def device_overlap(batches: list[dict]) -> dict:
    """From batch device intervals: the time with at least one batch on the
    device, the part of it with two or more (on different streams), and the
    most batches at once."""
    ev = []
    for b in batches:
        ev.append((b["start_ms"], 1))
        ev.append((b["end_ms"], -1))
    ev.sort()
    busy = multi = 0.0
    cur = peak = 0
    last = None
    for t, d in ev:
        if last is not None:
            if cur >= 1:
                busy += t - last
            if cur >= 2:
                multi += t - last
        cur += d
        peak = max(peak, cur)
        last = t
    return {"device_busy_ms": busy, "device_overlap_ms": multi,
            "overlap_frac": multi / busy if busy > 0 else 0.0, "max_batches_at_once": peak}


def replay(server: Server, tables, arrivals_s, warmup: int = 0, release: bool = True) -> TraceResult:
    """Submits tables[i] at arrivals_s[i] (seconds from start), waits for all
    of them, and returns the latencies of the requests after the first
    `warmup` ones.  With release, each graph is released once measured;
    without, graphs stay resident and the budget evicts the least recently
    used ones."""
    ids = []
    t0 = time.perf_counter()
    for (src, dst), at in zip(tables, arrivals_s):
        while True:
            dt = at - (time.perf_counter() - t0)
            if dt <= 0:
                break
            time.sleep(min(dt, 0.0005) if dt > 0.0002 else 0)
        ids.append(server.submit(src, dst))
    t_first = t0 + (arrivals_s[warmup] if warmup < len(arrivals_s) else 0.0)
    lat, rows, failed, evicted = [], 0, 0, 0
    t_last = t_first
    for i, rid in enumerate(ids):
        rc, g, l = server.wait(rid)
        if i >= warmup:
            # a graph evicted before this poll was converted all the same
            if rc in (0, ringo.STATUS_EVICTED) and l is not None:
                lat.append(l)
                rows += int(tables[i][0].size)
                t_last = max(t_last, t0 + arrivals_s[i] + l)
                evicted += rc == ringo.STATUS_EVICTED
            else:
                failed += 1
        if release:
            server.release(rid)
    return TraceResult(np.array(lat), rows, t_last - t_first, failed, evicted, server.stats())
