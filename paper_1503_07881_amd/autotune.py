"""Autotuner of the radix-pass schedule.

For every table-size bucket (powers of two of rows), the conversion is timed
on the device with each supported tile shape (items per thread of the
scatter tile), each radix digit width (8 to 11 bits) and each node-numbering
method (radix sort of all identifiers, or the node hash table), and the
fastest is kept.  Results are cached as JSON (RINGO_TUNE_CACHE, else the
in-tree tuned_schedules.json measured on an MI355X) and applied to the
library through ringo_tune_set.  The schedule changes only the tiling and
the number of passes: the output is the same bit for bit whichever schedule
runs.

    python -m paper_1503_07881_amd.autotune                 # tune and save
    python -m paper_1503_07881_amd.autotune --emit-header   # cache -> csrc/tuned_schedule.h
    from paper_1503_07881_amd import autotune; autotune.apply()   # load and apply

The library's built-in schedule table is generated from the committed
cache (csrc/tuned_schedule.h), so the tuned schedules apply from the
library's first call on; apply() sets another cache at run time.
"""
from __future__ import annotations

import json
import os
import time

from . import ringo, workloads

ITEMS = (8, 12, 16)
METHODS = (ringo.NODES_SORT, ringo.NODES_HASH)
DIGIT_BITS = (8, 9, 10, 11)


def cache_path() -> str:
    return os.environ.get("RINGO_TUNE_CACHE",
                          os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_schedules.json"))


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_properties(0).name if torch.cuda.is_available() else "none"


def tune(log2_sizes=range(10, 27), rounds: int = 0, margin: float = 0.03, verbose: bool = False) -> dict:
    """Times every schedule for R-MAT tables of 2^k rows; returns
    {"device": ..., "buckets": {str(rows): {"items": i, "digit_bits": d, "node_method": m,
    "ms": {...}}}}.  Every schedule runs twice first (allocations, graph
    captures), then the schedules take turns, one call each per round, so
    that drifts of the device affect them alike; the median per schedule
    counts (each timed call follows an untimed one of the same schedule, and
    each round starts at another schedule).  The library's built-in schedule
    for the size is kept unless
    another is faster by more than `margin` (calls of a few milliseconds or
    less vary by a few percent from call to call)."""
    import torch
    dev = torch.device("cuda:0")
    sh = torch.cuda.current_stream().cuda_stream
    out = {"device": _device_name(), "margin": margin, "buckets": {}}
    builtin = {k: ringo.tune_get(1 << k) for k in log2_sizes}
    scheds = [(m, b, i) for m in METHODS for b in DIGIT_BITS for i in ITEMS]

    def call(src, dst, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ringo.graph_free(ringo.table_to_graph_raw(src.data_ptr(), dst.data_ptr(), n, sh))
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for k in log2_sizes:
        n = 1 << k
        spec = workloads.TableSpec("rmat", n, seed=99, table=k, scale=workloads.rmat_scale_for(n))
        src = torch.empty(n, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), sh)
        first = 0.0
        for method, bits, items in scheds:
            ringo.tune_set(n, bits, items, method)
            call(src, dst, n)
            first = max(first, call(src, dst, n))
        # about a second of timed calls per size, 5 to 20 rounds
        r = rounds or max(5, min(20, int(1.0 / max(2 * first * len(scheds), 1e-6))))
        ts = {sc: [] for sc in scheds}
        for rd in range(r):
            # each round starts at another schedule, and each schedule's timed
            # call follows an untimed one of its own (the first call after a
            # change of schedule pays for buffers of other sizes)
            for j in range(len(scheds)):
                sc = scheds[(j + rd * 7) % len(scheds)]
                ringo.tune_set(n, sc[1], sc[2], sc[0])
                call(src, dst, n)
                ts[sc].append(call(src, dst, n))
        times = {sc: sorted(v)[len(v) // 2] * 1e3 for sc, v in ts.items()}
        d0, i0, m0 = builtin[k]
        best = min(times, key=times.get)
        if (m0, d0, i0) in times and times[(m0, d0, i0)] <= times[best] * (1 + margin):
            best = (m0, d0, i0)
        method, bits, items = best
        out["buckets"][str(n)] = {"items": items, "digit_bits": bits, "node_method": method,
                                  "ms": {f"{'hash' if m else 'sort'}/d{d}/{i}": round(v, 4)
                                         for (m, d, i), v in times.items()}}
        if verbose:
            print(f"rows 2^{k}: best {'hash' if method else 'sort'}/d{bits}/{items} "
                  f"({times[best]:.4f} ms; built-in {'hash' if m0 else 'sort'}/d{d0}/{i0} "
                  f"{times.get((m0, d0, i0), float('nan')):.4f} ms)", flush=True)
        del src, dst
    apply(out)
    return out


def save(cache: dict, path: str | None = None) -> str:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return path


def load(path: str | None = None) -> dict | None:
    path = path or cache_path()
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def apply(cache: dict | None = None) -> int:
    """Sets the library's schedule for the size buckets the cache covers;
    buckets between two tuned sizes take the schedule of the nearest tuned
    size below (the smallest tuned size for buckets below it), and buckets
    above the largest tuned size keep the library's.  A cached bucket
    without a node method keeps the library's; one without a digit width
    takes the cache's top-level "digit_bits", else 8.  Buckets with an
    unsupported entry are ignored.  Returns the number of buckets set."""
    cache = cache if cache is not None else load()
    if not cache:
        return 0
    default_bits = cache.get("digit_bits", 8)
    buckets = sorted((int(k), v.get("digit_bits", default_bits), v["items"], v.get("node_method"))
                     for k, v in cache.get("buckets", {}).items()
                     if v.get("items") in ITEMS and v.get("node_method", 0) in METHODS
                     and v.get("digit_bits", default_bits) in DIGIT_BITS)
    if not buckets:
        return 0
    applied = 0
    largest = buckets[-1][0]
    for e in range(0, 63):
        rows = 1 << e
        if rows > largest:
            break
        below = [(d, it, m) for n, d, it, m in buckets if n <= rows]
        bits, items, method = below[-1] if below else buckets[0][1:]
        ringo.tune_set(rows, bits, items, method)
        applied += 1
    return applied


HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "tuned_schedule.h")


def header_text(cache: dict) -> str:
    """The library's built-in schedule table (csrc/tuned_schedule.h) for a
    cache: one row per tuned size, in ascending order, that the library
    applies to the size buckets the cache covers as apply() does."""
    rows = sorted((int(k), v.get("digit_bits", 8), v["items"], v.get("node_method", 0))
                  for k, v in cache.get("buckets", {}).items()
                  if v.get("items") in ITEMS and v.get("node_method", 0) in METHODS
                  and v.get("digit_bits", 8) in DIGIT_BITS)
    lines = ["// Generated from tuned_schedules.json by `python -m paper_1503_07881_amd.autotune --emit-header`;",
             "// do not edit.  Schedules measured on " + str(cache.get("device", "?")) + " for R-MAT tables:",
             "// {log2 rows, digit bits, items per thread, node method (0 sort, 1 hash)}.",
             "#pragma once", "", "namespace ringo {", "",
             "struct TunedBucket {", "  int log2_rows, digit_bits, items, node_method;", "};", "",
             f"constexpr int NUM_TUNED = {len(rows)};",
             "constexpr TunedBucket TUNED[NUM_TUNED > 0 ? NUM_TUNED : 1] = {"]
    for n, d, it, m in rows:
        lines.append(f"    {{{n.bit_length() - 1}, {d}, {it}, {m}}},")
    if not rows:
        lines.append("    {0, 8, 8, 0},")
    lines += ["};", "", "}  // namespace ringo", ""]
    return "\n".join(lines)


def emit_header(cache: dict | None = None, path: str | None = None) -> str:
    cache = cache if cache is not None else load()
    path = path or HEADER
    with open(path, "w") as f:
        f.write(header_text(cache or {}))
    return path


if __name__ == "__main__":
    import sys
    if "--emit-header" in sys.argv:
        print("wrote", emit_header())
    else:
        c = tune(verbose=True)
        print("saved", save(c))
