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

    python -m paper_1503_07881_amd.autotune            # tune and save
    from paper_1503_07881_amd import autotune; autotune.apply()   # load and apply
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


def tune(log2_sizes=range(10, 27, 2), reps: int = 3, verbose: bool = False) -> dict:
    """Times every schedule for R-MAT tables of 2^k rows; returns
    {"device": ..., "buckets": {str(rows): {"items": i, "digit_bits": d, "node_method": m,
    "ms": {...}}}}."""
    import torch
    dev = torch.device("cuda:0")
    sh = torch.cuda.current_stream().cuda_stream
    out = {"device": _device_name(), "buckets": {}}
    for k in log2_sizes:
        n = 1 << k
        spec = workloads.TableSpec("rmat", n, seed=99, table=k, scale=workloads.rmat_scale_for(n))
        src = torch.empty(n, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), sh)
        times = {}
        for method in METHODS:
            for bits in DIGIT_BITS:
                for items in ITEMS:
                    ringo.tune_set(n, bits, items, method)
                    t0 = time.perf_counter()
                    ringo.graph_free(ringo.table_to_graph_raw(src.data_ptr(), dst.data_ptr(), n, sh))
                    torch.cuda.synchronize()
                    # small tables take milliseconds or less and vary from call
                    # to call: enough repetitions for about 50 ms each
                    first = time.perf_counter() - t0
                    ts = []
                    for _ in range(max(reps, min(50, int(0.05 / max(first, 1e-6))))):
                        t0 = time.perf_counter()
                        ringo.graph_free(ringo.table_to_graph_raw(src.data_ptr(), dst.data_ptr(), n, sh))
                        torch.cuda.synchronize()
                        ts.append(time.perf_counter() - t0)
                    times[(method, bits, items)] = sorted(ts)[len(ts) // 2] * 1e3
        method, bits, items = min(times, key=times.get)
        out["buckets"][str(n)] = {"items": items, "digit_bits": bits, "node_method": method,
                                  "ms": {f"{'hash' if m else 'sort'}/d{d}/{i}": round(v, 4)
                                         for (m, d, i), v in times.items()}}
        if verbose:
            print(f"rows 2^{k}: best {'hash' if method else 'sort'}/d{bits}/{items}  "
                  f"{out['buckets'][str(n)]['ms']}", flush=True)
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


if __name__ == "__main__":
    c = tune(verbose=True)
    print("saved", save(c))
