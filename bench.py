#!/usr/bin/env python3
"""Throughput of the table-to-graph conversion (Section 2.4) on one MI355X.

A step is one full conversion of the 1.5e9-row R-MAT scale-26 edge table
(the Twitter2010-shaped stand-in of Table 2, the largest single-GPU
workload): node numbering, edge-key sort, dedupe, out-CSR, in-key sort,
in-CSR, output allocation and the size read-backs.  The input columns are
generated on the device and are resident in HBM before the timed region
starts.

Prints one JSON line: edges/s (input rows per second, the paper's "Edges/s"
of Table 5), the roofline position of the dominant kernel measured with HIP
events on the conversion's stream inside the timed region, the whole
conversion's algorithmic-byte and counter-traffic fractions of HBM peak, the
CPU oracle timed on a bounded prefix of the same workload, and as extra keys
the 2^26-row (LiveJournal-shaped) workload, the batched speedup over 4096
tables, and the oracle's time on the whole 2^26-row table.

--config 1|2 time the 1e6-row or 2^26-row workload instead; --config 4 the
batched form alone; --config 5 the served form (p50/p99 latency).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
KERNEL_DIR = os.path.join(ROOT, "paper_1503_07881_amd", "csrc")

# Trace entry -> kernel name in a rocprofv3 summary ({items}: items per thread,
# {bits}: the schedule's digit width; a|b: either instantiation, one entry
# covering both).  Radix-pass instantiations: <256, items, mode, digit bits>,
# mode 1 node (first pass), 3 node, 4 distinct nodes, 5 edge, 2 in (first
# pass), 6 in, 10 in (first pass, dedupe folded), 11 and 12 the groupings of
# the partitioned numbering, 13 its rank grouping.  Passes take 8-bit digits
# where the key width leaves room, so an entry may cover both widths.
ROCPROF_NAME = {
    "hash_estimate": "k_hll", "hash_insert": "k_hash_insert|k_hash_insert_keys",
    "hash_compact": "k_hash_compact",
    "hash_rank": "k_hash_rank", "hash_remap_pack": "k_hash_remap", "hash_bucket_sort": "k_bucket_sort",
    "hash_pack_parts": "k_hash_pack_parts", "hash_rank_slots": "k_hash_rank_slots",
    "hash_part_scatter": "k_downsweep<256, {items}, 11, 8>",
    "hash_part_dst_scatter": "k_downsweep<256, {items}, 12, 8>",
    "hash_part_rank": "k_downsweep<256, {items}, 13, 8>",
    "unique": "k_dedupe_write<false>",
    "directory": "k_dir", "remap_pack": "k_remap", "dedupe_out_csr": "k_dedupe_write<true>", "in_csr": "k_in_csr",
    "sort_node_scatter": "k_downsweep<256, {items}, 1|3, 8|{bits}>",
    "sort_vnode_scatter": "k_downsweep<256, {items}, 4, 8|{bits}>",
    # plain edge and in-passes of 16-key schedules with digits of at most
    # 9 bits run on two-half tiles (k_downsweep_pair<16, mode, digit bits>)
    "sort_edge_scatter": ("k_downsweep<256, {items}, 5, 8|{bits}>", "k_downsweep_pair<16, 5, 8|{bits}>"),
    "sort_in_scatter": ("k_downsweep<256, {items}, 2|6|10, 8|{bits}>", "k_downsweep_pair<16, 6, 8|{bits}>"),
}


def rocprof_names(entry: str, items: int, bits: int) -> list:
    """Every kernel name a trace entry may stand for in a rocprofv3 summary."""
    import itertools
    pats = ROCPROF_NAME.get(entry, entry)
    names = []
    for pat in (pats,) if isinstance(pats, str) else pats:
        pat = pat.format(items=items, bits=bits)
        if "<" not in pat:
            names += pat.split("|")
            continue
        head, args = pat[:-1].split("<", 1)
        alts = [sorted(set(a.strip().split("|")), key=lambda x: (len(x), x)) for a in args.split(",")]
        names += [f"{head}<{', '.join(c)}>" for c in itertools.product(*alts)]
    return names


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_file(kernel: str) -> str:
    if kernel == "edge_table":
        return "to_table.hip"
    pats = ROCPROF_NAME.get(kernel, "")
    if kernel.startswith("sort_") or any(p.startswith("k_downsweep") for p in
                                         ((pats,) if isinstance(pats, str) else pats)):
        return "lsd.h"
    return "hash.hip" if kernel.startswith("hash_") else "kernels.hip"


def kernel_source_sha(kernel: str) -> str:
    """Digest of the source file that holds `kernel` and of the device
    helpers it includes: counter summaries taken before a change to them no
    longer describe the kernel."""
    h = hashlib.sha256()
    for name in (kernel_source_file(kernel), "device_common.h", "ringo_internal.h"):
        with open(os.path.join(KERNEL_DIR, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_file(kernel: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, or None when the kernels changed since."""
    path = traffic_file(kernel, workload)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_sha(kernel):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


CONVERSION_SOURCES = ("kernels.hip", "lsd.h", "hash.hip", "pipeline.hip", "device_common.h",
                      "ringo_internal.h")


def conversion_source_sha() -> str:
    """Digest of every source that decides which kernels one conversion runs
    and how they touch memory."""
    h = hashlib.sha256()
    for name in CONVERSION_SOURCES:
        with open(os.path.join(KERNEL_DIR, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def read_conversion_traffic(workload: str):
    """HBM bytes (fetched + written) of one whole conversion on `workload`,
    summed over all of its kernels, from the committed rocprofv3 counter
    summary; None when the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_conversion_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("conversion_source_sha") != conversion_source_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_conversion"])
    except (KeyError, ValueError):
        return None


def host_info() -> dict:
    """The host the CPU baseline ran on: logical CPUs, CPU model, memory."""
    info = {"logical_cpus": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["mem_GiB"] = round(int(line.split()[1]) / (1 << 20), 1)
                    break
    except OSError:
        pass
    return info


def cpu_baseline(spec, rows: int):
    """The oracle as it stands, on the first `rows` rows of the benchmarked
    workload (generated on the host with the same seeded generator)."""
    import numpy as np  # noqa: F401
    import oracle
    from paper_1503_07881_amd import workloads
    sample = workloads.TableSpec(spec.kind, min(rows, spec.n), seed=spec.seed, scale=spec.scale)
    src, dst = workloads.generate_host(sample)
    t0 = time.perf_counter()
    oracle.table_to_graph(src, dst)
    dt = time.perf_counter() - t0
    what = (f"first {sample.n:,} rows of the {_workload_name(spec)} workload (rows are i.i.d., so a prefix "
            f"is a sample of the same distribution)")
    single = {"value": sample.n / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
              "sample": f"{what}; single-threaded std::sort oracle, {dt:.2f} s"}
    # the same oracle with its sorts on every host thread (the rest of its
    # steps stay serial)
    t0 = time.perf_counter()
    oracle.table_to_graph(src, dst, all_cores=True)
    dp = time.perf_counter() - t0
    par = {"value": sample.n / dp, "unit": "edges/s", "cores": oracle.last_threads, "kind": "oracle",
           "sample": f"{what}; the oracle with a parallel sort (libstdc++ parallel mode) on "
                     f"{oracle.last_threads} threads, {dp:.2f} s"}
    single["host"] = par["host"] = host_info()
    return single, par


def bench_batched(args):
    """4096 tables, rows log-uniform in [1e3, 2e6]: one batched call against
    one call per table, same GPU, outputs compared bit for bit."""
    import torch
    from paper_1503_07881_amd import ringo, workloads
    dev = torch.device("cuda:0")
    specs = workloads.config4()
    total = sum(s.n for s in specs)
    log(f"bench: batched workload, {len(specs)} tables, {total:,} rows")
    src = torch.empty(total, dtype=torch.int64, device=dev)
    dst = torch.empty(total, dtype=torch.int64, device=dev)
    sh = torch.cuda.current_stream().cuda_stream
    offs, off = [], 0
    for s in specs:
        workloads.generate_device(s, src.data_ptr() + 8 * off, dst.data_ptr() + 8 * off, sh)
        offs.append((off, s.n))
        off += s.n
    torch.cuda.synchronize()
    sp = [src.data_ptr() + 8 * o for o, _ in offs]
    dp = [dst.data_ptr() + 8 * o for o, _ in offs]
    ns = [n for _, n in offs]

    def batched():
        return ringo.table_to_graph_batched_raw(sp, dp, ns, sh)

    def singles():
        out = []
        for s_, d_, n_ in zip(sp, dp, ns):
            out.append(ringo.table_to_graph_raw(s_, d_, n_, sh))
        return out

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gs = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            for g in gs:
                ringo.graph_free(g)
        return sorted(ts)[len(ts) // 2]

    for g in batched():
        ringo.graph_free(g)
    for g in singles():
        ringo.graph_free(g)
    t_b = timed(batched, max(1, args.steps))
    log(f"bench: batched {t_b * 1e3:.1f} ms")
    t_s = timed(singles, max(1, min(args.steps, 3)))
    log(f"bench: one call per table {t_s * 1e3:.1f} ms")
    # identical output, table by table, on the device
    gb = [ringo._wrap(r, dev) for r in batched()]
    mismatches = 0
    for i, (s_, d_, n_) in enumerate(zip(sp, dp, ns)):
        g1 = ringo._wrap(ringo.table_to_graph_raw(s_, d_, n_, sh), dev)
        for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs"):
            if not torch.equal(getattr(gb[i], f), getattr(g1, f)):
                mismatches += 1
                break
    out = {
        "metric": "batched speedup: one batched call vs one call per table (same GPU, identical output)",
        "value": t_s / t_b, "unit": "x", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic (seeded uniform and R-MAT tables generated on the device)",
        "config": {"workload": "batch_4096_tables_rows_1e3_to_2e6", "tables": len(specs), "rows": total},
        "batched_edges_per_s": total / t_b, "single_calls_edges_per_s": total / t_s,
        "single_calls_ms": t_s * 1e3, "tables_differing": mismatches,
    }
    print(json.dumps(out), flush=True)


def _device_table(spec, dev):
    import torch
    from paper_1503_07881_amd import workloads
    src = torch.empty(spec.n, dtype=torch.int64, device=dev)
    dst = torch.empty(spec.n, dtype=torch.int64, device=dev)
    if spec.kind == "rmat" or (spec.ndup == 0 and not spec.shuffle):
        workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), torch.cuda.current_stream().cuda_stream)
    else:
        hs, hd = workloads.generate_host(spec)
        src.copy_(torch.from_numpy(hs))
        dst.copy_(torch.from_numpy(hd))
    return src, dst


def _workload_name(spec) -> str:
    return (f"{spec.kind}_scale{spec.scale}_rows{spec.n}" if spec.kind == "rmat"
            else f"uniform_rows{spec.n}_pool{spec.pool}")


def bench_to_table(args):
    """Graph-to-table conversion: the edge table of the graph built from the
    workload (edges/s = graph edges per second), one kernel per call."""
    import numpy as np
    import torch
    from paper_1503_07881_amd import ringo, workloads
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = {1: workloads.config1, 2: workloads.config2, 3: workloads.config3}[args.config]()
    src, dst = _device_table(spec, dev)
    g = ringo.to_graph(src, dst)
    del src, dst
    V, E = g.num_nodes, g.num_edges
    es = torch.empty(E, dtype=torch.int64, device=dev)
    ed = torch.empty(E, dtype=torch.int64, device=dev)
    raw = ringo.raw_of(g)
    sh = torch.cuda.current_stream().cuda_stream
    for _ in range(args.warmup):
        ringo.graph_to_edge_table_raw(raw, es.data_ptr(), ed.data_ptr(), sh)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        ringo.graph_to_edge_table_raw(raw, es.data_ptr(), ed.data_ptr(), sh)
        b.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    kms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    nbytes = 36.0 * E + 8.0 * (V + 1)   # offsets, neighbours, two id reads and two id writes per edge
    achieved = nbytes / (kms / 1e3) / 1e9
    workload = _workload_name(spec)
    out = {"metric": "edges/s converted (graph to edge table, 1 GPU)", "value": E / (ms / 1e3),
           "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic (the graph of the seeded workload table)",
           "config": {"workload": workload, "rows": spec.n, "nodes": V, "edges": E},
           "roofline": {"bound": "hbm", "kernel": "edge_table", "rocprof_kernel": "k_edge_table",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBPS, 4),
                        "traffic": read_traffic("edge_table", workload),
                        "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": round(kms, 5)}}
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph(g.node_ids.cpu().numpy(), g.out_offsets.cpu().numpy(), g.out_nbrs.cpu().numpy(),
                          g.in_offsets.cpu().numpy(), g.in_nbrs.cpu().numpy())
        t1 = time.perf_counter()
        oracle.graph_to_edge_table(og)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": E / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole graph ({E:,} edges), numpy oracle, {dt:.2f} s"}
    print(json.dumps(out), flush=True)


def bench_pagerank(args):
    """PageRank, ten iterations (the count the paper times), on the graph of
    the workload; value = edges x iterations per second."""
    import torch
    from paper_1503_07881_amd import ringo, workloads
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = {1: workloads.config1, 2: workloads.config2, 3: workloads.config3}[args.config]()
    src, dst = _device_table(spec, dev)
    g = ringo.to_graph(src, dst)
    del src, dst
    V, E, iters = g.num_nodes, g.num_edges, 10
    ranks = torch.empty(V, dtype=torch.float64, device=dev)
    raw = ringo.raw_of(g)
    sh = torch.cuda.current_stream().cuda_stream
    for _ in range(args.warmup):
        ringo.pagerank_raw(raw, 0.85, iters, ranks.data_ptr(), sh)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        ringo.pagerank_raw(raw, 0.85, iters, ranks.data_ptr(), sh)
        b.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    kms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    # per iteration: in-neighbour index + gathered contribution per edge; per
    # node the two offsets, the rank, the contribution (written, then read) and
    # the new rank
    nbytes = iters * (12.0 * E + 48.0 * V)
    achieved = nbytes / (kms / 1e3) / 1e9
    workload = _workload_name(spec)
    out = {"metric": "PageRank edge-iterations/s (10 iterations, fp64, 1 GPU)", "value": E * iters / (ms / 1e3),
           "unit": "edges*iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (the graph of the seeded workload table)",
           "config": {"workload": workload, "rows": spec.n, "nodes": V, "edges": E, "iterations": iters,
                      "damping": 0.85},
           "roofline": {"bound": "hbm", "kernel": "pagerank_10_iterations", "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                        "traffic": None, "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": round(kms, 5)}}
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph(g.node_ids.cpu().numpy(), g.out_offsets.cpu().numpy(), g.out_nbrs.cpu().numpy(),
                          g.in_offsets.cpu().numpy(), g.in_nbrs.cpu().numpy())
        t1 = time.perf_counter()
        oracle.pagerank(og, 0.85, iters)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": E * iters / dt, "unit": "edges*iterations/s", "cores": 1,
                               "kind": "oracle", "sample": f"the whole graph, 10 iterations, numpy oracle, {dt:.2f} s"}
    print(json.dumps(out), flush=True)


def serve_runs(pool: int, n_req: int, warm: int, rates, budgets, streams: int, batch_rows: int):
    """The served workload: a pool of request tables (rows log-uniform in
    [1e4, 5e7], uniform or R-MAT) in pinned host memory, replayed with
    Poisson arrivals at each rate (a fraction of the measured one-at-a-time
    capacity) under each HBM budget, graphs left resident (the budget evicts
    least recently used ones); continuous batching against FIFO
    one-at-a-time on the same trace.  Returns the runs and the capacity."""
    import numpy as np
    import torch
    from paper_1503_07881_amd import serve, workloads
    torch.cuda.set_device(0)
    log(f"bench: serving pool of {pool} request tables (host generation, pinned)")
    tables = []
    for j in range(pool):
        sp = workloads.config5_request(j)
        hs, hd = workloads.generate_host(sp)
        tables.append((torch.from_numpy(hs).pin_memory().numpy(), torch.from_numpy(hd).pin_memory().numpy()))
    # one-at-a-time capacity: the pool back to back through a FIFO server
    with serve.Server(max(budgets), num_streams=1, max_batch_tables=1) as fifo:
        serve.replay(fifo, tables[:8], np.zeros(8))
        t0 = time.perf_counter()
        serve.replay(fifo, tables, np.zeros(pool))
        mu = pool / (time.perf_counter() - t0)
    log(f"bench: one-at-a-time capacity {mu:.1f} requests/s")
    trace = [tables[j % pool] for j in range(n_req + warm)]
    runs = {}
    for budget in budgets:
        for frac in rates:
            arrivals = workloads.config5_arrivals(n_req + warm, frac * mu)
            with serve.Server(budget, num_streams=streams, max_batch_tables=16, max_batch_rows=batch_rows) as srv:
                r = serve.replay(srv, trace, arrivals, warmup=warm, release=False)
                cb = r.summary()
                cb["device"] = serve.device_overlap(srv.batches())
                cb["peak_reserved_bytes"] = r.stats["peak_reserved_bytes"]
                cb["resident_bytes_at_end"] = r.stats["resident_bytes"]
            with serve.Server(budget, num_streams=1, max_batch_tables=1) as fifo:
                ff = serve.replay(fifo, trace, arrivals, warmup=warm, release=False).summary()
            key = f"{frac}mu_budget{budget >> 30}GiB"
            runs[key] = {"rate_per_s": frac * mu, "budget_bytes": budget, "continuous_batching": cb,
                         "fifo_one_at_a_time": ff}
            log(f"bench: {key}: p50/p99 {cb['p50_ms']:.2f}/{cb['p99_ms']:.2f} ms, evicted {cb['evicted']} "
                f"(FIFO {ff['p50_ms']:.2f}/{ff['p99_ms']:.2f} ms), device overlap "
                f"{cb['device']['overlap_frac']:.2f}")
    del tables, trace
    return runs, mu


def bench_serve(args):
    """Served form (--config 5): at least 2000 measured requests at 0.5 and
    0.8 of the one-at-a-time capacity, under the 200 GB budget and under one
    that binds."""
    budgets = (200 << 30, args.serve_small_budget_gib << 30)
    runs, mu = serve_runs(args.serve_pool, args.serve_requests, args.serve_warmup, (0.5, 0.8), budgets,
                          args.serve_streams, args.serve_batch_rows)
    hi = runs[f"0.8mu_budget{200}GiB"]["continuous_batching"]
    out = {
        "metric": "p50 serve latency (submission to resident graph) at 0.8x one-at-a-time capacity",
        "value": hi["p50_ms"], "unit": "ms", "n_gpus": 1, "steps": args.serve_requests,
        "warmup": args.serve_warmup, "ms_per_step": hi["mean_ms"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic (seeded uniform and R-MAT request tables, pinned host memory)",
        "config": {"workload": "serve_poisson_rows_1e4_to_5e7", "pool_tables": args.serve_pool,
                   "requests": args.serve_requests, "budgets_bytes": list(budgets),
                   "streams": args.serve_streams, "max_batch_rows": args.serve_batch_rows},
        "p99_ms": hi["p99_ms"], "edges_per_s": hi["edges_per_s"], "capacity_one_at_a_time_per_s": mu,
        "runs": runs,
    }
    print(json.dumps(out), flush=True)


def copy_bandwidth(dev, sh):
    """Achievable-bandwidth reference: a plain 16-byte copy of 2 GiB (five
    launches timed with events on the stream they run on)."""
    import torch
    from paper_1503_07881_amd import workloads
    cbytes = 1 << 31
    ca = torch.empty(cbytes // 8, dtype=torch.int64, device=dev)
    cb = torch.empty_like(ca)
    for _ in range(2):
        workloads.copy_device(cb.data_ptr(), ca.data_ptr(), cbytes, sh)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        workloads.copy_device(cb.data_ptr(), ca.data_ptr(), cbytes, sh)
    e1.record()
    torch.cuda.synchronize()
    del ca, cb
    return 2 * cbytes * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9


def measure_conversion(spec, args, kind, copy_gbps, steps, warmup):
    """Times `steps` conversions of `spec` (generated on the device, resident
    before the timed region): untraced, per step, and traced with the
    library's HIP events on the conversion's stream. Returns the pieces of
    the benchmark line."""
    import torch
    from paper_1503_07881_amd import ringo
    dev = torch.device("cuda:0")
    n = spec.n
    log(f"bench: generating {spec.kind} n={n:,} on the device")
    src, dst = _device_table(spec, dev)
    torch.cuda.synchronize()
    sh = torch.cuda.current_stream().cuda_stream

    def step():
        g = ringo.table_to_graph_raw(src.data_ptr(), dst.data_ptr(), n, sh, kind)
        V, E = g.num_nodes, g.num_edges
        ringo.graph_free(g)
        return V, E

    V = E = 0
    for i in range(warmup):
        V, E = step()
        log(f"bench: warmup {i + 1}/{warmup} V={V:,} E={E:,}")
    torch.cuda.synchronize()
    # untraced: K steps back to back, then each step alone (median)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms_untraced = (time.perf_counter() - t0) * 1e3 / steps
    per = []
    for _ in range(min(steps, 5)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t1) * 1e3)
    log(f"bench: untraced {ms_untraced:.3f} ms/step (median of {len(per)} single steps "
        f"{sorted(per)[len(per) // 2]:.3f})")
    # timed region, with per-kernel HIP events on the conversion's stream
    # (a single table on the sync-free path enqueues its kernels here rather
    # than replaying its captured graph, so that every kernel is timed)
    ringo.trace_enable(True)
    os.environ["RINGO_FIXED_GRAPH"] = "0"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        V, E = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    os.environ.pop("RINGO_FIXED_GRAPH", None)
    trace = ringo.trace_read()
    ringo.trace_enable(False)
    log(f"bench: timed {steps} steps: {ms:.3f} ms/step")
    del src, dst
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    kernels = {}
    for name, t in trace.items():
        avg_ms = t["ms"] / t["launches"]
        bpl = t["bytes"] / t["launches"]
        kernels[name] = {"launches_per_step": t["launches"] // steps,
                         "ms_per_step": round(t["ms"] / steps, 4),
                         "avg_launch_ms": round(avg_ms, 5),
                         "GBps": round(bpl / (avg_ms / 1e3) / 1e9, 1)}
    # the dominant kernel: most time per step among entries that are one kernel
    dom = max((k for k in trace if not k.endswith("_count")), key=lambda k: trace[k]["ms"])
    t = trace[dom]
    avg_s = t["ms"] / t["launches"] / 1e3
    bytes_per_launch = t["bytes"] / t["launches"]
    achieved = bytes_per_launch / avg_s / 1e9
    workload = _workload_name(spec)
    traffic = read_traffic(dom, workload)
    bits, items, method = ringo.tune_get(n)
    # the library's byte model of one whole conversion (every kernel's
    # algorithmic bytes, summed), over the untraced step time
    alg_bytes = sum(t2["bytes"] for t2 in trace.values()) / steps
    conv_bytes = read_conversion_traffic(workload) if kind == ringo.GRAPH_DIRECTED else None
    io_min = 16 * n + 24 * V + 8 + 8 * E
    sec = ms_untraced / 1e3
    return {
        "value": n / (ms / 1e3), "ms_per_step": ms, "ms_per_step_untraced": ms_untraced,
        "ms_single_step_median": sorted(per)[len(per) // 2],
        "workload": workload, "rows": n, "nodes": V, "edges": E, "seed": spec.seed,
        "digit_bits": bits, "items_per_thread": items,
        "node_method": "hash" if method == ringo.NODES_HASH else "sort",
        "roofline": {"bound": "hbm", "kernel": dom,
                     "rocprof_kernel": " | ".join(rocprof_names(dom, items, bits)),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     # the counter-measured bytes over the same launch time (line-granular
                     # traffic of random accesses included: raw traffic, not useful bytes)
                     "traffic_GBps": round(traffic / avg_s / 1e9, 1) if traffic else None,
                     "traffic_frac": round(traffic / avg_s / 1e9 / HBM_PEAK_GBPS, 4) if traffic else None,
                     "traffic_over_algorithmic": round(traffic / bytes_per_launch, 2) if traffic else None,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": round(avg_s * 1e3, 5)},
        # every kernel's algorithmic bytes (the library's byte model) over the
        # untraced conversion time: the useful-bandwidth fraction of the
        # whole conversion
        "conversion_alg": {"bytes": alg_bytes, "GBps": round(alg_bytes / sec / 1e9, 1),
                           "frac": round(alg_bytes / sec / 1e9 / HBM_PEAK_GBPS, 4)},
        # every kernel's counter-measured HBM bytes (FETCH_SIZE + WRITE_SIZE,
        # scaled) over the same time: raw traffic, wasted lines of the random
        # probes and gathers included
        "conversion_traffic": ({"bytes": conv_bytes, "GBps": round(conv_bytes / sec / 1e9, 1),
                                "frac": round(conv_bytes / sec / 1e9 / HBM_PEAK_GBPS, 4),
                                "frac_of_copy": round(conv_bytes / sec / 1e9 / copy_gbps, 4)}
                               if conv_bytes else None),
        # reading the table once and writing the graph once: 16n + 24V + 8 + 8E bytes
        "io_minimum": {"bytes": io_min, "GBps": round(io_min / sec / 1e9, 1),
                       "frac": round(io_min / sec / 1e9 / HBM_PEAK_GBPS, 4)},
        "kernels": kernels,
    }


def batched_extra(steps):
    """The batched workload's speedup for the headline line (fewer repetitions
    than --config 4): median batched call, median of one call per table,
    tables whose outputs differ."""
    import torch
    from paper_1503_07881_amd import ringo, workloads
    dev = torch.device("cuda:0")
    specs = workloads.config4()
    total = sum(s.n for s in specs)
    src = torch.empty(total, dtype=torch.int64, device=dev)
    dst = torch.empty(total, dtype=torch.int64, device=dev)
    sh = torch.cuda.current_stream().cuda_stream
    offs, off = [], 0
    for s in specs:
        workloads.generate_device(s, src.data_ptr() + 8 * off, dst.data_ptr() + 8 * off, sh)
        offs.append((off, s.n))
        off += s.n
    torch.cuda.synchronize()
    sp = [src.data_ptr() + 8 * o for o, _ in offs]
    dp = [dst.data_ptr() + 8 * o for o, _ in offs]
    ns = [n for _, n in offs]

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gs = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            for g in gs:
                ringo.graph_free(g)
        return sorted(ts)[len(ts) // 2]

    def batched():
        return ringo.table_to_graph_batched_raw(sp, dp, ns, sh)

    def singles():
        return [ringo.table_to_graph_raw(a, b, c, sh) for a, b, c in zip(sp, dp, ns)]

    for g in batched():
        ringo.graph_free(g)
    t_b = timed(batched, max(3, min(steps, 7)))
    t_s = timed(singles, 3)
    gb = [ringo._wrap(r, dev) for r in batched()]
    differing = 0
    for i, (a, b, c) in enumerate(zip(sp, dp, ns)):
        g1 = ringo._wrap(ringo.table_to_graph_raw(a, b, c, sh), dev)
        for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs"):
            if not torch.equal(getattr(gb[i], f), getattr(g1, f)):
                differing += 1
                break
    del gb, src, dst
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"bench: batched {t_b * 1e3:.1f} ms, one call per table {t_s * 1e3:.1f} ms, differing {differing}")
    return {"workload": "batch_4096_tables_rows_1e3_to_2e6", "tables": len(specs), "rows": total,
            "speedup": t_s / t_b, "batched_ms": t_b * 1e3, "single_calls_ms": t_s * 1e3,
            "batched_edges_per_s": total / t_b, "single_calls_edges_per_s": total / t_s,
            "tables_differing": differing}


def cpu_oracle_full(spec):
    """The oracle (single-threaded, as it stands) over a whole table."""
    import oracle
    from paper_1503_07881_amd import workloads
    src, dst = workloads.generate_host(spec)
    t0 = time.perf_counter()
    oracle.table_to_graph(src, dst)
    dt = time.perf_counter() - t0
    return {"value": spec.n / dt, "unit": "edges/s", "cores": 1, "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"the whole {_workload_name(spec)} table ({spec.n:,} rows), single-threaded std::sort oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3, choices=(1, 2, 3, 4, 5),
                    help="3 (default): the 1.5e9-row R-MAT headline, with the 2^26-row workload and the "
                         "batched speedup as extra keys")
    ap.add_argument("--serve-pool", type=int, default=128)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-streams", type=int, default=3)
    ap.add_argument("--serve-batch-rows", type=int, default=8 << 20,
                    help="rows a batch may hold (a larger request runs alone)")
    ap.add_argument("--serve-small-budget-gib", type=int, default=32,
                    help="the second, binding budget of --config 5")
    ap.add_argument("--cpu-rows", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the 2^26-row and batched extra keys")
    ap.add_argument("--kind", default="directed", choices=("directed", "undirected", "multi"),
                    help="graph kind of the table-to-graph conversion")
    ap.add_argument("--node-method", default="auto", choices=("auto", "sort", "hash"),
                    help="node numbering: the schedule table's choice per size, or one method")
    ap.add_argument("--op", default="to_graph", choices=("to_graph", "to_table", "pagerank"),
                    help="to_graph: table-to-graph conversion (default); to_table: graph-to-table; "
                         "pagerank: ten PageRank iterations on the converted graph")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the conversion runs on a single MI355X).",
              file=sys.stderr)
        sys.exit(2)

    if args.node_method != "auto":
        from paper_1503_07881_amd import ringo
        ringo.set_node_method(ringo.NODES_HASH if args.node_method == "hash" else ringo.NODES_SORT)
    if args.op == "to_table":
        bench_to_table(args)
        return
    if args.op == "pagerank":
        bench_pagerank(args)
        return
    if args.config == 4:
        bench_batched(args)
        return
    if args.config == 5:
        bench_serve(args)
        return

    import torch
    from paper_1503_07881_amd import ringo, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sh = torch.cuda.current_stream().cuda_stream
    copy_gbps = copy_bandwidth(dev, sh)
    log(f"bench: copy kernel {copy_gbps:.0f} GB/s")
    kind = {"directed": ringo.GRAPH_DIRECTED, "undirected": ringo.GRAPH_UNDIRECTED,
            "multi": ringo.GRAPH_MULTI}[args.kind]
    spec = {1: workloads.config1, 2: workloads.config2, 3: workloads.config3}[args.config]()
    m = measure_conversion(spec, args, kind, copy_gbps, args.steps, args.warmup)
    out = {
        "metric": ("edges/s converted (input rows per second, table to directed simple graph, 1 GPU)"
                   if args.kind == "directed" else
                   f"edges/s converted (input rows per second, table to {args.kind} graph, 1 GPU)"),
        "value": m["value"], "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64",
        "data": ("synthetic (seeded R-MAT on the device, hashed 64-bit identifiers)" if spec.kind == "rmat"
                 else "synthetic (seeded uniform table, hashed 64-bit identifiers)"),
        "config": {"workload": m["workload"], "graph_kind": args.kind, "rows": m["rows"], "nodes": m["nodes"],
                   "edges": m["edges"], "seed": m["seed"], "digit_bits": m["digit_bits"],
                   "items_per_thread": m["items_per_thread"], "node_method": m["node_method"]},
        "roofline": m["roofline"],
        "ms_per_step_untraced": m["ms_per_step_untraced"],
        "ms_single_step_median": m["ms_single_step_median"],
        "conversion_alg": m["conversion_alg"],
        "conversion_traffic": m["conversion_traffic"],
        "io_minimum": m["io_minimum"],
        "copy_kernel_GBps": round(copy_gbps, 1),
        "kernels": m["kernels"],
    }
    if args.config == 3 and not args.no_extras and args.kind == "directed":
        # the LiveJournal-shaped 2^26-row workload and the batched speedup
        c2 = measure_conversion(workloads.config2(), args, kind, copy_gbps, args.steps, min(args.warmup, 2))
        out["config2"] = {k: c2[k] for k in ("workload", "value", "ms_per_step", "ms_per_step_untraced",
                                             "ms_single_step_median", "nodes", "edges", "conversion_alg",
                                             "conversion_traffic")}
        out["config2"]["roofline"] = {k: c2["roofline"][k] for k in ("kernel", "frac", "achieved", "traffic",
                                                                      "avg_launch_ms")}
        out["batched"] = batched_extra(args.steps)
        # the served form: p50/p99 at 0.8x one-at-a-time capacity (a shorter
        # trace than --config 5 runs), continuous batching against FIFO
        runs, mu = serve_runs(48, 400, 40, (0.8,), (200 << 30,), args.serve_streams, args.serve_batch_rows)
        r = runs["0.8mu_budget200GiB"]
        out["serve"] = {"workload": "serve_poisson_rows_1e4_to_5e7", "requests": 400, "pool_tables": 48,
                        "rate_per_s": r["rate_per_s"], "capacity_one_at_a_time_per_s": mu,
                        "p50_ms": r["continuous_batching"]["p50_ms"], "p99_ms": r["continuous_batching"]["p99_ms"],
                        "edges_per_s": r["continuous_batching"]["edges_per_s"],
                        "fifo_p50_ms": r["fifo_one_at_a_time"]["p50_ms"],
                        "fifo_p99_ms": r["fifo_one_at_a_time"]["p99_ms"],
                        "device_overlap_frac": r["continuous_batching"]["device"]["overlap_frac"]}
    if not args.no_cpu_baseline and args.config in (2, 3):
        log(f"bench: CPU oracle on the first {args.cpu_rows:,} rows")
        out["cpu_baseline"], out["cpu_baseline_all_cores"] = cpu_baseline(spec, args.cpu_rows)
        if args.config == 3 and not args.no_extras:
            log("bench: CPU oracle on the whole 2^26-row table")
            out["cpu_oracle_config2_whole_table"] = cpu_oracle_full(workloads.config2())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
