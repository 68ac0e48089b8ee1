"""Parity of the HIP path with the CPU oracle, element by element, through
the C ABI (bit-exact: the conversion is integer work)."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from helpers import assert_same, check_invariants, check_invariants_torch, check_sampled
from paper_1503_07881_amd import ringo, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_graph(src, dst, dev):
    import torch
    s = torch.from_numpy(np.ascontiguousarray(src, dtype=np.int64)).to(dev)
    d = torch.from_numpy(np.ascontiguousarray(dst, dtype=np.int64)).to(dev)
    g = ringo.to_graph(s, d)
    torch.cuda.synchronize()
    return g


def test_hand_examples(cuda, method, small_path):
    for ex in json.load(open(GOLDEN))["examples"]:
        say("hand example", ex["name"], method, small_path)
        src = np.array(ex["src"], dtype=np.int64)
        dst = np.array(ex["dst"], dtype=np.int64)
        g = gpu_graph(src, dst, cuda)
        assert_same(g, oracle.table_to_graph(src, dst), ex["name"] + ": ")


def random_table(seed, n, pool):
    rng = np.random.default_rng(seed)
    ids = rng.integers(I64_MIN, I64_MAX, size=pool, dtype=np.int64, endpoint=True)
    if pool > 2:
        ids[0], ids[1] = I64_MIN, I64_MAX
    return ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]


# sizes around the tile edges of the kernels (2n node keys per tile of 4096,
# n edge keys per tile of 4096, remap tiles of 8192 rows, histogram chunks)
EDGE_SIZES = [1, 2, 3, 63, 64, 65, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 16385, 40000, 131072 + 7]


@pytest.mark.parametrize("n", EDGE_SIZES)
def test_tile_boundaries(cuda, method, small_path, n):
    for pool in (1, 7, max(1, n // 3), 4 * n):
        say("tile boundary case n", n, "pool", pool, method, small_path)
        src, dst = random_table(n * 31 + pool, n, pool)
        assert_same(gpu_graph(src, dst, cuda), oracle.table_to_graph(src, dst), f"n={n} pool={pool}: ")


@pytest.mark.parametrize("n", [(1 << 22) - 1, 1 << 22, (1 << 22) + 1])
def test_scan_paths_boundary(cuda, n):
    """Sort numbering of 2n node keys at 4096 tiles of 2048: the node passes
    sit on both sides of the switch between the one-kernel scan of small
    passes and the run scan plus tile prefixes."""
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    try:
        ringo.set_node_method(ringo.NODES_SORT)
        say("scan boundary conversion n", n)
        src, dst = random_table(n + 11, n, 1 << 20)
        assert_same(gpu_graph(src, dst, cuda), oracle.table_to_graph(src, dst), f"n={n}: ")
    finally:
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)


def test_hash_bucket_paths(cuda):
    """Hash numbering of one table: identifiers spread over the 64-bit range
    have their distinct keys sorted bucket by bucket in LDS; identifiers
    crowded into one bucket of the top key bits (more than 2048 of them) take
    the radix passes instead.  Both are the oracle's graph."""
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    try:
        ringo.set_node_method(ringo.NODES_HASH)
        # fewer distinct identifiers than half the rows, so the table is built
        spread = random_table(91, 400_000, 100_000)
        crowded = (np.tile(np.arange(0, 60_000, dtype=np.int64), 4),
                   np.tile(np.arange(7, 60_007, dtype=np.int64), 4))
        for name, (src, dst), want, not_want in (
                ("spread", spread, "hash_bucket_sort", "sort_vnode_count"),
                ("crowded", crowded, "sort_vnode_count", "hash_bucket_sort")):
            say("hash bucket path", name)
            ringo.trace_enable(True)
            g = gpu_graph(src, dst, cuda)
            names = set(ringo.trace_read())
            ringo.trace_enable(False)
            assert want in names and not_want not in names, (name, sorted(names))
            assert_same(g, oracle.table_to_graph(src, dst), name + ": ")
    finally:
        ringo.trace_enable(False)
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)


def test_hash_numbering_steps_aside_for_distinct_ids(cuda):
    """Under hash numbering, a table whose estimated distinct identifiers
    exceed half its rows is numbered by sorting (no table is built); one with
    fewer builds the table.  Both give the oracle's graph."""
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    try:
        ringo.set_node_method(ringo.NODES_HASH)
        n = 300_000
        for pool, built in ((n // 8, True), (n // 3, True), (2 * n, False), (8 * n, False)):
            src, dst = random_table(pool, n, pool)
            ringo.trace_enable(True)
            g = gpu_graph(src, dst, cuda)
            names = set(ringo.trace_read())
            ringo.trace_enable(False)
            say("hash or sort by distinct count: pool", pool, "V", g.num_nodes, sorted(names))
            assert ("hash_insert" in names) == built, (pool, g.num_nodes, sorted(names))
            assert "hash_estimate" in names
            assert_same(g, oracle.table_to_graph(src, dst), f"pool {pool}: ")
    finally:
        ringo.trace_enable(False)
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)


@pytest.mark.parametrize("seed", range(8))
def test_random_small(cuda, method, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(0, 300_000))
    pool = int(rng.integers(1, max(2, 2 * n)))
    say("random case seed", seed, "n", n, "pool", pool, method)
    src, dst = random_table(seed, n, pool)
    assert_same(gpu_graph(src, dst, cuda), oracle.table_to_graph(src, dst))


def test_special_structures(cuda, method, small_path):
    k = 61
    ids = np.array([workloads.mix64(i) - (1 << 63) for i in range(k)], dtype=np.int64)
    a, b = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    cases = {
        "complete_digraph": (ids[a.ravel()], ids[b.ravel()]),
        "star_hub_first": (np.full(5000, I64_MIN, dtype=np.int64), np.arange(5000, dtype=np.int64)),
        "star_hub_last": (np.full(5000, I64_MAX, dtype=np.int64), np.arange(5000, dtype=np.int64)),
        "self_loops": (np.arange(-3000, 3000, dtype=np.int64), np.arange(-3000, 3000, dtype=np.int64)),
        "one_node": (np.full(10000, 42, dtype=np.int64), np.full(10000, 42, dtype=np.int64)),
        "sequential_ids": (np.arange(0, 100000, dtype=np.int64), np.arange(1, 100001, dtype=np.int64)),
        "clustered_ids": (np.concatenate([np.arange(50), I64_MAX - np.arange(50)]).astype(np.int64),
                          np.concatenate([I64_MAX - np.arange(50), np.arange(50)]).astype(np.int64)),
    }
    for V in (2, 3, 4, 5, 255, 256, 257, 65536, 65537):
        vids = ids[:min(V, k)] if V <= k else np.array([workloads.mix64(i) - (1 << 63) for i in range(V)],
                                                         dtype=np.int64)
        cases[f"path_V{V}"] = (vids, np.roll(vids, -1))
    for name, (src, dst) in cases.items():
        say("special case", name, method, small_path)
        assert_same(gpu_graph(src, dst, cuda), oracle.table_to_graph(src, dst), name + ": ")


@pytest.mark.parametrize("n", [1 << 20, 1 << 22])
@pytest.mark.parametrize("hub", ["min", "max"])
def test_star_long_offset_runs(cuda, method, n, hub):
    """Out- and in-stars whose hub sits at either end of the signed range:
    the out- or in-offsets of every leaf form one run of about n equal
    entries, and (sort numbering) the directory has a run of about 2^b empty
    buckets; such runs are queued and written by a grid-wide fill.  2^20
    rows take the sync-free path under sort numbering, 2^22 the pipeline."""
    h = I64_MIN if hub == "min" else I64_MAX
    leaves = np.arange(n, dtype=np.int64)
    for direction in ("out", "in"):
        src, dst = (np.full(n, h, np.int64), leaves) if direction == "out" else (leaves, np.full(n, h, np.int64))
        say("star", direction, "hub", hub, "rows", n, method)
        assert_same(gpu_graph(src, dst, cuda), oracle.table_to_graph(src, dst, all_cores=True),
                    f"{direction}-star hub {hub} n={n}: ")


def test_config1_full(cuda, method):
    say("config 1: 1,000,000 rows", method)
    src, dst = workloads.generate_host(workloads.config1())
    g = gpu_graph(src, dst, cuda)
    assert g.num_nodes == 100_000
    assert_same(g, oracle.table_to_graph(src, dst))


def test_determinism(cuda, method):
    say("determinism: two runs of an R-MAT table", method)
    src, dst = workloads.generate_host(workloads.TableSpec("rmat", 3_000_000, seed=21, scale=18))
    g1 = gpu_graph(src, dst, cuda)
    g2 = gpu_graph(src, dst, cuda)
    assert_same(g1, g2)


def test_rmat_medium_vs_oracle(cuda, method):
    say("R-MAT scale 20, 4M rows vs oracle", method)
    spec = workloads.TableSpec("rmat", 1 << 22, seed=22, scale=20)
    src, dst = workloads.generate_host(spec)
    g = gpu_graph(src, dst, cuda)
    assert_same(g, oracle.table_to_graph(src, dst))


def test_batched_equals_singles_and_oracle(cuda, method):
    import torch
    specs = [workloads.mixed_table(77, i, 1, 300_000) for i in range(40)]
    specs += [workloads.TableSpec("uniform", 0, seed=1), workloads.TableSpec("uniform", 1, seed=2, pool=1)]
    tables = [workloads.generate_host(s) for s in specs]
    say("batched: tables", len(tables), "rows", sum(s.n for s in specs), method)
    ts = [(torch.from_numpy(s).to(cuda), torch.from_numpy(d).to(cuda)) for s, d in tables]
    gb = ringo.to_graph_batched([s for s, _ in ts], [d for _, d in ts])
    torch.cuda.synchronize()
    for i, ((s, d), (hs, hd)) in enumerate(zip(ts, tables)):
        g1 = ringo.to_graph(s, d)
        torch.cuda.synchronize()
        assert_same(gb[i], g1, f"table {i} batched vs single: ")
        assert_same(gb[i], oracle.table_to_graph(hs, hd), f"table {i} vs oracle: ")


def test_small_tables_batched(cuda, method):
    """Batches of small tables only (one workgroup each, one synchronisation)
    and small tables among large ones, against the oracle."""
    import torch
    rng = np.random.default_rng(404)
    sizes = [1, 2, 3, 64, 1000, 2047, 2048, 1500, 17, 999]
    tables = [random_table(int(rng.integers(1 << 30)), n, max(1, n // 4)) for n in sizes]
    big = [random_table(5, 9000, 700), random_table(6, 2049, 100)]
    for label, tabs in (("small only", tables), ("mixed", tables + big)):
        say("small tables batched:", label, method)
        ts = [(torch.from_numpy(s).to(cuda), torch.from_numpy(d).to(cuda)) for s, d in tabs]
        gb = ringo.to_graph_batched([s for s, _ in ts], [d for _, d in ts])
        torch.cuda.synchronize()
        for i, (hs, hd) in enumerate(tabs):
            assert_same(gb[i], oracle.table_to_graph(hs, hd), f"{label} table {i}: ")


@pytest.mark.parametrize("parts", ["0", "1"])
@pytest.mark.parametrize("cap", [1, 64, 4096])
def test_hash_overflow_falls_back_to_sort(cuda, cap, parts):
    """Node hash tables capped far below V (forced from the host): every probe
    sequence stops at its bound, the call numbers the nodes by sorting, and
    the graph is still the oracle's.  Tables that fit keep the hash path.
    parts: inserts in row order, or of keys grouped by table part."""
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    try:
        os.environ["RINGO_HASH_TEST_CAPACITY"] = str(cap)
        os.environ["RINGO_HASH_PARTS"] = parts
        ringo.set_node_method(ringo.NODES_HASH)
        for n, pool in ((5, 3), (1000, 40), (20000, 5000), (200_000, 150_000)):
            say("hash capacity", cap, "n", n, "pool", pool)
            src, dst = random_table(n + cap, n, pool)
            assert_same(gpu_graph(src, dst, cuda), oracle.table_to_graph(src, dst), f"cap={cap} n={n}: ")
    finally:
        del os.environ["RINGO_HASH_TEST_CAPACITY"]
        os.environ.pop("RINGO_HASH_PARTS", None)
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)


@pytest.mark.slow
def test_too_many_nodes_limit(cuda, method, small_path, monkeypatch):
    """The node-count limit (RINGO_MAX_NODES, int32 neighbours) lowered
    through the RINGO_TEST_MAX_NODES hook: a table over it fails with
    TOO_MANY_NODES (alone and in a batch, all-or-nothing, outputs zeroed), a
    table at it converts, and the library works on afterwards."""
    import ctypes
    import torch
    rng = np.random.default_rng(77)
    for rows in (300, 9000):  # LDS-sized and pipeline-sized tables
        src = rng.integers(0, 1 << 40, rows, dtype=np.int64)
        dst = rng.integers(0, 1 << 40, rows, dtype=np.int64)
        V = np.unique(np.concatenate([src, dst])).size
        s, d = (torch.from_numpy(a).to(cuda) for a in (src, dst))
        say("node limit", rows, "rows", V, "nodes", method, small_path)
        monkeypatch.setenv("RINGO_TEST_MAX_NODES", str(V - 1))
        with pytest.raises(ringo.RingoError) as err:
            ringo.to_graph(s, d)
        assert err.value.status == 2
        # a batch with one table over the limit: every output zeroed
        ok_s, ok_d = s[:5].contiguous(), d[:5].contiguous()
        P = (ctypes.c_void_p * 2)(ok_s.data_ptr(), s.data_ptr())
        Q = (ctypes.c_void_p * 2)(ok_d.data_ptr(), d.data_ptr())
        N = (ctypes.c_int64 * 2)(5, rows)
        outs = (ringo.RawGraph * 2)()
        rc = ringo.lib().ringo_table_to_graph_batched(2, P, Q, N, outs, torch.cuda.current_stream().cuda_stream)
        assert rc == 2
        assert all(o.num_nodes == 0 and o.node_ids is None and o.out_nbrs is None for o in outs)
        monkeypatch.setenv("RINGO_TEST_MAX_NODES", str(V))
        g = ringo.to_graph(s, d)
        torch.cuda.synchronize()
        assert g.num_nodes == V
        monkeypatch.delenv("RINGO_TEST_MAX_NODES")
        assert_same(gpu_graph(src, dst, cuda), oracle.table_to_graph(src, dst), "after the limit: ")


def test_config2_full_size(cuda):
    """The 2^26-row R-MAT workload at full size, in the configuration the
    benchmark times: complete invariants (torch on the device) and the exact
    lists of sampled nodes from the definition."""
    import torch
    say("config 2: 2^26 rows, device generation")
    spec = workloads.config2()
    src = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    dst = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), torch.cuda.current_stream().cuda_stream)
    # spot-check the device generator against the host generator
    hs, hd = workloads.generate_host(workloads.TableSpec("rmat", 100_000, seed=spec.seed, scale=spec.scale))
    assert np.array_equal(src[:100_000].cpu().numpy(), hs) and np.array_equal(dst[:100_000].cpu().numpy(), hd)
    g = ringo.to_graph(src, dst)
    torch.cuda.synchronize()
    say("config 2: V", g.num_nodes, "E", g.num_edges, "method", ringo.tune_get(spec.n)[2])
    check_invariants_torch(g, src, dst)
    check_sampled(g, src, dst, num_samples=200)
    # the other node-numbering method gives the same bytes
    d, it, m = ringo.tune_get(spec.n)
    try:
        ringo.tune_set(spec.n, d, it, 1 - m)
        g2 = ringo.to_graph(src, dst)
        torch.cuda.synchronize()
    finally:
        ringo.tune_set(spec.n, d, it, m)
    say("config 2: method", 1 - m, "V", g2.num_nodes, "E", g2.num_edges)
    assert _same_on_device(g, g2) is None


def _device_tables(specs, dev):
    """Generate every table of `specs` on the device, back to back in two
    buffers; returns the buffers and per-table (offset, rows)."""
    import torch
    total = sum(s.n for s in specs)
    src = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    dst = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    sh = torch.cuda.current_stream().cuda_stream
    offs = []
    off = 0
    for s in specs:
        if s.n:
            workloads.generate_device(s, src.data_ptr() + 8 * off, dst.data_ptr() + 8 * off, sh)
        offs.append((off, s.n))
        off += s.n
    torch.cuda.synchronize()
    return src, dst, offs


def _same_on_device(g1, g2):
    import torch
    for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs"):
        a, b = getattr(g1, f), getattr(g2, f)
        if a.shape != b.shape or not torch.equal(a, b):
            return f
    return None


@pytest.mark.slow
def test_config4_batched_full(cuda):
    """All 4096 tables of the batched workload: the batched call equals one
    call per table bit for bit, and every table equals the oracle's graph
    (the oracle runs on a pool of host threads; its C calls release the
    interpreter lock)."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    specs = workloads.config4()
    say("config 4: 4096 tables, rows", sum(s.n for s in specs))
    src, dst, offs = _device_tables(specs, cuda)
    sh = torch.cuda.current_stream().cuda_stream
    raws = ringo.table_to_graph_batched_raw([src.data_ptr() + 8 * o for o, _ in offs],
                                            [dst.data_ptr() + 8 * o for o, _ in offs],
                                            [n for _, n in offs], sh)
    gb = [ringo._wrap(r, cuda) for r in raws]
    torch.cuda.synchronize()
    for i, (o, n) in enumerate(offs):
        g1 = ringo._wrap(ringo.table_to_graph_raw(src.data_ptr() + 8 * o, dst.data_ptr() + 8 * o, n, sh), cuda)
        bad = _same_on_device(gb[i], g1)
        assert bad is None, f"table {i} ({specs[i]}): batched {bad} differs from the single call"
        assert gb[i].num_nodes == g1.num_nodes and gb[i].num_edges == g1.num_edges
    say("config 4: batched equals single calls; every table against the oracle")
    hsrc, hdst = src.cpu().numpy(), dst.cpu().numpy()
    del src, dst

    def check(i, got):
        o, n = offs[i]
        assert_same(got, oracle.table_to_graph(hsrc[o:o + n], hdst[o:o + n]), f"config 4 table {i}: ")
        return n

    done = 0
    with ThreadPoolExecutor(max_workers=16) as ex:
        futs = []
        for i in range(len(specs)):
            got = {f: getattr(gb[i], f).cpu().numpy() for f in ("node_ids", "out_offsets", "out_nbrs",
                                                                  "in_offsets", "in_nbrs")}
            gb[i] = None
            futs.append(ex.submit(check, i, got))
            if len(futs) >= 64:
                done += futs.pop(0).result()
        for f in futs:
            done += f.result()
    assert done == sum(s.n for s in specs)
    say("config 4: all", len(specs), "tables equal the oracle")


@pytest.mark.slow
def test_config3_full_size(cuda):
    """The 1.5e9-row R-MAT scale-26 workload at full size: complete
    invariants with torch on the device and exact lists of sampled nodes."""
    import torch
    spec = workloads.config3()
    say("config 3: 1.5e9 rows, device generation")
    src = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    dst = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), torch.cuda.current_stream().cuda_stream)
    hs, hd = workloads.generate_host(workloads.TableSpec("rmat", 50_000, seed=spec.seed, scale=spec.scale))
    assert np.array_equal(src[:50_000].cpu().numpy(), hs) and np.array_equal(dst[:50_000].cpu().numpy(), hd)
    g = ringo.to_graph(src, dst)
    torch.cuda.synchronize()
    say("config 3: V", g.num_nodes, "E", g.num_edges)
    check_sampled(g, src, dst, num_samples=64)
    say("config 3: sampled lists match; invariants")
    check_invariants_torch(g, src, dst)
