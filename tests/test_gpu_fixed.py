"""The sync-free single-table path (directed tables of 2049 to 2^20 rows
numbered by sorting): every kernel enqueued at once, V and E moved into the
plan on the device, outputs sized for the worst case.  Its graph must equal
the oracle's (Section 2.4's conversion, bit-exact) and the pass pipeline's,
element by element."""
import os
import sys

import numpy as np
import pytest

import oracle
from helpers import assert_same
from paper_1503_07881_amd import ringo, workloads

pytestmark = pytest.mark.gpu

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
FIXED_MAX_ROWS = 1 << 20
# trace entries of the sync-free path: its kernels enqueued, or its graph
# replayed (a size met before)
SYNC_FREE = {"plan_device", "fixed_graph_replay"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def convert(src, dst, dev, fixed=True):
    """Converts on the device; returns (host graph dict, trace names)."""
    import torch
    s = torch.from_numpy(np.ascontiguousarray(src, dtype=np.int64)).to(dev)
    d = torch.from_numpy(np.ascontiguousarray(dst, dtype=np.int64)).to(dev)
    if not fixed:
        os.environ["RINGO_FIXED_PATH"] = "0"
    try:
        ringo.trace_enable(True)
        g = ringo.to_graph(s, d)
        torch.cuda.synchronize()
        names = set(ringo.trace_read())
    finally:
        ringo.trace_enable(False)
        os.environ.pop("RINGO_FIXED_PATH", None)
    host = {f: getattr(g, f).cpu().numpy() for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets",
                                                     "in_nbrs")}
    return host, names


@pytest.fixture
def sort_numbering():
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    ringo.set_node_method(ringo.NODES_SORT)
    yield
    for e, (d, it, m) in enumerate(saved):
        ringo.tune_set(1 << e, d, it, m)


def random_table(seed, n, pool):
    rng = np.random.default_rng(seed)
    ids = rng.integers(I64_MIN, I64_MAX, size=pool, dtype=np.int64, endpoint=True)
    if pool > 2:
        ids[0], ids[1] = I64_MIN, I64_MAX
    return ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]


# the LDS path's limit, sort and scan tile edges (2048 keys per sort tile,
# 4096 per scan tile, 8192 rows per remap tile), and the path's own limit
SIZES = [2049, 2050, 3000, 4095, 4096, 4097, 8191, 8193, 16385, 65537, 100_003,
         FIXED_MAX_ROWS - 1, FIXED_MAX_ROWS]


@pytest.mark.parametrize("n", SIZES)
def test_sizes_vs_oracle_and_pipeline(cuda, sort_numbering, n):
    for pool in (1, 7, max(1, n // 3), 4 * n):
        say("sync-free path n", n, "pool", pool)
        src, dst = random_table(n * 17 + pool, n, pool)
        got, names = convert(src, dst, cuda)
        assert names & SYNC_FREE, sorted(names)
        assert_same(got, oracle.table_to_graph(src, dst), f"n={n} pool={pool}: ")
        if pool in (7, 4 * n):
            pipe, pnames = convert(src, dst, cuda, fixed=False)
            assert not pnames & SYNC_FREE
            assert_same(got, pipe, f"n={n} pool={pool} against the pipeline: ")


def test_structures(cuda, sort_numbering):
    """Shapes that stress the device-side sizes: V = 2n (every identifier
    distinct, so b = ceil(log2 2n) exactly), one node, stars with the hub at
    either end of the signed range, sequential and clustered identifiers,
    V at powers of two."""
    n = 300_000
    ids = np.array([workloads.mix64(i) - (1 << 63) for i in range(2 * n)], dtype=np.int64)
    cases = {
        "all_distinct": (ids[:n], ids[n:]),
        "all_distinct_max": (np.arange(0, FIXED_MAX_ROWS, dtype=np.int64),
                             np.arange(FIXED_MAX_ROWS, 2 * FIXED_MAX_ROWS, dtype=np.int64)),
        "one_node": (np.full(n, 42, dtype=np.int64), np.full(n, 42, dtype=np.int64)),
        "star_out_hub_min": (np.full(n, I64_MIN, dtype=np.int64), np.arange(n, dtype=np.int64)),
        "star_in_hub_max": (np.arange(n, dtype=np.int64), np.full(n, I64_MAX, dtype=np.int64)),
        "sequential": (np.arange(n, dtype=np.int64), np.arange(1, n + 1, dtype=np.int64)),
        "clustered": (np.concatenate([np.arange(n // 2), I64_MAX - np.arange(n // 2)]).astype(np.int64),
                      np.concatenate([I64_MAX - np.arange(n // 2), np.arange(n // 2)]).astype(np.int64)),
    }
    for V in (4096, 4097, 65536, 65537):
        vids = ids[:V]
        cases[f"cycle_V{V}"] = (vids, np.roll(vids, -1))
    for name, (src, dst) in cases.items():
        say("sync-free structure", name, "rows", src.size)
        got, names = convert(src, dst, cuda)
        assert names & SYNC_FREE, (name, sorted(names))
        assert_same(got, oracle.table_to_graph(src, dst), name + ": ")


@pytest.mark.parametrize("bits,items", [(9, 8), (10, 12), (11, 16), (8, 16)])
def test_schedules(cuda, sort_numbering, bits, items):
    """The path under other digit widths and tile shapes of the schedule."""
    n = 200_001
    saved = ringo.tune_get(n)
    try:
        ringo.tune_set(n, bits, items, ringo.NODES_SORT)
        for pool in (5, 3 * n):
            say("sync-free schedule", bits, items, "pool", pool)
            src, dst = random_table(bits * 100 + items + pool, n, pool)
            got, names = convert(src, dst, cuda)
            assert names & SYNC_FREE
            assert_same(got, oracle.table_to_graph(src, dst), f"d={bits} items={items} pool={pool}: ")
    finally:
        ringo.tune_set(n, *saved)


def test_config1_and_repeat(cuda, sort_numbering):
    """The 10^6-row uniform workload through the path, twice in a row (the
    second call reuses pooled memory) and after a larger and a smaller call."""
    spec = workloads.config1()
    src, dst = workloads.generate_host(spec)
    want = oracle.table_to_graph(src, dst)
    big = random_table(5, FIXED_MAX_ROWS, 3 * FIXED_MAX_ROWS)
    small = random_table(6, 5000, 900)
    for label, (s, d) in (("config1", (src, dst)), ("big", big), ("config1 again", (src, dst)),
                          ("small", small), ("config1 last", (src, dst))):
        say("sync-free sequence", label)
        got, names = convert(s, d, cuda)
        assert names & SYNC_FREE
        if s is src:
            assert_same(got, want, label + ": ")
        else:
            assert_same(got, oracle.table_to_graph(s, d), label + ": ")


def test_outside_the_range_uses_the_pipeline(cuda, sort_numbering):
    for n in (2048, FIXED_MAX_ROWS + 1):
        src, dst = random_table(n, n, n)
        got, names = convert(src, dst, cuda)
        assert not names & SYNC_FREE, (n, sorted(names))
        assert_same(got, oracle.table_to_graph(src, dst), f"n={n}: ")


def _convert_on(src_t, dst_t, stream=None):
    import torch
    ringo.trace_enable(True)
    try:
        g = ringo.to_graph(src_t, dst_t, stream=stream)
        torch.cuda.synchronize()
        names = set(ringo.trace_read())
    finally:
        ringo.trace_enable(False)
    return {f: getattr(g, f).cpu().numpy() for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets",
                                                     "in_nbrs")}, names


def test_graph_replay_matches_eager(cuda, sort_numbering):
    """A size met a second time is captured into a HIP graph and replayed.
    Every replay, with other conversions, torch work and synchronisations in
    between, on the default and on a side stream, equals the eager path
    (replay off) and the oracle."""
    import torch
    hs1, hd1 = random_table(71, 300_001, 90_000)
    hs2, hd2 = random_table(72, 50_000, 120_000)
    s1, d1 = torch.from_numpy(hs1).to(cuda), torch.from_numpy(hd1).to(cuda)
    s2, d2 = torch.from_numpy(hs2).to(cuda), torch.from_numpy(hd2).to(cuda)
    os.environ["RINGO_FIXED_GRAPH"] = "0"
    try:
        ref1, n1 = _convert_on(s1, d1)
        ref2, _ = _convert_on(s2, d2)
    finally:
        os.environ.pop("RINGO_FIXED_GRAPH", None)
    assert "plan_device" in n1 and "fixed_graph_replay" not in n1
    assert_same(ref1, oracle.table_to_graph(hs1, hd1), "eager: ")
    side = torch.cuda.Stream(device=cuda)
    replays = 0
    for i in range(6):
        say("graph replay round", i)
        got, names = _convert_on(s1, d1, stream=side if i % 2 else None)
        replays += "fixed_graph_replay" in names
        if i >= 1:
            assert "fixed_graph_replay" in names and "plan_device" not in names, (i, sorted(names))
        assert_same(got, ref1, f"round {i}: ")
        # other work in between: another size, torch kernels, the pipeline
        got2, _ = _convert_on(s2, d2)
        assert_same(got2, ref2, f"round {i}, second table: ")
        x = torch.arange(1 << 20, device=cuda, dtype=torch.int64)
        assert int((x * 3).sum()) == 3 * ((1 << 20) - 1) * (1 << 20) // 2
        os.environ["RINGO_FIXED_PATH"] = "0"
        try:
            got3, _ = _convert_on(s2, d2)
        finally:
            os.environ.pop("RINGO_FIXED_PATH", None)
        assert_same(got3, ref2, f"round {i}, pipeline: ")
    assert replays >= 5


def test_graph_cache_eviction(cuda, sort_numbering):
    """More sizes than graphs kept: sizes come back after their graphs were
    evicted; every result equals the oracle's."""
    import torch
    tables = [random_table(300 + k, 3000 + 997 * k, 2000 + 50 * k) for k in range(11)]
    want = [oracle.table_to_graph(s, d) for s, d in tables]
    dev_tabs = [(torch.from_numpy(s).to(cuda), torch.from_numpy(d).to(cuda)) for s, d in tables]
    for r in range(3):
        for k, (s, d) in enumerate(dev_tabs):
            got, names = _convert_on(s, d)
            assert names & SYNC_FREE
            assert_same(got, want[k], f"round {r} table {k}: ")
