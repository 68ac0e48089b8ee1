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
        assert "plan_device" in names, sorted(names)
        assert_same(got, oracle.table_to_graph(src, dst), f"n={n} pool={pool}: ")
        if pool in (7, 4 * n):
            pipe, pnames = convert(src, dst, cuda, fixed=False)
            assert "plan_device" not in pnames
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
        assert "plan_device" in names, (name, sorted(names))
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
            assert "plan_device" in names
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
        assert "plan_device" in names
        if s is src:
            assert_same(got, want, label + ": ")
        else:
            assert_same(got, oracle.table_to_graph(s, d), label + ": ")


def test_outside_the_range_uses_the_pipeline(cuda, sort_numbering):
    for n in (2048, FIXED_MAX_ROWS + 1):
        src, dst = random_table(n, n, n)
        got, names = convert(src, dst, cuda)
        assert "plan_device" not in names, (n, sorted(names))
        assert_same(got, oracle.table_to_graph(src, dst), f"n={n}: ")
