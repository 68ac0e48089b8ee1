"""ringo_table_to_graph_noalloc (the entry point for callers that cannot
allocate): its graph equals ringo_table_to_graph's, element by element, on
consecutive calls that share the library's one device workspace, the second
with a smaller table; its limits and argument checks."""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
from helpers import assert_same
from paper_1503_07881_amd import ringo

pytestmark = pytest.mark.gpu

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
SENTINEL = -12345


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def table(seed, n, pool, dev):
    import torch
    rng = np.random.default_rng(seed)
    ids = rng.integers(I64_MIN, I64_MAX, size=pool, dtype=np.int64, endpoint=True)
    s = ids[rng.integers(0, pool, n)]
    d = ids[rng.integers(0, pool, n)]
    return s, d, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev)


class Outputs:
    """Worst-case output arrays (filled with a sentinel) for n rows."""

    def __init__(self, n, dev):
        import torch
        self.n = n
        self.node_ids = torch.full((2 * n,), SENTINEL, dtype=torch.int64, device=dev)
        self.out_off = torch.full((2 * n + 1,), SENTINEL, dtype=torch.int64, device=dev)
        self.out_nbr = torch.full((n,), SENTINEL, dtype=torch.int32, device=dev)
        self.in_off = torch.full((2 * n + 1,), SENTINEL, dtype=torch.int64, device=dev)
        self.in_nbr = torch.full((n,), SENTINEL, dtype=torch.int32, device=dev)
        self.counts = torch.full((2,), SENTINEL, dtype=torch.int64, device=dev)

    def call(self, src, dst, stream):
        ringo.table_to_graph_noalloc_raw(src.data_ptr(), dst.data_ptr(), self.n, self.node_ids.data_ptr(),
                                         self.out_off.data_ptr(), self.out_nbr.data_ptr(), self.in_off.data_ptr(),
                                         self.in_nbr.data_ptr(), self.counts.data_ptr(), stream)

    def graph(self):
        """The graph part of the arrays; the rest must still hold the sentinel."""
        V, E = (int(x) for x in self.counts.cpu().tolist())
        arrs = {"node_ids": (self.node_ids, V), "out_offsets": (self.out_off, V + 1), "out_nbrs": (self.out_nbr, E),
                "in_offsets": (self.in_off, V + 1), "in_nbrs": (self.in_nbr, E)}
        out = {}
        for f, (t, k) in arrs.items():
            h = t.cpu().numpy()
            assert np.all(h[k:] == SENTINEL), f"{f}: written past its {k} entries"
            out[f] = h[:k]
        return out


def entry_point_graph(src_t, dst_t, pipeline):
    import torch
    if pipeline:
        os.environ["RINGO_FIXED_PATH"] = "0"
    try:
        g = ringo.to_graph(src_t, dst_t)
        torch.cuda.synchronize()
    finally:
        os.environ.pop("RINGO_FIXED_PATH", None)
    return {f: getattr(g, f).cpu().numpy() for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets",
                                                     "in_nbrs")}


def test_two_calls_second_smaller(cuda):
    """Two calls in a row on one stream, the second with a smaller table
    (nothing synchronised between them), each equal to the existing entry
    point's graph (default routing and the pass pipeline) and the oracle's."""
    import torch
    sh = torch.cuda.current_stream().cuda_stream
    cases = [table(1, 700_001, 200_000, cuda), table(2, 3_000, 700, cuda)]
    outs = [Outputs(c[2].numel(), cuda) for c in cases]
    say("no-alloc: two calls, 700001 then 3000 rows")
    for (_, _, s, d), o in zip(cases, outs):
        o.call(s, d, sh)
    torch.cuda.synchronize()
    for (hs, hd, s, d), o in zip(cases, outs):
        got = o.graph()
        assert_same(got, entry_point_graph(s, d, pipeline=False), f"n={o.n} against ringo_table_to_graph: ")
        assert_same(got, entry_point_graph(s, d, pipeline=True), f"n={o.n} against the pass pipeline: ")
        assert_same(got, oracle.table_to_graph(hs, hd), f"n={o.n} against the oracle: ")


def test_repeated_calls_reuse_the_workspace(cuda):
    """Larger, smaller, larger again, and a repeat: every result is exact
    although each call finds the previous call's contents in the workspace."""
    import torch
    sh = torch.cuda.current_stream().cuda_stream
    for seed, n, pool in ((3, 1 << 20, 3 << 20), (4, 2049, 5), (5, 250_000, 30), (5, 250_000, 30), (6, 70_000, 1)):
        hs, hd, s, d = table(seed, n, pool, cuda)
        say("no-alloc call n", n, "pool", pool)
        o = Outputs(n, cuda)
        o.call(s, d, sh)
        torch.cuda.synchronize()
        assert_same(o.graph(), entry_point_graph(s, d, pipeline=True), f"n={n} pool={pool}: ")


def test_small_and_empty_tables(cuda):
    """Tables the existing entry point converts in LDS (at most 2048 rows),
    and the empty table."""
    import torch
    sh = torch.cuda.current_stream().cuda_stream
    for n in (1, 2, 63, 2048):
        hs, hd, s, d = table(100 + n, n, max(1, n // 2), cuda)
        o = Outputs(n, cuda)
        o.call(s, d, sh)
        torch.cuda.synchronize()
        assert_same(o.graph(), entry_point_graph(s, d, pipeline=False), f"n={n}: ")
    o = Outputs(0, cuda)
    ringo.table_to_graph_noalloc_raw(0, 0, 0, 0, o.out_off.data_ptr(), 0, o.in_off.data_ptr(), 0,
                                     o.counts.data_ptr(), sh)
    torch.cuda.synchronize()
    assert o.counts.cpu().tolist() == [0, 0]
    assert o.out_off.cpu().tolist() == [0] and o.in_off.cpu().tolist() == [0]


def test_argument_checks(cuda):
    """Rejected on the host, before anything is enqueued."""
    import torch
    sh = torch.cuda.current_stream().cuda_stream
    L = ringo.lib()
    o = Outputs(4, cuda)
    s = torch.zeros(4, dtype=torch.int64, device=cuda)
    p = [o.node_ids.data_ptr(), o.out_off.data_ptr(), o.out_nbr.data_ptr(), o.in_off.data_ptr(),
         o.in_nbr.data_ptr(), o.counts.data_ptr()]
    assert L.ringo_table_to_graph_noalloc(s.data_ptr(), s.data_ptr(), ringo.NOALLOC_MAX_ROWS + 1, *p, sh) == 1
    assert L.ringo_table_to_graph_noalloc(s.data_ptr(), s.data_ptr(), -1, *p, sh) == 1
    assert L.ringo_table_to_graph_noalloc(None, s.data_ptr(), 4, *p, sh) == 1
    for k in range(6):
        q = list(p)
        q[k] = None
        assert L.ringo_table_to_graph_noalloc(s.data_ptr(), s.data_ptr(), 4, *q, sh) == 1, k
    torch.cuda.synchronize()
    assert o.counts.cpu().tolist() == [SENTINEL, SENTINEL], "nothing enqueued by a rejected call"


def test_captured_in_a_caller_graph(cuda):
    """Captured into the caller's graph (what a caller that cannot allocate
    usually does) and replayed three times, with eager conversions between the
    replays that leave other contents in the shared workspace: every replay
    equals the eager call's graph, which equals the oracle's."""
    import torch
    hs, hd, s, d = table(7, 300_001, 90_000, cuda)
    n = s.numel()
    eager = Outputs(n, cuda)
    # the first eager call also resolves the workspace's address, outside any capture
    eager.call(s, d, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    want = eager.graph()
    assert_same(want, oracle.table_to_graph(hs, hd), "eager call against the oracle: ")

    o = Outputs(n, cuda)
    g = torch.cuda.CUDAGraph()
    say("no-alloc: capture, n", n)
    with torch.cuda.graph(g):
        o.call(s, d, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    other = [table(20 + k, 5_000 + 777 * k, 1_000, cuda) for k in range(3)]
    for k, (_, _, s2, d2) in enumerate(other):
        for t in (o.node_ids, o.out_off, o.out_nbr, o.in_off, o.in_nbr, o.counts):
            t.fill_(SENTINEL)
        between = Outputs(s2.numel(), cuda)
        between.call(s2, d2, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        say("no-alloc: replay", k)
        g.replay()
        torch.cuda.synchronize()
        assert_same(o.graph(), want, f"replay {k}: ")
        assert_same(between.graph(), entry_point_graph(s2, d2, pipeline=True), f"eager call {k}: ")
