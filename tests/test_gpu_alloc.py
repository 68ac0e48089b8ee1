"""Caller-supplied device allocator (ringo_set_allocator) and the
out-of-memory path: a counting allocator that refuses its k-th request makes
the conversion fail with RINGO_ERR_OUT_OF_MEMORY, every block handed out
before is returned, the outputs are zeroed, and conversions work again
afterwards (with the hook and with the built-in allocator)."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from helpers import assert_same
from paper_1503_07881_amd import ringo, workloads

pytestmark = pytest.mark.gpu

ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class CountingAllocator:
    """torch's caching allocator behind the hook; refuses request number
    `fail_at` (1-based; 0 never) and records the live blocks."""

    def __init__(self, dev):
        import torch
        self.torch = torch
        self.dev = dev
        self.fail_at = 0
        self.requests = 0
        self.live = {}
        self.c_alloc = ALLOC(self._alloc)
        self.c_free = FREE(self._free)

    def _alloc(self, nbytes, stream, ctx):
        self.requests += 1
        if self.fail_at and self.requests == self.fail_at:
            return None
        ptr = self.torch.cuda.caching_allocator_alloc(max(int(nbytes), 1), self.dev.index, stream)
        self.live[ptr] = nbytes
        return ptr

    def _free(self, ptr, stream, ctx):
        if ptr:
            self.live.pop(ptr)
            self.torch.cuda.caching_allocator_delete(ptr)

    def install(self):
        assert ringo.lib().ringo_set_allocator(ctypes.cast(self.c_alloc, ctypes.c_void_p),
                                               ctypes.cast(self.c_free, ctypes.c_void_p), None) == 0


def convert_raw(src, dst, kind=ringo.GRAPH_DIRECTED):
    import torch
    g = ringo.RawGraph()
    sh = torch.cuda.current_stream().cuda_stream
    rc = ringo.lib().ringo_table_to_graph_ex(src.data_ptr(), dst.data_ptr(), src.numel(), kind,
                                             ctypes.byref(g), sh)
    torch.cuda.synchronize()
    return rc, g


KINDS = {"directed": ringo.GRAPH_DIRECTED, "undirected": ringo.GRAPH_UNDIRECTED,
         "multi": ringo.GRAPH_MULTI}


# the sync-free path converts directed tables only
ALLOC_CASES = [(m, k) for m in ("sort", "hash", "hash_parts", "sync_free") for k in KINDS
               if m != "sync_free" or k == "directed"]


@pytest.mark.parametrize("method,kname", ALLOC_CASES)
def test_allocator_hook_and_out_of_memory(cuda, method, kname, monkeypatch):
    """method: the node numbering of the pass pipeline (hash_parts: through
    keys grouped by table part, whose every request is refused in turn), or
    (directed tables numbered by sorting) the sync-free single-table path,
    whose workspace and outputs are two requests."""
    import torch
    if method != "sync_free":
        monkeypatch.setenv("RINGO_FIXED_PATH", "0")
    monkeypatch.setenv("RINGO_HASH_PARTS", "1" if method == "hash_parts" else "0")
    rng = np.random.default_rng(5)
    n = 300_000  # above the small-table size
    # identifiers from a pool of n / 8, so that hash numbering builds its table
    ids = rng.integers(-(1 << 62), 1 << 62, n // 8, dtype=np.int64)
    src_h = ids[rng.integers(0, ids.size, n)]
    dst_h = src_h[rng.permutation(n)]
    src, dst = (torch.from_numpy(a).to(cuda) for a in (src_h, dst_h))
    kind = KINDS[kname]
    want = oracle.table_to_graph_kind(src_h, dst_h, {"directed": oracle.DIRECTED, "undirected": oracle.UNDIRECTED,
                                                     "multi": oracle.MULTIGRAPH}[kname])
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    al = CountingAllocator(cuda)
    try:
        ringo.set_node_method(ringo.NODES_HASH if method.startswith("hash") else ringo.NODES_SORT)
        al.install()
        # a full conversion through the hook: how many requests it makes
        rc, g = convert_raw(src, dst, kind)
        assert rc == 0
        total = al.requests
        assert (total == 2 if method == "sync_free" else total > 3) and al.live
        ringo.graph_free(g)
        assert not al.live, "blocks left after graph_free"
        # refuse every request in turn (a sample of them for speed)
        ks = range(1, total + 1) if method == "hash_parts" else {1, 2, 3, total // 2, total - 1, total}
        for k in sorted(set(ks) & set(range(1, total + 1))):
            say("allocator refuses request", k, "of", total, method, kname)
            al.requests, al.fail_at = 0, k
            rc, g = convert_raw(src, dst, kind)
            assert rc == 3, (k, rc)  # RINGO_ERR_OUT_OF_MEMORY
            assert g.num_nodes == 0 and g.node_ids is None and g.out_nbrs is None
            assert not al.live, f"blocks leaked after a failure at request {k}"
        al.fail_at = 0
        rc, g = convert_raw(src, dst, kind)
        assert rc == 0
        got = ringo._wrap(g, cuda)
        assert_same(got, want, "through the hook after failures: ")
        del got
    finally:
        assert ringo.lib().ringo_set_allocator(None, None, None) == 0
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)
    # the built-in allocator again
    g2 = ringo.to_graph(src, dst, kind=kind)
    torch.cuda.synchronize()
    assert_same(g2, want, "built-in allocator: ")


@pytest.mark.gpu
def test_release_cached_returns_idle_blocks(cuda):
    """After a conversion whose graph is freed, the built-in allocator holds
    idle blocks; ringo_release_cached returns them (a second call finds
    none), and a later conversion allocates again and gives the same graph."""
    import torch
    spec = workloads.TableSpec("rmat", 1 << 22, seed=71, scale=18)
    src = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    dst = torch.empty_like(src)
    workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), torch.cuda.current_stream().cuda_stream)
    first = ringo.to_graph(src, dst)
    keep = {f: getattr(first, f).clone() for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs")}
    del first
    torch.cuda.synchronize()
    freed = ringo.release_cached()
    say("released", freed, "bytes")
    assert freed > 16 * spec.n  # at least the two key buffers of the call
    assert ringo.release_cached() == 0
    again = ringo.to_graph(src, dst)
    torch.cuda.synchronize()
    for f, t in keep.items():
        assert torch.equal(getattr(again, f), t), f
