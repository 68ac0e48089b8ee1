"""Radix digit widths of 8 to 11 bits (the schedule's digit_bits): every
conversion kind with both node-numbering methods, against the oracle
element by element, bit-exact. The graph is the same whatever digit width
the radix passes use; only the number of passes and the counts per tile
change."""
import contextlib
import sys

import numpy as np
import pytest

import oracle
from paper_1503_07881_amd import ringo, workloads

pytestmark = pytest.mark.gpu

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
KINDS = {"directed": (ringo.GRAPH_DIRECTED, oracle.DIRECTED),
         "undirected": (ringo.GRAPH_UNDIRECTED, oracle.UNDIRECTED),
         "multigraph": (ringo.GRAPH_MULTI, oracle.MULTIGRAPH)}
FIELDS = ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@contextlib.contextmanager
def schedule(digit_bits, items=None, method=None):
    """Every size bucket on digit_bits (and items / method when given); the
    library's schedule is restored afterwards."""
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    try:
        for e, (_, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, digit_bits, items or it, m if method is None else method)
        yield
    finally:
        for e, (d, it, m) in enumerate(saved):
            ringo.tune_set(1 << e, d, it, m)


@contextlib.contextmanager
def numbering(method):
    """NODES_SORT, NODES_HASH, or "parts": the hash numbering through keys
    grouped by table part at every size."""
    import os
    if method == "parts":
        os.environ["RINGO_HASH_PARTS"] = "1"
    try:
        yield ringo.NODES_HASH if method == "parts" else method
    finally:
        os.environ.pop("RINGO_HASH_PARTS", None)


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(dev)


def assert_same_kind(g, og, kind, label):
    import torch
    torch.cuda.synchronize()
    for f in FIELDS:
        got, want = getattr(g, f).cpu().numpy(), getattr(og, f)
        assert got.shape == want.shape, f"{label}{f}: shape {got.shape} != {want.shape}"
        if not np.array_equal(got, want):
            bad = np.flatnonzero(got != want)
            raise AssertionError(f"{label}{f}: {bad.size} mismatches, first at {bad[0]}")
    if kind == ringo.GRAPH_MULTI:
        assert np.array_equal(g.out_eids.cpu().numpy(), og.out_eids), label + "out_eids"
        assert np.array_equal(g.in_eids.cpu().numpy(), og.in_eids), label + "in_eids"


def random_table(seed, n, pool):
    rng = np.random.default_rng(seed)
    ids = rng.integers(I64_MIN, I64_MAX, size=pool, dtype=np.int64, endpoint=True)
    if pool > 2:
        ids[0], ids[1] = I64_MIN, I64_MAX
    return ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]


@pytest.mark.parametrize("bits", [9, 10, 11])
@pytest.mark.parametrize("kname", sorted(KINDS))
def test_kinds_and_methods(cuda, bits, kname):
    kind, okind = KINDS[kname]
    # pool sizes give V from 1 to about 2n, so b (and the pass counts) vary;
    # n spans several 2048-key tiles with a ragged end
    cases = [(4097, 1), (4097, 3), (20011, 500), (20011, 40000), (150001, 30000), (150001, 1 << 40)]
    for method in (ringo.NODES_SORT, ringo.NODES_HASH):
        with schedule(bits, method=method):
            for n, pool in cases:
                say("digit bits", bits, kname, "method", method, "n", n, "pool", pool)
                src, dst = random_table(n * 7 + pool % 1000 + bits, n, min(pool, 1 << 20))
                g = ringo.to_graph(to_dev(src, cuda), to_dev(dst, cuda), kind=kind)
                assert_same_kind(g, oracle.table_to_graph_kind(src, dst, okind), kind,
                                 f"bits {bits} {kname} method {method} n {n} pool {pool}: ")


@pytest.mark.parametrize("items", [8, 12, 16])
@pytest.mark.parametrize("bits", [8, 9, 11])
def test_items_with_digit_bits(cuda, items, bits):
    spec = workloads.TableSpec("rmat", 1 << 19, seed=71, scale=16)
    src, dst = workloads.generate_host(spec)
    for kname in ("directed", "multigraph"):
        kind, okind = KINDS[kname]
        # parts at 12 items: grouping tiles of 3072 rows, which the estimate's
        # tiles do not divide, so the grouping counts the parts itself
        for method in (ringo.NODES_SORT, ringo.NODES_HASH, "parts"):
            say("R-MAT 2^19 rows, digit bits", bits, "items", items, kname, "method", method)
            with numbering(method) as m, schedule(bits, items=items, method=m):
                g = ringo.to_graph(to_dev(src, cuda), to_dev(dst, cuda), kind=kind)
                assert_same_kind(g, oracle.table_to_graph_kind(src, dst, okind), kind,
                                 f"bits {bits} items {items} {kname} method {method}: ")


@pytest.mark.parametrize("bits", [9, 11])
def test_batched(cuda, bits):
    import torch
    specs = [workloads.mixed_table(93, i, 1, 120_000) for i in range(20)]
    specs += [workloads.TableSpec("uniform", 0, seed=1), workloads.TableSpec("uniform", 1, seed=2, pool=1)]
    tables = [workloads.generate_host(s) for s in specs]
    ts = [(torch.from_numpy(s).to(cuda), torch.from_numpy(d).to(cuda)) for s, d in tables]
    for method in (ringo.NODES_SORT, ringo.NODES_HASH):
        say("batched, digit bits", bits, "method", method, len(tables), "tables")
        with schedule(bits, method=method):
            gb = ringo.to_graph_batched([s for s, _ in ts], [d for _, d in ts])
        for i, (hs, hd) in enumerate(tables):
            assert_same_kind(gb[i], oracle.table_to_graph_kind(hs, hd, oracle.DIRECTED), ringo.GRAPH_DIRECTED,
                             f"bits {bits} method {method} table {i}: ")


@pytest.mark.parametrize("bits", [9, 10, 11])
def test_rmat_large(cuda, bits):
    """2^22 rows: passes of more than 4096 tiles (the two-kernel scan), the
    bucketed distinct-key sort of the hash numbering, and 2b = 38 to 40 bit
    edge keys."""
    spec = workloads.TableSpec("rmat", 1 << 22, seed=77, scale=19)
    src, dst = workloads.generate_host(spec)
    want = oracle.table_to_graph(src, dst)
    for method in (ringo.NODES_SORT, ringo.NODES_HASH, "parts"):
        say("R-MAT 2^22 rows, digit bits", bits, "method", method)
        with numbering(method) as m, schedule(bits, method=m):
            g = ringo.to_graph(to_dev(src, cuda), to_dev(dst, cuda))
        assert_same_kind(g, want, ringo.GRAPH_DIRECTED, f"bits {bits} method {method}: ")


@contextlib.contextmanager
def tile_pairs(on):
    """RINGO_TILE_PAIRS: the plain edge and in-passes of 16-key schedules on
    two-half 8192-key tiles (on, the default) or one-half 4096-key tiles."""
    import os
    os.environ["RINGO_TILE_PAIRS"] = "1" if on else "0"
    try:
        yield
    finally:
        os.environ.pop("RINGO_TILE_PAIRS", None)


@pytest.mark.parametrize("bits", [8, 9])
def test_tile_halves(cuda, bits):
    """16 keys per thread with 8- or 9-bit digits: the plain passes on
    two-half tiles and on one-half tiles give the oracle's graph, for the
    directed and undirected kinds (the multigraph's key-value passes keep
    one-half tiles) and every numbering; a ragged last tile."""
    spec = workloads.TableSpec("rmat", (1 << 19) + 4097, seed=73, scale=16)
    src, dst = workloads.generate_host(spec)
    for kname in ("directed", "undirected"):
        kind, okind = KINDS[kname]
        want = oracle.table_to_graph_kind(src, dst, okind)
        for method in (ringo.NODES_SORT, ringo.NODES_HASH, "parts"):
            for on in (True, False):
                say("R-MAT 2^19 + 4097 rows, digit bits", bits, "16 items", kname, "method", method, "pairs", on)
                with tile_pairs(on), numbering(method) as m, schedule(bits, items=16, method=m):
                    g = ringo.to_graph(to_dev(src, cuda), to_dev(dst, cuda), kind=kind)
                    assert_same_kind(g, want, kind, f"bits {bits} {kname} method {method} pairs {on}: ")
