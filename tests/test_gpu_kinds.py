"""Undirected and multigraph conversions on the GPU through the C ABI,
element by element against the oracle (bit-exact, integer work), with
both node-numbering methods; full-size checks by properties that fix the
answer."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1503_07881_amd import ringo, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "graph_kinds_examples.json")
I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
KINDS = {"undirected": ringo.GRAPH_UNDIRECTED, "multigraph": ringo.GRAPH_MULTI}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(dev)


FIELDS = ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs")


def assert_same_kind(g, og, kind, label=""):
    import torch
    torch.cuda.synchronize()
    assert g.kind == kind
    for f in FIELDS:
        got = getattr(g, f).cpu().numpy()
        want = getattr(og, f)
        assert np.array_equal(got, want), f"{label}{f} differs"
    if kind == ringo.GRAPH_MULTI:
        assert np.array_equal(g.out_eids.cpu().numpy(), og.out_eids), label + "out_eids"
        assert np.array_equal(g.in_eids.cpu().numpy(), og.in_eids), label + "in_eids"
    else:
        assert g.out_eids is None and g.in_eids is None
    if kind == ringo.GRAPH_UNDIRECTED and g.num_edges:
        assert g.in_nbrs.data_ptr() == g.out_nbrs.data_ptr()


def check(src, dst, kind, dev, label=""):
    g = ringo.to_graph(to_dev(src, dev), to_dev(dst, dev), kind=kind)
    assert_same_kind(g, oracle.table_to_graph_kind(src, dst, kind), kind, label)
    return g


@pytest.mark.parametrize("kname", sorted(KINDS))
def test_hand_examples(cuda, kname, method):
    kind = KINDS[kname]
    for ex in json.load(open(GOLDEN))["examples"]:
        say("kinds hand example", ex["name"], kname, method)
        g = ringo.to_graph(to_dev(ex["src"], cuda), to_dev(ex["dst"], cuda), kind=kind)
        assert g.node_ids.cpu().tolist() == ex["node_ids"]
        if kind == ringo.GRAPH_UNDIRECTED:
            u = ex["undirected"]
            assert g.out_offsets.cpu().tolist() == u["offsets"] and g.out_nbrs.cpu().tolist() == u["nbrs"]
            assert g.in_offsets.cpu().tolist() == u["offsets"] and g.in_nbrs.cpu().tolist() == u["nbrs"]
        else:
            for f, v in ex["multigraph"].items():
                assert getattr(g, f).cpu().tolist() == v, (ex["name"], f)


def random_table(seed, n, pool):
    rng = np.random.default_rng(seed)
    ids = rng.integers(I64_MIN, I64_MAX, size=pool, dtype=np.int64, endpoint=True)
    if pool > 2:
        ids[0], ids[1] = I64_MIN, I64_MAX
    return ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]


SIZES = [1, 2, 63, 2047, 2048, 2049, 4097, 8193, 40000, 131072 + 7]


@pytest.mark.parametrize("kname", sorted(KINDS))
@pytest.mark.parametrize("n", SIZES)
def test_tile_boundaries(cuda, kname, n, method):
    for pool in (1, 7, max(1, n // 3), 4 * n):
        say("kinds tile case", kname, "n", n, "pool", pool, method)
        src, dst = random_table(n * 13 + pool, n, pool)
        check(src, dst, KINDS[kname], cuda, f"{kname} n={n} pool={pool}: ")


@pytest.mark.parametrize("kname", sorted(KINDS))
def test_special_structures(cuda, kname, method):
    m = 30_000
    leaves = np.arange(-m, m, 2, dtype=np.int64)
    cases = {
        "same_row": (np.full(9000, 3, np.int64), np.full(9000, -3, np.int64)),
        "loops": (np.arange(-4000, 4000, dtype=np.int64), np.arange(-4000, 4000, dtype=np.int64)),
        "star_both_ways": (np.concatenate([np.full(leaves.size, 11), leaves]),
                           np.concatenate([leaves, np.full(leaves.size, 11)])),
        "extremes": (np.array([I64_MAX, I64_MIN, 0, I64_MAX], np.int64), np.array([I64_MIN, I64_MAX, 0, I64_MAX], np.int64)),
    }
    for name, (s, d) in cases.items():
        say("kinds special", kname, name, method)
        check(s, d, KINDS[kname], cuda, f"{kname} {name}: ")


@pytest.mark.parametrize("kname", sorted(KINDS))
def test_rmat_medium(cuda, kname):
    spec = workloads.TableSpec("rmat", 1 << 21, seed=31, scale=19)
    src, dst = workloads.generate_host(spec)
    say("kinds R-MAT scale 19, 2M rows", kname)
    check(src, dst, KINDS[kname], cuda, kname + " rmat: ")


@pytest.mark.parametrize("kname", sorted(KINDS))
def test_batched_equals_oracle(cuda, kname):
    import torch
    kind = KINDS[kname]
    specs = [workloads.mixed_table(91, i, 1, 200_000) for i in range(24)]
    specs += [workloads.TableSpec("uniform", 0, seed=1), workloads.TableSpec("uniform", 1, seed=2, pool=1)]
    tables = [workloads.generate_host(s) for s in specs]
    say("kinds batched", kname, len(tables), "tables")
    ts = [(torch.from_numpy(s).to(cuda), torch.from_numpy(d).to(cuda)) for s, d in tables]
    gb = ringo.to_graph_batched([s for s, _ in ts], [d for _, d in ts], kind=kind)
    for i, (hs, hd) in enumerate(tables):
        assert_same_kind(gb[i], oracle.table_to_graph_kind(hs, hd, kind), kind, f"{kname} table {i}: ")


def test_invalid_kind(cuda):
    import ctypes
    g = ringo.RawGraph()
    s = to_dev([1, 2], cuda)
    assert ringo.lib().ringo_table_to_graph_ex(s.data_ptr(), s.data_ptr(), 2, 3, ctypes.byref(g), None) == 1


def _lex_increasing(*cols):
    """Rows (c0[i], c1[i], ...) strictly increasing, lexicographically."""
    import torch
    n = cols[0].numel()
    if n < 2:
        return True
    gt = torch.zeros(n - 1, dtype=torch.bool, device=cols[0].device)
    eq = torch.ones(n - 1, dtype=torch.bool, device=cols[0].device)
    for c in cols:
        a, b = c[:-1], c[1:]
        gt |= eq & (b > a)
        eq &= b == a
    return bool(gt.all())


@pytest.mark.slow
def test_config2_full_size(cuda):
    """2^26-row R-MAT table.  Multigraph: E = n, the row lists are
    permutations of the rows, every entry is its row's (source, destination),
    and entries ascend by (owner, neighbour, row): that fixes the answer.
    Undirected: the adjacency equals the distinct pairs of the directed
    graph's out- and in-lists together (computed with torch)."""
    import torch
    spec = workloads.config2()
    say("kinds: config 2, device generation")
    src = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    dst = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), torch.cuda.current_stream().cuda_stream)
    n = spec.n
    gm = ringo.to_graph(src, dst, kind=ringo.GRAPH_MULTI)
    torch.cuda.synchronize()
    say("multigraph V", gm.num_nodes, "E", gm.num_edges)
    assert gm.num_edges == n
    for off, nbr, eid, own_col, nb_col in ((gm.out_offsets, gm.out_nbrs, gm.out_eids, src, dst),
                                           (gm.in_offsets, gm.in_nbrs, gm.in_eids, dst, src)):
        e = eid.long()
        assert torch.equal(torch.sort(e).values, torch.arange(n, device=cuda))
        owner = torch.repeat_interleave(torch.arange(gm.num_nodes, device=cuda), off[1:] - off[:-1])
        assert torch.equal(gm.node_ids[owner], own_col[e])
        assert torch.equal(gm.node_ids[nbr.long()], nb_col[e])
        assert _lex_increasing(owner, nbr.long(), e)
        del e, owner
    del gm
    gd = ringo.to_graph(src, dst)
    gu = ringo.to_graph(src, dst, kind=ringo.GRAPH_UNDIRECTED)
    torch.cuda.synchronize()
    say("undirected V", gu.num_nodes, "E", gu.num_edges)
    assert torch.equal(gu.node_ids, gd.node_ids)
    V = gd.num_nodes
    own_out = torch.repeat_interleave(torch.arange(V, device=cuda), gd.out_offsets[1:] - gd.out_offsets[:-1])
    own_in = torch.repeat_interleave(torch.arange(V, device=cuda), gd.in_offsets[1:] - gd.in_offsets[:-1])
    keys = torch.cat([own_out * V + gd.out_nbrs.long(), own_in * V + gd.in_nbrs.long()])
    want = torch.unique(keys)
    assert gu.num_edges == want.numel()
    own_u = torch.repeat_interleave(torch.arange(V, device=cuda), gu.out_offsets[1:] - gu.out_offsets[:-1])
    assert torch.equal(own_u * V + gu.out_nbrs.long(), want)
    assert torch.equal(gu.in_offsets, gu.out_offsets) and torch.equal(gu.in_nbrs, gu.out_nbrs)


@pytest.mark.parametrize("kname", sorted(KINDS))
@pytest.mark.parametrize("hub", ["min", "max"])
def test_star_long_offset_runs(cuda, kname, method, hub):
    """Stars of 2^21 leaves whose hub sits at either end of the signed range:
    the offsets of every leaf form one long run, written by the queued fill
    rather than by the lane that finds it."""
    n = 1 << 21
    h = I64_MIN if hub == "min" else I64_MAX
    leaves = np.arange(-(n // 2), n // 2, dtype=np.int64)
    for direction in ("out", "in"):
        s, d = (np.full(n, h, np.int64), leaves) if direction == "out" else (leaves, np.full(n, h, np.int64))
        say("kinds star", kname, direction, "hub", hub, method)
        check(s, d, KINDS[kname], cuda, f"{kname} {direction}-star hub {hub}: ")
