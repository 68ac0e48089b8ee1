"""Graph-to-table conversion on the GPU through the C ABI, element by element
against the oracle (bit-exact), plus a full-size round trip."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1503_07881_amd import ringo, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "graph_to_table_examples.json")
I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(dev)


def check_against_oracle(src, dst, dev, label=""):
    import torch
    g = ringo.to_graph(to_dev(src, dev), to_dev(dst, dev))
    es, ed = ringo.to_edge_table(g)
    ids, od, idg = ringo.to_node_table(g)
    torch.cuda.synchronize()
    og = oracle.table_to_graph(src, dst)
    os_, od_ = oracle.graph_to_edge_table(og)
    oi, oo, oin = oracle.graph_to_node_table(og)
    assert np.array_equal(es.cpu().numpy(), os_), label + "edge src"
    assert np.array_equal(ed.cpu().numpy(), od_), label + "edge dst"
    assert np.array_equal(ids.cpu().numpy(), oi), label + "node ids"
    assert np.array_equal(od.cpu().numpy(), oo), label + "out degree"
    assert np.array_equal(idg.cpu().numpy(), oin), label + "in degree"
    return g, es, ed


def test_hand_examples(cuda):
    for ex in json.load(open(GOLDEN))["examples"]:
        say("graph to table, hand example", ex["name"])
        g = ringo.to_graph(to_dev(ex["src"], cuda), to_dev(ex["dst"], cuda))
        es, ed = ringo.to_edge_table(g)
        ids, od, idg = ringo.to_node_table(g)
        assert es.cpu().tolist() == ex["edge_src"] and ed.cpu().tolist() == ex["edge_dst"]
        assert ids.cpu().tolist() == ex["node_ids"]
        assert od.cpu().tolist() == ex["out_degree"] and idg.cpu().tolist() == ex["in_degree"]


def random_table(seed, n, pool):
    rng = np.random.default_rng(seed)
    ids = rng.integers(I64_MIN, I64_MAX, size=pool, dtype=np.int64, endpoint=True)
    return ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]


# V + E around multiples of the merge tile (2048 items)
@pytest.mark.parametrize("n,pool", [(1, 1), (2, 3), (1000, 1000), (1024, 1), (1500, 600), (3000, 1100),
                                    (4096, 4096), (20000, 300), (100_000, 70_000), (333_333, 5000)])
def test_random_tables(cuda, n, pool):
    say("graph to table, random n", n, "pool", pool)
    src, dst = random_table(n * 7 + pool, n, pool)
    check_against_oracle(src, dst, cuda, f"n={n} pool={pool}: ")


def test_degree_skew(cuda):
    """Runs of zero-degree nodes and one huge list, both ways round."""
    leaves = np.arange(-50_000, 50_000, dtype=np.int64)
    hub = np.full(leaves.size, 7, dtype=np.int64)
    cases = {"out_star": (hub, leaves), "in_star": (leaves, hub),
             "two_hubs": (np.concatenate([hub, leaves[:100]]), np.concatenate([leaves, np.full(100, I64_MAX)]))}
    for name, (s, d) in cases.items():
        say("graph to table, skew case", name)
        check_against_oracle(s, d, cuda, name + ": ")


def test_empty_graph_and_invalid_args(cuda):
    import torch
    g = ringo.to_graph(torch.zeros(0, dtype=torch.int64, device=cuda), torch.zeros(0, dtype=torch.int64, device=cuda))
    es, ed = ringo.to_edge_table(g)
    assert es.numel() == 0 and ed.numel() == 0
    raw = ringo.raw_of(ringo.to_graph(to_dev([1, 2], cuda), to_dev([2, 3], cuda)))
    with pytest.raises(ringo.RingoError):
        ringo.graph_to_edge_table_raw(raw, 0, 0, 0)


@pytest.mark.slow
def test_config2_round_trip(cuda):
    """2^26-row R-MAT table: the edge table is strictly increasing in (src, dst),
    every sampled row is the definition's, and converting it back gives the
    same graph bit for bit."""
    import torch
    spec = workloads.config2()
    say("graph to table: config 2, device generation")
    src = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    dst = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), torch.cuda.current_stream().cuda_stream)
    g = ringo.to_graph(src, dst)
    es, ed = ringo.to_edge_table(g)
    torch.cuda.synchronize()
    E = g.num_edges
    assert es.numel() == E
    # strictly increasing rows in signed (src, dst) order
    same = es[1:] == es[:-1]
    assert bool(((es[1:] > es[:-1]) | (same & (ed[1:] > ed[:-1]))).all())
    # sampled rows from the definition (source by searching the offsets)
    rng = np.random.default_rng(3)
    idx = torch.from_numpy(rng.integers(0, E, 4096)).to(cuda)
    srcpos = torch.searchsorted(g.out_offsets, idx, right=True) - 1
    assert torch.equal(es[idx], g.node_ids[srcpos])
    assert torch.equal(ed[idx], g.node_ids[g.out_nbrs[idx].long()])
    # round trip
    g2 = ringo.to_graph(es, ed)
    torch.cuda.synchronize()
    for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs"):
        assert torch.equal(getattr(g, f), getattr(g2, f)), f
