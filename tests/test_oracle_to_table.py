"""Pins of the oracle's graph-to-table conversion (Section 2.4, "Conversion
of graphs to tables"), CPU only: hand-worked fixtures, the round trip
table -> graph -> table against numpy's set of distinct rows, a loop form of
the definition, closed forms, and planted mistakes that the pins must catch."""
import inspect
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "graph_to_table_examples.json")


def load_examples():
    return json.load(open(GOLDEN))["examples"]


def distinct_rows(src, dst):
    """Sorted distinct (src, dst) rows by numpy (signed lexicographic)."""
    rows = np.unique(np.stack([np.asarray(src, np.int64), np.asarray(dst, np.int64)], axis=1), axis=0)
    return rows[:, 0], rows[:, 1]


def random_table(seed, n, pool):
    rng = np.random.default_rng(seed)
    ids = rng.integers(-(1 << 63), (1 << 63) - 1, size=pool, dtype=np.int64, endpoint=True)
    return ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]


def run_pins(to_edges, to_nodes):
    """Returns the first pin the given functions fail, or None."""
    try:
        for ex in load_examples():
            g = oracle.table_to_graph(np.array(ex["src"], np.int64), np.array(ex["dst"], np.int64))
            s, d = to_edges(g)
            assert list(s) == ex["edge_src"] and list(d) == ex["edge_dst"], ex["name"]
            ids, od, idg = to_nodes(g)
            assert list(ids) == ex["node_ids"] and list(od) == ex["out_degree"] and list(idg) == ex["in_degree"]
        for seed in range(10):
            src, dst = random_table(seed, 200, 1 + seed * 7)
            g = oracle.table_to_graph(src, dst)
            s, d = to_edges(g)
            es, ed = distinct_rows(src, dst)
            assert np.array_equal(s, es) and np.array_equal(d, ed), f"round trip seed {seed}"
            ids, od, idg = to_nodes(g)
            assert od.sum() == idg.sum() == len(es)
            # degrees from the distinct rows
            assert np.array_equal(od, np.array([(es == v).sum() for v in ids]))
            assert np.array_equal(idg, np.array([(ed == v).sum() for v in ids]))
    except AssertionError as e:
        return str(e) or "assertion"
    return None


def test_fixtures_and_round_trip():
    assert run_pins(oracle.graph_to_edge_table, oracle.graph_to_node_table) is None


@pytest.mark.parametrize("seed", range(6))
def test_loop_form_agrees(seed):
    src, dst = random_table(100 + seed, 300, 40)
    g = oracle.table_to_graph(src, dst)
    s, d = oracle.graph_to_edge_table(g)
    ls, ld = oracle.graph_to_edge_table_loops(g)
    assert list(s) == ls and list(d) == ld


def test_complete_digraph_closed_form():
    k = 13
    ids = np.array([(i * 0x9E3779B97F4A7C15) % (1 << 64) - (1 << 63) for i in range(k)], dtype=np.int64)
    a, b = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    perm = np.random.default_rng(5).permutation(k * k)
    g = oracle.table_to_graph(ids[a.ravel()][perm], ids[b.ravel()][perm])
    s, d = oracle.graph_to_edge_table(g)
    sid = np.sort(ids)
    assert np.array_equal(s, np.repeat(sid, k)) and np.array_equal(d, np.tile(sid, k))
    _, od, idg = oracle.graph_to_node_table(g)
    assert (od == k).all() and (idg == k).all()


def test_empty_graph():
    g = oracle.table_to_graph(np.zeros(0, np.int64), np.zeros(0, np.int64))
    s, d = oracle.graph_to_edge_table(g)
    assert s.size == 0 and d.size == 0
    assert all(c.size == 0 for c in oracle.graph_to_node_table(g))


# Each mutant is a plausible slip in the oracle's inverse conversion.
MUTANTS = {
    "columns_swapped": ("return ids[src_idx], ids[nbr]", "return ids[nbr], ids[src_idx]"),
    "source_off_by_one": ("np.repeat(np.arange(V, dtype=np.int64), np.diff(off))",
                          "np.repeat(np.arange(V, dtype=np.int64), np.diff(off))[::-1]"),
    "dense_index_not_id": ("return ids[src_idx], ids[nbr]", "return src_idx, nbr"),
    "degrees_swapped": ("return (ids.copy(), np.diff(np.asarray(g.out_offsets, dtype=np.int64)),\n"
                        "            np.diff(np.asarray(g.in_offsets, dtype=np.int64)))",
                        "return (ids.copy(), np.diff(np.asarray(g.in_offsets, dtype=np.int64)),\n"
                        "            np.diff(np.asarray(g.out_offsets, dtype=np.int64)))"),
}


def _mutated(fn, old, new):
    src = inspect.getsource(fn)
    assert old in src, f"mutation anchor not found in {fn.__name__}"
    ns = {"np": np}
    exec(src.replace(old, new), ns)
    return ns[fn.__name__]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    old, new = MUTANTS[name]
    to_edges, to_nodes = oracle.graph_to_edge_table, oracle.graph_to_node_table
    if old in inspect.getsource(to_edges):
        to_edges = _mutated(to_edges, old, new)
    else:
        to_nodes = _mutated(to_nodes, old, new)
    assert run_pins(to_edges, to_nodes) is not None, f"mutant {name} passed every pin"
