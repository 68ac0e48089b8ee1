"""Pins of the oracle's undirected and multigraph conversions (the paper
discusses directed graphs, Section 2.4; these kinds use the same
definition with another edge rule).  CPU only: hand-worked fixtures, brute
force over Python sets and sorted lists, a scipy route (A + A^T) for the
undirected kind, a numpy lexsort route for the multigraph, closed forms,
and planted mistakes compiled into copies of the oracle."""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "graph_kinds_examples.json")


def examples():
    return json.load(open(GOLDEN))["examples"]


def tiny_table(rng, n, pool):
    ids = np.array([-(1 << 63), -3, 0, 4, (1 << 63) - 1, 17, -99, 5, 8, 123456789, -7, 2][:pool], dtype=np.int64)
    return ids[rng.integers(0, len(ids), n)], ids[rng.integers(0, len(ids), n)]


def brute_undirected(src, dst):
    nodes = sorted(set(src.tolist()) | set(dst.tolist()))
    idx = {v: i for i, v in enumerate(nodes)}
    adj = [set() for _ in nodes]
    for s, d in zip(src.tolist(), dst.tolist()):
        adj[idx[s]].add(idx[d])
        adj[idx[d]].add(idx[s])
    off = np.cumsum([0] + [len(a) for a in adj])
    nbrs = [w for a in adj for w in sorted(a)]
    return np.array(nodes, np.int64), off, np.array(nbrs, np.int32)


def brute_multi(src, dst):
    nodes = sorted(set(src.tolist()) | set(dst.tolist()))
    idx = {v: i for i, v in enumerate(nodes)}
    out = [[] for _ in nodes]
    inn = [[] for _ in nodes]
    for r, (s, d) in enumerate(zip(src.tolist(), dst.tolist())):
        out[idx[s]].append((idx[d], r))
        inn[idx[d]].append((idx[s], r))
    res = {}
    for name, lists in (("out", out), ("in", inn)):
        lists = [sorted(l) for l in lists]
        res[name + "_offsets"] = np.cumsum([0] + [len(l) for l in lists])
        res[name + "_nbrs"] = np.array([w for l in lists for w, _ in l], np.int32)
        res[name + "_eids"] = np.array([r for l in lists for _, r in l], np.int32)
    return np.array(nodes, np.int64), res


def scipy_undirected(src, dst):
    nodes, inv = np.unique(np.concatenate([src, dst]), return_inverse=True)
    n, V = src.size, nodes.size
    A = sp.coo_matrix((np.ones(n), (inv[:n], inv[n:])), shape=(V, V))
    S = (A + A.T).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return nodes, S.indptr.astype(np.int64), S.indices.astype(np.int32)


def lexsort_multi(src, dst):
    nodes, inv = np.unique(np.concatenate([src, dst]), return_inverse=True)
    n, V = src.size, nodes.size
    s, d, r = inv[:n], inv[n:], np.arange(n)
    res = {}
    for name, own, nb in (("out", s, d), ("in", d, s)):
        order = np.lexsort((r, nb, own))
        res[name + "_offsets"] = np.concatenate([[0], np.cumsum(np.bincount(own, minlength=V))])
        res[name + "_nbrs"] = nb[order].astype(np.int32)
        res[name + "_eids"] = r[order].astype(np.int32)
    return nodes, res


def run_pins(lib):
    def kind(s, d, k):
        return oracle.table_to_graph_kind(np.asarray(s, np.int64), np.asarray(d, np.int64), k, lib_path=lib)
    try:
        for ex in examples():
            g = kind(ex["src"], ex["dst"], 1)
            u = ex["undirected"]
            assert g.node_ids.tolist() == ex["node_ids"], ex["name"]
            assert g.out_offsets.tolist() == u["offsets"] and g.out_nbrs.tolist() == u["nbrs"], ex["name"]
            assert g.in_offsets.tolist() == u["offsets"] and g.in_nbrs.tolist() == u["nbrs"], ex["name"]
            g = kind(ex["src"], ex["dst"], 2)
            for f, v in ex["multigraph"].items():
                assert getattr(g, f).tolist() == v, (ex["name"], f)
        for seed in range(25):
            rng = np.random.default_rng(seed)
            src, dst = tiny_table(rng, int(rng.integers(1, 60)), int(rng.integers(1, 13)))
            nodes, off, nbrs = brute_undirected(src, dst)
            g = kind(src, dst, 1)
            assert np.array_equal(g.node_ids, nodes) and np.array_equal(g.out_offsets, off)
            assert np.array_equal(g.out_nbrs, nbrs) and np.array_equal(g.in_nbrs, nbrs)
            nodes, res = brute_multi(src, dst)
            g = kind(src, dst, 2)
            assert np.array_equal(g.node_ids, nodes)
            for f, v in res.items():
                assert np.array_equal(getattr(g, f), v), f
    except (AssertionError, oracle.OracleError) as e:
        return str(e) or "assertion"
    return None


def test_pins_hold():
    assert run_pins(oracle.LIB_PATH) is None


@pytest.mark.parametrize("seed", range(5))
def test_library_routes(seed):
    rng = np.random.default_rng(50 + seed)
    n, pool = 20_000, 3000
    ids = rng.integers(-(1 << 63), (1 << 63) - 1, size=pool, dtype=np.int64, endpoint=True)
    src, dst = ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]
    g = oracle.table_to_graph_kind(src, dst, 1)
    nodes, off, nbrs = scipy_undirected(src, dst)
    assert np.array_equal(g.node_ids, nodes) and np.array_equal(g.out_offsets, off)
    assert np.array_equal(g.out_nbrs, nbrs)
    g = oracle.table_to_graph_kind(src, dst, 2)
    nodes, res = lexsort_multi(src, dst)
    for f, v in res.items():
        assert np.array_equal(getattr(g, f), v), f


def test_closed_forms():
    # undirected star: centre adjacent to every leaf, each leaf to the centre
    m = 40
    g = oracle.table_to_graph_kind(np.arange(1, m + 1), np.zeros(m, np.int64), 1)
    assert g.out_offsets.tolist() == [0, m] + list(range(m + 1, 2 * m + 1))
    assert g.out_nbrs.tolist() == list(range(1, m + 1)) + [0] * m
    # multigraph keeps every row: E = n, degrees are the row counts
    rng = np.random.default_rng(9)
    s, d = rng.integers(0, 10, 500), rng.integers(0, 10, 500)
    g = oracle.table_to_graph_kind(s, d, 2)
    assert g.num_edges == 500
    assert np.array_equal(np.diff(g.out_offsets), np.bincount(np.searchsorted(g.node_ids, s), minlength=g.num_nodes))
    assert sorted(g.out_eids.tolist()) == list(range(500)) and sorted(g.in_eids.tolist()) == list(range(500))
    # undirected adjacency is symmetric and the directed graph's edges are a subset
    u = oracle.table_to_graph_kind(s, d, 1)
    pairs = {(v, int(w)) for v in range(u.num_nodes) for w in u.out_nbrs[u.out_offsets[v]:u.out_offsets[v + 1]]}
    assert all((w, v) in pairs for v, w in pairs)
    dg = oracle.table_to_graph(s, d)
    assert all((v, int(w)) in pairs for v in range(dg.num_nodes)
               for w in dg.out_nbrs[dg.out_offsets[v]:dg.out_offsets[v + 1]])


def test_errors():
    with pytest.raises(oracle.OracleError):
        oracle.table_to_graph_kind(np.zeros(3, np.int64), np.zeros(3, np.int64), 7)


MUTANTS = {
    "undirected_one_orientation": ("        both.push_back({d, s});\n", ""),
    "undirected_no_dedupe": ("      both.erase(std::unique(both.begin(), both.end()), both.end());\n", ""),
    "multi_row_tiebreak_dropped": ("    return row < o.row;", "    return false;"),
    "multi_in_not_swapped": ("      for (auto &x : t3) std::swap(x.owner, x.nbr);\n", ""),
    "multi_row_not_recorded": ("    eid[i] = t[i].row;", "    eid[i] = (int32_t)i;"),
    "multi_deduped": ("      std::sort(t3.begin(), t3.end());\n      build_direction_rows(t3, V, g->out_off",
                      "      std::sort(t3.begin(), t3.end());\n      t3.erase(std::unique(t3.begin(), t3.end(), "
                      "[](const Triple &a, const Triple &b) { return a.owner == b.owner && a.nbr == b.nbr; }), t3.end());\n"
                      "      build_direction_rows(t3, V, g->out_off"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    text = open(oracle.SRC_PATH).read()
    old, new = MUTANTS[name]
    assert text.count(old) == 1, f"mutation anchor for {name} not found"
    src = tmp_path / "mutant.cpp"
    src.write_text(text.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", lib, str(src)], check=True)
    assert run_pins(lib) is not None, f"mutant {name} passed every pin"
