"""Pins of the oracle's PageRank (Page, Brin, Motwani & Winograd 1999; ten
iterations in the paper's Section 3), CPU only: hand-worked iterations and
fixed points, a dense matrix-power route, the stationary vector from an
eigen-decomposition, closed forms, invariants, and planted mistakes."""
import inspect
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pagerank_examples.json")


def graph(src, dst):
    return oracle.table_to_graph(np.asarray(src, np.int64), np.asarray(dst, np.int64))


def random_graph(seed, n, pool):
    rng = np.random.default_rng(seed)
    return graph(rng.integers(0, pool, n), rng.integers(0, pool, n))


def stationary(g, d):
    """Eigenvector of the Google matrix for eigenvalue 1 (numpy eig)."""
    V = len(g.node_ids)
    off = np.asarray(g.out_offsets)
    A = np.zeros((V, V))
    for u in range(V):
        A[u, np.asarray(g.out_nbrs[off[u]:off[u + 1]], dtype=np.int64)] = 1.0
    deg = A.sum(1)
    P = np.where(deg[:, None] > 0, A / np.maximum(deg, 1)[:, None], 1.0 / V)
    M = d * P.T + (1 - d) / V
    w, vecs = np.linalg.eig(M)
    x = np.real(vecs[:, np.argmin(np.abs(w - 1))])
    return x / x.sum()


def run_pins(pr):
    try:
        for ex in json.load(open(GOLDEN))["examples"]:
            g = graph(ex["src"], ex["dst"])
            for it, want in ex["iterations"].items():
                assert np.allclose(pr(g, ex["damping"], int(it)), want, rtol=0, atol=1e-15), (ex["name"], it)
            assert np.allclose(pr(g, ex["damping"], 400), ex["limit"], rtol=0, atol=1e-12), ex["name"]
        for seed in range(8):
            g = random_graph(seed, 40, 12)
            for d in (0.85, 0.5):
                dense = oracle.pagerank_dense(g, d, 10)
                assert np.allclose(pr(g, d, 10), dense, rtol=1e-12, atol=0), f"dense seed {seed}"
                assert abs(pr(g, d, 10).sum() - 1.0) < 1e-12
            assert np.allclose(pr(g, 0.85, 300), stationary(g, 0.85), rtol=1e-9, atol=0), f"eig seed {seed}"
    except AssertionError as e:
        return str(e) or "assertion"
    return None


def test_pins_hold():
    assert run_pins(oracle.pagerank) is None


def test_closed_forms():
    # complete digraph with loops, any damping: uniform at every iteration
    k = 9
    a, b = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    g = graph(a.ravel() * 1000 - 7, b.ravel() * 1000 - 7)
    for d in (0.0, 0.3, 0.85, 1.0):
        assert np.allclose(oracle.pagerank(g, d, 10), 1.0 / k, rtol=1e-14)
    # damping 0: pure teleport
    g = random_graph(3, 500, 60)
    assert np.allclose(oracle.pagerank(g, 0.0, 7), 1.0 / len(g.node_ids), rtol=1e-14)
    # zero iterations: the start vector
    assert np.allclose(oracle.pagerank(g, 0.85, 0), 1.0 / len(g.node_ids), rtol=0)
    # star into a sink from m sources: sources share one value, the sink another
    m = 50
    g = graph(np.arange(m) + 1, np.zeros(m, np.int64))
    r = oracle.pagerank(g, 0.85, 10)
    assert np.allclose(r[1:], r[1]) and r[0] > r[1]


def test_sum_is_one_every_iteration():
    g = random_graph(11, 3000, 700)
    for t in range(12):
        assert abs(oracle.pagerank(g, 0.85, t).sum() - 1.0) < 1e-12


MUTANTS = {
    "no_dangling_mass": ("r = (1.0 - damping) / V + damping * (s + dangling / V)",
                         "r = (1.0 - damping) / V + damping * s"),
    "no_teleport": ("r = (1.0 - damping) / V + damping * (s + dangling / V)",
                    "r = damping * (s + dangling / V)"),
    "damping_swapped": ("r = (1.0 - damping) / V + damping * (s + dangling / V)",
                        "r = damping / V + (1.0 - damping) * (s + dangling / V)"),
    "not_divided_by_outdeg": ("contrib[has] = r[has] / outdeg[has]", "contrib[has] = r[has]"),
    "pull_along_out_edges": ("s = np.bincount(nbr, weights=contrib[src], minlength=V)",
                             "s = np.bincount(src, weights=contrib[nbr], minlength=V)"),
    "one_iteration_short": ("for _ in range(iterations):", "for _ in range(max(0, iterations - 1)):"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    old, new = MUTANTS[name]
    src = inspect.getsource(oracle.pagerank)
    assert old in src
    ns = {"np": np}
    exec(src.replace(old, new), ns)
    assert run_pins(ns["pagerank"]) is not None, f"mutant {name} passed every pin"
