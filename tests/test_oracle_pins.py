"""Pins of the CPU oracle against facts that do not come from the oracle:
hand-worked examples of the definition (Section 2.4), brute force over
Python sets, an independent numpy/scipy route, closed forms, special cases
and invariants.  A mutation test plants plausible mistakes in the oracle's
source and checks that these pins catch every one."""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from helpers import assert_same, brute_force, check_invariants, scipy_route
from paper_1503_07881_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def load_examples():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


def as_np(ex):
    return {"node_ids": np.array(ex["node_ids"], dtype=np.int64),
            "out_offsets": np.array(ex["out_offsets"], dtype=np.int64),
            "out_nbrs": np.array(ex["out_nbrs"], dtype=np.int32),
            "in_offsets": np.array(ex["in_offsets"], dtype=np.int64),
            "in_nbrs": np.array(ex["in_nbrs"], dtype=np.int32)}


@pytest.mark.parametrize("ex", load_examples(), ids=lambda e: e["name"])
def test_hand_examples(ex):
    src = np.array(ex["src"], dtype=np.int64)
    dst = np.array(ex["dst"], dtype=np.int64)
    assert_same(oracle.table_to_graph(src, dst), as_np(ex), ex["name"] + ": ")
    # the independent routes agree with the hand-worked values too
    assert_same(brute_force(src, dst), as_np(ex), "brute: ")
    if src.size:
        assert_same(scipy_route(src, dst), as_np(ex), "scipy: ")


def tiny_table(rng, n, pool):
    ids = rng.integers(I64_MIN, I64_MAX, size=pool, dtype=np.int64, endpoint=True)
    if pool > 2:
        ids[0], ids[1] = I64_MIN, I64_MAX
    return ids[rng.integers(0, pool, n)], ids[rng.integers(0, pool, n)]


@pytest.mark.parametrize("seed", range(60))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 65))
    pool = int(rng.integers(1, 12))
    src, dst = tiny_table(rng, n, pool)
    g = oracle.table_to_graph(src, dst)
    assert_same(g, brute_force(src, dst))
    assert g.num_nodes == len(set(src.tolist()) | set(dst.tolist()))
    assert g.num_edges == len(set(zip(src.tolist(), dst.tolist())))
    check_invariants(g, src, dst)


@pytest.mark.parametrize("seed,n,pool", [(1, 1000, 30), (2, 5000, 5000), (3, 20000, 700), (4, 100000, 100000),
                                         (5, 50000, 3)])
def test_scipy_route(seed, n, pool):
    rng = np.random.default_rng(seed)
    src, dst = tiny_table(rng, n, pool)
    g = oracle.table_to_graph(src, dst)
    assert_same(g, scipy_route(src, dst))
    check_invariants(g, src, dst)


def test_complete_digraph_closed_form():
    k = 37
    ids = np.array(sorted(workloads.mix64(i) - (1 << 63) for i in range(k)), dtype=np.int64)
    a, b = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    rng = np.random.default_rng(7)
    perm = rng.permutation(k * k)
    src = np.concatenate([ids[a.ravel()[perm]], ids[a.ravel()[:50]]])  # with repeats
    dst = np.concatenate([ids[b.ravel()[perm]], ids[b.ravel()[:50]]])
    g = oracle.table_to_graph(src, dst)
    assert g.num_nodes == k and g.num_edges == k * k
    assert np.array_equal(g.out_offsets, np.arange(k + 1) * k)
    assert np.array_equal(g.out_nbrs, np.tile(np.arange(k), k))
    assert np.array_equal(g.in_offsets, np.arange(k + 1) * k)
    assert np.array_equal(g.in_nbrs, np.tile(np.arange(k), k))
    assert np.array_equal(g.node_ids, ids)


def test_star_closed_form():
    m = 500
    leaves = np.arange(1, m + 1, dtype=np.int64) * -3
    c = np.int64(0)
    rng = np.random.default_rng(3)
    order = rng.permutation(m)
    g = oracle.table_to_graph(np.full(m, c), leaves[order])
    nodes = np.sort(np.append(leaves, c))
    ci = int(np.searchsorted(nodes, c))
    assert np.array_equal(g.node_ids, nodes)
    deg_out = np.diff(g.out_offsets)
    assert deg_out[ci] == m and deg_out.sum() == m
    assert np.array_equal(g.out_nbrs, np.array([i for i in range(m + 1) if i != ci], dtype=np.int32))
    deg_in = np.diff(g.in_offsets)
    assert deg_in[ci] == 0 and np.all(np.delete(deg_in, ci) == 1)
    assert np.all(g.in_nbrs == ci)


def test_self_loops_closed_form():
    k = 1000
    ids = np.random.default_rng(5).permutation(np.arange(-k, k, 2, dtype=np.int64))
    g = oracle.table_to_graph(ids, ids)
    n = ids.size
    assert np.array_equal(g.out_nbrs, np.arange(n)) and np.array_equal(g.in_nbrs, np.arange(n))
    assert np.array_equal(g.out_offsets, np.arange(n + 1)) and np.array_equal(g.in_offsets, np.arange(n + 1))


@pytest.mark.parametrize("V", [1, 2, 3, 4, 5, 255, 256, 257, 1023, 1024, 1025, 65536, 65537])
def test_node_count_boundaries(V):
    """V = 2^j and 2^j + 1: a path over V nodes plus a loop at the last one."""
    ids = np.array([workloads.mix64(i) - (1 << 63) for i in range(V)], dtype=np.int64)
    src = ids
    dst = np.roll(ids, -1) if V > 1 else ids
    g = oracle.table_to_graph(src, dst)
    assert g.num_nodes == V and g.num_edges == V
    check_invariants(g, src, dst)
    if V <= 1100:
        assert_same(g, brute_force(src, dst))
    else:
        assert_same(g, scipy_route(src, dst))


def test_single_row_and_extremes():
    for s, d in [(0, 0), (I64_MIN, I64_MAX), (I64_MAX, I64_MIN), (-1, 1), (I64_MIN, I64_MIN)]:
        src = np.array([s], dtype=np.int64)
        dst = np.array([d], dtype=np.int64)
        assert_same(oracle.table_to_graph(src, dst), brute_force(src, dst))


def test_errors():
    L = oracle.load()
    import ctypes
    h, V, E = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int64()
    assert L.oracle_table_to_graph(None, None, -1, ctypes.byref(h), ctypes.byref(V), ctypes.byref(E)) == 1
    assert L.oracle_table_to_graph(None, None, 5, ctypes.byref(h), ctypes.byref(V), ctypes.byref(E)) == 1


@pytest.mark.parametrize("seed,n,pool", [(11, 0, 1), (12, 1, 1), (13, 64, 5), (14, 50_000, 2_000),
                                         (15, 400_000, 1 << 40)])
def test_all_cores_mode_same_result(seed, n, pool):
    """The timing mode on every host thread (a parallel sort in place of
    std::sort) gives the serial oracle's graph."""
    rng = np.random.default_rng(seed)
    src, dst = tiny_table(rng, n, min(pool, 1 << 20))
    serial = oracle.table_to_graph(src, dst)
    assert_same(oracle.table_to_graph(src, dst, all_cores=True), serial)
    assert oracle.last_threads >= 1
    for ex in load_examples():
        s, d = np.array(ex["src"], np.int64), np.array(ex["dst"], np.int64)
        assert_same(oracle.table_to_graph(s, d, all_cores=True), as_np(ex), ex["name"] + ": ")


def test_config1_full_invariants():
    """The 1M-row workload: oracle vs the scipy route, plus the invariants."""
    src, dst = workloads.generate_host(workloads.config1())
    g = oracle.table_to_graph(src, dst)
    assert g.num_nodes == 100_000
    assert_same(g, scipy_route(src, dst))
    check_invariants(g, src, dst)
    # ~1% injected duplicates: E is at most n - 10,000 and close to it
    assert 980_000 < g.num_edges <= 990_000


# ------------------------------------------------------------- mutation test
#
# Each mutant is a plausible slip in the oracle (a dropped step, a swapped
# operand, an off-by-one, a wrong comparison).  The pins above must reject
# every one.

MUTANTS = {
    "no_edge_dedupe": ("e.erase(std::unique(e.begin(), e.end()), e.end());", ""),
    "no_node_dedupe": ("all.erase(std::unique(all.begin(), all.end()), all.end());", ""),
    "unsigned_node_order": ("    sort(all.begin(), all.end());",
                            "    std::sort(all.begin(), all.end(), [](int64_t a, int64_t b) { return (uint64_t)a < (uint64_t)b; });"),
    "swapped_columns": ("e[(size_t)r] = {index_of(src[r]), index_of(dst[r])};",
                        "e[(size_t)r] = {index_of(dst[r]), index_of(src[r])};"),
    "offset_off_by_one": ("for (const auto &p : pairs) off[(size_t)p.first + 1] += 1;",
                          "for (const auto &p : pairs) off[(size_t)p.first] += 1;"),
    "in_not_transposed": ("for (auto &p : e) std::swap(p.first, p.second);", ""),
    "in_unsorted": ("std::swap(p.first, p.second);\n    sort(e.begin(), e.end());",
                    "std::swap(p.first, p.second);"),
    "only_src_nodes": ("all.insert(all.end(), dst, dst + n);", ""),
    "prefix_sum_skips_last": ("for (int64_t v = 0; v < V; ++v) off[(size_t)v + 1] += off[(size_t)v];",
                              "for (int64_t v = 0; v + 1 < V; ++v) off[(size_t)v + 1] += off[(size_t)v];"),
    "neighbour_is_owner": ("nbr[i] = pairs[i].second;", "nbr[i] = pairs[i].first;"),
}


def run_pins(lib_path):
    """Returns the first pin a given oracle build fails, or None."""
    def tt(s, d):
        return oracle.table_to_graph(np.asarray(s, np.int64), np.asarray(d, np.int64), lib_path=lib_path)
    try:
        for ex in load_examples():
            assert_same(tt(ex["src"], ex["dst"]), as_np(ex))
        for seed in range(20):
            rng = np.random.default_rng(seed)
            src, dst = tiny_table(rng, int(rng.integers(1, 65)), int(rng.integers(1, 12)))
            assert_same(tt(src, dst), brute_force(src, dst))
    except (AssertionError, oracle.OracleError) as e:
        return str(e) or "assertion"
    return None


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
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", lib, str(src)], check=True)
    assert run_pins(lib) is not None, f"mutant {name} passed every pin"


def test_unmutated_oracle_passes_pins():
    assert run_pins(oracle.LIB_PATH) is None
