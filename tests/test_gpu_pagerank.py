"""PageRank on the GPU through the C ABI against the oracle.

Tolerance, derived from the arithmetic: contributions r[u]/outdeg(u) are
the same IEEE divisions on both sides; only the order of the fp64 sums
differs.  A sum of k positive terms is within gamma_{k-1} ~ (k-1) u of the
exact value (u = 2^-53), for each side, so two orders differ by at most
2 (k-1) u relative; the dangling mass is a sum of at most V terms.  The
iteration is a contraction (factor d <= 1), so per-iteration differences
add up over t iterations at most:  rtol = 2 t (max in-degree + V) u."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1503_07881_amd import ringo, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pagerank_examples.json")
U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(dev)


def rtol_for(og, iterations):
    indeg = np.diff(np.asarray(og.in_offsets))
    return 2.0 * max(iterations, 1) * (int(indeg.max(initial=0)) + len(og.node_ids)) * U


def check(src, dst, dev, d=0.85, it=10, label=""):
    import torch
    g = ringo.to_graph(to_dev(src, dev), to_dev(dst, dev))
    r = ringo.pagerank(g, d, it)
    torch.cuda.synchronize()
    og = oracle.table_to_graph(np.asarray(src, np.int64), np.asarray(dst, np.int64))
    want = oracle.pagerank(og, d, it)
    got = r.cpu().numpy()
    tol = rtol_for(og, it)
    err = np.max(np.abs(got - want) / want) if want.size else 0.0
    assert err <= tol, f"{label}max relative difference {err:.3g} > {tol:.3g}"
    return g, r


def test_hand_examples(cuda):
    import torch
    for ex in json.load(open(GOLDEN))["examples"]:
        say("pagerank hand example", ex["name"])
        g = ringo.to_graph(to_dev(ex["src"], cuda), to_dev(ex["dst"], cuda))
        for it, want in ex["iterations"].items():
            got = ringo.pagerank(g, ex["damping"], int(it)).cpu().numpy()
            assert np.allclose(got, want, rtol=0, atol=1e-15), (ex["name"], it, got)
        got = ringo.pagerank(g, ex["damping"], 400).cpu().numpy()
        torch.cuda.synchronize()
        assert np.allclose(got, ex["limit"], rtol=0, atol=1e-12), ex["name"]


def random_table(seed, n, pool):
    rng = np.random.default_rng(seed)
    return rng.integers(0, pool, n), rng.integers(0, pool, n)


# V + E around multiples of the merge tile (2048 items), small and large pools
@pytest.mark.parametrize("n,pool", [(1, 1), (5, 3), (1000, 1048), (1500, 548), (2047, 1), (4096, 100),
                                    (50_000, 20_000), (200_000, 3000), (300_000, 400_000)])
def test_random_graphs(cuda, n, pool):
    say("pagerank random n", n, "pool", pool)
    src, dst = random_table(n + pool, n, pool)
    check(src, dst, cuda, label=f"n={n} pool={pool}: ")


def test_hubs_straddling_tiles(cuda):
    """In-stars whose lists span many tiles, sinks (no out-edges), and zero
    in-degree runs."""
    m = 200_000
    leaves = np.arange(1, m + 1, dtype=np.int64)
    cases = {
        "in_star": (leaves, np.zeros(m, np.int64)),
        "two_in_stars": (np.concatenate([leaves, leaves]),
                         np.concatenate([np.zeros(m, np.int64), np.full(m, -5, np.int64)])),
        "out_star": (np.zeros(m, np.int64), leaves),
        "chain_plus_star": (np.concatenate([leaves[:-1], leaves]), np.concatenate([leaves[1:], np.zeros(m, np.int64)])),
    }
    for name, (s, d) in cases.items():
        say("pagerank structure", name)
        check(s, d, cuda, label=name + ": ")


def test_damping_and_iteration_edges(cuda):
    src, dst = random_table(5, 30_000, 9000)
    for d, it in ((0.0, 3), (1.0, 10), (0.85, 0), (0.85, 1), (0.5, 25)):
        say("pagerank damping", d, "iterations", it)
        check(src, dst, cuda, d, it, f"d={d} it={it}: ")


def test_rmat_medium_and_determinism(cuda):
    import torch
    spec = workloads.TableSpec("rmat", 1 << 22, seed=22, scale=20)
    src, dst = workloads.generate_host(spec)
    say("pagerank R-MAT scale 20, 4M rows")
    g, r1 = check(src, dst, cuda, label="rmat: ")
    r2 = ringo.pagerank(g, 0.85, 10)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)


def test_invalid_arguments(cuda):
    g = ringo.to_graph(to_dev([1, 2], cuda), to_dev([2, 3], cuda))
    raw = ringo.raw_of(g)
    import torch
    ranks = torch.empty(3, dtype=torch.float64, device=cuda)
    for d, it in ((-0.1, 10), (1.5, 10), (float("nan"), 10), (0.85, -1)):
        with pytest.raises(ringo.RingoError):
            ringo.pagerank_raw(raw, d, it, ranks.data_ptr(), 0)
    with pytest.raises(ringo.RingoError):
        ringo.pagerank_raw(raw, 0.85, 10, 0, 0)


@pytest.mark.slow
def test_config2_full_size(cuda):
    import torch
    spec = workloads.config2()
    say("pagerank: config 2, device generation")
    src = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    dst = torch.empty(spec.n, dtype=torch.int64, device=cuda)
    workloads.generate_device(spec, src.data_ptr(), dst.data_ptr(), torch.cuda.current_stream().cuda_stream)
    g = ringo.to_graph(src, dst)
    r = ringo.pagerank(g, 0.85, 10)
    torch.cuda.synchronize()
    og = oracle.Graph(g.node_ids.cpu().numpy(), g.out_offsets.cpu().numpy(), g.out_nbrs.cpu().numpy(),
                      g.in_offsets.cpu().numpy(), g.in_nbrs.cpu().numpy())
    say("pagerank: config 2 oracle on the host, V", g.num_nodes, "E", g.num_edges)
    want = oracle.pagerank(og, 0.85, 10)
    err = np.max(np.abs(r.cpu().numpy() - want) / want)
    assert err <= rtol_for(og, 10), err
