"""The C-ABI library loads, exports every symbol include/ringo.h declares,
and rejects invalid arguments before touching the device (CPU only)."""
import ctypes
import os
import re

import pytest

from paper_1503_07881_amd import ringo, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ringo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ringo_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("ringo_table_to_graph", "ringo_table_to_graph_batched", "ringo_graph_free", "ringo_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(ringo.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"
    assert set(declared_functions()) == set(ringo.EXPORTED_SYMBOLS)


def test_status_strings():
    for code in range(7):
        assert ringo.status_string(code)
    assert ringo.status_string(0) == "ok"
    assert "gfx950" in ringo.version()


def test_invalid_arguments_rejected_on_host():
    L = ringo.lib()
    g = ringo.RawGraph()
    assert L.ringo_table_to_graph(None, None, -1, ctypes.byref(g), None) == 1
    assert L.ringo_table_to_graph(None, None, 10, ctypes.byref(g), None) == 1
    assert L.ringo_table_to_graph(None, None, (1 << 31), ctypes.byref(g), None) == 1
    assert L.ringo_table_to_graph(None, None, 0, None, None) == 1
    assert g.num_nodes == 0 and g.node_ids is None
    n = (ctypes.c_int64 * 2)(5, -1)
    p = (ctypes.c_void_p * 2)(None, None)
    outs = (ringo.RawGraph * 2)()
    assert L.ringo_table_to_graph_batched(2, p, p, n, outs, None) == 1
    assert L.ringo_table_to_graph_batched(-1, p, p, n, outs, None) == 1
    assert L.ringo_table_to_graph_batched(0, None, None, None, None, None) == 0
    ringo.graph_free(g)  # zeroed struct: no-op
    L.ringo_graph_free(None)
    # graph to table: checked on the host, nothing launched
    assert L.ringo_graph_to_edge_table(None, None, None, None) == 1
    assert L.ringo_graph_to_node_table(None, None, None, None, None) == 1
    g.num_nodes, g.num_edges = 3, 5
    assert L.ringo_graph_to_edge_table(ctypes.byref(g), None, None, None) == 1
    g.num_edges = -1
    assert L.ringo_graph_to_edge_table(ctypes.byref(g), None, None, None) == 1
    g.num_nodes, g.num_edges = 0, 0
    assert L.ringo_graph_to_edge_table(ctypes.byref(g), None, None, None) == 0
    assert L.ringo_graph_to_node_table(ctypes.byref(g), None, None, None, None) == 0
    # pagerank: argument checks on the host
    assert L.ringo_pagerank(None, ctypes.c_double(0.85), 10, None, None) == 1
    assert L.ringo_pagerank(ctypes.byref(g), ctypes.c_double(0.85), 10, None, None) == 0  # V = 0
    g.num_nodes = 4
    assert L.ringo_pagerank(ctypes.byref(g), ctypes.c_double(0.85), 10, None, None) == 1
    assert L.ringo_pagerank(ctypes.byref(g), ctypes.c_double(1.5), 10, None, None) == 1
    assert L.ringo_pagerank(ctypes.byref(g), ctypes.c_double(0.85), -2, None, None) == 1
    # sort primitive: argument checks on the host (the pointers are never read)
    a, b = 0x10000, 0x10008
    assert L.ringo_sort_keys(None, None, 0, 64, None) == 0
    assert L.ringo_sort_keys(None, None, -1, 64, None) == 1
    assert L.ringo_sort_keys(None, None, 5, 64, None) == 1
    assert L.ringo_sort_keys(a, b, 5, 0, None) == 1
    assert L.ringo_sort_keys(a, b, 5, 65, None) == 1
    assert L.ringo_sort_keys(a, b, 2, 64, None) == 1        # out starts inside in
    assert L.ringo_sort_keys(b, a, 2, 64, None) == 1        # in starts inside out
    assert L.ringo_sort_keys(a, a, 1, 64, None) == 1        # in place
    assert L.ringo_sort_keys(a, b, 1 << 33, 64, None) == 1  # above 2 * RINGO_MAX_ROWS


def test_tune_schedule_roundtrip():
    d, it, m = ringo.tune_get(1000)
    assert d == 8 and it in (8, 12, 16) and m == ringo.NODES_SORT
    # built-in tile shape and digit width by table size
    assert ringo.tune_get(1 << 26)[:2] == (8, 8)
    assert ringo.tune_get(1 << 28)[:2] == (8, 16)
    assert ringo.tune_get(1_500_000_000)[:2] == (9, 16)
    assert ringo.tune_get(1 << 24)[2] == ringo.NODES_HASH   # built-in default for large tables
    assert ringo.tune_get(1 << 20)[2] == ringo.NODES_SORT   # built-in default below 2^24 rows
    ringo.tune_set(1 << 20, 8, 12)
    assert ringo.tune_get(1 << 20) == (8, 12, ringo.NODES_SORT)
    ringo.tune_set(1 << 20, 8, 12, ringo.NODES_HASH)
    assert ringo.tune_get(1 << 20) == (8, 12, ringo.NODES_HASH)
    assert ringo.tune_get(1 << 21)[2] == ringo.NODES_SORT   # other buckets untouched
    ringo.tune_set(1 << 20, 8, 8, ringo.NODES_SORT)         # back to the built-in default
    with pytest.raises(ringo.RingoError):
        ringo.tune_set(1000, 8, 16, 2)
    for bits in (9, 10, 11, 8):                                # digit widths 8 to 11
        ringo.tune_set(1000, bits, 16)
        assert ringo.tune_get(1000)[:2] == (bits, 16)
    for bits in (0, 7, 12, 16):
        with pytest.raises(ringo.RingoError):
            ringo.tune_set(1000, bits, 16)
    assert ringo.tune_get(1000)[0] == 8
    with pytest.raises(ringo.RingoError):
        ringo.tune_set(1000, 8, 7)
    ringo.tune_set(1000, d, it, m)


def test_generators_deterministic_and_shaped():
    spec = workloads.TableSpec("uniform", 50_000, seed=9, pool=1000, ndup=500, shuffle=True)
    a = workloads.generate_host(spec)
    b = workloads.generate_host(spec, threads=1)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    import numpy as np
    assert np.unique(np.concatenate(a)).size <= 1000
    r = workloads.generate_host(workloads.TableSpec("rmat", 100_000, seed=2, scale=10))
    assert np.unique(np.concatenate(r)).size <= 1024
    # R-MAT skew: the most frequent source carries far more than 1/1024 of rows
    _, counts = np.unique(r[0], return_counts=True)
    assert counts.max() > 20 * 100_000 / 1024
    # the splitmix64 finaliser matches the library's
    L = workloads.lib()
    for x in (0, 1, 12345, (1 << 64) - 1):
        assert L.ringo_gen_mix64(x) == workloads.mix64(x)


def test_config4_sizes():
    specs = workloads.config4()
    assert len(specs) == 4096
    ns = [s.n for s in specs]
    assert min(ns) >= 1000 and max(ns) <= 2_000_000
    total = sum(ns)
    assert 0.9e9 < total < 1.25e9
    assert all(s.kind == ("uniform" if i % 2 == 0 else "rmat") for i, s in enumerate(specs))


def test_autotune_cache_roundtrip(tmp_path):
    from paper_1503_07881_amd import autotune
    saved = [ringo.tune_get(1 << e) for e in range(63)]
    cache = {"device": "test",
             "buckets": {str(1 << 10): {"items": 8, "digit_bits": 9, "node_method": 0},
                         str(1 << 20): {"items": 12, "digit_bits": 11, "node_method": 1},
                         str(1 << 24): {"items": 16}}}
    path = autotune.save(cache, str(tmp_path / "tune.json"))
    assert autotune.load(path) == cache
    assert autotune.apply(autotune.load(path)) == 25  # buckets 2^0 .. 2^24
    assert ringo.tune_get(1 << 5)[:2] == (9, 8)      # below the first tuned size: nearest
    assert ringo.tune_get(1 << 15)[:2] == (9, 8)
    assert ringo.tune_get(1 << 21) == (11, 12, 1)
    assert ringo.tune_get(1 << 24)[:2] == (8, 16)     # no digit width in the bucket: 8
    assert ringo.tune_get(1 << 30)[:2] == (9, 16)     # above the largest tuned size: the library's
    assert ringo.tune_get(1 << 15)[2] == 0
    assert autotune.apply({"digit_bits": 11, "buckets": {}}) == 0
    # an unsupported digit width or tile shape is ignored
    assert autotune.apply({"buckets": {"1": {"items": 8, "digit_bits": 12}, "2": {"items": 10}}}) == 0
    # a cache whose top-level width covers every bucket it sets
    assert autotune.apply({"digit_bits": 10, "buckets": {"1": {"items": 12, "node_method": 0},
                                                         str(1 << 40): {"items": 12, "node_method": 1}}}) == 41
    assert ringo.tune_get(1 << 40)[:2] == (10, 12)
    # restore the library's schedule
    for e, (d, it, m) in enumerate(saved):
        ringo.tune_set(1 << e, d, it, m)


def test_builtin_schedule_is_the_tuned_cache():
    """The library's built-in schedule table is the committed autotuner cache:
    the generated header matches the cache, and in a fresh process (no
    schedule set at run time) every size bucket the cache covers has the
    schedule that autotune.apply() would give it from the cache."""
    import json
    import subprocess
    import sys
    from paper_1503_07881_amd import autotune
    pkg = os.path.dirname(autotune.__file__)
    cache = autotune.load(os.path.join(pkg, "tuned_schedules.json"))
    assert cache and cache["buckets"], "no committed cache"
    with open(autotune.HEADER) as f:
        assert f.read() == autotune.header_text(cache), "csrc/tuned_schedule.h is stale: re-emit it"
    rows = sorted((int(k), v["digit_bits"], v["items"], v["node_method"]) for k, v in cache["buckets"].items())
    largest = rows[-1][0].bit_length() - 1
    code = ("import json, sys; sys.path.insert(0, %r); from paper_1503_07881_amd import ringo; "
            "print(json.dumps([ringo.tune_get(1 << e) for e in range(%d)]))" % (ROOT, largest + 1))
    got = json.loads(subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                                    check=True).stdout)
    for e in range(largest + 1):
        below = [r for r in rows if r[0] <= (1 << e)]
        n, d, it, m = below[-1] if below else rows[0]
        assert tuple(got[e]) == (d, it, m), (e, got[e], (d, it, m))
