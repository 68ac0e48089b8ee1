"""bench.py's host logic (no GPU): which kernel names a trace entry stands
for in a rocprofv3 summary, which source file decides a kernel's counter
summary, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_edge_scatter_names_both_tile_shapes():
    names = bench.rocprof_names("sort_edge_scatter", 16, 9)
    # one-half tiles (any mode's kernel) and the plain passes' two-half tiles,
    # each with 8-bit digits where the key width leaves room
    assert set(names) == {"k_downsweep<256, 16, 5, 8>", "k_downsweep<256, 16, 5, 9>",
                          "k_downsweep_pair<16, 5, 8>", "k_downsweep_pair<16, 5, 9>"}
    names = bench.rocprof_names("sort_in_scatter", 8, 8)
    assert "k_downsweep<256, 8, 10, 8>" in names and "k_downsweep_pair<16, 6, 8>" in names


def test_plain_and_alternative_names():
    assert bench.rocprof_names("hash_insert", 16, 9) == ["k_hash_insert", "k_hash_insert_keys"]
    assert bench.rocprof_names("in_csr", 8, 8) == ["k_in_csr"]
    assert bench.rocprof_names("hash_part_scatter", 16, 9) == ["k_downsweep<256, 16, 11, 8>"]
    assert bench.rocprof_names("unknown_entry", 8, 8) == ["unknown_entry"]


def test_kernel_source_files():
    assert bench.kernel_source_file("sort_edge_scatter") == "lsd.h"
    assert bench.kernel_source_file("hash_part_rank") == "lsd.h"  # a radix pass
    assert bench.kernel_source_file("hash_insert") == "hash.hip"
    assert bench.kernel_source_file("edge_table") == "to_table.hip"
    for name in bench.CONVERSION_SOURCES:
        assert os.path.exists(os.path.join(bench.KERNEL_DIR, name)), name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
