"""MI355X-native table-to-graph conversion (Ringo's "sort-first" ToGraph,
Section 2.4 of the paper), as a C-ABI HIP library with a thin binding."""
from .ringo import (Graph, RingoError, graph_free, lib, status_string, table_to_graph_batched_raw,
                    table_to_graph_raw, to_graph, to_graph_batched, tune_get, tune_set, version)

__all__ = ["Graph", "RingoError", "graph_free", "lib", "status_string", "table_to_graph_batched_raw",
           "table_to_graph_raw", "to_graph", "to_graph_batched", "tune_get", "tune_set", "version"]
