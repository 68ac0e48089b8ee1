// CPU oracle of the table-to-graph conversion -- TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg
// may load this library.  The product path never calls it and shares no code,
// header or helper with it.
//
// What it computes is the plain definition of the conversion (Section 2.4,
// "Conversion of tables to graphs"): table T with source column S and
// destination column D gives the directed graph G = (V, E) where
//   * V is the set of distinct values of S and D, and
//   * every row r gives the edge (r_S, r_D);
// and a directed graph keeps, per node, a sorted out-neighbour vector and a
// sorted in-neighbour vector (Section 2.4; CSR layout as in Section 2.2).
//
// Readings taken where the paper is silent:
//   * E is a set: repeated rows give one edge (a simple directed graph);
//     self-loops are kept.
//   * Nodes are listed in ascending signed 64-bit order; a neighbour is
//     stored as its dense position in that list (a 32-bit index), so sorted
//     by position equals sorted by identifier.
//   * Offsets are 64-bit; the empty table gives V = 0, E = 0, offsets {0}.
//   * V and the row count must stay below 2^31.
//
// The steps follow the paper's "sort-first" outline (Section 2.4): copy the
// two columns, sort the copies, count neighbours per node, then copy the
// neighbour lists into place.  std::sort and std::unique serve as the sort
// and the duplicate removal; there is no blocking, packing or fusion.
//
// Parity: pinned by hand-worked fixtures, brute force over Python sets,
// an independent numpy/scipy route, closed forms and invariants (tests/).
//
// oracle_table_to_graph_par is the same computation with libstdc++'s
// parallel-mode sort (OpenMP, all host threads) in place of std::sort and the
// rows' independent lookups spread over the threads, for running the oracle
// on every core (timing, and the largest tables); sorting values of a total
// order gives the same sequence either way, so the result is identical.
//
// Two further graph kinds (oracle_table_to_graph_kind), the same definition
// with another edge rule (the paper limits its discussion to directed graphs,
// Section 2.4; these are the readings taken for the other two):
//   * undirected: the adjacency of v is the set of w with a row (v, w) or
//     (w, v), ascending; a self-loop appears once; the in-direction is the
//     out-direction.
//   * multigraph: every row is its own edge, identified by its row index;
//     out-lists ascend by (destination, row), in-lists by (source, row).

#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <new>
#include <parallel/algorithm>
#include <utility>
#include <vector>

namespace {

struct OracleGraph {
  std::vector<int64_t> nodes;
  std::vector<int64_t> out_off, in_off;
  std::vector<int32_t> out_nbr, in_nbr;
  std::vector<int32_t> out_eid, in_eid;  // multigraph only
};

struct Triple {
  int32_t owner, nbr, row;
  bool operator<(const Triple &o) const {
    if (owner != o.owner) return owner < o.owner;
    if (nbr != o.nbr) return nbr < o.nbr;
    return row < o.row;
  }
};

// Offsets, neighbour list and row list of one direction from sorted triples.
void build_direction_rows(const std::vector<Triple> &t, int64_t V, std::vector<int64_t> &off,
                          std::vector<int32_t> &nbr, std::vector<int32_t> &eid) {
  off.assign((size_t)V + 1, 0);
  for (const auto &x : t) off[(size_t)x.owner + 1] += 1;
  for (size_t v = 1; v < off.size(); ++v) off[v] += off[v - 1];
  nbr.resize(t.size());
  eid.resize(t.size());
  for (size_t i = 0; i < t.size(); ++i) {
    nbr[i] = t[i].nbr;
    eid[i] = t[i].row;
  }
}

// Offsets and neighbour list of one direction from (owner, neighbour) pairs
// that are already sorted and distinct: count the neighbours of each node,
// prefix-sum the counts, copy the neighbours.
void build_direction(const std::vector<std::pair<int32_t, int32_t>> &pairs, int64_t V,
                     std::vector<int64_t> &off, std::vector<int32_t> &nbr) {
  off.assign((size_t)V + 1, 0);
  for (const auto &p : pairs) off[(size_t)p.first + 1] += 1;
  for (int64_t v = 0; v < V; ++v) off[(size_t)v + 1] += off[(size_t)v];
  nbr.resize(pairs.size());
  for (size_t i = 0; i < pairs.size(); ++i) nbr[i] = pairs[i].second;
}

// ORACLE_PROGRESS=1: the parallel mode names each finished step on stderr
// (runs on the largest tables take minutes).
void progress(bool parallel, const char *what) {
  static const bool on = getenv("ORACLE_PROGRESS") && getenv("ORACLE_PROGRESS")[0] == '1';
  if (parallel && on) {
    fprintf(stderr, "oracle: %s\n", what);
    fflush(stderr);
  }
}

struct SerialSort {
  static constexpr bool parallel = false;
  template <class It> void operator()(It b, It e) const { std::sort(b, e); }
};
struct ParallelSort {
  static constexpr bool parallel = true;
  template <class It> void operator()(It b, It e) const { __gnu_parallel::sort(b, e); }
};

// Returns 0 on success, 1 on invalid arguments, 2 when V > 2^31 - 1,
// 3 when host memory runs out.  On success *handle owns the result.
template <class Sort>
int table_to_graph(const int64_t *src, const int64_t *dst, int64_t n, void **handle,
                   int64_t *num_nodes, int64_t *num_edges, Sort sort) {
  if (!handle || !num_nodes || !num_edges || n < 0 || n > INT32_MAX) return 1;
  if (n > 0 && (!src || !dst)) return 1;
  *handle = nullptr;
  try {
    OracleGraph *g = new OracleGraph();
    // Node set: copy both columns, sort the copy, keep distinct values.
    std::vector<int64_t> all;
    all.reserve((size_t)2 * n);
    all.insert(all.end(), src, src + n);
    all.insert(all.end(), dst, dst + n);
    sort(all.begin(), all.end());
    progress(Sort::parallel, "node keys sorted");
    all.erase(std::unique(all.begin(), all.end()), all.end());
    g->nodes.swap(all);
    const int64_t V = (int64_t)g->nodes.size();
    if (V > INT32_MAX) {
      delete g;
      return 2;
    }
    auto index_of = [&](int64_t id) {
      return (int32_t)(std::lower_bound(g->nodes.begin(), g->nodes.end(), id) - g->nodes.begin());
    };
    // Edge set: one (source index, destination index) pair per row, sorted,
    // repeated pairs removed.
    std::vector<std::pair<int32_t, int32_t>> e((size_t)n);
    // (each row's lookup is independent: the parallel mode spreads the rows
    // over the host threads, in eight slices, which gives the same pairs)
    for (int part = 0; part < 8; ++part) {
      const int64_t r0 = n * part / 8, r1 = n * (part + 1) / 8;
#pragma omp parallel for schedule(static) if (Sort::parallel)
      for (int64_t r = r0; r < r1; ++r) e[(size_t)r] = {index_of(src[r]), index_of(dst[r])};
      progress(Sort::parallel, "an eighth of the rows looked up");
    }
    sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    progress(Sort::parallel, "edges sorted");
    build_direction(e, V, g->out_off, g->out_nbr);
    // In-direction: the same edges keyed by destination.
    for (auto &p : e) std::swap(p.first, p.second);
    sort(e.begin(), e.end());
    build_direction(e, V, g->in_off, g->in_nbr);
    progress(Sort::parallel, "in-direction built");
    *num_nodes = V;
    *num_edges = (int64_t)e.size();
    *handle = g;
    return 0;
  } catch (const std::bad_alloc &) {
    return 3;
  }
}

}  // namespace

extern "C" {

int oracle_table_to_graph(const int64_t *src, const int64_t *dst, int64_t n, void **handle,
                          int64_t *num_nodes, int64_t *num_edges) {
  return table_to_graph(src, dst, n, handle, num_nodes, num_edges, SerialSort());
}

// The same on all host threads (timing only); returns the thread count
// used in *threads.
int oracle_table_to_graph_par(const int64_t *src, const int64_t *dst, int64_t n, void **handle,
                              int64_t *num_nodes, int64_t *num_edges, int32_t *threads) {
  if (threads) *threads = omp_get_max_threads();
  return table_to_graph(src, dst, n, handle, num_nodes, num_edges, ParallelSort());
}

// Copies the result into caller-owned arrays of sizes V, V+1, E, V+1, E.
void oracle_copy(const void *handle, int64_t *nodes, int64_t *out_off, int32_t *out_nbr,
                 int64_t *in_off, int32_t *in_nbr) {
  const OracleGraph *g = (const OracleGraph *)handle;
  std::copy(g->nodes.begin(), g->nodes.end(), nodes);
  std::copy(g->out_off.begin(), g->out_off.end(), out_off);
  std::copy(g->out_nbr.begin(), g->out_nbr.end(), out_nbr);
  std::copy(g->in_off.begin(), g->in_off.end(), in_off);
  std::copy(g->in_nbr.begin(), g->in_nbr.end(), in_nbr);
}

// kind 0: as oracle_table_to_graph; 1: undirected; 2: multigraph (see the
// header).  Same return codes.
int oracle_table_to_graph_kind(const int64_t *src, const int64_t *dst, int64_t n, int kind,
                               void **handle, int64_t *num_nodes, int64_t *num_edges) {
  if (kind == 0) return oracle_table_to_graph(src, dst, n, handle, num_nodes, num_edges);
  if (kind != 1 && kind != 2) return 1;
  if (!handle || !num_nodes || !num_edges || n < 0 || n > INT32_MAX) return 1;
  if (n > 0 && (!src || !dst)) return 1;
  *handle = nullptr;
  try {
    OracleGraph *g = new OracleGraph();
    std::vector<int64_t> ids(src, src + n);
    ids.insert(ids.end(), dst, dst + n);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    g->nodes.swap(ids);
    const int64_t V = (int64_t)g->nodes.size();
    if (V > INT32_MAX) {
      delete g;
      return 2;
    }
    auto index_of = [&](int64_t id) {
      return (int32_t)(std::lower_bound(g->nodes.begin(), g->nodes.end(), id) - g->nodes.begin());
    };
    if (kind == 1) {
      // both orientations of every row, sorted, repeats removed
      std::vector<std::pair<int32_t, int32_t>> both;
      both.reserve((size_t)2 * n);
      for (int64_t r = 0; r < n; ++r) {
        const int32_t s = index_of(src[r]), d = index_of(dst[r]);
        both.push_back({s, d});
        both.push_back({d, s});
      }
      std::sort(both.begin(), both.end());
      both.erase(std::unique(both.begin(), both.end()), both.end());
      build_direction(both, V, g->out_off, g->out_nbr);
      g->in_off = g->out_off;
      g->in_nbr = g->out_nbr;
      *num_edges = (int64_t)both.size();
    } else {
      // every row an edge: (source, destination, row), then (destination, source, row)
      std::vector<Triple> t3((size_t)n);
      for (int64_t r = 0; r < n; ++r) t3[(size_t)r] = {index_of(src[r]), index_of(dst[r]), (int32_t)r};
      std::sort(t3.begin(), t3.end());
      build_direction_rows(t3, V, g->out_off, g->out_nbr, g->out_eid);
      for (auto &x : t3) std::swap(x.owner, x.nbr);
      std::sort(t3.begin(), t3.end());
      build_direction_rows(t3, V, g->in_off, g->in_nbr, g->in_eid);
      *num_edges = n;
    }
    *num_nodes = V;
    *handle = g;
    return 0;
  } catch (const std::bad_alloc &) {
    return 3;
  }
}

// Multigraph row indices (arrays of E), after oracle_table_to_graph_kind(2).
void oracle_copy_eids(const void *handle, int32_t *out_eid, int32_t *in_eid) {
  const OracleGraph *g = (const OracleGraph *)handle;
  std::copy(g->out_eid.begin(), g->out_eid.end(), out_eid);
  std::copy(g->in_eid.begin(), g->in_eid.end(), in_eid);
}

void oracle_free(void *handle) { delete (OracleGraph *)handle; }

}  // extern "C"
