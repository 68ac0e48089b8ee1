// Graph-to-table conversion (Section 2.4, "Conversion of graphs to tables").
//
// The paper splits the nodes or edges of the graph among workers, allocates
// the output table up front, and lets every worker fill its own part.  On the
// GPU the edge table is one load-balanced pass over the out-CSR:
//
//   edge table  row i = (node_ids[source of edge i], node_ids[out_nbrs[i]]),
//               edges in out-CSR order, i.e. (source, destination) ascending
//   node table  row v = (node_ids[v], out-degree, in-degree)
//
// The source of every edge comes from a merge-path split (Green, McColl &
// Bader 2012) of the sequence of node ends out_off[1..V] against the edge
// positions 0..E-1: every tile of the merge takes the same number of items
// (nodes + edges), so hubs and runs of zero-degree nodes cost the same as
// anything else.  Each tile finds its two end points by binary search over
// the whole offsets array, stages its part of the offsets in LDS, and each
// thread merges its own share of the tile there.  Sources land in LDS and
// the tile writes both columns with coalesced stores.

#include <stdint.h>

#include <algorithm>

#include "device_common.h"
#include "ringo.h"

namespace ringo {
namespace {

constexpr int TT_BLOCK = 256;
constexpr int TT_ITEMS = 8;
constexpr int TT_TILE = TT_BLOCK * TT_ITEMS;  // merge items (nodes + edges) per tile

// End of node i's out-range (the i-th entry of the merged node sequence).
__device__ __forceinline__ int64_t node_end(const int64_t *out_off, int64_t i) {
  return G(out_off)[i + 1];
}

// Merge-path split of diagonal d: the number i of node ends that precede the
// (d - i)-th edge position, node ends first on ties (a node whose range ends
// at position j is finished before edge j).
__device__ int64_t merge_split_global(const int64_t *out_off, int64_t V, int64_t E, int64_t d) {
  int64_t lo = std::max<int64_t>(0, d - E), hi = std::min<int64_t>(d, V);
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (node_end(out_off, mid) <= d - mid - 1) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(TT_BLOCK) void k_edge_table(const int64_t *node_ids,
                                                         const int64_t *out_off,
                                                         const int32_t *out_nbr, int64_t V,
                                                         int64_t E, int64_t *src_ids,
                                                         int64_t *dst_ids) {
  __shared__ int64_t s_end[TT_TILE];   // node ends of the tile
  __shared__ int32_t s_src[TT_TILE];   // source (node index - i0) of each edge of the tile
  __shared__ int64_t s_split[2];
  const int tid = threadIdx.x;
  const int64_t total = V + E;
  const int64_t tiles = (total + TT_TILE - 1) / TT_TILE;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t d0 = tile * TT_TILE;
    const int64_t d1 = std::min<int64_t>(d0 + TT_TILE, total);
    if (tid < 2) s_split[tid] = merge_split_global(out_off, V, E, tid == 0 ? d0 : d1);
    __syncthreads();
    const int64_t i0 = s_split[0], i1 = s_split[1];
    const int64_t j0 = d0 - i0, j1 = d1 - i1;
    const int ni = (int)(i1 - i0), nj = (int)(j1 - j0);
    for (int k = tid; k < ni; k += TT_BLOCK) s_end[k] = node_end(out_off, i0 + k);
    __syncthreads();
    // this thread's diagonal inside the tile, split in LDS
    const int dl = std::min(tid * TT_ITEMS, ni + nj);
    int lo = std::max(0, dl - nj), hi = std::min(dl, ni);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_end[mid] <= j0 + (dl - mid - 1)) lo = mid + 1; else hi = mid;
    }
    int i = lo, j = dl - lo;
    const int steps = std::min(TT_ITEMS, ni + nj - dl);
    for (int s = 0; s < steps; ++s) {
      if (i < ni && (j >= nj || s_end[i] <= j0 + j)) {
        ++i;
      } else {
        s_src[j] = i;  // edge j0 + j belongs to node i0 + i
        ++j;
      }
    }
    __syncthreads();
    for (int k = tid; k < nj; k += TT_BLOCK) {
      const int64_t e = j0 + k;
      G(src_ids)[e] = G(node_ids)[i0 + s_src[k]];
      G(dst_ids)[e] = G(node_ids)[G(out_nbr)[e]];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_node_table(const int64_t *node_ids, const int64_t *out_off,
                                                    const int64_t *in_off, int64_t V, int64_t *ids,
                                                    int64_t *out_deg, int64_t *in_deg) {
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
    if (ids) G(ids)[v] = G(node_ids)[v];
    if (out_deg) G(out_deg)[v] = G(out_off)[v + 1] - G(out_off)[v];
    if (in_deg) G(in_deg)[v] = G(in_off)[v + 1] - G(in_off)[v];
  }
}

int cu_count() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      n = 256;
    return n > 0 ? n : 256;
  }();
  return cus;
}

}  // namespace
}  // namespace ringo

using namespace ringo;

extern "C" ringo_status_t ringo_graph_to_edge_table(const ringo_graph_t *g, int64_t *src_ids,
                                                    int64_t *dst_ids, hipStream_t stream) {
  if (!g || g->num_nodes < 0 || g->num_edges < 0) return RINGO_ERR_INVALID_ARG;
  const int64_t V = g->num_nodes, E = g->num_edges;
  if (E == 0) return RINGO_OK;
  if (!src_ids || !dst_ids || !g->node_ids || !g->out_offsets || !g->out_nbrs || V == 0)
    return RINGO_ERR_INVALID_ARG;
  const int64_t tiles = (V + E + TT_TILE - 1) / TT_TILE;
  const int grid = (int)std::min<int64_t>(tiles, (int64_t)cu_count() * 8);
  hipLaunchKernelGGL(k_edge_table, dim3(grid), dim3(TT_BLOCK), 0, stream, g->node_ids,
                     g->out_offsets, g->out_nbrs, V, E, src_ids, dst_ids);
  return hipGetLastError() == hipSuccess ? RINGO_OK : RINGO_ERR_HIP;
}

extern "C" ringo_status_t ringo_graph_to_node_table(const ringo_graph_t *g, int64_t *node_ids,
                                                    int64_t *out_degree, int64_t *in_degree,
                                                    hipStream_t stream) {
  if (!g || g->num_nodes < 0 || g->num_edges < 0) return RINGO_ERR_INVALID_ARG;
  const int64_t V = g->num_nodes;
  if (V == 0 || (!node_ids && !out_degree && !in_degree)) return RINGO_OK;
  if ((node_ids && !g->node_ids) || (out_degree && !g->out_offsets) ||
      (in_degree && !g->in_offsets))
    return RINGO_ERR_INVALID_ARG;
  const int grid = (int)std::min<int64_t>((V + 255) / 256, (int64_t)cu_count() * 8);
  hipLaunchKernelGGL(k_node_table, dim3(grid), dim3(256), 0, stream, g->node_ids, g->out_offsets,
                     g->in_offsets, V, node_ids, out_degree, in_degree);
  return hipGetLastError() == hipSuccess ? RINGO_OK : RINGO_ERR_HIP;
}
