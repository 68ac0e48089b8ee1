// PageRank on a converted graph: the consumer of the conversion in the
// paper's workflow (a graph built from a table, then its PageRank scores;
// Section 4), timed there over ten iterations (Section 3, Table 3).
//
// Definition (Page, Brin, Motwani & Winograd 1999), teleport and the mass
// of nodes without out-edges both spread uniformly, in fp64:
//   r_0[v]     = 1 / V
//   r_{t+1}[v] = (1 - d) / V + d * (sum over edges u -> v of r_t[u] / outdeg(u)
//                                   + D_t / V)
//   D_t        = sum of r_t[u] over nodes u with outdeg(u) = 0
//
// One iteration is a pull over the in-CSR:
//   contrib   contrib[u] = r[u] / outdeg(u) (0 without out-edges), and a
//             per-block partial sum of the dangling mass
//   dsum      the partial sums added in a fixed order -> D_t
//   pull      merge-path split (Merrill & Garland 2016, merge-based SpMV) of
//             the node ends in_off[1..V] against the in-edges: every tile
//             takes the same number of nodes + edges; inside the tile each
//             thread sums its share of the neighbour contributions, a walk
//             back over the threads' partial sums finishes the nodes that
//             straddle threads, and nodes that straddle tiles leave partial
//             sums for
//   fixup     which finishes each of them by walking back over the tiles.
// Every sum runs in an order fixed by the tiling, so results are the same
// bit for bit from run to run.

#include <stdint.h>

#include <algorithm>

#include "device_common.h"
#include "ringo.h"
#include "ringo_internal.h"

namespace ringo {
namespace {

constexpr int PR_BLOCK = 256;
constexpr int PR_ITEMS = 8;
constexpr int PR_TILE = PR_BLOCK * PR_ITEMS;  // merge items (node ends + edges) per tile
constexpr int PR_DPARTS = 1024;               // blocks of the contribution kernel

__global__ __launch_bounds__(256) void k_pr_init(double *r, int64_t V) {
  const double x = 1.0 / (double)V;
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256)
    G(r)[v] = x;
}

// Block sum of one double per thread, fixed order (wave shuffles, then waves).
__device__ double block_sum(double x, double *s_w) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) s_w[w] = x;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)blockDim.x / 64; ++i) t += s_w[i];
  __syncthreads();
  return t;  // valid in thread 0
}

__global__ __launch_bounds__(256) void k_pr_contrib(const int64_t *out_off, const double *r,
                                                    double *contrib, double *dpart, int64_t V) {
  __shared__ double s_w[4];
  double dang = 0;
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < V; u += (int64_t)gridDim.x * 256) {
    const int64_t deg = G(out_off)[u + 1] - G(out_off)[u];
    const double x = G(r)[u];
    if (deg > 0) {
      G(contrib)[u] = x / (double)deg;
    } else {
      G(contrib)[u] = 0.0;
      dang += x;
    }
  }
  const double t = block_sum(dang, s_w);
  if (threadIdx.x == 0) dpart[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_pr_dsum(const double *dpart, int n, double *dsum) {
  __shared__ double s_w[4];
  double x = 0;
  for (int i = threadIdx.x; i < n; i += 256) x += dpart[i];
  const double t = block_sum(x, s_w);
  if (threadIdx.x == 0) *dsum = t;
}

__device__ int64_t merge_split_global(const int64_t *in_off, int64_t V, int64_t E, int64_t d) {
  int64_t lo = std::max<int64_t>(0, d - E), hi = std::min<int64_t>(d, V);
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (G(in_off)[mid + 1] <= d - mid - 1) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct PrParams {
  const int64_t *in_off;
  const int32_t *in_nbr;
  const double *contrib;
  const double *dsum;
  double *r_new;
  int64_t V, E;
  double damping;
  int64_t *carry_node;  // [tiles] node finishing in the tile but begun before it, or -1
  double *carry_part;   // [tiles] its sum over the tile's items
  double *tail_part;    // [tiles] sum of the items after the tile's last node end
  int32_t *has_end;     // [tiles] whether any node ends in the tile
};

__device__ __forceinline__ double pr_value(const PrParams &p, double s, double dangling) {
  const double Vd = (double)p.V;
  return (1.0 - p.damping) / Vd + p.damping * (s + dangling / Vd);
}

__global__ __launch_bounds__(PR_BLOCK) void k_pr_pull(PrParams p) {
  __shared__ int64_t s_end[PR_TILE];
  __shared__ double s_x[PR_TILE];
  __shared__ double s_tail[PR_BLOCK];
  __shared__ int32_t s_flag[PR_BLOCK];
  __shared__ int64_t s_split[2];
  const int tid = threadIdx.x;
  const int64_t total = p.V + p.E;
  const int64_t tiles = (total + PR_TILE - 1) / PR_TILE;
  const double dangling = *p.dsum;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t d0 = tile * PR_TILE;
    const int64_t d1 = std::min<int64_t>(d0 + PR_TILE, total);
    if (tid < 2) s_split[tid] = merge_split_global(p.in_off, p.V, p.E, tid == 0 ? d0 : d1);
    __syncthreads();
    const int64_t i0 = s_split[0], i1 = s_split[1];
    const int64_t j0 = d0 - i0, j1 = d1 - i1;
    const int ni = (int)(i1 - i0), nj = (int)(j1 - j0);
    for (int k = tid; k < ni; k += PR_BLOCK) s_end[k] = G(p.in_off)[i0 + k + 1];
    for (int k = tid; k < nj; k += PR_BLOCK) s_x[k] = G(p.contrib)[G(p.in_nbr)[j0 + k]];
    __syncthreads();
    const int dl = std::min(tid * PR_ITEMS, ni + nj);
    int lo = std::max(0, dl - nj), hi = std::min(dl, ni);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_end[mid] <= j0 + (dl - mid - 1)) lo = mid + 1; else hi = mid;
    }
    int i = lo, j = dl - lo;
    const int steps = std::min(PR_ITEMS, ni + nj - dl);
    double acc = 0, head_sum = 0;
    int head = -1;
    for (int s = 0; s < steps; ++s) {
      if (i < ni && (j >= nj || s_end[i] <= j0 + j)) {
        if (head < 0) {
          head = i;
          head_sum = acc;
        } else {
          G(p.r_new)[i0 + i] = pr_value(p, acc, dangling);  // all its edges are this thread's
        }
        acc = 0;
        ++i;
      } else {
        acc += s_x[j];
        ++j;
      }
    }
    s_tail[tid] = acc;
    s_flag[tid] = head >= 0;
    __syncthreads();
    if (head >= 0) {
      // the head node's earlier edges are the tails of the threads back to
      // (and including) the previous one that saw a node end
      double c = 0;
      int t = tid - 1;
      for (; t >= 0; --t) {
        c += s_tail[t];
        if (s_flag[t]) break;
      }
      const double sum = head_sum + c;
      if (t < 0 && G(p.in_off)[i0] < j0) {  // tile's first node end, node begun in an earlier tile
        p.carry_node[tile] = i0 + head;
        p.carry_part[tile] = sum;
      } else {
        G(p.r_new)[i0 + head] = pr_value(p, sum, dangling);
      }
    }
    if (tid == PR_BLOCK - 1) {
      double c = 0;
      int t = PR_BLOCK - 1;
      for (; t >= 0; --t) {
        c += s_tail[t];
        if (s_flag[t]) break;
      }
      p.tail_part[tile] = c;
      p.has_end[tile] = t >= 0;
    }
    if (tid == 0) {
      // no node finishing here began earlier: mark so the fixup skips the tile
      bool begun_before = false;
      for (int t = 0; t < PR_BLOCK; ++t)
        if (s_flag[t]) { begun_before = G(p.in_off)[i0] < j0; break; }
      if (!begun_before) p.carry_node[tile] = -1;
    }
    __syncthreads();
  }
}

// Nodes whose in-edges straddle tiles: the tile where the node ends holds
// the partial sum of its last part; every earlier tile back to (and
// including) the one where it begins adds its tail sum.
__global__ __launch_bounds__(256) void k_pr_fixup(PrParams p, int64_t tiles) {
  const double dangling = *p.dsum;
  for (int64_t tile = (int64_t)blockIdx.x * 256 + threadIdx.x; tile < tiles;
       tile += (int64_t)gridDim.x * 256) {
    const int64_t v = p.carry_node[tile];
    if (v < 0) continue;
    double s = p.carry_part[tile];
    for (int64_t t = tile - 1; t >= 0; --t) {
      s += p.tail_part[t];
      if (p.has_end[t]) break;
    }
    G(p.r_new)[v] = pr_value(p, s, dangling);
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

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace
}  // namespace ringo

using namespace ringo;

extern "C" ringo_status_t ringo_pagerank(const ringo_graph_t *g, double damping, int32_t iterations,
                                         double *ranks, hipStream_t stream) {
  if (!g || g->num_nodes < 0 || g->num_edges < 0 || iterations < 0 || !(damping >= 0.0) ||
      !(damping <= 1.0))
    return RINGO_ERR_INVALID_ARG;
  const int64_t V = g->num_nodes, E = g->num_edges;
  if (V == 0) return RINGO_OK;
  if (!ranks || !g->out_offsets || !g->in_offsets || (E > 0 && !g->in_nbrs))
    return RINGO_ERR_INVALID_ARG;
  const int64_t tiles = (V + E + PR_TILE - 1) / PR_TILE;
  const size_t b_r = align256(sizeof(double) * V);
  const size_t b_dp = align256(sizeof(double) * (PR_DPARTS + 1));
  const size_t b_t = align256(sizeof(int64_t) * tiles);
  const size_t bytes = 2 * b_r + b_dp + 4 * b_t;
  char *ws = (char *)workspace_alloc(bytes, stream);
  if (!ws) return RINGO_ERR_OUT_OF_MEMORY;
  double *tmp = (double *)ws;
  double *contrib = (double *)(ws + b_r);
  double *dpart = (double *)(ws + 2 * b_r);
  double *dsum = dpart + PR_DPARTS;
  PrParams p;
  p.in_off = g->in_offsets;
  p.in_nbr = g->in_nbrs;
  p.contrib = contrib;
  p.dsum = dsum;
  p.V = V;
  p.E = E;
  p.damping = damping;
  p.carry_node = (int64_t *)(ws + 2 * b_r + b_dp);
  p.carry_part = (double *)(ws + 2 * b_r + b_dp + b_t);
  p.tail_part = (double *)(ws + 2 * b_r + b_dp + 2 * b_t);
  p.has_end = (int32_t *)(ws + 2 * b_r + b_dp + 3 * b_t);

  // ping-pong so that the last iteration writes `ranks`
  double *buf[2] = {ranks, tmp};
  const int node_grid = (int)std::min<int64_t>((V + 255) / 256, PR_DPARTS);
  const int pull_grid = (int)std::min<int64_t>(tiles, (int64_t)cu_count() * 8);
  const int fix_grid = (int)std::min<int64_t>((tiles + 255) / 256, 1024);
  hipLaunchKernelGGL(k_pr_init, dim3(node_grid), dim3(256), 0, stream, buf[iterations & 1], V);
  for (int it = 0; it < iterations; ++it) {
    const double *r = buf[(iterations - it) & 1];
    p.r_new = buf[(iterations - it - 1) & 1];
    hipLaunchKernelGGL(k_pr_contrib, dim3(PR_DPARTS), dim3(256), 0, stream, g->out_offsets, r,
                       contrib, dpart, V);
    hipLaunchKernelGGL(k_pr_dsum, dim3(1), dim3(256), 0, stream, dpart, PR_DPARTS, dsum);
    hipLaunchKernelGGL(k_pr_pull, dim3(pull_grid), dim3(PR_BLOCK), 0, stream, p);
    hipLaunchKernelGGL(k_pr_fixup, dim3(fix_grid), dim3(256), 0, stream, p, tiles);
  }
  const hipError_t e = hipGetLastError();
  workspace_free(ws, stream);
  return e == hipSuccess ? RINGO_OK : RINGO_ERR_HIP;
}
