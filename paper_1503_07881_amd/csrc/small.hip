// Small tables converted entirely in LDS by one workgroup.
//
// The same conversion as the pass pipeline (Section 2.4: copy the two
// columns, sort the copies, count neighbours, place the sorted lists), for a
// table of at most SMALL_ROWS rows, by one 1024-thread workgroup that keeps
// everything in LDS:
//
//   node keys   2n keys uint64(id) ^ 2^63, bitonic sort (Batcher 1968)
//   unique      head flags + block scan -> sorted distinct nodes, node_ids
//   remap       binary search of every row's src and dst -> (s << 32) | d
//   edges       bitonic sort, head flags + block scan -> distinct edges,
//               out_nbrs and out_offsets (boundary fill)
//   in          (d << 32) | s of the distinct edges, bitonic sort,
//               in_nbrs and in_offsets
//
// One launch covers any number of small tables (one workgroup each), and a
// lone small table costs one launch and one read-back instead of the
// pipeline's many passes.  Outputs go to arrays sized for the worst case
// (V <= 2n, E <= n); V and E are written to vres[2i] and vres[2i+1].

#include "device_common.h"
#include "ringo_internal.h"

namespace ringo {

namespace {

constexpr int SB = 1024;  // threads per workgroup
constexpr int SB_WAVES = SB / 64;

// Ascending bitonic sort of s[0, p) (p a power of two), all threads.
__device__ void bitonic_sort(uint64_t *s, int p) {
  for (int k = 2; k <= p; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < p / 2; t += SB) {
        // the t-th pair (i, i + j) with i's bit j clear
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int l = i + j;
        const uint64_t a = s[i], b = s[l];
        const bool up = (i & k) == 0;
        if ((a > b) == up) {
          s[i] = b;
          s[l] = a;
        }
      }
      __syncthreads();
    }
  }
}

__host__ __device__ inline int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Head flags of s[0, cnt) under `same`, compacted into out[0, total); returns
// the total.  Each thread takes SMALL_PER consecutive elements.
constexpr int SMALL_PER = 2 * SMALL_ROWS / SB;

template <class Same>
__device__ int compact_heads(const uint64_t *s, int cnt, uint64_t *out, uint32_t *s_w,
                             Same same) {
  const int i0 = threadIdx.x * SMALL_PER;
  uint32_t mine = 0;
  for (int i = i0; i < i0 + SMALL_PER && i < cnt; ++i) mine += (i == 0 || !same(s[i - 1], s[i]));
  uint32_t total;
  uint32_t pos = block_excl_scan<SB>(mine, s_w, total);
  for (int i = i0; i < i0 + SMALL_PER && i < cnt; ++i)
    if (i == 0 || !same(s[i - 1], s[i])) out[pos++] = s[i];
  __syncthreads();
  return (int)total;
}

}  // namespace

__global__ __launch_bounds__(SB) void k_small_convert(const SmallTable *tabs, int64_t *vres) {
  __shared__ uint64_t s_a[2 * SMALL_ROWS];  // node keys, later the distinct edges
  __shared__ uint64_t s_n[2 * SMALL_ROWS];  // distinct nodes
  __shared__ uint64_t s_e[SMALL_ROWS];      // edge keys, later the in-keys
  __shared__ uint32_t s_w[SB_WAVES];
  const SmallTable T = tabs[blockIdx.x];
  const int n = (int)T.n;
  const int tid = threadIdx.x;

  // node keys
  const int pn = pow2_at_least(2 * n);
  for (int i = tid; i < pn; i += SB) {
    uint64_t k = ~0ull;  // padding sorts last; equal real keys are interchangeable
    if (i < n) k = (uint64_t)G(T.src)[i] ^ SIGN_FLIP;
    else if (i < 2 * n) k = (uint64_t)G(T.dst)[i - n] ^ SIGN_FLIP;
    s_a[i] = k;
  }
  __syncthreads();
  bitonic_sort(s_a, pn);
  const int V = compact_heads(s_a, 2 * n, s_n, s_w, [](uint64_t x, uint64_t y) { return x == y; });
  for (int v = tid; v < V; v += SB) G(T.node_ids)[v] = (int64_t)(s_n[v] ^ SIGN_FLIP);

  // remap: position of every row's src and dst among the nodes
  auto rank_of = [&](uint64_t key) {
    int lo = 0, hi = V;  // first position with node >= key (the key is present)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_n[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (uint64_t)lo;
  };
  const int pe = pow2_at_least(n);
  for (int r = tid; r < pe; r += SB) {
    uint64_t k = ~0ull;
    if (r < n) {
      const uint64_t s = rank_of((uint64_t)G(T.src)[r] ^ SIGN_FLIP);
      const uint64_t d = rank_of((uint64_t)G(T.dst)[r] ^ SIGN_FLIP);
      k = (s << 32) | d;
    }
    s_e[r] = k;
  }
  __syncthreads();
  bitonic_sort(s_e, pe);
  // distinct edges, into s_a (the node keys are no longer needed)
  const int E = compact_heads(s_e, n, s_a, s_w, [](uint64_t x, uint64_t y) { return x == y; });

  // out-CSR: out_off[v] = first position whose source is >= v
  for (int j = tid; j < E; j += SB) {
    const uint64_t k = s_a[j];
    const int64_t s = (int64_t)(k >> 32);
    G(T.out_nbr)[j] = (int32_t)(uint32_t)k;
    const int64_t hp = j == 0 ? -1 : (int64_t)(s_a[j - 1] >> 32);
    for (int64_t v = hp + 1; v <= s; ++v) G(T.out_off)[v] = j;
    if (j == E - 1)
      for (int64_t v = s + 1; v <= V; ++v) G(T.out_off)[v] = E;
  }
  // in-keys (d << 32) | s of the distinct edges
  const int pi = pow2_at_least(E);
  for (int j = tid; j < pi; j += SB) {
    uint64_t k = ~0ull;
    if (j < E) {
      const uint64_t x = s_a[j];
      k = (x << 32) | (x >> 32);
    }
    s_e[j] = k;
  }
  __syncthreads();
  bitonic_sort(s_e, pi);
  for (int j = tid; j < E; j += SB) {
    const uint64_t k = s_e[j];
    const int64_t d = (int64_t)(k >> 32);
    G(T.in_nbr)[j] = (int32_t)(uint32_t)k;
    const int64_t hp = j == 0 ? -1 : (int64_t)(s_e[j - 1] >> 32);
    for (int64_t v = hp + 1; v <= d; ++v) G(T.in_off)[v] = j;
    if (j == E - 1)
      for (int64_t v = d + 1; v <= V; ++v) G(T.in_off)[v] = E;
  }
  if (tid == 0) {
    vres[2 * blockIdx.x] = V;
    vres[2 * blockIdx.x + 1] = E;
  }
}

hipError_t launch_small(const SmallTable *tabs, int count, int64_t *vres, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_convert, dim3(count), dim3(SB), 0, s, tabs, vres);
  return hipGetLastError();
}

}  // namespace ringo
