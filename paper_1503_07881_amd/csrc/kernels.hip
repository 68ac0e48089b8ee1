// gfx950 kernels of the table-to-graph conversion.
//
// The method is the paper's "sort-first" conversion (Converting Between
// Tables and Graphs, Section 2.4): copy the source and destination columns,
// sort the copies, count neighbours per node and place the sorted neighbour
// lists.  On the GPU every step is a tiled, HBM-streaming pass over all
// tables of a batch at once:
//
//   node keys   2n (id ^ 2^63) keys per table, least-significant-digit radix
//               sort, ceil(64 / d) passes of d-bit digits (8 by default)
//   unique      head flags on the sorted keys + stream compaction -> nodes
//   directory   bucket index over the sorted nodes for the remap lookups
//   remap       every row's (src, dst) -> dense positions, packed into
//               (s << b) | d with b = ceil(log2 V)
//   edge keys   radix sort of the packed keys over their 2b low bits
//   in keys     repack to (d << 32) | s, stable radix sort on d only; the
//               first in-pass also drops repeated edges (first copy only)
//               and writes out-neighbours and out-offsets
//   in-CSR      in-neighbours + in-offsets
//   dedupe      adjacent compare + compaction (undirected graphs,
//               multigraph offsets)
//
// (lsd.h holds the radix pass kernels, hash.hip the alternative node
// numbering through a node hash table, small.hip the single-workgroup
// conversion of small tables.)
//
// Each radix pass is a tile-granular reduce-then-scan: an upsweep counts the
// digits of every tile, a scan over tiles turns the counts into per-tile
// digit offsets, and a downsweep ranks every key stably inside its tile with
// 64-lane wavefront ballots and writes each digit run of the tile as one
// contiguous LDS-staged store.  Stream compaction (unique, dedupe) counts
// the heads of every tile, scans the counts, then writes; no block waits on
// another.

#include "device_common.h"
#include "ringo_internal.h"

namespace ringo {

// ------------------------------------------------------------------ fills

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)g), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

// Tables with no rows: both offset arrays are the single value 0.
__global__ void k_empty_offsets(const SegPlan *plan, int32_t S) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) {
    if (plan[i].n == 0) {
      plan[i].out_off[0] = 0;
      plan[i].in_off[0] = 0;
    }
  }
}

// The runs queued by fill_run: one block per chunk of up to GAP_CHUNK units,
// grid-stride over the chunks (their count is read on the device).
__global__ __launch_bounds__(256) void k_gap_fill(const GapEntry *e, const uint32_t *count,
                                                  uint32_t cap) {
  const uint32_t n = std::min(*count, cap);
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const GapEntry g = e[i];
    if (g.words == 2) {
      __attribute__((address_space(1))) u64x2 *p = (__attribute__((address_space(1))) u64x2 *)G(g.dst);
      u64x2 v;
      v.x = g.w0;
      v.y = g.w1;
      for (int64_t u = threadIdx.x; u < g.len; u += 256) p[u] = v;
    } else {
      __attribute__((address_space(1))) uint64_t *p = G(g.dst);
      for (int64_t u = threadIdx.x; u < g.len; u += 256) p[u] = g.w0;
    }
  }
}

hipError_t launch_gap_fill(const GapQueue &q, hipStream_t s) {
  if (!q.e || q.cap == 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<uint32_t>(q.cap, (uint32_t)device_cu_count() * 4);
  hipLaunchKernelGGL(k_gap_fill, dim3(g), dim3(256), 0, s, (const GapEntry *)q.e, (const uint32_t *)q.count,
                     q.cap);
  return hipGetLastError();
}

hipError_t launch_empty_offsets(const SegPlan *plan, int32_t S, hipStream_t s) {
  hipLaunchKernelGGL(k_empty_offsets, dim3((S + 255) / 256), dim3(256), 0, s, plan, S);
  return hipGetLastError();
}

// --------------------------------------------- sync-free single table
//
// A call whose sizes all follow from n (worst-case tile maps, outputs sized
// V <= 2n and E <= n) enqueues every kernel at once: the metadata is
// written by a kernel from its arguments, and V and E pass from the kernels
// that count them into the plan on the device.

__global__ void k_meta_init(MetaWords m, int32_t nwords, uint64_t *dst, int64_t *results,
                            int32_t nres) {
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = m.w[i];
  for (int i = threadIdx.x; i < nres; i += blockDim.x) results[i] = 0;
}

// V (results[0]) into the plan, and the directory's bucket bits from it.
__global__ void k_plan_nodes(SegPlan *plan, const int64_t *results, int32_t dirk_cap) {
  if (threadIdx.x != 0) return;
  const int64_t V = results[0];
  plan->V = V;
  plan->dirk = std::min(V > 0 ? ceil_log2(V) : 0, (int)dirk_cap);
}

// E (results[1]) into the plan; V and E to the caller's pair.
__global__ void k_plan_edges(SegPlan *plan, const int64_t *results, int64_t *ve) {
  if (threadIdx.x != 0) return;
  plan->E = results[1];
  ve[0] = plan->V;
  ve[1] = results[1];
}

// A table with no rows: both offset arrays are {0}, V = E = 0.
__global__ void k_fixed_empty(int64_t *out_off, int64_t *in_off, int64_t *ve) {
  if (threadIdx.x != 0) return;
  out_off[0] = 0;
  in_off[0] = 0;
  ve[0] = 0;
  ve[1] = 0;
}

hipError_t launch_meta_init(const MetaWords &m, int32_t nwords, uint64_t *dst, int64_t *results,
                            int32_t nres, hipStream_t s) {
  if (nwords < 0 || nwords > META_WORDS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_meta_init, dim3(1), dim3(64), 0, s, m, nwords, dst, results, nres);
  return hipGetLastError();
}

const void *meta_init_kernel() { return reinterpret_cast<const void *>(&k_meta_init); }

hipError_t launch_plan_nodes(SegPlan *plan, const int64_t *results, int32_t dirk_cap,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_plan_nodes, dim3(1), dim3(64), 0, s, plan, results, dirk_cap);
  return hipGetLastError();
}

hipError_t launch_plan_edges(SegPlan *plan, const int64_t *results, int64_t *ve, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_edges, dim3(1), dim3(64), 0, s, plan, results, ve);
  return hipGetLastError();
}

hipError_t launch_fixed_empty(int64_t *out_off, int64_t *in_off, int64_t *ve, hipStream_t s) {
  hipLaunchKernelGGL(k_fixed_empty, dim3(1), dim3(64), 0, s, out_off, in_off, ve);
  return hipGetLastError();
}

// ------------------------------------------------------------ LSD pass
//
// The pass kernels are in lsd.h, one translation unit per digit width.

int sort_tile(int items) { return 256 * items; }

int64_t sort_runs(int64_t tiles) {
  const int rt = run_tiles_for(tiles);
  return (tiles + rt - 1) / rt;
}

// Upper bound of sort_runs(t) over t <= max_tiles: below 2^16 tiles there
// are at most 4096 runs, above it every run holds 32 tiles.
int64_t sort_runs_bound(int64_t max_tiles) {
  return std::max<int64_t>(4096, (max_tiles + 31) / 32) + 1;
}

hipError_t launch_sort_part(const SortLaunch &a, int mode, int items, int digit_bits, int parts,
                            hipStream_t s) {
  if (a.total_tiles == 0) return hipSuccess;
  switch (digit_bits) {
    case 8: return launch_sort_part_rb<8>(a, mode, items, parts, s);
    case 9: return launch_sort_part_rb<9>(a, mode, items, parts, s);
    case 10: return launch_sort_part_rb<10>(a, mode, items, parts, s);
    case 11: return launch_sort_part_rb<11>(a, mode, items, parts, s);
    default: return hipErrorInvalidValue;
  }
}


// ------------------------------------------------------ unique (node set)
//
// Head flags on the sorted node keys, stream compaction of the heads into
// the node list, per-table node count: launch_unique, with the compaction
// kernels of the dedupe section below.

// ------------------------------------------------------- node directory
//
// Bucket index over the sorted node keys of a table: bucket q holds the
// keys whose (key - lo) >> shift equals q, with 2^dirk buckets (about one
// key per bucket for spread-out identifiers).  Entry q holds the bucket's
// first key and its position range [start, next), so a lookup whose key is
// the first of its bucket costs one 16-byte read.  The same pass writes the
// node identifiers of the output.

__device__ __forceinline__ int dir_shift(uint64_t lo, uint64_t hi, int dirk) {
  const uint64_t range = hi - lo;
  const int bits = range == 0 ? 0 : 64 - __clzll((long long)range);
  return bits > dirk ? bits - dirk : 0;
}

__global__ __launch_bounds__(256) void k_dir(TileLaunch t, const uint64_t *nodes, DirEntry *dir) {
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint64_t *nd = nodes + 2 * P.row_off;
    const uint64_t lo = nd[0], hi = nd[P.V - 1];
    const int shift = dir_shift(lo, hi, P.dirk);
    __attribute__((address_space(1))) DirEntry *D = G(dir + P.dir_off);
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)DIR_TILE;
    const int64_t end = std::min<int64_t>(base + DIR_TILE, P.V);
    for (int64_t j = base + threadIdx.x; j < end; j += 256) {
      const uint64_t u = nd[j];
      G(P.node_ids)[j] = (int64_t)(u ^ SIGN_FLIP);
      const int64_t q = (int64_t)((u - lo) >> shift);
      const int64_t qp = j == 0 ? -1 : (int64_t)((nd[j - 1] - lo) >> shift);
      const int64_t qn = j == P.V - 1 ? ((int64_t)1 << P.dirk) + 1 : (int64_t)((nd[j + 1] - lo) >> shift);
      if (q != qp) {  // first key of bucket q; the buckets skipped before it are empty
        // {key 0, start j, next j} for each of them
        fill_run(t.gaps, (uint64_t *)(dir + P.dir_off + qp + 1), q - qp - 1, 0,
                 (uint64_t)(uint32_t)j | ((uint64_t)(uint32_t)j << 32), 2);
        D[q].key = u;
        D[q].start = (uint32_t)j;
      }
      if (q != qn) {  // last key of bucket q
        D[q].next = (uint32_t)(j + 1);
        if (j == P.V - 1) {
          const int64_t nb = (int64_t)1 << P.dirk;
          fill_run(t.gaps, (uint64_t *)(dir + P.dir_off + q + 1), nb - q, 0,
                   (uint64_t)(uint32_t)P.V | ((uint64_t)(uint32_t)P.V << 32), 2);
        }
      }
    }
  }
}

hipError_t launch_dir(const TileLaunch &t, const uint64_t *nodes, DirEntry *dir, int grid,
                      hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dir, dim3(grid), dim3(256), 0, s, t, nodes, dir);
  return hipGetLastError();
}

// ---------------------------------------------------------------- remap
//
// Dense position of every row's source and destination (merge-rank against
// the sorted node list through the bucket directory), packed into the edge
// key (s << b) | d.  Keys that open their bucket are found by the directory
// read alone; the others by a binary search inside the bucket.  All keys of
// a thread advance together so that their loads overlap.

template <int K>
__device__ __forceinline__ void node_rank_n(const uint64_t *nd, const DirEntry *D, uint64_t lo,
                                            int shift, uint64_t nbuckets, const uint64_t *u,
                                            uint32_t *rank) {
  uint32_t a[K], e[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    uint64_t q = (u[j] - lo) >> shift;
    if (q >= nbuckets) q = nbuckets - 1;  // only for keys outside the table's range
    // one 16-byte load: {key, start | next << 32}
    const u64x2 de = G((const u64x2 *)(D + q))[0];
    const uint32_t start = (uint32_t)de.y, next = (uint32_t)(de.y >> 32);
    a[j] = start;
    e[j] = de.x == u[j] ? start + 1 : next;
  }
  bool more = true;
  while (more) {
    more = false;
    uint32_t m[K];
    uint64_t x[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      m[j] = (a[j] + e[j]) >> 1;
      // unconditional load (finished searches read node 0, always present)
      x[j] = G(nd)[e[j] - a[j] > 1 ? m[j] : 0u];
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (e[j] - a[j] > 1) {
        if (x[j] <= u[j]) a[j] = m[j]; else e[j] = m[j];
        more |= e[j] - a[j] > 1;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) rank[j] = a[j];
}

__global__ __launch_bounds__(256) void k_remap(TileLaunch t, const uint64_t *nodes,
                                               const DirEntry *dir, uint64_t *ekeys, int sym) {
  const int tid = threadIdx.x;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint64_t *nd = nodes + 2 * P.row_off;
    const uint64_t lo = nd[0], hi = nd[P.V - 1];
    const int shift = dir_shift(lo, hi, P.dirk);
    const DirEntry *D = dir + P.dir_off;
    const uint64_t nb = 1ull << P.dirk;
    const int b = P.b;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)REMAP_TILE;
    const int64_t end = std::min<int64_t>(base + REMAP_TILE, P.n);
    constexpr int U = 4;  // rows per thread in flight
    for (int64_t r0 = base + tid; r0 < end; r0 += U * 256) {
      uint64_t u[2 * U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int64_t r = std::min<int64_t>(r0 + j * 256, end - 1);
        u[j] = (uint64_t)G(P.src)[r] ^ SIGN_FLIP;
        u[U + j] = (uint64_t)G(P.dst)[r] ^ SIGN_FLIP;
      }
      uint32_t rk[2 * U];
      node_rank_n<2 * U>(nd, D, lo, shift, nb, u, rk);
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (r0 + j * 256 < end) {
          if (sym) {
            G(ekeys)[2 * P.row_off + r0 + j * 256] = ((uint64_t)rk[j] << b) | rk[U + j];
            G(ekeys)[2 * P.row_off + P.n + r0 + j * 256] = ((uint64_t)rk[U + j] << b) | rk[j];
          } else {
            G(ekeys)[P.row_off + r0 + j * 256] = ((uint64_t)rk[j] << b) | rk[U + j];
          }
        }
    }
  }
}

hipError_t launch_remap(const TileLaunch &t, const uint64_t *nodes, const DirEntry *dir,
                        uint64_t *ekeys, int sym, int grid, hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_remap, dim3(grid), dim3(256), 0, s, t, nodes, dir, ekeys, sym);
  return hipGetLastError();
}

// --------------------------------------------------------------- dedupe
//
// Adjacent compare of the sorted edge keys, compaction of the first copy of
// every edge, and out-offsets by boundary fill (out_off[v] = position of
// the first edge whose source is >= v).
//
// Undirected graphs: the sorted keys of both orientations keep the first
// copy of every key (stream compaction) and give the out-offsets, in three
// launches: head counts per tile, one scan over the tiles, then the
// compacted keys and the offsets (each tile recomputes its heads).  Tiles
// never wait on each other; a single pass with decoupled look-back was
// slower on this device.

// Keys of ITEMS rows of a tile (row i = keys i * BLOCK + tid, coalesced),
// each key's predecessor (from the lane below; lane 0 loads its own), and
// the ballot of the heads (first copies) of every row.
__device__ __forceinline__ void dedupe_heads(const uint64_t *in, int64_t start, int64_t base,
                                             int cnt, uint64_t k[SCAN_ITEMS],
                                             uint64_t kp[SCAN_ITEMS],
                                             uint64_t heads[SCAN_ITEMS]) {
  constexpr int BLOCK = SCAN_BLOCK, ITEMS = SCAN_ITEMS;
  const int tid = threadIdx.x, lane = tid & 63;
  const __attribute__((address_space(1))) uint64_t *K = G(in) + start;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int idx = std::min(i * BLOCK + tid, cnt - 1);
    k[i] = K[base + idx];
    kp[i] = (lane == 0 && base + idx > 0) ? K[base + idx - 1] : 0ull;
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint64_t below = __shfl_up(k[i], 1, 64);
    if (lane != 0) kp[i] = below;
    const int idx = i * BLOCK + tid;
    heads[i] = __ballot(idx < cnt && (base + idx == 0 || k[i] != kp[i]));
  }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_dedupe_count(TileLaunch t, const uint64_t *in,
                                                             uint32_t *tcnt) {
  constexpr int WAVES = SCAN_BLOCK / 64;
  __shared__ uint32_t s_w[WAVES];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)SCAN_TILE;
    const int cnt = (int)std::min<int64_t>(SCAN_TILE, range_count(P, t.range_kind) - base);
    uint64_t k[SCAN_ITEMS], kp[SCAN_ITEMS], heads[SCAN_ITEMS];
    dedupe_heads(in, range_start(P, t.range_kind), base, cnt, k, kp, heads);
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) c += (uint32_t)__popcll(heads[i]);
    if (lane == 0) s_w[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (int w = 0; w < WAVES; ++w) tot += s_w[w];
      tcnt[tile] = tot;
    }
    __syncthreads();
  }
}

// Exclusive scan of the tile counts in place (one block), the grand total
// after the last tile; 32-bit and wrapping (only differences inside one
// table are used).
__global__ __launch_bounds__(1024) void k_dedupe_scan(uint32_t *tcnt, int64_t tiles) {
  __shared__ uint32_t s_w[16];
  const int tid = threadIdx.x;
  const int64_t per = (tiles + 1023) / 1024;
  const int64_t t0 = std::min<int64_t>(tid * per, tiles), t1 = std::min<int64_t>(t0 + per, tiles);
  uint32_t sum = 0;
  for (int64_t t = t0; t < t1; ++t) sum += tcnt[t];
  uint32_t total;
  uint32_t run = block_excl_scan<1024>(sum, s_w, total);
  for (int64_t t = t0; t < t1; ++t) {
    const uint32_t v = tcnt[t];
    tcnt[t] = run;
    run += v;
  }
  if (tid == 0) tcnt[tiles] = total;
}

// OFFSETS: also the out-offsets by boundary fill (edge keys); without, the
// compaction alone (the distinct node keys).
template <bool OFFSETS>
__global__ __launch_bounds__(SCAN_BLOCK) void k_dedupe_write(TileLaunch t, const uint64_t *in,
                                                             uint64_t *out, int64_t *seg_count,
                                                             const uint32_t *tpre) {
  constexpr int BLOCK = SCAN_BLOCK, ITEMS = SCAN_ITEMS, WAVES = BLOCK / 64;
  __shared__ uint32_t s_cnt[64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const int64_t first = t.tmap[seg];
    const int64_t base = (tile - first) * (int64_t)SCAN_TILE;
    const int64_t start = range_start(P, t.range_kind);
    const int64_t count = range_count(P, t.range_kind);
    const int cnt = (int)std::min<int64_t>(SCAN_TILE, count - base);
    const int b = P.b;
    uint64_t k[ITEMS], kp[ITEMS], heads[ITEMS];
    dedupe_heads(in, start, base, cnt, k, kp, heads);
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) s_cnt[i * WAVES + wave] = (uint32_t)__popcll(heads[i]);
    __syncthreads();
    if (wave == 0) {
      const uint32_t v = s_cnt[lane];
      const uint32_t inc = wave_incl_scan(v, lane);
      s_cnt[lane] = inc - v;
    }
    __syncthreads();
    // keys of this table in its earlier tiles, and the table's total
    const int64_t prefix = (int64_t)(uint32_t)(tpre[tile] - tpre[first]);
    const bool last_tile = base + cnt == count;
    const int64_t E = (int64_t)(uint32_t)(tpre[t.tmap[seg + 1]] - tpre[first]);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = i * BLOCK + tid;
      if ((heads[i] >> lane) & 1ull) {
        const int64_t j = prefix + s_cnt[i * WAVES + wave] + lanes_below(heads[i]);
        if (j < count) G(out)[start + j] = k[i];
        if (OFFSETS) {
          const int64_t hsrc = std::min<int64_t>((int64_t)(k[i] >> b), P.V - 1);
          const int64_t hp = (base + idx == 0) ? -1 : (int64_t)(kp[i] >> b);
          fill_run(t.gaps, (uint64_t *)(P.out_off + hp + 1), hsrc - hp, (uint64_t)j, 0, 1);
        }
      }
      if (OFFSETS && last_tile && idx == cnt - 1) {
        // the last row of the table closes the offsets
        const int64_t h = std::min<int64_t>((int64_t)(k[i] >> b), P.V - 1);
        fill_run(t.gaps, (uint64_t *)(P.out_off + h + 1), P.V - h, (uint64_t)E, 0, 1);
      }
    }
    if (tid == 0 && last_tile) seg_count[seg] = E;
    __syncthreads();
  }
}

hipError_t launch_dedupe_scan(const TileLaunch &t, const uint64_t *in, uint64_t *out,
                              int64_t *seg_count, uint32_t *tcnt, int grid, hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dedupe_count, dim3(grid), dim3(SCAN_BLOCK), 0, s, t, in, tcnt);
  hipLaunchKernelGGL(k_dedupe_scan, dim3(1), dim3(1024), 0, s, tcnt, t.total_tiles);
  hipLaunchKernelGGL(k_dedupe_write<true>, dim3(grid), dim3(SCAN_BLOCK), 0, s, t, in, out,
                     seg_count, (const uint32_t *)tcnt);
  return hipGetLastError();
}

// Unique node keys: the same compaction of the sorted node keys, without
// offsets; each table's count is its V.
hipError_t launch_unique(const TileLaunch &t, const uint64_t *in, uint64_t *out, int64_t *seg_count,
                         uint32_t *tcnt, int grid, hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dedupe_count, dim3(grid), dim3(SCAN_BLOCK), 0, s, t, in, tcnt);
  hipLaunchKernelGGL(k_dedupe_scan, dim3(1), dim3(1024), 0, s, tcnt, t.total_tiles);
  hipLaunchKernelGGL(k_dedupe_write<false>, dim3(grid), dim3(SCAN_BLOCK), 0, s, t, in, out,
                     seg_count, (const uint32_t *)tcnt);
  return hipGetLastError();
}

// Multigraph: every sorted key is its own edge, so an edge's position is its
// index and only the out-offsets need writing (a boundary fill over the
// sources of neighbouring keys, as k_in_csr does for the destinations); the
// table's edge count is its key count.
__global__ __launch_bounds__(256) void k_multi_offsets(TileLaunch t, const uint64_t *in,
                                                       int64_t *seg_count) {
  constexpr int U = 4;  // keys per thread in flight
  const int lane = threadIdx.x & 63;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const __attribute__((address_space(1))) uint64_t *K = G(in) + range_start(P, t.range_kind);
    const int64_t count = range_count(P, t.range_kind);
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)SCAN_TILE;
    const int64_t end = std::min<int64_t>(base + SCAN_TILE, count);
    const int64_t last = P.V - 1;
    const int b = P.b;
    for (int64_t j0 = base + threadIdx.x; j0 < end; j0 += U * 256) {
      uint64_t k[U], kp[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = std::min<int64_t>(j0 + u * 256, end - 1);
        k[u] = K[j];
        kp[u] = (lane == 0 && j > 0) ? K[j - 1] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t below = __shfl_up(k[u], 1, 64);
        if (lane != 0) kp[u] = below;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + u * 256;
        if (j < end) {
          const int64_t h = std::min<int64_t>((int64_t)(k[u] >> b), last);
          const int64_t hp = j == 0 ? -1 : std::min<int64_t>((int64_t)(kp[u] >> b), last);
          fill_run(t.gaps, (uint64_t *)(P.out_off + hp + 1), h - hp, (uint64_t)j, 0, 1);
          if (j == count - 1) {
            fill_run(t.gaps, (uint64_t *)(P.out_off + h + 1), P.V - h, (uint64_t)count, 0, 1);
            seg_count[seg] = count;
          }
        }
      }
    }
  }
}

hipError_t launch_multi_offsets(const TileLaunch &t, const uint64_t *in, int64_t *seg_count,
                                int grid, hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_multi_offsets, dim3(grid), dim3(256), 0, s, t, in, seg_count);
  return hipGetLastError();
}

// --------------------------------------------------------------- in-CSR
//
// The unique edges sorted by (d, s): in-neighbours are the low words, and
// in_off[v] is the position of the first edge whose destination is >= v.

__global__ __launch_bounds__(256) void k_in_csr(TileLaunch t, const uint64_t *in,
                                                const uint32_t *vals) {
  constexpr int U = 4;  // keys per thread in flight
  const int lane = threadIdx.x & 63;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const __attribute__((address_space(1))) uint64_t *K = G(in) + P.row_off;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)SCAN_TILE;
    const int64_t end = std::min<int64_t>(base + SCAN_TILE, P.E);
    const int64_t last = P.V - 1;
    for (int64_t j0 = base + threadIdx.x; j0 < end; j0 += U * 256) {
      // A wave's lanes hold consecutive keys, so each key's predecessor is
      // the lane below's key; lane 0 loads its own.
      uint64_t k[U], kp[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = std::min<int64_t>(j0 + u * 256, end - 1);
        k[u] = K[j];
        kp[u] = (lane == 0 && j > 0) ? K[j - 1] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t below = __shfl_up(k[u], 1, 64);
        if (lane != 0) kp[u] = below;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + u * 256;
        if (j < end) {
          G(P.in_nbr)[j] = (int32_t)(uint32_t)k[u];
          if (vals) G(P.in_eid)[j] = (int32_t)G(vals)[P.row_off + j];
          const int64_t h = std::min<int64_t>((int64_t)(k[u] >> 32), last);
          const int64_t hp = j == 0 ? -1 : std::min<int64_t>((int64_t)(kp[u] >> 32), last);
          fill_run(t.gaps, (uint64_t *)(P.in_off + hp + 1), h - hp, (uint64_t)j, 0, 1);
          if (j == P.E - 1)
            fill_run(t.gaps, (uint64_t *)(P.in_off + h + 1), P.V - h, (uint64_t)P.E, 0, 1);
        }
      }
    }
  }
}

hipError_t launch_in_csr(const TileLaunch &t, const uint64_t *in, const uint32_t *vals, int grid,
                         hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_in_csr, dim3(grid), dim3(256), 0, s, t, in, vals);
  return hipGetLastError();
}

// ------------------------------------------------- undirected / multigraph
//
// Undirected graphs: the unique keys of both orientations are the adjacency
// (in (v, w) order), so the neighbours are their low b bits.
__global__ __launch_bounds__(256) void k_out_nbr(TileLaunch t, const uint64_t *in) {
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint64_t *K = in + range_start(P, t.range_kind);
    const uint64_t mask = (1ull << P.b) - 1;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)SCAN_TILE;
    const int64_t end = std::min<int64_t>(base + SCAN_TILE, P.E);
    for (int64_t j = base + threadIdx.x; j < end; j += 256)
      G(P.out_nbr)[j] = (int32_t)(uint32_t)(G(K)[j] & mask);
  }
}

hipError_t launch_out_nbr(const TileLaunch &t, const uint64_t *in, int grid, hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_out_nbr, dim3(grid), dim3(256), 0, s, t, in);
  return hipGetLastError();
}

// Multigraph: every edge starts out as its row.
__global__ __launch_bounds__(256) void k_iota(TileLaunch t, uint32_t *v) {
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)REMAP_TILE;
    const int64_t end = std::min<int64_t>(base + REMAP_TILE, P.n);
    for (int64_t r = base + threadIdx.x; r < end; r += 256) G(v)[P.row_off + r] = (uint32_t)r;
  }
}

hipError_t launch_iota(const TileLaunch &rows, uint32_t *v, int grid, hipStream_t s) {
  if (rows.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(grid), dim3(256), 0, s, rows, v);
  return hipGetLastError();
}

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

}  // namespace ringo
