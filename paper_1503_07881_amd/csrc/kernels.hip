// gfx950 kernels of the table-to-graph conversion.
//
// The method is the paper's "sort-first" conversion (Converting Between
// Tables and Graphs, Section 2.4): copy the source and destination columns,
// sort the copies, count neighbours per node and place the sorted neighbour
// lists.  On the GPU every step is a tiled, HBM-streaming pass over all
// tables of a batch at once:
//
//   node keys   2n (id ^ 2^63) keys per table, least-significant-digit radix
//               sort, 8-bit digits, 8 passes
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
// (hash.hip holds the alternative node numbering through a node hash table,
// small.hip the single-workgroup conversion of small tables.)
//
// Each radix pass is a tile-granular reduce-then-scan: an upsweep counts the
// digits of every tile, a scan over tiles turns the counts into per-tile
// digit offsets, and a downsweep ranks every key stably inside its tile with
// 64-lane wavefront ballots and writes each digit run of the tile as one
// contiguous LDS-staged store.  Stream compaction (unique, dedupe) uses a
// single pass with decoupled look-back (Merrill & Garland 2016).

#include "device_common.h"
#include "ringo_internal.h"

namespace ringo {

// ----------------------------------------------------- decoupled look-back
//
// Status word of (tile, digit): [63:56] launch epoch, [55:54] flag
// (1 = tile aggregate, 2 = inclusive prefix), [53:0] value.  A word whose
// epoch differs from the current launch's is "not yet published", so the
// buffer is cleared once per call rather than once per pass.

constexpr uint64_t ST_AGG = 1, ST_INC = 2;
constexpr uint64_t ST_VMASK = (1ull << 54) - 1;

__device__ __forceinline__ uint64_t st_pack(uint32_t epoch, uint64_t flag, uint64_t v) {
  return ((uint64_t)epoch << 56) | (flag << 54) | v;
}
__device__ __forceinline__ void st_store(uint64_t *p, uint64_t w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
#ifndef RINGO_SPIN_SLEEP
#define RINGO_SPIN_SLEEP 1
#endif
__device__ __forceinline__ uint64_t st_wait(const uint64_t *p, uint32_t epoch) {
  uint64_t w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while ((uint32_t)(w >> 56) != epoch) {
    __builtin_amdgcn_s_sleep(RINGO_SPIN_SLEEP);
    w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return w;
}

// First half of the look-back: publish this tile's aggregate, or its
// inclusive prefix straight away when it opens its table or when the
// predecessor's inclusive prefix is already visible.  Returns true with
// *excl set when the prefix is resolved.
__device__ __forceinline__ bool lb_publish(uint64_t *status, int64_t tile, int64_t first,
                                           int stride, int d, uint32_t epoch, uint64_t total,
                                           uint64_t *excl) {
  uint64_t *own = status + tile * stride + d;
  if (tile == first) {
    st_store(own, st_pack(epoch, ST_INC, total));
    *excl = 0;
    return true;
  }
  const uint64_t w = __hip_atomic_load(status + (tile - 1) * stride + d, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  if ((uint32_t)(w >> 56) == epoch && ((w >> 54) & 3) == ST_INC) {
    *excl = w & ST_VMASK;
    st_store(own, st_pack(epoch, ST_INC, *excl + total));
    return true;
  }
  st_store(own, st_pack(epoch, ST_AGG, total));
  return false;
}

// Second half: walk back over predecessors until an inclusive prefix is
// found (the first tile of a table always publishes one), then publish ours.
// The status words of LB_WINDOW predecessors are requested together, so a
// walk over k published aggregates costs k / LB_WINDOW dependent round trips.
#ifndef RINGO_LB_WINDOW
#define RINGO_LB_WINDOW 8
#endif
constexpr int LB_WINDOW = RINGO_LB_WINDOW;

__device__ __forceinline__ uint64_t lb_resolve(uint64_t *status, int64_t tile, int64_t first,
                                               int stride, int d, uint32_t epoch, uint64_t total) {
  uint64_t acc = 0;
  bool done = false;
  for (int64_t p = tile - 1; !done; p -= LB_WINDOW) {
    uint64_t w[LB_WINDOW];
#pragma unroll
    for (int k = 0; k < LB_WINDOW; ++k)
      w[k] = p - k >= first ? __hip_atomic_load(status + (p - k) * stride + d, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : 0;
#pragma unroll
    for (int k = 0; k < LB_WINDOW; ++k) {
      if (done) break;
      uint64_t x = w[k];
      // the walk ends at the table's first tile at the latest, which always
      // publishes an inclusive prefix, so p - k >= first here
      if ((uint32_t)(x >> 56) != epoch) x = st_wait(status + (p - k) * stride + d, epoch);
      acc += x & ST_VMASK;
      done = ((x >> 54) & 3) == ST_INC;
    }
  }
  st_store(status + tile * stride + d, st_pack(epoch, ST_INC, acc + total));
  return acc;
}

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

hipError_t launch_empty_offsets(const SegPlan *plan, int32_t S, hipStream_t s) {
  hipLaunchKernelGGL(k_empty_offsets, dim3((S + 255) / 256), dim3(256), 0, s, plan, S);
  return hipGetLastError();
}

// ------------------------------------------------------------ LSD pass
//
// One stable counting-sort pass on RADIX_BITS digits, reduce-then-scan at
// tile granularity, with every kernel walking the tiles in global order:
//   upsweep      digit counts of every tile (and of every run of
//                run_tiles consecutive tiles)
//   block scan   exclusive prefix of the run counts, per digit
//   tile prefix  exclusive prefix of the tile counts, per digit: the
//                position of a tile's first key of each digit, relative to
//                the first tile of its table (passes of at most
//                SMALL_SCAN_TILES tiles do both scans in one kernel)
//   seg base     every table's digit bases
//   downsweep    wave-ballot stable rank inside the tile, LDS staging in
//                digit order, contiguous write-out of every digit run
// No block waits on another.  Tiles in flight are always neighbours in
// the input, so the runs they write land next to each other in every
// digit's output range.  Prefixes are 32-bit and wrap: only differences
// inside one table (fewer than 2^32 keys) are used.

constexpr int NUM_XCD = 8;    // accelerator complex dies of the MI355X
// s_waitcnt immediate: lgkmcnt(0), vmcnt and expcnt left at their maxima
constexpr int LGKMCNT_0 = 0xC07F;

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The key of element e of a table's range, as the pass sorts it.
template <int MODE>
__device__ __forceinline__ uint64_t pass_key(const SortLaunch &a, const SegPlan &P, int64_t start,
                                             int64_t e) {
  if (MODE == SORT_NODE_FIRST) {
    // one load from a selected pointer: no branch, so loads stay in flight
    const __attribute__((address_space(1))) int64_t *ptr = e < P.n ? G(P.src) + e : G(P.dst) + (e - P.n);
    return (uint64_t)*ptr ^ SIGN_FLIP;
  } else if (MODE == SORT_IN_FIRST || MODE == SORT_IN_FIRST_KV || MODE == SORT_IN_FIRST_DEDUP) {
    const uint64_t x = G(a.in)[start + e];
    const uint64_t d = x & ((1ull << P.b) - 1);
    return (d << 32) | (x >> P.b);
  }
  return G(a.in)[start + e];
}

// Header of the table holding a tile; tiles only move forward in a block.
struct TileHeader {
  int seg = -1;
  int64_t first = 0, end = 0, start = 0, count = 0;
  SegPlan P;
  __device__ __forceinline__ void at(const SortLaunch &a, int64_t tile) {
    if (tile < end) return;
    seg = find_seg(a.tmap, a.num_segs, tile);
    P = a.plan[seg];
    first = a.tmap[seg];
    end = a.tmap[seg + 1];
    start = range_start(P, a.range_kind);
    count = range_count(P, a.range_kind);
  }
};

// Each wave counts whole tiles on its own, in a wave-private LDS histogram;
// the block only meets once, to add up the four waves' sums over its run of
// run_tiles tiles.  LDS atomics of a wave are not ordered with its later LDS
// reads and writes, so the wave waits for its LDS operations to complete
// (lgkmcnt(0)) between clearing, counting and reading the histogram.  Plain
// passes read their keys in place two per lane (16-byte loads) where the
// tile's first key is 16-byte aligned.
template <int MODE>
__global__ __launch_bounds__(256) void k_upsweep(SortLaunch a, int tile_keys, int run_tiles) {
  // Every wave counts its tiles in a private LDS histogram whose bins are
  // split over SUB sub-counters (lane % SUB, adjacent words): lanes with an
  // equal digit (clustered identifiers) meet at most 64 / SUB to a counter,
  // and a plain atomic add per key costs less than finding the runs.
  constexpr int W = 4, U = 16, U2 = 4, SUB = 4;
  // the passes that read their keys from elsewhere, or compare neighbours
  constexpr bool FIRST = MODE == SORT_NODE_FIRST || MODE == SORT_IN_FIRST ||
                         MODE == SORT_IN_FIRST_KV || MODE == SORT_IN_FIRST_DEDUP;
  __shared__ uint4 s_h4[W * RADIX];
  uint32_t *s_h = (uint32_t *)s_h4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int shift = a.shift;
  const int64_t t0 = (int64_t)blockIdx.x * run_tiles;
  const int64_t t1 = std::min<int64_t>(t0 + run_tiles, a.total_tiles);
  TileHeader H;
  uint32_t run_sum[RADIX / 64] = {0, 0, 0, 0};
  uint4 *h4 = s_h4 + wave * RADIX;  // h4[d] = the SUB counters of digit d
  uint32_t *h = s_h + wave * RADIX * SUB + (lane & (SUB - 1));
  for (int64_t t = t0 + wave; t < t1; t += W) {
#pragma unroll
    for (int j = 0; j < RADIX / 64; ++j) h4[lane + 64 * j] = make_uint4(0, 0, 0, 0);
    __builtin_amdgcn_s_waitcnt(LGKMCNT_0);
    __builtin_amdgcn_wave_barrier();
    H.at(a, t);
    const int64_t k0 = (t - H.first) * tile_keys;
    const int64_t k1 = std::min<int64_t>(k0 + tile_keys, H.count);
    if (!FIRST && ((uintptr_t)(a.in + H.start + k0) & 15) == 0) {
      // keys read in place, two per lane (16-byte loads); an odd last key
      // on its own
      const int cnt = (int)(k1 - k0);
      const int np = cnt >> 1;
      const __attribute__((address_space(1))) u64x2 *p2 =
          (const __attribute__((address_space(1))) u64x2 *)(G(a.in) + H.start + k0);
      for (int q0 = lane; q0 < np; q0 += U2 * 64) {
        u64x2 k[U2];
#pragma unroll
        for (int j = 0; j < U2; ++j) k[j] = p2[std::min(q0 + j * 64, np - 1)];
#pragma unroll
        for (int j = 0; j < U2; ++j)
          if (q0 + j * 64 < np) {
            atomicAdd(&h[((uint32_t)(k[j].x >> shift) & (RADIX - 1)) * SUB], 1u);
            atomicAdd(&h[((uint32_t)(k[j].y >> shift) & (RADIX - 1)) * SUB], 1u);
          }
      }
      if ((cnt & 1) && lane == 0)
        atomicAdd(&h[((uint32_t)(G(a.in)[H.start + k1 - 1] >> shift) & (RADIX - 1)) * SUB], 1u);
    } else {
      for (int64_t e0 = k0 + lane; e0 < k1; e0 += U * 64) {
        uint64_t k[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
          k[j] = pass_key<MODE>(a, H.P, H.start, std::min<int64_t>(e0 + j * 64, k1 - 1));
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int64_t e = e0 + j * 64;
          bool valid = e < k1;
          if (MODE == SORT_IN_FIRST_DEDUP) {
            // only the first copy of every key counts
            uint64_t prev = __shfl_up(k[j], 1, 64);
            // lane 0 reads its predecessor, only for elements inside the tile
            if (lane == 0) prev = (e > 0 && e < k1) ? pass_key<MODE>(a, H.P, H.start, e - 1) : ~k[j];
            valid = valid && (e == 0 || k[j] != prev);
          }
          if (valid) atomicAdd(&h[((uint32_t)(k[j] >> shift) & (RADIX - 1)) * SUB], 1u);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(LGKMCNT_0);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < RADIX / 64; ++j) {
      const uint4 c = h4[lane + 64 * j];
      const uint32_t v = c.x + c.y + c.z + c.w;
      a.counts[t * RADIX + lane + 64 * j] = v;
      run_sum[j] += v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RADIX / 64; ++j) s_h[wave * RADIX + lane + 64 * j] = run_sum[j];
  __syncthreads();
  uint32_t v = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) v += s_h[w * RADIX + tid];
  a.bsum[(int64_t)blockIdx.x * RADIX + tid] = v;
}

// Run sums from tile counts written elsewhere (SORT_PART_PREFIX): one block
// per run of run_tiles tiles, one thread per digit.
__global__ __launch_bounds__(RADIX) void k_run_sums(SortLaunch a, int run_tiles) {
  const int d = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * run_tiles;
  const int64_t t1 = std::min<int64_t>(t0 + run_tiles, a.total_tiles);
  uint32_t sum = 0;
  for (int64_t t = t0; t < t1; ++t) sum += a.counts[t * RADIX + d];
  a.bsum[(int64_t)blockIdx.x * RADIX + d] = sum;
}

// Exclusive scan of the run counts over all runs, one block per digit.
__global__ __launch_bounds__(1024) void k_block_scan(SortLaunch a, int64_t runs) {
  __shared__ uint32_t s_w[16];
  const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < runs; b0 += 1024) {
    const int64_t b = b0 + tid;
    const uint32_t v = b < runs ? a.bsum[b * RADIX + d] : 0u;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t x = s_w[i];
      off += (i < w) ? x : 0u;
      tot += x;
    }
    if (b < runs) a.bsum[b * RADIX + d] = carry + off + inc - v;
    carry += tot;
    __syncthreads();
  }
  // sentinel row: prefix one past the last tile
  if (tid == 0) a.counts[a.total_tiles * RADIX + d] = carry;
}

// Tile counts become exclusive prefixes, in place; one block per run.
__global__ __launch_bounds__(RADIX) void k_tile_prefix(SortLaunch a, int run_tiles) {
  const int d = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * run_tiles;
  const int64_t t1 = std::min<int64_t>(t0 + run_tiles, a.total_tiles);
  uint32_t run = a.bsum[(int64_t)blockIdx.x * RADIX + d];
  // C tiles at a time: their loads are in flight together
  constexpr int C = 8;
  for (int64_t t = t0; t < t1; t += C) {
    uint32_t v[C];
#pragma unroll
    for (int i = 0; i < C; ++i) v[i] = t + i < t1 ? a.counts[(t + i) * RADIX + d] : 0u;
#pragma unroll
    for (int i = 0; i < C; ++i) {
      if (t + i < t1) a.counts[(t + i) * RADIX + d] = run;
      run += v[i];
    }
  }
}

// Small passes (at most SMALL_SCAN_TILES tiles): the run scan and the tile
// prefixes in one kernel, one block per digit.  Each thread takes a
// contiguous group of tiles; the block scan of the group sums gives each
// group's start.  Same result as k_block_scan followed by k_tile_prefix.
constexpr int SMALL_SCAN_TILES = 16 * 256;

__global__ __launch_bounds__(256) void k_scan_small(SortLaunch a) {
  __shared__ uint32_t s_w[4];
  const int d = blockIdx.x, tid = threadIdx.x;
  const int64_t T = a.total_tiles;
  const int64_t per = (T + 255) / 256;
  const int64_t t0 = std::min<int64_t>(tid * per, T), t1 = std::min<int64_t>(t0 + per, T);
  uint32_t v[16];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    v[i] = t0 + i < t1 ? a.counts[(t0 + i) * RADIX + d] : 0u;
    sum += v[i];
  }
  uint32_t total;
  uint32_t run = block_excl_scan<256>(sum, s_w, total);
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (t0 + i < t1) {
      a.counts[(t0 + i) * RADIX + d] = run;
      run += v[i];
    }
  // sentinel row: prefix one past the last tile
  if (tid == 0) a.counts[T * RADIX + d] = total;
}

// Digit bases of every table for this pass: the table's digit totals are
// differences of tile prefixes across its tiles; their exclusive scan over
// digits, plus the table's range start, is where each digit's run begins.
__global__ __launch_bounds__(RADIX) void k_seg_base(SortLaunch a) {
  __shared__ uint32_t s_w[RADIX / 64];
  const int seg = blockIdx.x, d = threadIdx.x;
  const int64_t f = a.tmap[seg], l = a.tmap[seg + 1];
  const uint32_t tot = l > f ? a.counts[l * RADIX + d] - a.counts[f * RADIX + d] : 0u;
  uint32_t all;
  const uint32_t ex = block_excl_scan<RADIX>(tot, s_w, all);
  a.digit_base[(int64_t)seg * RADIX + d] = range_start(a.plan[seg], a.range_kind) + (int64_t)ex;
  if (a.seg_total && d == 0) a.seg_total[seg] = (int64_t)all;
}

// Waves per SIMD the downsweep is compiled for: as many as the kernel's
// registers allow without spilling (a tile of 8 keys per thread needs about
// 105 VGPRs, 12 about 140, 16 about 175 and fits 168; carrying values and
// folding the dedupe take more).
constexpr int ds_waves(int items, int mode) {
  return mode == SORT_IN_FIRST_DEDUP ? (items <= 8 ? 3 : 2)
         : (mode == SORT_EDGE_KV || mode == SORT_IN_FIRST_KV || mode == SORT_IN_KV)
             ? (items <= 8 ? 4 : items <= 12 ? 3 : 2)
             : (items <= 8 ? 4 : 3);
}

template <int BLOCK, int ITEMS, int MODE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ds_waves(ITEMS, MODE), 8))) void k_downsweep(SortLaunch a) {
  constexpr int WAVES = BLOCK / 64;
  constexpr int TILE = BLOCK * ITEMS;
  constexpr bool KV = MODE == SORT_EDGE_KV || MODE == SORT_IN_FIRST_KV || MODE == SORT_IN_KV;
  constexpr bool DEDUP = MODE == SORT_IN_FIRST_DEDUP;
  constexpr bool IN_FIRST = MODE == SORT_IN_FIRST || MODE == SORT_IN_FIRST_KV;
  static_assert(BLOCK >= RADIX, "one thread per digit");
  __shared__ uint64_t s_stage[TILE];
  __shared__ uint32_t s_vstage[KV ? TILE : 1];
  __shared__ uint32_t s_whist[WAVES * RADIX];
  __shared__ uint32_t s_lstart[RADIX];
  __shared__ int64_t s_goff[RADIX];
  __shared__ uint32_t s_w[WAVES];
  __shared__ uint32_t s_wu[DEDUP ? WAVES : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int shift = a.shift;
  TileHeader H;
  int64_t dbase = 0;     // this thread's digit: first output position in the table
  uint32_t pfirst = 0;   // prefix of the table's first tile
  for (int i = tid; i < WAVES * RADIX; i += BLOCK) s_whist[i] = 0;
  __syncthreads();

  // Tiles in contiguous ranges per XCD (blocks go to the XCDs round-robin,
  // and the grid is a multiple of their count): tiles that run together on
  // one XCD are neighbours, so the partial cache lines shared by their digit
  // runs meet in the same L2.  Any mapping is correct; this one is faster.
  const int xcd = blockIdx.x % NUM_XCD;
  const int64_t per = gridDim.x / NUM_XCD;
  const int64_t t_hi = a.total_tiles * (xcd + 1) / NUM_XCD;
  for (int64_t tile = a.total_tiles * xcd / NUM_XCD + blockIdx.x / NUM_XCD; tile < t_hi;
       tile += per) {
    if (tile >= H.end) {
      H.at(a, tile);
      if (tid < RADIX) {
        dbase = a.digit_base[(int64_t)H.seg * RADIX + tid];
        pfirst = a.counts[H.first * RADIX + tid];
      }
    }
    const int64_t base = (tile - H.first) * (int64_t)TILE;
    const int cnt = (int)std::min<int64_t>(TILE, H.count - base);

    // Wave w owns the contiguous run [w * ITEMS * 64, (w + 1) * ITEMS * 64)
    // of the tile, one coalesced 64-key row per item.  Lanes past the end
    // load the tile's first key and are masked out of the rank; the loads
    // are unconditional so that all of them are in flight before the first
    // wait.
    uint64_t keys[ITEMS];
    uint32_t vals[KV ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = wave * (ITEMS * 64) + i * 64 + lane;
      keys[i] = pass_key<MODE>(a, H.P, H.start, base + (idx < cnt ? idx : 0));
      if (KV) vals[KV ? i : 0] = G(a.vin)[H.start + base + (idx < cnt ? idx : 0)];
    }
    if (IN_FIRST) {
      // out-neighbours (and multigraph rows), already in (s, d) order; stored
      // after all loads are issued so that no load waits for another
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int idx = wave * (ITEMS * 64) + i * 64 + lane;
        if (idx < cnt) {
          G(H.P.out_nbr)[base + idx] = (int32_t)(uint32_t)(keys[i] >> 32);
          if (KV) G(H.P.out_eid)[base + idx] = (int32_t)vals[KV ? i : 0];
        }
      }
    }
    // Live keys: all keys of the tile, or (dedupe folded into the pass) the
    // first copy of every key; ub[i] is row i's ballot of live lanes.
    uint32_t live_bits = 0;
    uint32_t wave_live = 0;
    uint32_t psrc[DEDUP ? ITEMS : 1];  // DEDUP: source of each key's predecessor
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = wave * (ITEMS * 64) + i * 64 + lane;
      bool live = idx < cnt;
      if (DEDUP) {
        const int64_t e = base + idx;
        uint64_t prev = __shfl_up(keys[i], 1, 64);
        const uint64_t above = __shfl(keys[i > 0 ? i - 1 : 0], 63, 64);
        // lane 0 reads its predecessor, only for elements inside the tile
        if (lane == 0 && idx < cnt)
          prev = i > 0 ? above : (e > 0 ? pass_key<MODE>(a, H.P, H.start, e - 1) : ~keys[i]);
        live = live && (e == 0 || keys[i] != prev);
        psrc[DEDUP ? i : 0] = (uint32_t)prev;
        wave_live += (uint32_t)__popcll(__ballot(live));
      }
      live_bits |= (uint32_t)live << i;
    }
    if (DEDUP && lane == 0) s_wu[DEDUP ? wave : 0] = wave_live;
    const uint32_t tprefix = tid < RADIX ? a.counts[tile * RADIX + tid] : 0u;

    // Stable rank inside the wave: lanes with an equal digit are found with
    // RADIX_BITS ballots; the lowest such lane bumps the wave's digit count.
    uint32_t rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const bool valid = (live_bits >> i) & 1u;
      const uint32_t d = (uint32_t)(keys[i] >> shift) & (RADIX - 1);
      uint64_t m = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < RADIX_BITS; ++bit) {
        const bool set = (d >> bit) & 1u;
        const uint64_t bb = __ballot(set);
        m &= set ? bb : ~bb;
      }
      const uint32_t below = lanes_below(m);
      uint32_t rk = 0;
      if (valid) {
        const uint32_t old = s_whist[wave * RADIX + d];
        if (below == 0) s_whist[wave * RADIX + d] = old + (uint32_t)__popcll(m);
        rk = old + below;
      }
      rank[i] = rk;
    }
    __syncthreads();

    // Tile digit counts; per-wave counts become exclusive offsets.
    uint32_t total = 0;
    if (tid < RADIX) {
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = s_whist[w * RADIX + tid];
        s_whist[w * RADIX + tid] = total;
        total += c;
      }
    }
    uint32_t tile_total;
    const uint32_t lstart = block_excl_scan<BLOCK>(tid < RADIX ? total : 0u, s_w, tile_total);
    if (tid < RADIX) {
      s_lstart[tid] = lstart;
      s_goff[tid] = dbase + (int64_t)(uint32_t)(tprefix - pfirst) - (int64_t)lstart;
    }
    uint32_t dpos = 0;  // DEDUP: de-duplicated position of this wave's first live key
    if (DEDUP) {
      // the table's live keys in earlier tiles (the digit prefixes summed),
      // then in earlier waves of this tile
      uint32_t tile_hp;
      (void)block_excl_scan<BLOCK>(tid < RADIX ? (uint32_t)(tprefix - pfirst) : 0u, s_w, tile_hp);
      dpos = tile_hp;
      for (int w = 0; w < wave; ++w) dpos += s_wu[w];
    }
    __syncthreads();

    // Stage the tile in LDS in digit order.
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      if ((live_bits >> i) & 1u) {
        const uint32_t d = (uint32_t)(keys[i] >> shift) & (RADIX - 1);
        const uint32_t slot = s_lstart[d] + s_whist[wave * RADIX + d] + rank[i];
        s_stage[slot] = keys[i];
        if (KV) s_vstage[KV ? slot : 0] = vals[KV ? i : 0];
      }
    }
    if (DEDUP) {
      // out-neighbours and out-offsets at the de-duplicated positions (rank
      // is dead here, which keeps the kernel within its registers)
      const int64_t V = H.P.V;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int idx = wave * (ITEMS * 64) + i * 64 + lane;
        const int64_t e = base + idx;
        const bool live = (live_bits >> i) & 1u;
        const uint64_t lb = __ballot(live);
        const int64_t s_own = (int64_t)(uint32_t)keys[i];
        if (live) {
          const int64_t j = (int64_t)dpos + lanes_below(lb);
          G(H.P.out_nbr)[j] = (int32_t)(uint32_t)(keys[i] >> 32);
          // out_off[v] = first position whose source is >= v
          const int64_t hp = e == 0 ? -1 : (int64_t)psrc[DEDUP ? i : 0];
          for (int64_t v = hp + 1; v <= s_own; ++v) G(H.P.out_off)[v] = j;
        }
        if (idx < cnt && e == H.count - 1)  // the table's last key closes the offsets
          for (int64_t v = s_own + 1; v <= V; ++v) G(H.P.out_off)[v] = H.P.E;
        dpos += (uint32_t)__popcll(lb);
      }
    }
    __syncthreads();

    // Write out: consecutive threads take consecutive staged keys, so every
    // digit run is stored contiguously.
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int p = i * BLOCK + tid;
      if (p < (int)tile_total) {
        const uint64_t k = s_stage[p];
        const int64_t pos = s_goff[(uint32_t)(k >> shift) & (RADIX - 1)] + p;
        if ((uint64_t)(pos - H.start) < (uint64_t)H.count) {  // in range by construction
          G(a.out)[pos] = k;
          if (KV) G(a.vout)[pos] = s_vstage[KV ? p : 0];
        }
      }
    }
    for (int i = tid; i < WAVES * RADIX; i += BLOCK) s_whist[i] = 0;
    __syncthreads();
  }
}

int sort_tile(int items) { return 256 * items; }

// Tiles per upsweep run: the power of two in [4, 32] that gives about 2048
// runs (blocks), so that small inputs still spread over the device.
static int run_tiles_for(int64_t tiles) {
  const int64_t r = tiles / 2048;
  int rt = 4;
  while (rt < 32 && 2 * rt <= r) rt *= 2;
  return rt;
}

int64_t sort_runs(int64_t tiles) {
  const int rt = run_tiles_for(tiles);
  return (tiles + rt - 1) / rt;
}

// Upper bound of sort_runs(t) over t <= max_tiles: below 2^16 tiles there
// are at most 4096 runs, above it every run holds 32 tiles.
int64_t sort_runs_bound(int64_t max_tiles) {
  return std::max<int64_t>(4096, (max_tiles + 31) / 32) + 1;
}

// Blocks of the downsweep that fit on the device at once.
template <int ITEMS>
static int resident_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_downsweep<256, ITEMS, SORT_PLAIN>, 256,
                                                   0) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb * device_cu_count();
}

template <int ITEMS, int MODE>
static hipError_t launch_pass_t(const SortLaunch &a, int parts, hipStream_t s) {
  if (parts & (SORT_PART_COUNT | SORT_PART_PREFIX)) {
    const int rt = run_tiles_for(a.total_tiles);
    const int64_t runs = (a.total_tiles + rt - 1) / rt;
    if (parts & SORT_PART_COUNT)
      hipLaunchKernelGGL((k_upsweep<MODE>), dim3((unsigned)runs), dim3(256), 0, s, a, 256 * ITEMS,
                         rt);
    else if (a.total_tiles > SMALL_SCAN_TILES)
      hipLaunchKernelGGL(k_run_sums, dim3((unsigned)runs), dim3(RADIX), 0, s, a, rt);
    if (a.total_tiles <= SMALL_SCAN_TILES) {
      hipLaunchKernelGGL(k_scan_small, dim3(RADIX), dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL(k_block_scan, dim3(RADIX), dim3(1024), 0, s, a, runs);
      hipLaunchKernelGGL(k_tile_prefix, dim3((unsigned)runs), dim3(RADIX), 0, s, a, rt);
    }
    hipLaunchKernelGGL(k_seg_base, dim3(a.num_segs), dim3(RADIX), 0, s, a);
  }
  if (parts & SORT_PART_SCATTER) {
    // four blocks per resident slot: blocks that finish early make room for
    // the next ones (measured faster than one persistent block per slot)
    const int64_t g = std::max<int64_t>(
        NUM_XCD, std::min<int64_t>(a.total_tiles, 4 * resident_t<ITEMS>()) / NUM_XCD * NUM_XCD);
    hipLaunchKernelGGL((k_downsweep<256, ITEMS, MODE>), dim3((unsigned)g), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// Every use of the pass has its own instantiation (the kernels differ only
// for the two first passes that read their keys from elsewhere), so that a
// profile names the pass a kernel belongs to.
template <int ITEMS>
static hipError_t launch_pass_items(const SortLaunch &a, int mode, int parts, hipStream_t s) {
  switch (mode) {
    case SORT_NODE_FIRST: return launch_pass_t<ITEMS, SORT_NODE_FIRST>(a, parts, s);
    case SORT_IN_FIRST: return launch_pass_t<ITEMS, SORT_IN_FIRST>(a, parts, s);
    case SORT_NODE: return launch_pass_t<ITEMS, SORT_NODE>(a, parts, s);
    case SORT_VNODE: return launch_pass_t<ITEMS, SORT_VNODE>(a, parts, s);
    case SORT_EDGE: return launch_pass_t<ITEMS, SORT_EDGE>(a, parts, s);
    case SORT_IN: return launch_pass_t<ITEMS, SORT_IN>(a, parts, s);
    case SORT_EDGE_KV: return launch_pass_t<ITEMS, SORT_EDGE_KV>(a, parts, s);
    case SORT_IN_FIRST_KV: return launch_pass_t<ITEMS, SORT_IN_FIRST_KV>(a, parts, s);
    case SORT_IN_KV: return launch_pass_t<ITEMS, SORT_IN_KV>(a, parts, s);
    case SORT_IN_FIRST_DEDUP: return launch_pass_t<ITEMS, SORT_IN_FIRST_DEDUP>(a, parts, s);
    default: return launch_pass_t<ITEMS, SORT_PLAIN>(a, parts, s);
  }
}

hipError_t launch_sort_part(const SortLaunch &a, int mode, int items, int parts, hipStream_t s) {
  if (a.total_tiles == 0) return hipSuccess;
  switch (items) {
    case 8: return launch_pass_items<8>(a, mode, parts, s);
    case 12: return launch_pass_items<12>(a, mode, parts, s);
    default: return launch_pass_items<16>(a, mode, parts, s);
  }
}


// ------------------------------------------------------ unique (node set)
//
// Head flags on the sorted node keys, stream compaction of the heads into
// the node list, per-table node count.  A tile is processed as ITEMS rows
// of BLOCK keys; the head count of each (row, wave) pair is a ballot, and
// the pairs are scanned in index order by one wave.

template <int BLOCK, int ITEMS>
struct CompactTile {
  static constexpr int WAVES = BLOCK / 64;
  static constexpr int TILE = BLOCK * ITEMS;
  static_assert(ITEMS * WAVES <= 64, "one wave scans the row counts");
};

__global__ __launch_bounds__(SCAN_BLOCK) void k_unique(TileLaunch t, const uint64_t *in,
                                                       uint64_t *out, int64_t *seg_count,
                                                       uint64_t *status, uint32_t *counter,
                                                       uint32_t epoch) {
  constexpr int BLOCK = SCAN_BLOCK, ITEMS = SCAN_ITEMS, WAVES = BLOCK / 64, TILE = SCAN_TILE;
  __shared__ uint64_t s_k[TILE];
  __shared__ uint32_t s_cnt[64];
  __shared__ int64_t s_tile, s_prefix, s_total;
  __shared__ int32_t s_seg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (;;) {
    if (tid == 0) {
      const int64_t tt = (int64_t)atomicAdd(counter, 1u);
      s_tile = tt;
      s_seg = tt < t.total_tiles ? find_seg(t.tmap, t.num_segs, tt) : 0;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile >= t.total_tiles) break;
    const int seg = s_seg;
    const SegPlan P = t.plan[seg];
    const int64_t first = t.tmap[seg];
    const int64_t base = (tile - first) * (int64_t)TILE;
    const int64_t start = range_start(P, t.range_kind);
    const int64_t count = range_count(P, t.range_kind);
    const int cnt = (int)std::min<int64_t>(TILE, count - base);
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = i * BLOCK + tid;
      if (idx < cnt) s_k[idx] = in[start + base + idx];
    }
    const uint64_t before = base > 0 ? in[start + base - 1] : 0;
    __syncthreads();
    uint64_t heads[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = i * BLOCK + tid;
      bool h = false;
      if (idx < cnt) {
        const uint64_t k = s_k[idx];
        h = (base + idx == 0) || k != (idx > 0 ? s_k[idx - 1] : before);
      }
      heads[i] = __ballot(h);
      if (lane == 0) s_cnt[i * WAVES + wave] = (uint32_t)__popcll(heads[i]);
    }
    __syncthreads();
    if (wave == 0) {
      const uint32_t v = s_cnt[lane];
      const uint32_t inc = wave_incl_scan(v, lane);
      s_cnt[lane] = inc - v;
      const uint32_t tot = __shfl(inc, 63, 64);
      if (lane == 0) {
        uint64_t ex;
        if (!lb_publish(status, tile, first, 1, 0, epoch, tot, &ex))
          ex = lb_resolve(status, tile, first, 1, 0, epoch, tot);
        s_prefix = (int64_t)ex;
        s_total = (int64_t)ex + tot;
      }
    }
    __syncthreads();
    const int64_t prefix = s_prefix;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = i * BLOCK + tid;
      if ((heads[i] >> lane) & 1ull) {
        const int64_t j = prefix + s_cnt[i * WAVES + wave] + lanes_below(heads[i]);
        if (j < count) out[start + j] = s_k[idx];
      }
    }
    if (tid == 0 && base + cnt == count) seg_count[seg] = s_total;
    __syncthreads();
  }
}

hipError_t launch_unique(const TileLaunch &t, const uint64_t *in, uint64_t *out, int64_t *seg_count,
                         uint64_t *status, uint32_t *counter, uint32_t epoch, int grid,
                         hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unique, dim3(grid), dim3(SCAN_BLOCK), 0, s, t, in, out, seg_count, status,
                     counter, epoch);
  return hipGetLastError();
}

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
        for (int64_t x = qp + 1; x < q; ++x) {
          D[x].key = 0;
          D[x].start = (uint32_t)j;
          D[x].next = (uint32_t)j;
        }
        D[q].key = u;
        D[q].start = (uint32_t)j;
      }
      if (q != qn) {  // last key of bucket q
        D[q].next = (uint32_t)(j + 1);
        if (j == P.V - 1) {
          const int64_t nb = (int64_t)1 << P.dirk;
          for (int64_t x = q + 1; x <= nb; ++x) {
            D[x].key = 0;
            D[x].start = (uint32_t)P.V;
            D[x].next = (uint32_t)P.V;
          }
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

__global__ __launch_bounds__(SCAN_BLOCK) void k_dedupe(TileLaunch t, const uint64_t *in,
                                                       uint64_t *out, int64_t *seg_count,
                                                       uint64_t *status, uint32_t *counter,
                                                       uint32_t epoch, int keep_all) {
  constexpr int BLOCK = SCAN_BLOCK, ITEMS = SCAN_ITEMS, WAVES = BLOCK / 64, TILE = SCAN_TILE;
  __shared__ uint64_t s_k[TILE];
  __shared__ uint32_t s_cnt[64];
  __shared__ int64_t s_tile, s_prefix, s_total;
  __shared__ int32_t s_seg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (;;) {
    if (tid == 0) {
      const int64_t tt = (int64_t)atomicAdd(counter, 1u);
      s_tile = tt;
      s_seg = tt < t.total_tiles ? find_seg(t.tmap, t.num_segs, tt) : 0;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile >= t.total_tiles) break;
    const int seg = s_seg;
    const SegPlan P = t.plan[seg];
    const int64_t first = t.tmap[seg];
    const int64_t base = (tile - first) * (int64_t)TILE;
    const int64_t start = range_start(P, t.range_kind);
    const int64_t count = range_count(P, t.range_kind);
    const int cnt = (int)std::min<int64_t>(TILE, count - base);
    const int b = P.b;
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = i * BLOCK + tid;
      if (idx < cnt) s_k[idx] = in[start + base + idx];
    }
    const uint64_t before = base > 0 ? in[start + base - 1] : 0;
    __syncthreads();
    uint64_t heads[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = i * BLOCK + tid;
      bool h = false;
      if (idx < cnt) {
        const uint64_t k = s_k[idx];
        h = keep_all || (base + idx == 0) || k != (idx > 0 ? s_k[idx - 1] : before);
      }
      heads[i] = __ballot(h);
      if (lane == 0) s_cnt[i * WAVES + wave] = (uint32_t)__popcll(heads[i]);
    }
    __syncthreads();
    if (wave == 0) {
      const uint32_t v = s_cnt[lane];
      const uint32_t inc = wave_incl_scan(v, lane);
      s_cnt[lane] = inc - v;
      const uint32_t tot = __shfl(inc, 63, 64);
      if (lane == 0) {
        uint64_t ex;
        if (!lb_publish(status, tile, first, 1, 0, epoch, tot, &ex))
          ex = lb_resolve(status, tile, first, 1, 0, epoch, tot);
        s_prefix = (int64_t)ex;
        s_total = (int64_t)ex + tot;
      }
    }
    __syncthreads();
    const int64_t prefix = s_prefix;
    const bool last_tile = base + cnt == count;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = i * BLOCK + tid;
      if ((heads[i] >> lane) & 1ull) {
        const uint64_t k = s_k[idx];
        const int64_t j = prefix + s_cnt[i * WAVES + wave] + lanes_below(heads[i]);
        if (j < count) out[start + j] = k;
        const int64_t hsrc = std::min<int64_t>((int64_t)(k >> b), P.V - 1);
        const int64_t hp =
            (base + idx == 0) ? -1 : (int64_t)((idx > 0 ? s_k[idx - 1] : before) >> b);
        for (int64_t v = hp + 1; v <= hsrc; ++v) G(P.out_off)[v] = j;
      }
      if (last_tile && idx == cnt - 1) {
        // the last row of the table closes the offsets
        const int64_t E = s_total;
        for (int64_t v = std::min<int64_t>((int64_t)(s_k[idx] >> b), P.V - 1) + 1; v <= P.V; ++v)
          G(P.out_off)[v] = E;
      }
    }
    if (tid == 0 && last_tile) seg_count[seg] = s_total;
    __syncthreads();
  }
}

hipError_t launch_dedupe(const TileLaunch &t, const uint64_t *in, uint64_t *out,
                         int64_t *seg_count, uint64_t *status, uint32_t *counter,
                         uint32_t epoch, int keep_all, int grid, hipStream_t s) {
  if (t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dedupe, dim3(grid), dim3(SCAN_BLOCK), 0, s, t, in, out, seg_count,
                     status, counter, epoch, keep_all);
  return hipGetLastError();
}

// --------------------------------------------------------------- in-CSR
//
// The unique edges sorted by (d, s): in-neighbours are the low words, and
// in_off[v] is the position of the first edge whose destination is >= v.

__global__ __launch_bounds__(256) void k_in_csr(TileLaunch t, const uint64_t *in,
                                                const uint32_t *vals) {
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint64_t *K = in + P.row_off;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)SCAN_TILE;
    const int64_t end = std::min<int64_t>(base + SCAN_TILE, P.E);
    for (int64_t j = base + threadIdx.x; j < end; j += 256) {
      const uint64_t k = K[j];
      G(P.in_nbr)[j] = (int32_t)(uint32_t)k;
      if (vals) G(P.in_eid)[j] = (int32_t)G(vals)[P.row_off + j];
      const int64_t h = std::min<int64_t>((int64_t)(k >> 32), P.V - 1);
      const int64_t hp = j == 0 ? -1 : std::min<int64_t>((int64_t)(K[j - 1] >> 32), P.V - 1);
      for (int64_t v = hp + 1; v <= h; ++v) G(P.in_off)[v] = j;
      if (j == P.E - 1)
        for (int64_t v = h + 1; v <= P.V; ++v) G(P.in_off)[v] = P.E;
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
