// One least-significant-digit radix sort pass of the table-to-graph
// conversion, for digits of RB bits (8 to 11; R = 2^RB digits).  Each digit
// width is instantiated in a translation unit of its own (lsd_d8.hip to
// lsd_d11.hip), which defines launch_sort_part_rb<RB>.
//
// A pass is a stable counting sort, reduce-then-scan at tile granularity,
// with every kernel walking the tiles in global order:
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
//
// Wider digits mean fewer passes over the keys (a 44-bit edge key takes 6
// passes of 8 bits, 4 of 11) but R counters per tile in the counts array
// and in LDS; which width is faster depends on the table size, and the
// schedule table picks it.
#pragma once

#include <atomic>
#include <type_traits>

#include "device_common.h"
#include "ringo_internal.h"

namespace ringo {

// s_waitcnt immediate: lgkmcnt(0), vmcnt and expcnt left at their maxima
constexpr int LGKMCNT_0 = 0xC07F;

template <int MODE>
constexpr bool part_mode() {
  return MODE == SORT_PART_ROWS || MODE == SORT_PART_DST || MODE == SORT_PART_RANK;
}

// Digit of key k in the pass: bits [shift, shift + RB) of the key, or
// (partition passes) the key's part of the node hash tables.
template <int MODE, int RB>
__device__ __forceinline__ uint32_t key_digit(uint64_t k, int shift) {
  if constexpr (part_mode<MODE>()) {
    static_assert(RB == PART_BITS, "partition passes have PART_BITS-bit digits");
    return slot_part(k);
  } else {
    return (uint32_t)(k >> shift) & ((1u << RB) - 1);
  }
}

// The key of element e of a table's range, as the pass sorts it.  A pass
// reads each key twice (count, then scatter) and never again, so the reads
// are non-temporal: they leave the caches to the scatter's partial lines,
// which meet there with their neighbours' before going to memory.
template <int MODE>
__device__ __forceinline__ uint64_t pass_key(const SortLaunch &a, const SegPlan &P, int64_t start,
                                             int64_t e) {
  if (MODE == SORT_PART_ROWS) {
    return (uint64_t)G(P.src)[e] ^ SIGN_FLIP;
  } else if (MODE == SORT_NODE_FIRST) {
    // one load from a selected pointer: no branch, so loads stay in flight
    const __attribute__((address_space(1))) int64_t *ptr = e < P.n ? G(P.src) + e : G(P.dst) + (e - P.n);
    return (uint64_t)*ptr ^ SIGN_FLIP;
  } else if (MODE == SORT_IN_FIRST || MODE == SORT_IN_FIRST_KV || MODE == SORT_IN_FIRST_DEDUP) {
    const uint64_t x = __builtin_nontemporal_load(&G(a.in)[start + e]);
    const uint64_t d = x & ((1ull << P.b) - 1);
    return (d << 32) | (x >> P.b);
  }
  return __builtin_nontemporal_load(&G(a.in)[start + e]);
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

// The SUB sub-counters of one upsweep histogram bin, read and cleared as one
// LDS access.
template <int SUB> struct SubBin;
template <> struct SubBin<4> {
  typedef uint4 T;
  static __device__ __forceinline__ uint32_t sum(T c) { return c.x + c.y + c.z + c.w; }
  static __device__ __forceinline__ T zero() { return make_uint4(0, 0, 0, 0); }
};
template <> struct SubBin<2> {
  typedef uint2 T;
  static __device__ __forceinline__ uint32_t sum(T c) { return c.x + c.y; }
  static __device__ __forceinline__ T zero() { return make_uint2(0, 0); }
};
template <> struct SubBin<1> {
  typedef uint32_t T;
  static __device__ __forceinline__ uint32_t sum(T c) { return c; }
  static __device__ __forceinline__ T zero() { return 0u; }
};

// Each wave counts whole tiles on its own, in a wave-private LDS histogram;
// the block only meets once, to add up the four waves' sums over its run of
// run_tiles tiles.  LDS atomics of a wave are not ordered with its later LDS
// reads and writes, so the wave waits for its LDS operations to complete
// (lgkmcnt(0)) between clearing, counting and reading the histogram.  Plain
// passes read their keys in place two per lane (16-byte loads) where the
// tile's first key is 16-byte aligned.
template <int MODE, int RB>
__global__ __launch_bounds__(256) void k_upsweep(SortLaunch a, int tile_keys, int run_tiles) {
  constexpr int R = 1 << RB;
  // Every bin is split over SUB sub-counters (lane % SUB, adjacent words):
  // lanes with an equal digit (clustered identifiers) meet at most 64 / SUB
  // to a counter, and a plain atomic add per key costs less than finding the
  // runs.  Wider digits collide less often and keep the histogram small.
  constexpr int SUB = RB == 8 ? 4 : RB == 9 ? 2 : 1;
  constexpr int W = 4, U = 16, U2 = 4, DL = R / 64;
  typedef SubBin<SUB> Bin;
  // the passes that read their keys from elsewhere, or compare neighbours
  constexpr bool FIRST = MODE == SORT_NODE_FIRST || MODE == SORT_IN_FIRST ||
                         MODE == SORT_IN_FIRST_KV || MODE == SORT_IN_FIRST_DEDUP ||
                         MODE == SORT_PART_ROWS;
  __shared__ typename Bin::T s_hb[W * R];
  uint32_t *s_h = (uint32_t *)s_hb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int shift = a.shift;
  const int64_t t0 = (int64_t)blockIdx.x * run_tiles;
  const int64_t t1 = std::min<int64_t>(t0 + run_tiles, a.total_tiles);
  TileHeader H;
  uint32_t run_sum[DL];
#pragma unroll
  for (int j = 0; j < DL; ++j) run_sum[j] = 0;
  typename Bin::T *hb = s_hb + wave * R;  // hb[d] = the SUB counters of digit d
  uint32_t *h = s_h + wave * R * SUB + (lane & (SUB - 1));
  for (int64_t t = t0 + wave; t < t1; t += W) {
#pragma unroll
    for (int j = 0; j < DL; ++j) hb[lane + 64 * j] = Bin::zero();
    __builtin_amdgcn_s_waitcnt(LGKMCNT_0);
    __builtin_amdgcn_wave_barrier();
    H.at(a, t);
    const int64_t k0 = (t - H.first) * tile_keys;
    // a tile past the table's key count (tile maps sized for the worst case,
    // the count set on the device) is empty
    const int64_t k1 = std::max<int64_t>(k0, std::min<int64_t>(k0 + tile_keys, H.count));
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
        for (int j = 0; j < U2; ++j) k[j] = __builtin_nontemporal_load(&p2[std::min(q0 + j * 64, np - 1)]);
#pragma unroll
        for (int j = 0; j < U2; ++j)
          if (q0 + j * 64 < np) {
            atomicAdd(&h[key_digit<MODE, RB>(k[j].x, shift) * SUB], 1u);
            atomicAdd(&h[key_digit<MODE, RB>(k[j].y, shift) * SUB], 1u);
          }
      }
      if ((cnt & 1) && lane == 0)
        atomicAdd(&h[key_digit<MODE, RB>(G(a.in)[H.start + k1 - 1], shift) * SUB], 1u);
    } else {
      // DEDUP: lane 63's key of the previous group of rows, the predecessor
      // of lane 0's first key in the next group
      uint64_t carry = 0;
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
            // only the first copy of every key counts; lane 0's predecessor
            // is lane 63's key of the row above (a shuffle, or the carry of
            // the previous group), read from memory only for the tile's
            // first row (the keys are read non-temporally, so a second read
            // of a line goes to memory again)
            uint64_t prev = __shfl_up(k[j], 1, 64);
            const uint64_t above = j > 0 ? __shfl(k[j > 0 ? j - 1 : 0], 63, 64) : carry;
            if (lane == 0)
              prev = e != k0 ? above
                             : (e > 0 && e < k1) ? pass_key<MODE>(a, H.P, H.start, e - 1) : ~k[j];
            valid = valid && (e == 0 || k[j] != prev);
          }
          if (valid) atomicAdd(&h[key_digit<MODE, RB>(k[j], shift) * SUB], 1u);
        }
        if (MODE == SORT_IN_FIRST_DEDUP) carry = __shfl(k[U - 1], 63, 64);
      }
    }
    __builtin_amdgcn_s_waitcnt(LGKMCNT_0);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < DL; ++j) {
      const uint32_t v = Bin::sum(hb[lane + 64 * j]);
      a.counts[t * R + lane + 64 * j] = v;
      run_sum[j] += v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < DL; ++j) s_h[wave * R + lane + 64 * j] = run_sum[j];
  __syncthreads();
  for (int d = tid; d < R; d += 256) {
    uint32_t v = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) v += s_h[w * R + d];
    a.bsum[(int64_t)blockIdx.x * R + d] = v;
  }
}

// Run sums from tile counts written elsewhere (SORT_PART_PREFIX): one block
// per run of run_tiles tiles and 256 digits.
template <int RB>
__global__ __launch_bounds__(256) void k_run_sums(SortLaunch a, int run_tiles) {
  constexpr int R = 1 << RB;
  const int d = blockIdx.y * 256 + threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * run_tiles;
  const int64_t t1 = std::min<int64_t>(t0 + run_tiles, a.total_tiles);
  uint32_t sum = 0;
  for (int64_t t = t0; t < t1; ++t) sum += a.counts[t * R + d];
  a.bsum[(int64_t)blockIdx.x * R + d] = sum;
}

// Exclusive scan of the run counts over all runs, one block per digit.
template <int RB>
__global__ __launch_bounds__(1024) void k_block_scan(SortLaunch a, int64_t runs) {
  constexpr int R = 1 << RB;
  __shared__ uint32_t s_w[16];
  const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < runs; b0 += 1024) {
    const int64_t b = b0 + tid;
    const uint32_t v = b < runs ? a.bsum[b * R + d] : 0u;
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
    if (b < runs) a.bsum[b * R + d] = carry + off + inc - v;
    carry += tot;
    __syncthreads();
  }
  // sentinel row: prefix one past the last tile
  if (tid == 0) a.counts[a.total_tiles * R + d] = carry;
}

// Tile counts become exclusive prefixes, in place; one block per run and
// 256 digits.
template <int RB>
__global__ __launch_bounds__(256) void k_tile_prefix(SortLaunch a, int run_tiles) {
  constexpr int R = 1 << RB;
  const int d = blockIdx.y * 256 + threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * run_tiles;
  const int64_t t1 = std::min<int64_t>(t0 + run_tiles, a.total_tiles);
  uint32_t run = a.bsum[(int64_t)blockIdx.x * R + d];
  // C tiles at a time: their loads are in flight together
  constexpr int C = 8;
  for (int64_t t = t0; t < t1; t += C) {
    uint32_t v[C];
#pragma unroll
    for (int i = 0; i < C; ++i) v[i] = t + i < t1 ? a.counts[(t + i) * R + d] : 0u;
#pragma unroll
    for (int i = 0; i < C; ++i) {
      if (t + i < t1) a.counts[(t + i) * R + d] = run;
      run += v[i];
    }
  }
}

// Small passes (at most SMALL_SCAN_TILES tiles): the run scan and the tile
// prefixes in one kernel, one block per digit.  Each thread takes a
// contiguous group of tiles; the block scan of the group sums gives each
// group's start.  Same result as k_block_scan followed by k_tile_prefix.
constexpr int SMALL_SCAN_TILES = 16 * 256;

template <int RB>
__global__ __launch_bounds__(256) void k_scan_small(SortLaunch a) {
  constexpr int R = 1 << RB;
  __shared__ uint32_t s_w[4];
  const int d = blockIdx.x, tid = threadIdx.x;
  const int64_t T = a.total_tiles;
  const int64_t per = (T + 255) / 256;
  const int64_t t0 = std::min<int64_t>(tid * per, T), t1 = std::min<int64_t>(t0 + per, T);
  uint32_t v[16];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    v[i] = t0 + i < t1 ? a.counts[(t0 + i) * R + d] : 0u;
    sum += v[i];
  }
  uint32_t total;
  uint32_t run = block_excl_scan<256>(sum, s_w, total);
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (t0 + i < t1) {
      a.counts[(t0 + i) * R + d] = run;
      run += v[i];
    }
  // sentinel row: prefix one past the last tile
  if (tid == 0) a.counts[T * R + d] = total;
}

// Digit bases of every table for this pass: the table's digit totals are
// differences of tile prefixes across its tiles; their exclusive scan over
// digits, plus the table's range start, is where each digit's run begins.
// One block per table, R / 256 consecutive digits per thread.
template <int RB>
__global__ __launch_bounds__(256) void k_seg_base(SortLaunch a) {
  constexpr int R = 1 << RB, DPT = R / 256;
  __shared__ uint32_t s_w[4];
  const int seg = blockIdx.x, tid = threadIdx.x;
  const int64_t f = a.tmap[seg], l = a.tmap[seg + 1];
  uint32_t tot[DPT];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int d = tid * DPT + j;
    tot[j] = l > f ? a.counts[l * R + d] - a.counts[f * R + d] : 0u;
    sum += tot[j];
  }
  uint32_t all;
  uint32_t ex = block_excl_scan<256>(sum, s_w, all);
  const int64_t rs = range_start(a.plan[seg], a.range_kind);
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    a.digit_base[(int64_t)seg * R + tid * DPT + j] = rs + (int64_t)ex;
    ex += tot[j];
  }
  if (a.seg_total && tid == 0) a.seg_total[seg] = (int64_t)all;
}

// Waves per SIMD the downsweep is compiled for: as many as the kernel's
// registers allow without spilling (a tile of 8 keys per thread needs about
// 105 VGPRs, 12 about 140, 16 about 175 and fits 168; carrying values and
// folding the dedupe take more, and so do the per-table digit bases of the
// wider digits, R / 256 per thread).
constexpr int ds_waves(int items, int mode, int rb) {
  return mode == SORT_IN_FIRST_DEDUP
             ? (items <= 8 ? (rb <= 9 ? 3 : 2) : items <= 12 ? 2 : (rb <= 9 ? 2 : 1))
         : mode == SORT_PART_ROWS ? (items <= 8 ? 3 : 2)
         : (mode == SORT_EDGE_KV || mode == SORT_IN_FIRST_KV || mode == SORT_IN_KV ||
            mode == SORT_PART_RANK)
             ? (items <= 8 ? (rb <= 9 ? 4 : 3) : items <= 12 ? (rb <= 9 ? 3 : 2) : 2)
             : (items <= 8 ? (rb <= 10 ? 4 : 3) : items <= 12 || rb == 8 ? 3 : 2);
}

template <int BLOCK, int ITEMS, int MODE, int RB>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ds_waves(ITEMS, MODE, RB), 8))) void k_downsweep(SortLaunch a) {
  constexpr int R = 1 << RB;
  constexpr int DPT = R / BLOCK;  // consecutive digits per thread
  static_assert(R % BLOCK == 0, "whole digits per thread");
  constexpr int WAVES = BLOCK / 64;
  constexpr int TILE = BLOCK * ITEMS;
  // RANKV: only the carried values (source positions) are written; WIDE:
  // 64-bit destination keys carried with the keys
  constexpr bool RANKV = MODE == SORT_PART_RANK;
  constexpr bool WIDE = MODE == SORT_PART_ROWS;
  constexpr bool KV = MODE == SORT_EDGE_KV || MODE == SORT_IN_FIRST_KV || MODE == SORT_IN_KV || RANKV;
  constexpr bool DEDUP = MODE == SORT_IN_FIRST_DEDUP;
  constexpr bool IN_FIRST = MODE == SORT_IN_FIRST || MODE == SORT_IN_FIRST_KV;
  // Per-wave digit counts, then slot bases; they never exceed TILE, so
  // 16 bits hold them and the wider digits' histograms stay small.
  typedef typename std::conditional<(RB > 8), uint16_t, uint32_t>::type hist_t;
  static_assert(TILE < 65536, "16-bit slot bases");
  __shared__ uint64_t s_stage[TILE];
  __shared__ uint32_t s_vstage[KV ? TILE : 1];
  __shared__ uint64_t s_wstage[WIDE ? TILE : 1];
  __shared__ hist_t s_whist[WAVES * R];
  __shared__ int64_t s_goff[R];
  __shared__ uint32_t s_w[WAVES];
  __shared__ uint32_t s_wu[DEDUP ? WAVES : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int shift = a.shift;
  TileHeader H;
  int64_t dbase[DPT];    // this thread's digits: first output position in the table
  uint32_t pfirst[DPT];  // prefix of the table's first tile
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    dbase[j] = 0;
    pfirst[j] = 0;
  }
  for (int i = tid; i < WAVES * R; i += BLOCK) s_whist[i] = 0;
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
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const int d = tid * DPT + j;
        dbase[j] = a.digit_base[(int64_t)H.seg * R + d];
        pfirst[j] = a.counts[H.first * R + d];
      }
    }
    const int64_t base = (tile - H.first) * (int64_t)TILE;
    // a tile past the key count (worst-case tile maps) is empty: its loads
    // read the tile's first slot, inside the buffer, and nothing is written
    const int cnt = (int)std::max<int64_t>(0, std::min<int64_t>(TILE, H.count - base));

    // Wave w owns the contiguous run [w * ITEMS * 64, (w + 1) * ITEMS * 64)
    // of the tile, one coalesced 64-key row per item.  Lanes past the end
    // load the tile's first key and are masked out of the rank; the loads
    // are unconditional so that all of them are in flight before the first
    // wait.
    uint64_t keys[ITEMS];
    uint32_t vals[KV ? ITEMS : 1];
    uint64_t wv[WIDE ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = wave * (ITEMS * 64) + i * 64 + lane;
      const int64_t e = base + (idx < cnt ? idx : 0);
      keys[i] = pass_key<MODE>(a, H.P, H.start, e);
      if (KV) vals[KV ? i : 0] = __builtin_nontemporal_load(&G(a.vin)[H.start + e]);
      if (WIDE) wv[WIDE ? i : 0] = (uint64_t)G(H.P.dst)[e] ^ SIGN_FLIP;
    }
    // This tile's digit counts are the differences of its prefixes and the
    // next tile's (the last tile's next row is the scan's sentinel row).
    // Their scan over the digits gives each digit's first slot in the tile
    // (lstart) and the output position of that slot (s_goff); it runs while
    // the keys are in flight.
    uint32_t tdig = 0;  // sum of this thread's digit counts
    uint32_t hdig = 0;  // sum of this thread's digit prefixes inside the table
    uint32_t dcnt[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = tid * DPT + j;
      const uint32_t tp = a.counts[tile * R + d];
      dcnt[j] = a.counts[(tile + 1) * R + d] - tp;
      tdig += dcnt[j];
      const uint32_t rel = tp - pfirst[j];  // keys of digit d in the table's earlier tiles
      hdig += rel;
      // s_goff[d] is completed below, once lstart is known
      s_goff[d] = dbase[j] + (int64_t)rel;
    }
    uint32_t tile_total;
    uint32_t lstart = block_excl_scan<BLOCK>(tdig, s_w, tile_total);
    {
      uint32_t ls = lstart;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        s_goff[tid * DPT + j] -= (int64_t)ls;
        ls += dcnt[j];
      }
    }
    uint32_t dpos = 0;  // DEDUP: de-duplicated position of this wave's first live key
    if (DEDUP) {
      // the table's live keys in earlier tiles (the digit prefixes summed)
      uint32_t tile_hp;
      (void)block_excl_scan<BLOCK>(hdig, s_w, tile_hp);
      dpos = tile_hp;
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
    // first copy of every key.
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

    // Stable rank inside the wave: lanes with an equal digit are found with
    // RB ballots; the lowest such lane bumps the wave's digit count.  The
    // partition passes keep each key's digit (a hash) beside its rank, in
    // the upper 16 bits.
    uint32_t rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const bool valid = (live_bits >> i) & 1u;
      const uint32_t d = key_digit<MODE, RB>(keys[i], shift);
      const uint64_t mv = __ballot(valid);
      // Per bit: s = -1 where this lane's bit is set, else 0 (one v_bfe_i32);
      // the lanes that disagree with it on the bit are the ballot of set bits
      // XOR s.  Their union over the bits, starting from the lanes without a
      // key, takes one v_bitop3_b32 per half and bit: table 0xDE with the
      // union as the middle operand is union | (s ^ ballot) whichever outer
      // operand indexes the table's high bit.  Builtins, not inline
      // assembly: the compiler then keeps the wait states that a VALU read
      // of the ballot's SGPRs needs after the compare that wrote them.
      uint32_t alo = ~(uint32_t)mv, ahi = ~(uint32_t)(mv >> 32);
#pragma unroll
      for (int bit = 0; bit < RB; ++bit) {
        const int32_t sb = __builtin_amdgcn_sbfe((int32_t)d, bit, 1);
        const uint64_t bb = __ballot(sb < 0);
        alo = __builtin_amdgcn_bitop3_b32((uint32_t)sb, alo, (uint32_t)bb, 0xDE);
        ahi = __builtin_amdgcn_bitop3_b32((uint32_t)sb, ahi, (uint32_t)(bb >> 32), 0xDE);
      }
      const uint64_t m = ~(((uint64_t)ahi << 32) | alo);
      const uint32_t below = lanes_below(m);
      uint32_t rk = 0;
      if (valid) {
        const uint32_t old = s_whist[wave * R + d];
        if (below == 0) s_whist[wave * R + d] = (hist_t)(old + (uint32_t)__popcll(m));
        rk = old + below;
      }
      rank[i] = part_mode<MODE>() ? rk | d << 16 : rk;
    }
    __syncthreads();

    // Per-wave digit counts become slot bases: the digit's first slot in
    // the tile plus the digit's keys in earlier waves.
    {
      uint32_t ls = lstart;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const int d = tid * DPT + j;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
          const uint32_t c = s_whist[w * R + d];
          s_whist[w * R + d] = (hist_t)ls;
          ls += c;
        }
      }
    }
    if (DEDUP)
      for (int w = 0; w < wave; ++w) dpos += s_wu[w];
    __syncthreads();

    // Stage the tile in LDS in digit order.
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      if ((live_bits >> i) & 1u) {
        const uint32_t d = part_mode<MODE>() ? rank[i] >> 16 : key_digit<MODE, RB>(keys[i], shift);
        const uint32_t slot = (uint32_t)s_whist[wave * R + d] + (rank[i] & 0xffffu);
        s_stage[slot] = keys[i];
        if (KV) s_vstage[KV ? slot : 0] = vals[KV ? i : 0];
        if (WIDE) s_wstage[WIDE ? slot : 0] = wv[WIDE ? i : 0];
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
          fill_run(a.gaps, (uint64_t *)(H.P.out_off + hp + 1), s_own - hp, (uint64_t)j, 0, 1);
        }
        if (idx < cnt && e == H.count - 1)  // the table's last key closes the offsets
          fill_run(a.gaps, (uint64_t *)(H.P.out_off + s_own + 1), V - s_own, (uint64_t)H.P.E, 0, 1);
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
        const int64_t pos = s_goff[key_digit<MODE, RB>(k, shift)] + p;
        if ((uint64_t)(pos - H.start) < (uint64_t)H.count) {  // in range by construction
          if (!RANKV) G(a.out)[pos] = k;
          if (KV) G(a.vout)[pos] = s_vstage[KV ? p : 0];
          if (WIDE) G(a.wout)[pos] = s_wstage[WIDE ? p : 0];
        }
      }
    }
    for (int i = tid; i < WAVES * R; i += BLOCK) s_whist[i] = 0;
    __syncthreads();
  }
}

// The plain passes over tiles of two halves (2 x 256 x ITEMS keys): each
// half is loaded, ranked and staged in turn with the registers of one (in
// every digit the second half's slots follow the first's), then the whole
// tile is written out.  A tile's digit runs are twice as long as those of
// the one-half tile at the same registers and blocks per CU, so fewer of
// the lines they write are shared with a neighbouring tile.
// (The staging buffer holds two blocks per CU, so the kernel is compiled
// for two waves per SIMD.)
template <int ITEMS, int MODE, int RB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_downsweep_pair(SortLaunch a) {
  static_assert(MODE == SORT_PLAIN || MODE == SORT_EDGE || MODE == SORT_IN, "plain passes only");
  constexpr int BLOCK = 256;
  constexpr int R = 1 << RB;
  constexpr int DPT = R / BLOCK;
  static_assert(R % BLOCK == 0, "whole digits per thread");
  constexpr int WAVES = BLOCK / 64;
  constexpr int HALF = BLOCK * ITEMS;
  constexpr int TILE = 2 * HALF;
  static_assert(ITEMS <= 32, "one live bit per item");
  typedef typename std::conditional<(RB > 8), uint16_t, uint32_t>::type hist_t;
  static_assert(TILE < 65536, "16-bit slot bases");
  __shared__ uint64_t s_stage[TILE];
  __shared__ hist_t s_whist[WAVES * R];
  __shared__ int64_t s_goff[R];
  __shared__ uint32_t s_w[WAVES];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int shift = a.shift;
  TileHeader H;
  int64_t dbase[DPT];
  uint32_t pfirst[DPT];
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    dbase[j] = 0;
    pfirst[j] = 0;
  }
  for (int i = tid; i < WAVES * R; i += BLOCK) s_whist[i] = 0;
  __syncthreads();

  // tiles in contiguous ranges per XCD, as in k_downsweep
  const int xcd = blockIdx.x % NUM_XCD;
  const int64_t per = gridDim.x / NUM_XCD;
  const int64_t t_hi = a.total_tiles * (xcd + 1) / NUM_XCD;
  for (int64_t tile = a.total_tiles * xcd / NUM_XCD + blockIdx.x / NUM_XCD; tile < t_hi;
       tile += per) {
    if (tile >= H.end) {
      H.at(a, tile);
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const int d = tid * DPT + j;
        dbase[j] = a.digit_base[(int64_t)H.seg * R + d];
        pfirst[j] = a.counts[H.first * R + d];
      }
    }
    const int64_t base = (tile - H.first) * (int64_t)TILE;
    const int cnt = (int)std::max<int64_t>(0, std::min<int64_t>(TILE, H.count - base));

    // the first half's keys are in flight while the digit bases are found
    uint64_t keys[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int idx = wave * (ITEMS * 64) + i * 64 + lane;
      keys[i] = pass_key<MODE>(a, H.P, H.start, base + (idx < cnt ? idx : 0));
    }
    uint32_t tdig = 0;
    uint32_t dcnt[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = tid * DPT + j;
      const uint32_t tp = a.counts[tile * R + d];
      dcnt[j] = a.counts[(tile + 1) * R + d] - tp;
      tdig += dcnt[j];
      s_goff[d] = dbase[j] + (int64_t)(tp - pfirst[j]);
    }
    uint32_t tile_total;
    const uint32_t lstart = block_excl_scan<BLOCK>(tdig, s_w, tile_total);
    uint32_t next[DPT];  // next free slot of each of this thread's digits
    {
      uint32_t ls = lstart;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        s_goff[tid * DPT + j] -= (int64_t)ls;
        next[j] = ls;
        ls += dcnt[j];
      }
    }

#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int h0 = h * HALF + wave * (ITEMS * 64);  // this wave's first key of the half
      if (h == 1) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const int idx = h0 + i * 64 + lane;
          keys[i] = pass_key<MODE>(a, H.P, H.start, base + (idx < cnt ? idx : 0));
        }
      }
      // stable rank inside the wave, as in k_downsweep
      uint32_t rank[ITEMS];
      uint32_t live_bits = 0;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const bool valid = h0 + i * 64 + lane < cnt;
        live_bits |= (uint32_t)valid << i;
        const uint32_t d = key_digit<MODE, RB>(keys[i], shift);
        const uint64_t mv = __ballot(valid);
        uint32_t alo = ~(uint32_t)mv, ahi = ~(uint32_t)(mv >> 32);
#pragma unroll
        for (int bit = 0; bit < RB; ++bit) {
          const int32_t sb = __builtin_amdgcn_sbfe((int32_t)d, bit, 1);
          const uint64_t bb = __ballot(sb < 0);
          alo = __builtin_amdgcn_bitop3_b32((uint32_t)sb, alo, (uint32_t)bb, 0xDE);
          ahi = __builtin_amdgcn_bitop3_b32((uint32_t)sb, ahi, (uint32_t)(bb >> 32), 0xDE);
        }
        const uint64_t m = ~(((uint64_t)ahi << 32) | alo);
        const uint32_t below = lanes_below(m);
        uint32_t rk = 0;
        if (valid) {
          const uint32_t old = s_whist[wave * R + d];
          if (below == 0) s_whist[wave * R + d] = (hist_t)(old + (uint32_t)__popcll(m));
          rk = old + below;
        }
        rank[i] = rk;
      }
      __syncthreads();
      // this half's per-wave digit counts become slot bases
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const int d = tid * DPT + j;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
          const uint32_t c = s_whist[w * R + d];
          s_whist[w * R + d] = (hist_t)next[j];
          next[j] += c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        if ((live_bits >> i) & 1u) {
          const uint32_t d = key_digit<MODE, RB>(keys[i], shift);
          s_stage[(uint32_t)s_whist[wave * R + d] + rank[i]] = keys[i];
        }
      }
      __syncthreads();
      for (int i = tid; i < WAVES * R; i += BLOCK) s_whist[i] = 0;
      __syncthreads();
    }

    // write out the whole tile: consecutive threads take consecutive staged
    // keys, so every digit run is stored contiguously
#pragma unroll
    for (int i = 0; i < 2 * ITEMS; ++i) {
      const int p = i * BLOCK + tid;
      if (p < (int)tile_total) {
        const uint64_t k = s_stage[p];
        const int64_t pos = s_goff[key_digit<MODE, RB>(k, shift)] + p;
        if ((uint64_t)(pos - H.start) < (uint64_t)H.count) G(a.out)[pos] = k;  // in range by construction
      }
    }
    __syncthreads();
  }
}

// Blocks of the downsweep that fit on the device at once.  The occupancy
// query is host work on the launch path of small tables, so its answer is
// kept (per instantiation; the blocks per CU do not depend on the device
// among gfx950 parts, the CU count is itself cached per device).
template <int ITEMS, int RB>
static int resident_t() {
  static std::atomic<int> per_cu{0};
  int nb = per_cu.load(std::memory_order_relaxed);
  if (nb == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_downsweep<256, ITEMS, SORT_PLAIN, RB>,
                                                     256, 0) != hipSuccess ||
        nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    per_cu.store(nb, std::memory_order_relaxed);
  }
  return nb * device_cu_count();
}

template <int RB>
static int resident_pair() {
  static std::atomic<int> per_cu{0};
  int nb = per_cu.load(std::memory_order_relaxed);
  if (nb == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_downsweep_pair<16, SORT_PLAIN, RB>,
                                                     256, 0) != hipSuccess ||
        nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    per_cu.store(nb, std::memory_order_relaxed);
  }
  return nb * device_cu_count();
}

// Counting parts of a pass over tiles of tile_keys keys: upsweep (or the
// run sums of counts written elsewhere), scans and digit bases.
template <int MODE, int RB>
static void launch_counts(const SortLaunch &a, int tile_keys, int parts, hipStream_t s) {
  constexpr int R = 1 << RB;
  if (parts & (SORT_PART_COUNT | SORT_PART_PREFIX)) {
    const int rt = run_tiles_for(a.total_tiles);
    const int64_t runs = (a.total_tiles + rt - 1) / rt;
    if (parts & SORT_PART_COUNT)
      hipLaunchKernelGGL((k_upsweep<MODE, RB>), dim3((unsigned)runs), dim3(256), 0, s, a,
                         tile_keys, rt);
    else if (a.total_tiles > SMALL_SCAN_TILES)
      hipLaunchKernelGGL(k_run_sums<RB>, dim3((unsigned)runs, R / 256), dim3(256), 0, s, a, rt);
    if (a.total_tiles <= SMALL_SCAN_TILES) {
      hipLaunchKernelGGL(k_scan_small<RB>, dim3(R), dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL(k_block_scan<RB>, dim3(R), dim3(1024), 0, s, a, runs);
      hipLaunchKernelGGL(k_tile_prefix<RB>, dim3((unsigned)runs, R / 256), dim3(256), 0, s, a,
                         rt);
    }
    hipLaunchKernelGGL(k_seg_base<RB>, dim3(a.num_segs), dim3(256), 0, s, a);
  }
}

template <int ITEMS, int MODE, int RB>
static hipError_t launch_pass_t(const SortLaunch &a, int parts, hipStream_t s) {
  launch_counts<MODE, RB>(a, 256 * ITEMS, parts, s);
  if (parts & SORT_PART_SCATTER) {
    // four blocks per resident slot: blocks that finish early make room for
    // the next ones (measured faster than one persistent block per slot)
    const int64_t g = std::max<int64_t>(
        NUM_XCD, std::min<int64_t>(a.total_tiles, 4 * resident_t<ITEMS, RB>()) / NUM_XCD * NUM_XCD);
    hipLaunchKernelGGL((k_downsweep<256, ITEMS, MODE, RB>), dim3((unsigned)g), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// Every use of the pass has its own instantiation (the kernels differ only
// for the two first passes that read their keys from elsewhere), so that a
// profile names the pass a kernel belongs to.
template <int ITEMS, int RB>
static hipError_t launch_pass_items(const SortLaunch &a, int mode, int parts, hipStream_t s) {
  switch (mode) {
    case SORT_NODE_FIRST: return launch_pass_t<ITEMS, SORT_NODE_FIRST, RB>(a, parts, s);
    case SORT_IN_FIRST: return launch_pass_t<ITEMS, SORT_IN_FIRST, RB>(a, parts, s);
    case SORT_NODE: return launch_pass_t<ITEMS, SORT_NODE, RB>(a, parts, s);
    case SORT_VNODE: return launch_pass_t<ITEMS, SORT_VNODE, RB>(a, parts, s);
    case SORT_EDGE: return launch_pass_t<ITEMS, SORT_EDGE, RB>(a, parts, s);
    case SORT_IN: return launch_pass_t<ITEMS, SORT_IN, RB>(a, parts, s);
    case SORT_EDGE_KV: return launch_pass_t<ITEMS, SORT_EDGE_KV, RB>(a, parts, s);
    case SORT_IN_FIRST_KV: return launch_pass_t<ITEMS, SORT_IN_FIRST_KV, RB>(a, parts, s);
    case SORT_IN_KV: return launch_pass_t<ITEMS, SORT_IN_KV, RB>(a, parts, s);
    case SORT_IN_FIRST_DEDUP: return launch_pass_t<ITEMS, SORT_IN_FIRST_DEDUP, RB>(a, parts, s);
    case SORT_PART_ROWS:
    case SORT_PART_DST:
    case SORT_PART_RANK:
      if constexpr (RB == PART_BITS) {
        if (mode == SORT_PART_ROWS) return launch_pass_t<ITEMS, SORT_PART_ROWS, RB>(a, parts, s);
        if (mode == SORT_PART_DST) return launch_pass_t<ITEMS, SORT_PART_DST, RB>(a, parts, s);
        return launch_pass_t<ITEMS, SORT_PART_RANK, RB>(a, parts, s);
      } else {
        return hipErrorInvalidValue;  // partition passes have PART_BITS-bit digits
      }
    default: return launch_pass_t<ITEMS, SORT_PLAIN, RB>(a, parts, s);
  }
}

// Plain passes over two-half tiles (items code PAIR_ITEMS: 2 x 16 keys per
// thread); the two halves' staging fits two blocks per CU up to 9-bit digits.
template <int MODE, int RB>
static hipError_t launch_pair_t(const SortLaunch &a, int parts, hipStream_t s) {
  launch_counts<MODE, RB>(a, 2 * 256 * 16, parts, s);
  if (parts & SORT_PART_SCATTER) {
    const int64_t g = std::max<int64_t>(
        NUM_XCD, std::min<int64_t>(a.total_tiles, 4 * resident_pair<RB>()) / NUM_XCD * NUM_XCD);
    hipLaunchKernelGGL((k_downsweep_pair<16, MODE, RB>), dim3((unsigned)g), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <int RB>
static hipError_t launch_pair_items(const SortLaunch &a, int mode, int parts, hipStream_t s) {
  if constexpr (RB <= 9) {
    switch (mode) {
      case SORT_PLAIN: return launch_pair_t<SORT_PLAIN, RB>(a, parts, s);
      case SORT_EDGE: return launch_pair_t<SORT_EDGE, RB>(a, parts, s);
      case SORT_IN: return launch_pair_t<SORT_IN, RB>(a, parts, s);
      default: return hipErrorInvalidValue;  // the other modes use one-half tiles
    }
  } else {
    return hipErrorInvalidValue;
  }
}

template <int RB>
hipError_t launch_sort_part_rb(const SortLaunch &a, int mode, int items, int parts,
                               hipStream_t s) {
  switch (items) {
    case PAIR_ITEMS: return launch_pair_items<RB>(a, mode, parts, s);
    case 8: return launch_pass_items<8, RB>(a, mode, parts, s);
    case 12: return launch_pass_items<12, RB>(a, mode, parts, s);
    default: return launch_pass_items<16, RB>(a, mode, parts, s);
  }
}

}  // namespace ringo
