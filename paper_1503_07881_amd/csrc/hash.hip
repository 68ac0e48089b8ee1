// Node numbering through a node hash table.
//
// The paper keeps a graph's nodes in a hash table whose collisions go to the
// next free slot (Section 2.5, the paragraph on concurrent hash tables), and
// its Twitter2010 walk-through (Section 3) inserts both identifiers of every
// row into that table.  Here that table replaces the
// 2n-key radix sort of the node keys: only the V distinct keys are sorted,
// which is what fixes the dense positions, so the output is identical to
// the sort-based numbering.
//
//   estimate   HyperLogLog count of the distinct keys of each table
//              (Flajolet, Fusy, Gandouet & Meunier 2007), 2^10 registers;
//              the host sizes each table's slots from it (load <= 2/3)
//   insert     every row's two keys, lock-free compare-and-swap into the
//              first free slot of the probe sequence; the slot of every
//              key is written out (32-bit, src then dst per table)
//   compact    occupied slots -> the table's distinct keys (unordered; for
//              one table, grouped by bucket of their top 12 bits)
//   (sort)     the V keys: bucket by bucket in LDS when no bucket is over
//              BUCKET_CAP keys (node ids and ranks written directly), else
//              with the radix passes of kernels.hip
//   rank       after the radix passes: position of every sorted key, stored
//              beside its slot; node ids
//   remap      every row's (src, dst) slots -> positions (a gather from the
//              rank array), packed (s << b) | d
//
// The slots hold keys only (8 bytes) and the ranks live in their own 4-byte
// array, so the probe phase walks a table half the size, and the remap reads
// only the rank array, a quarter of it.
//
// Large tables probed often (partitioned numbering): a probe in row order
// misses every cache once the table outgrows them, so the keys are first
// grouped by the part of the table their home slot lies in (2^PART_BITS
// contiguous parts), with the radix pass kernels:
//   group rows   the rows by their source key's part, destination keys
//                carried beside them (grouped sources, then destinations)
//   group dst    the carried destination keys by their own part
//   insert       both groupings, tiles in contiguous ranges per XCD, so the
//                probes of one XCD meet one part at a time in its L2; the
//                slot of every key is written beside it (grouped order)
//   (compact, sort, rank as above)
//   rank slots   the grouped source keys' slots become their positions (a
//                gather from the part's slice of the rank array)
//   group rank   the grouping of the destination keys again, now carrying
//                the position of the source key beside each
//   pack         (source position, destination position) edge keys in the
//                destinations' grouped order, the destination positions
//                gathered through their slots; the edge sort does not need
//                row order
// Multigraph edges keep their rows through the sorts, so they stay in row
// order and take the remap.
//
// Keys are uint64(id) ^ 2^63 as in the sort-based path.  The key ~0 marks a
// free slot; a table holding that key sets a flag instead (its elements get
// the slot index NO_SLOT), and since ~0 is the largest key its position is
// always V - 1.  A probe sequence longer than min(capacity, MAX_PROBES) sets
// an overflow flag and stops; the host then converts that call with the
// sort-based numbering instead.

#include "device_common.h"
#include "ringo_internal.h"

namespace ringo {

constexpr uint32_t NO_SLOT = 0xffffffffu;

// ------------------------------------------------------------- estimate

__device__ __forceinline__ void hll_add(uint32_t *R, uint64_t h) {
  const uint32_t idx = (uint32_t)(h >> (64 - HLL_BITS));
  const uint64_t w = h << HLL_BITS;
  const uint32_t rho = w == 0 ? 64 - HLL_BITS + 1 : (uint32_t)__clzll((long long)w) + 1;
  if (R[idx] < rho) atomicMax(&R[idx], rho);  // the read only skips redundant atomics
}

// With pcounts, the estimate also counts the source keys' parts for the
// rows' grouping pass: per grouping tile of ptile rows (tile map ptmap,
// ptile dividing HLL_TILE), pcounts [tile][2^PART_BITS].  Each bin is split
// over four sub-counters (lane mod 4), as in the radix passes' counting, so
// the lanes of a hub's rows do not all meet at one counter.
__global__ __launch_bounds__(256) void k_hll(TileLaunch t, uint32_t *regs, uint32_t *pcounts,
                                             const int64_t *ptmap, int ptile) {
  constexpr int PR = 1 << PART_BITS, PSUB = 4, MAX_PSUB = HLL_TILE / 2048;
  __shared__ uint32_t R[HLL_M];
  __shared__ uint32_t s_pc[MAX_PSUB * PR * PSUB];
  const int tid = threadIdx.x;
  const int nsub = pcounts ? HLL_TILE / ptile : 0;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    for (int i = tid; i < HLL_M; i += 256) R[i] = 0;
    for (int i = tid; i < nsub * PR * PSUB; i += 256) s_pc[i] = 0;
    __syncthreads();
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)HLL_TILE;
    const int64_t end = std::min<int64_t>(base + HLL_TILE, P.n);
    constexpr int U = 4;
    for (int64_t r0 = base + tid; r0 < end; r0 += U * 256) {
      uint64_t s[U], d[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int64_t r = std::min<int64_t>(r0 + j * 256, end - 1);
        s[j] = (uint64_t)__builtin_nontemporal_load(&G(P.src)[r]) ^ SIGN_FLIP;
        d[j] = (uint64_t)__builtin_nontemporal_load(&G(P.dst)[r]) ^ SIGN_FLIP;
      }
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (r0 + j * 256 < end) {
          const uint64_t hs = fmix64(s[j]);
          hll_add(R, hs);
          hll_add(R, fmix64(d[j]));
          if (pcounts)
            atomicAdd(&s_pc[((int)((r0 + j * 256 - base) / ptile) * PR +
                             (int)(hs >> (64 - PART_BITS))) * PSUB + (tid & (PSUB - 1))], 1u);
        }
    }
    __syncthreads();
    uint32_t *g = regs + (int64_t)seg * HLL_M;
    for (int i = tid; i < HLL_M; i += 256) {
      const uint32_t v = R[i];
      if (v > G(g)[i]) atomicMax(&g[i], v);
    }
    if (pcounts) {
      // the grouping tiles of this estimate tile that hold rows of the table
      const int64_t first = base / ptile;
      for (int i = tid; i < nsub * PR; i += 256) {
        const int st = i / PR;
        if ((first + st) * ptile < P.n) {
          const uint32_t *c = s_pc + i * PSUB;
          G(pcounts)[(ptmap[seg] + first + st) * PR + i % PR] = c[0] + c[1] + c[2] + c[3];
        }
      }
    }
    __syncthreads();
  }
}

// One block per table: the bias-corrected harmonic-mean estimate, with
// linear counting while it is below 2.5 m and registers are still zero.
__global__ __launch_bounds__(256) void k_hll_estimate(const SegPlan *plan, int S,
                                                      const uint32_t *regs, int64_t *est) {
  __shared__ double s_sum[4];
  __shared__ int s_zero[4];
  const int seg = blockIdx.x;
  if (seg >= S) return;
  const uint32_t *g = regs + (int64_t)seg * HLL_M;
  double sum = 0;
  int zeros = 0;
  for (int i = threadIdx.x; i < HLL_M; i += 256) {
    const uint32_t v = g[i];
    sum += ldexp(1.0, -(int)v);
    zeros += v == 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_down(sum, o, 64);
    zeros += __shfl_down(zeros, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    s_sum[w] = sum;
    s_zero[w] = zeros;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sum = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
    zeros = s_zero[0] + s_zero[1] + s_zero[2] + s_zero[3];
    const double m = HLL_M;
    const double alpha = 0.7213 / (1.0 + 1.079 / m);
    double e = alpha * m * m / sum;
    if (e <= 2.5 * m && zeros > 0) e = m * log(m / zeros);
    est[seg] = plan[seg].n == 0 ? 0 : (int64_t)ceil(e);
  }
}

hipError_t launch_hll(const TileLaunch &rows, uint32_t *regs, int64_t *est, uint32_t *pcounts,
                      const int64_t *ptmap, int ptile, int grid, hipStream_t s) {
  if (pcounts && (ptile < 2048 || HLL_TILE % ptile != 0)) return hipErrorInvalidValue;
  if (rows.total_tiles > 0)
    hipLaunchKernelGGL(k_hll, dim3(grid), dim3(256), 0, s, rows, regs, pcounts, ptmap, ptile);
  hipLaunchKernelGGL(k_hll_estimate, dim3(rows.num_segs), dim3(256), 0, s, rows.plan,
                     rows.num_segs, regs, est);
  return hipGetLastError();
}

// --------------------------------------------------------------- insert
//
// The row columns, the slots and the edge keys are each read or written once
// per kernel, in order, so those accesses are non-temporal: the caches stay
// with the table and rank gathers, which are reused.
//
// Each thread carries the keys of U rows through their probe sequences at
// once so that their loads overlap.  A slot goes from free to its key exactly
// once, so a plain load that still sees it free is corrected by the
// compare-and-swap, and a plain load that sees a key sees the final value.

__global__ __launch_bounds__(256) void k_hash_insert(TileLaunch t, uint64_t *hkeys,
                                                     uint32_t *slots, uint32_t *flags) {
  const int tid = threadIdx.x;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    uint64_t *T = hkeys + P.tab_off;
    uint32_t *sl = slots + 2 * P.row_off;
    const uint64_t mask = (uint64_t)P.tab_cap - 1;
    const int lcap = __builtin_ctzll((uint64_t)P.tab_cap);  // tables with rows have slots
    const uint32_t max_probes = (uint32_t)std::min<int64_t>(P.tab_cap, MAX_PROBES);
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)REMAP_TILE;
    const int64_t end = std::min<int64_t>(base + REMAP_TILE, P.n);
    uint32_t flag = 0;
    constexpr int U = 4;
    for (int64_t r0 = base + tid; r0 < end; r0 += U * 256) {
      uint64_t u[2 * U], pos[2 * U];
      uint32_t left[2 * U];
      bool act[2 * U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int64_t r = std::min<int64_t>(r0 + j * 256, end - 1);
        u[j] = (uint64_t)__builtin_nontemporal_load(&G(P.src)[r]) ^ SIGN_FLIP;
        u[U + j] = (uint64_t)__builtin_nontemporal_load(&G(P.dst)[r]) ^ SIGN_FLIP;
      }
#pragma unroll
      for (int j = 0; j < 2 * U; ++j) {
        const bool valid = r0 + (j % U) * 256 < end;
        if (valid && u[j] == EMPTY_KEY) flag |= HFLAG_MAX_KEY;
        act[j] = valid && u[j] != EMPTY_KEY;
        pos[j] = home_slot(fmix64(u[j]), lcap);
        left[j] = max_probes;
      }
      // First probe of every key unconditionally (all loads in flight at
      // once); later probes only for the keys still walking, so that lanes
      // that are done add no memory traffic.
      bool more = true;
      bool first = true;
      while (more) {
        uint64_t k[2 * U];
        if (first) {
#pragma unroll
          for (int j = 0; j < 2 * U; ++j) k[j] = G(T)[pos[j]];
          first = false;
        } else {
#pragma unroll
          for (int j = 0; j < 2 * U; ++j) k[j] = act[j] ? G(T)[pos[j]] : 0ull;
        }
        more = false;
#pragma unroll
        for (int j = 0; j < 2 * U; ++j) {
          if (!act[j]) continue;
          uint64_t seen = k[j];
          if (seen == EMPTY_KEY) seen = atomicCAS((unsigned long long *)&T[pos[j]],
                                                  (unsigned long long)EMPTY_KEY,
                                                  (unsigned long long)u[j]);
          if (seen == EMPTY_KEY || seen == u[j]) {
            act[j] = false;
          } else if (--left[j] == 0) {
            flag |= HFLAG_OVERFLOW;
            act[j] = false;
          } else {
            pos[j] = (pos[j] + 1) & mask;
            more = true;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (r0 + j * 256 < end) {
          __builtin_nontemporal_store(u[j] == EMPTY_KEY ? NO_SLOT : (uint32_t)pos[j], &G(sl)[r0 + j * 256]);
          __builtin_nontemporal_store(u[U + j] == EMPTY_KEY ? NO_SLOT : (uint32_t)pos[U + j], &G(sl)[P.n + r0 + j * 256]);
        }
    }
    if (flag) atomicOr(&flags[seg], flag);
  }
}

// ------------------------------------------------- partitioned numbering
//
// With the keys grouped by the part of the table their home slot lies in,
// the blocks of one XCD walk a contiguous range of tiles (blocks go to the
// XCDs round-robin, and the grid is a multiple of their count), so the
// probes of that XCD meet one part of the table at a time, which stays in
// its L2.

__device__ __forceinline__ int64_t xcd_first_tile(int64_t total) {
  return total * (blockIdx.x % NUM_XCD) / NUM_XCD + blockIdx.x / NUM_XCD;
}
__device__ __forceinline__ int64_t xcd_end_tile(int64_t total) {
  return total * (blockIdx.x % NUM_XCD + 1) / NUM_XCD;
}
inline int xcd_grid(int grid) { return std::max(NUM_XCD, grid / NUM_XCD * NUM_XCD); }

// The insert of k_hash_insert over grouped keys; the slot of every key
// goes to slots + row_off (sequential in the grouped order).
__global__ __launch_bounds__(256) void k_hash_insert_keys(TileLaunch t, const uint64_t *keys,
                                                          uint64_t *hkeys, uint32_t *slots,
                                                          uint32_t *flags) {
  const int tid = threadIdx.x;
  const int64_t t_end = xcd_end_tile(t.total_tiles);
  for (int64_t tile = xcd_first_tile(t.total_tiles); tile < t_end; tile += gridDim.x / NUM_XCD) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    uint64_t *T = hkeys + P.tab_off;
    const uint64_t *K = keys + P.row_off;
    const uint64_t mask = (uint64_t)P.tab_cap - 1;
    const int lcap = __builtin_ctzll((uint64_t)P.tab_cap);  // tables with rows have slots
    const uint32_t max_probes = (uint32_t)std::min<int64_t>(P.tab_cap, MAX_PROBES);
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)REMAP_TILE;
    const int64_t end = std::min<int64_t>(base + REMAP_TILE, P.n);
    uint32_t flag = 0;
    constexpr int U = 8;
    for (int64_t r0 = base + tid; r0 < end; r0 += U * 256) {
      uint64_t u[U], pos[U];
      uint32_t left[U];
      bool act[U];
#pragma unroll
      for (int j = 0; j < U; ++j)
        u[j] = __builtin_nontemporal_load(&G(K)[std::min<int64_t>(r0 + j * 256, end - 1)]);
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const bool valid = r0 + j * 256 < end;
        if (valid && u[j] == EMPTY_KEY) flag |= HFLAG_MAX_KEY;
        act[j] = valid && u[j] != EMPTY_KEY;
        pos[j] = home_slot(fmix64(u[j]), lcap);
        left[j] = max_probes;
      }
      bool more = true;
      bool first = true;
      while (more) {
        uint64_t k[U];
        if (first) {
#pragma unroll
          for (int j = 0; j < U; ++j) k[j] = G(T)[pos[j]];
          first = false;
        } else {
#pragma unroll
          for (int j = 0; j < U; ++j) k[j] = act[j] ? G(T)[pos[j]] : 0ull;
        }
        more = false;
#pragma unroll
        for (int j = 0; j < U; ++j) {
          if (!act[j]) continue;
          uint64_t seen = k[j];
          if (seen == EMPTY_KEY) seen = atomicCAS((unsigned long long *)&T[pos[j]],
                                                  (unsigned long long)EMPTY_KEY,
                                                  (unsigned long long)u[j]);
          if (seen == EMPTY_KEY || seen == u[j]) {
            act[j] = false;
          } else if (--left[j] == 0) {
            flag |= HFLAG_OVERFLOW;
            act[j] = false;
          } else {
            pos[j] = (pos[j] + 1) & mask;
            more = true;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (r0 + j * 256 < end)
          __builtin_nontemporal_store(u[j] == EMPTY_KEY ? NO_SLOT : (uint32_t)pos[j], &G(slots)[P.row_off + r0 + j * 256]);
    }
    if (flag) atomicOr(&flags[seg], flag);
  }
}

hipError_t launch_hash_insert_keys(const TileLaunch &rows, const uint64_t *keys, uint64_t *hkeys,
                                   uint32_t *slots, uint32_t *flags, int grid, hipStream_t s) {
  if (rows.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_insert_keys, dim3(xcd_grid(grid)), dim3(256), 0, s, rows, keys, hkeys,
                     slots, flags);
  return hipGetLastError();
}

// Positions of grouped keys from their recorded slots, in place: the
// slots of one part lie in one slice of the rank array, which stays in the
// L2 of the XCD walking that part.
__global__ __launch_bounds__(256) void k_hash_rank_slots(TileLaunch t, uint32_t *slot_rank,
                                                         const uint32_t *hrank) {
  const int tid = threadIdx.x;
  const int64_t t_end = xcd_end_tile(t.total_tiles);
  for (int64_t tile = xcd_first_tile(t.total_tiles); tile < t_end; tile += gridDim.x / NUM_XCD) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint32_t *R = hrank + P.tab_off;
    uint32_t *SR = slot_rank + P.row_off;
    const uint32_t last = (uint32_t)(P.V - 1);
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)REMAP_TILE;
    const int64_t end = std::min<int64_t>(base + REMAP_TILE, P.n);
    constexpr int U = 8;
    for (int64_t r0 = base + tid; r0 < end; r0 += U * 256) {
      uint32_t q[U], rk[U];
#pragma unroll
      for (int j = 0; j < U; ++j) q[j] = __builtin_nontemporal_load(&G(SR)[std::min<int64_t>(r0 + j * 256, end - 1)]);
#pragma unroll
      for (int j = 0; j < U; ++j) rk[j] = G(R)[q[j] == NO_SLOT ? 0u : q[j]];
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (r0 + j * 256 < end) __builtin_nontemporal_store(q[j] == NO_SLOT ? last : rk[j], &G(SR)[r0 + j * 256]);
    }
  }
}

hipError_t launch_hash_rank_slots(const TileLaunch &rows, uint32_t *slot_rank,
                                  const uint32_t *hrank, int grid, hipStream_t s) {
  if (rows.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_rank_slots, dim3(xcd_grid(grid)), dim3(256), 0, s, rows, slot_rank,
                     hrank);
  return hipGetLastError();
}

// Edge keys from the destination keys' recorded slots (grouped order) and
// the source positions beside them; the counts of the first edge pass as in
// k_hash_remap.
__global__ __launch_bounds__(256) void k_hash_pack_parts(TileLaunch t, const uint32_t *dslots,
                                                         const uint32_t *spos,
                                                         const uint32_t *hrank, uint64_t *ekeys,
                                                         int sym, uint32_t *counts0, int sort_tile,
                                                         const int64_t *esort_tmap) {
  constexpr int MAX_SUB = REMAP_TILE / 2048;  // sort tiles of at least 2048 keys
  __shared__ uint32_t s_c[MAX_SUB * FUSED_RADIX];
  const int tid = threadIdx.x;
  const int nsub = counts0 ? REMAP_TILE / sort_tile : 0;
  for (int i = tid; i < nsub * FUSED_RADIX; i += 256) s_c[i] = 0;
  __syncthreads();
  const int64_t t_end = xcd_end_tile(t.total_tiles);
  for (int64_t tile = xcd_first_tile(t.total_tiles); tile < t_end; tile += gridDim.x / NUM_XCD) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint32_t *R = hrank + P.tab_off;
    const uint32_t last = (uint32_t)(P.V - 1);
    const int b = P.b;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)REMAP_TILE;
    const int64_t end = std::min<int64_t>(base + REMAP_TILE, P.n);
    constexpr int U = 8;
    for (int64_t r0 = base + tid; r0 < end; r0 += U * 256) {
      uint32_t q[U], rs[U], rd[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int64_t r = P.row_off + std::min<int64_t>(r0 + j * 256, end - 1);
        q[j] = __builtin_nontemporal_load(&G(dslots)[r]);
        rs[j] = __builtin_nontemporal_load(&G(spos)[r]);
      }
#pragma unroll
      for (int j = 0; j < U; ++j) rd[j] = G(R)[q[j] == NO_SLOT ? 0u : q[j]];
#pragma unroll
      for (int j = 0; j < U; ++j) rd[j] = q[j] == NO_SLOT ? last : rd[j];
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (r0 + j * 256 < end) {
          const uint64_t key = ((uint64_t)rs[j] << b) | rd[j];
          if (sym) {  // both orientations, 2n keys at 2 * row_off
            G(ekeys)[2 * P.row_off + r0 + j * 256] = key;
            G(ekeys)[2 * P.row_off + P.n + r0 + j * 256] = ((uint64_t)rd[j] << b) | rs[j];
          } else {
            __builtin_nontemporal_store(key, &G(ekeys)[P.row_off + r0 + j * 256]);
            if (counts0)
              atomicAdd(&s_c[(int)((r0 + j * 256 - base) / sort_tile) * FUSED_RADIX +
                             (uint32_t)(key & (FUSED_RADIX - 1))], 1u);
          }
        }
    }
    if (counts0) {
      __syncthreads();
      const int64_t first = (tile - t.tmap[seg]) * nsub;
      for (int i = tid; i < nsub * FUSED_RADIX; i += 256) {
        const int st = i / FUSED_RADIX;
        if ((first + st) * sort_tile < P.n)
          G(counts0)[(esort_tmap[seg] + first + st) * FUSED_RADIX + i % FUSED_RADIX] = s_c[i];
        s_c[i] = 0;
      }
      __syncthreads();
    }
  }
}

hipError_t launch_hash_pack_parts(const TileLaunch &rows, const uint32_t *dslots,
                                  const uint32_t *spos, const uint32_t *hrank, uint64_t *ekeys, int sym,
                                  uint32_t *counts0, int sort_tile, const int64_t *esort_tmap,
                                  int grid, hipStream_t s) {
  if (rows.total_tiles == 0) return hipSuccess;
  if (counts0 && (sym || sort_tile < 2048 || REMAP_TILE % sort_tile != 0))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hash_pack_parts, dim3(xcd_grid(grid)), dim3(256), 0, s, rows, dslots, spos,
                     hrank, ekeys, sym, counts0, sort_tile, esort_tmap);
  return hipGetLastError();
}

// Exclusive scan of the bucket counts (bstart [NBUCKETS + 1], bcur a copy of
// its first NBUCKETS entries), the largest bucket into *max_bucket and the
// total into *count.
__global__ __launch_bounds__(1024) void k_bucket_plan(const uint32_t *bcnt, uint32_t *bstart,
                                                      uint32_t *bcur, int64_t *max_bucket,
                                                      uint64_t *count) {
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_m[16];
  constexpr int PER = NBUCKETS / 1024;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t v[PER], sum = 0, mx = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    v[i] = bcnt[tid * PER + i];
    sum += v[i];
    mx = std::max(mx, v[i]);
  }
  uint32_t total;
  uint32_t run = block_excl_scan<1024>(sum, s_w, total);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    bstart[tid * PER + i] = run;
    bcur[tid * PER + i] = run;
    run += v[i];
  }
  if (tid == 0) {
    bstart[NBUCKETS] = total;
    *count = total;  // the table's distinct keys
  }
  for (int o = 32; o > 0; o >>= 1) mx = std::max(mx, (uint32_t)__shfl_down((int)mx, o, 64));
  if (lane == 0) s_m[w] = mx;
  __syncthreads();
  if (tid == 0) {
    uint32_t m = 0;
    for (int i = 0; i < 16; ++i) m = std::max(m, s_m[i]);
    *max_bucket = m;
  }
}

hipError_t launch_hash_insert(const TileLaunch &rows, uint64_t *hkeys, uint32_t *slots,
                              uint32_t *flags, int grid, hipStream_t s) {
  if (rows.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_insert, dim3(grid), dim3(256), 0, s, rows, hkeys, slots, flags);
  return hipGetLastError();
}

// Bucketed placement of one table's keys, by BP_BLOCKS blocks that each own a
// contiguous range of slots (the same ranges in both kernels):
//   count   keys per bucket, in LDS, added to bcnt once per block and bucket
//   place   after the scan of bcnt: each block reserves its range in every
//           bucket it holds keys of with one atomic, then places its keys
//           with LDS cursors (key to nodes, slot to bslot)
constexpr int BP_BLOCKS = 128;
constexpr int BP_THREADS = 1024;

__device__ __forceinline__ void slot_range(const SegPlan &P, int64_t &s0, int64_t &s1) {
  const int64_t per = (P.tab_cap + BP_BLOCKS - 1) / BP_BLOCKS;
  s0 = std::min<int64_t>((int64_t)blockIdx.x * per, P.tab_cap);
  s1 = std::min<int64_t>(s0 + per, P.tab_cap);
}

__global__ __launch_bounds__(BP_THREADS) void k_bucket_count(const SegPlan *plan,
                                                             const uint64_t *hkeys,
                                                             uint32_t *bcnt) {
  __shared__ uint32_t h[NBUCKETS];
  const int tid = threadIdx.x;
  for (int i = tid; i < NBUCKETS; i += BP_THREADS) h[i] = 0;
  __syncthreads();
  const SegPlan P = plan[0];
  const uint64_t *T = hkeys + P.tab_off;
  int64_t s0, s1;
  slot_range(P, s0, s1);
  constexpr int U = 8;
  for (int64_t i0 = s0 + tid; i0 < s1; i0 += U * BP_THREADS) {
    uint64_t k[U];
#pragma unroll
    for (int j = 0; j < U; ++j) k[j] = G(T)[std::min<int64_t>(i0 + j * BP_THREADS, s1 - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (i0 + j * BP_THREADS < s1 && k[j] != EMPTY_KEY)
        atomicAdd(&h[k[j] >> (64 - BUCKET_BITS)], 1u);
  }
  __syncthreads();
  for (int i = tid; i < NBUCKETS; i += BP_THREADS)
    if (h[i]) atomicAdd(&bcnt[i], h[i]);
}

__global__ __launch_bounds__(BP_THREADS) void k_bucket_place(const SegPlan *plan,
                                                             const uint64_t *hkeys,
                                                             uint32_t *bcur, uint64_t *nodes,
                                                             uint32_t *bslot) {
  __shared__ uint32_t h[NBUCKETS];  // this block's keys per bucket, then its cursors
  __shared__ uint32_t base[NBUCKETS];
  const int tid = threadIdx.x;
  for (int i = tid; i < NBUCKETS; i += BP_THREADS) h[i] = 0;
  __syncthreads();
  const SegPlan P = plan[0];
  const uint64_t *T = hkeys + P.tab_off;
  int64_t s0, s1;
  slot_range(P, s0, s1);
  constexpr int U = 8;
  for (int64_t i0 = s0 + tid; i0 < s1; i0 += U * BP_THREADS) {
    uint64_t k[U];
#pragma unroll
    for (int j = 0; j < U; ++j) k[j] = G(T)[std::min<int64_t>(i0 + j * BP_THREADS, s1 - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (i0 + j * BP_THREADS < s1 && k[j] != EMPTY_KEY)
        atomicAdd(&h[k[j] >> (64 - BUCKET_BITS)], 1u);
  }
  __syncthreads();
  for (int i = tid; i < NBUCKETS; i += BP_THREADS) {
    const uint32_t c = h[i];
    base[i] = c ? atomicAdd(&bcur[i], c) : 0u;
    h[i] = 0;
  }
  __syncthreads();
  for (int64_t i0 = s0 + tid; i0 < s1; i0 += U * BP_THREADS) {
    uint64_t k[U];
#pragma unroll
    for (int j = 0; j < U; ++j) k[j] = G(T)[std::min<int64_t>(i0 + j * BP_THREADS, s1 - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (i0 + j * BP_THREADS < s1 && k[j] != EMPTY_KEY) {
        const uint32_t bk = (uint32_t)(k[j] >> (64 - BUCKET_BITS));
        const uint32_t pos = base[bk] + atomicAdd(&h[bk], 1u);
        G(nodes)[pos] = k[j];
        G(bslot)[pos] = (uint32_t)(i0 + j * BP_THREADS);
      }
  }
}

// -------------------------------------------------------------- compact

constexpr int CMP_ITEMS = 16;
constexpr int CMP_TILE = 256 * CMP_ITEMS;

__global__ __launch_bounds__(256) void k_hash_compact(TileLaunch t, const uint64_t *hkeys,
                                                      uint64_t *nodes, uint64_t *count) {
  __shared__ uint32_t s_w[4];
  __shared__ uint64_t s_base;
  const int tid = threadIdx.x;
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint64_t *T = hkeys + P.tab_off;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)CMP_TILE;
    const int64_t cnt = std::min<int64_t>(CMP_TILE, P.tab_cap - base);
    uint64_t k[CMP_ITEMS];
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < CMP_ITEMS; ++i) {
      const int idx = i * 256 + tid;
      k[i] = G(T)[base + (idx < cnt ? idx : 0)];
      if (idx >= cnt) k[i] = EMPTY_KEY;
      mine += k[i] != EMPTY_KEY;
    }
    uint32_t total;
    const uint32_t off = block_excl_scan<256>(mine, s_w, total);
    if (tid == 0) s_base = total ? atomicAdd((unsigned long long *)&count[seg],
                                             (unsigned long long)total) : 0;
    __syncthreads();
    uint64_t *out = nodes + 2 * P.row_off + s_base + off;
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < CMP_ITEMS; ++i)
      if (k[i] != EMPTY_KEY) G(out)[o++] = k[i];
    __syncthreads();
  }
}

// One thread per table: the key ~0 goes after the others, and the count (or
// -1 after an overflow) becomes the table's V.
__global__ void k_hash_finish(const SegPlan *plan, int S, uint64_t *nodes, const uint64_t *count,
                              const uint32_t *flags, int64_t *seg_V) {
  const int seg = blockIdx.x * blockDim.x + threadIdx.x;
  if (seg >= S) return;
  const uint32_t f = flags[seg];
  int64_t v = (int64_t)count[seg];
  if (f & HFLAG_OVERFLOW) {
    v = -1;
  } else if (f & HFLAG_MAX_KEY) {
    nodes[2 * plan[seg].row_off + v] = EMPTY_KEY;
    ++v;
  }
  seg_V[seg] = v;
}

hipError_t launch_hash_compact(const TileLaunch &slots, const uint64_t *hkeys, uint64_t *nodes,
                               uint64_t *count, const uint32_t *flags, int64_t *seg_V,
                               const BucketLaunch *bk, int grid, hipStream_t s) {
  if (bk) {
    // one table, bucketed: the scan of the bucket counts gives the count
    if (slots.total_tiles > 0)
      hipLaunchKernelGGL(k_bucket_count, dim3(BP_BLOCKS), dim3(BP_THREADS), 0, s, slots.plan,
                         hkeys, bk->bcnt);
    hipLaunchKernelGGL(k_bucket_plan, dim3(1), dim3(1024), 0, s, bk->bcnt, bk->bstart, bk->bcur,
                       bk->max_bucket, count);
    if (slots.total_tiles > 0)
      hipLaunchKernelGGL(k_bucket_place, dim3(BP_BLOCKS), dim3(BP_THREADS), 0, s, slots.plan,
                         hkeys, bk->bcur, nodes, bk->bslot);
  } else if (slots.total_tiles > 0) {
    hipLaunchKernelGGL(k_hash_compact, dim3(grid), dim3(256), 0, s, slots, hkeys, nodes, count);
  }
  const int S = slots.num_segs;
  hipLaunchKernelGGL(k_hash_finish, dim3((S + 255) / 256), dim3(256), 0, s, slots.plan, S, nodes,
                     count, flags, seg_V);
  return hipGetLastError();
}

// ----------------------------------------------------------------- rank

__global__ __launch_bounds__(256) void k_hash_rank(TileLaunch t, const uint64_t *sorted,
                                                   const uint64_t *hkeys, uint32_t *hrank) {
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint64_t *nd = sorted + 2 * P.row_off;
    const uint64_t *T = hkeys + P.tab_off;
    const uint64_t mask = (uint64_t)P.tab_cap - 1;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)DIR_TILE;
    const int64_t end = std::min<int64_t>(base + DIR_TILE, P.V);
    for (int64_t j = base + threadIdx.x; j < end; j += 256) {
      const uint64_t u = G(nd)[j];
      G(P.node_ids)[j] = (int64_t)(u ^ SIGN_FLIP);
      if (u == EMPTY_KEY) continue;
      uint64_t pos = home_slot(fmix64(u), __builtin_ctzll((uint64_t)P.tab_cap));
      // the key is in the table (no overflow): the walk ends within tab_cap slots
      for (int64_t left = P.tab_cap; left > 0 && G(T)[pos] != u; --left) pos = (pos + 1) & mask;
      G(hrank)[P.tab_off + pos] = (uint32_t)j;
    }
  }
}

hipError_t launch_hash_rank(const TileLaunch &nodes_t, const uint64_t *sorted,
                            const uint64_t *hkeys, uint32_t *hrank, int grid, hipStream_t s) {
  if (nodes_t.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_rank, dim3(grid), dim3(256), 0, s, nodes_t, sorted, hkeys, hrank);
  return hipGetLastError();
}

// ----------------------------------------------------------- bucket sort
//
// One workgroup per bucket of the top BUCKET_BITS key bits (at most
// BUCKET_CAP keys, all distinct), in LDS: a counting sort on the next
// SUB_BITS bits puts the keys in sub-bucket order, and a key's rank inside
// the bucket is its sub-bucket's start plus the number of smaller keys in
// its sub-bucket (few: the sub-buckets split the bucket a thousandfold).
// Then node_ids and each key's position at its slot in hrank.  Buckets are
// in key order, so bucket start + rank inside the bucket is the key's
// position among all V keys.

constexpr int BS_THREADS = 256;
constexpr int SUB_BITS = 10;
constexpr int NSUB = 1 << SUB_BITS;

__global__ __launch_bounds__(BS_THREADS) void k_bucket_sort(const SegPlan *plan,
                                                            const uint32_t *bstart,
                                                            const uint64_t *keys,
                                                            const uint32_t *bslot,
                                                            const uint32_t *flags,
                                                            uint32_t *hrank) {
  __shared__ uint64_t s_k[BUCKET_CAP];  // the keys in sub-bucket order
  __shared__ uint32_t s_i[BUCKET_CAP];  // their indices in the bucket
  __shared__ uint32_t s_st[NSUB + 1];   // sub-bucket counts, then starts
  __shared__ uint32_t s_cur[NSUB];      // placement cursors
  __shared__ uint32_t s_w[BS_THREADS / 64];
  const int b = blockIdx.x, tid = threadIdx.x;
  const SegPlan P = plan[0];
  if (b == 0 && tid == 0 && (flags[0] & HFLAG_MAX_KEY))
    G(P.node_ids)[P.V - 1] = (int64_t)(EMPTY_KEY ^ SIGN_FLIP);  // the flagged key ~0 is last
  const uint32_t s = bstart[b];
  const int c = (int)(bstart[b + 1] - s);  // <= BUCKET_CAP, checked by the host
  if (c == 0) return;
  const __attribute__((address_space(1))) uint64_t *K = G(keys) + s;
  constexpr int SHIFT = 64 - BUCKET_BITS - SUB_BITS;
  for (int i = tid; i < NSUB; i += BS_THREADS) s_st[i] = 0;
  __syncthreads();
  for (int i = tid; i < c; i += BS_THREADS) atomicAdd(&s_st[(K[i] >> SHIFT) & (NSUB - 1)], 1u);
  __syncthreads();
  // exclusive scan of the NSUB counts: NSUB / BS_THREADS consecutive ones a thread
  constexpr int PER = NSUB / BS_THREADS;
  uint32_t v[PER], sum = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    v[q] = s_st[tid * PER + q];
    sum += v[q];
  }
  uint32_t total;
  uint32_t run = block_excl_scan<BS_THREADS>(sum, s_w, total);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    s_st[tid * PER + q] = run;
    s_cur[tid * PER + q] = run;
    run += v[q];
  }
  if (tid == 0) s_st[NSUB] = total;
  __syncthreads();
  for (int i = tid; i < c; i += BS_THREADS) {
    const uint64_t k = K[i];
    const uint32_t p = atomicAdd(&s_cur[(k >> SHIFT) & (NSUB - 1)], 1u);
    s_k[p] = k;
    s_i[p] = (uint32_t)i;
  }
  __syncthreads();
  uint32_t *R = hrank + P.tab_off;
  for (int p = tid; p < c; p += BS_THREADS) {
    const uint64_t k = s_k[p];
    const uint32_t sb = (uint32_t)(k >> SHIFT) & (NSUB - 1);
    const uint32_t q0 = s_st[sb], q1 = s_st[sb + 1];
    uint32_t r = q0;
    for (uint32_t q = q0; q < q1; ++q) r += s_k[q] < k;
    G(P.node_ids)[s + r] = (int64_t)(k ^ SIGN_FLIP);
    G(R)[G(bslot)[s + s_i[p]]] = s + r;
  }
}

hipError_t launch_bucket_sort(const SegPlan *plan, const BucketLaunch &bk, const uint64_t *keys,
                              const uint32_t *flags, uint32_t *hrank, hipStream_t s) {
  hipLaunchKernelGGL(k_bucket_sort, dim3(NBUCKETS), dim3(BS_THREADS), 0, s, plan, bk.bstart, keys,
                     bk.bslot, flags, hrank);
  return hipGetLastError();
}

// ---------------------------------------------------------------- remap

__global__ __launch_bounds__(256) void k_hash_remap(TileLaunch t, const uint32_t *slots,
                                                    const uint32_t *hrank, uint64_t *ekeys,
                                                    int sym, uint32_t *counts0, int sort_tile,
                                                    const int64_t *esort_tmap) {
  constexpr int MAX_SUB = REMAP_TILE / 2048;  // sort tiles of at least 2048 keys
  __shared__ uint32_t s_c[MAX_SUB * FUSED_RADIX];   // first-digit counts of the tile's sort tiles
  const int tid = threadIdx.x;
  const int nsub = counts0 ? REMAP_TILE / sort_tile : 0;
  for (int i = tid; i < nsub * FUSED_RADIX; i += 256) s_c[i] = 0;
  __syncthreads();
  for (int64_t tile = blockIdx.x; tile < t.total_tiles; tile += gridDim.x) {
    const int seg = find_seg(t.tmap, t.num_segs, tile);
    const SegPlan P = t.plan[seg];
    const uint32_t *sl = slots + 2 * P.row_off;
    const uint32_t *R = hrank + P.tab_off;
    const uint32_t last = (uint32_t)(P.V - 1);
    const int b = P.b;
    const int64_t base = (tile - t.tmap[seg]) * (int64_t)REMAP_TILE;
    const int64_t end = std::min<int64_t>(base + REMAP_TILE, P.n);
    constexpr int U = 8;
    for (int64_t r0 = base + tid; r0 < end; r0 += U * 256) {
      uint32_t q[2 * U], rk[2 * U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int64_t r = std::min<int64_t>(r0 + j * 256, end - 1);
        q[j] = __builtin_nontemporal_load(&G(sl)[r]);
        q[U + j] = __builtin_nontemporal_load(&G(sl)[P.n + r]);
      }
#pragma unroll
      for (int j = 0; j < 2 * U; ++j) rk[j] = G(R)[q[j] == NO_SLOT ? 0u : q[j]];
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (r0 + j * 256 < end) {
          const uint32_t rs = q[j] == NO_SLOT ? last : rk[j];
          const uint32_t rd = q[U + j] == NO_SLOT ? last : rk[U + j];
          const uint64_t key = ((uint64_t)rs << b) | rd;
          if (sym) {  // both orientations, 2n keys at 2 * row_off
            G(ekeys)[2 * P.row_off + r0 + j * 256] = key;
            G(ekeys)[2 * P.row_off + P.n + r0 + j * 256] = ((uint64_t)rd << b) | rs;
          } else {
            __builtin_nontemporal_store(key, &G(ekeys)[P.row_off + r0 + j * 256]);
            if (counts0)
              atomicAdd(&s_c[(int)((r0 + j * 256 - base) / sort_tile) * FUSED_RADIX +
                             (uint32_t)(key & (FUSED_RADIX - 1))], 1u);
          }
        }
    }
    if (counts0) {
      __syncthreads();
      // sort tiles of this remap tile that hold rows of the table
      const int64_t first = (tile - t.tmap[seg]) * nsub;
      for (int i = tid; i < nsub * FUSED_RADIX; i += 256) {
        const int st = i / FUSED_RADIX;
        if ((first + st) * sort_tile < P.n)
          G(counts0)[(esort_tmap[seg] + first + st) * FUSED_RADIX + i % FUSED_RADIX] = s_c[i];
        s_c[i] = 0;
      }
      __syncthreads();
    }
  }
}

hipError_t launch_hash_remap(const TileLaunch &rows, const uint32_t *slots, const uint32_t *hrank,
                             uint64_t *ekeys, int sym, uint32_t *counts0, int sort_tile,
                             const int64_t *esort_tmap, int grid, hipStream_t s) {
  if (rows.total_tiles == 0) return hipSuccess;
  if (counts0 && (sym || sort_tile < 2048 || REMAP_TILE % sort_tile != 0))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hash_remap, dim3(grid), dim3(256), 0, s, rows, slots, hrank, ekeys, sym,
                     counts0, sort_tile, esort_tmap);
  return hipGetLastError();
}

}  // namespace ringo
