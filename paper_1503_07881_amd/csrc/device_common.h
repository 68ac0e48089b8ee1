// Device helpers shared by the kernel files of libringo.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ringo_internal.h"

namespace ringo {

// --------------------------------------------------------------- helpers

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Pointers read from the plan are generic to the compiler; G() marks them as
// global-memory pointers so that accesses compile to global (not flat)
// instructions, which keep LDS waits independent of outstanding loads.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *G(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Index s of the table whose tiles hold tile t: tmap[s] <= t < tmap[s+1].
__device__ __forceinline__ int find_seg(const int64_t *tmap, int S, int64_t t) {
  int lo = 0, hi = S;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tmap[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// MurmurHash3's 64-bit finaliser (Appleby): a bijection with full avalanche.
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Home slot of a key with hash h in a node hash table of 2^lcap slots: the
// top lcap bits of the hash.
__device__ __forceinline__ uint64_t home_slot(uint64_t h, int lcap) {
  return lcap > 0 ? h >> (64 - lcap) : 0;
}

// Part of key u: the top PART_BITS bits of its hash.  The home slots of a
// part's keys form one contiguous range of every table of at least
// 2^PART_BITS slots (the table's 2^PART_BITS equal parts, in order), and
// the part does not depend on the table's size.
__device__ __forceinline__ uint32_t slot_part(uint64_t u) {
  return (uint32_t)(fmix64(u) >> (64 - PART_BITS));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan of one value per thread over the block; `total` receives
// the block sum.  Every thread of the block must call it.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v, lane);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BLOCK / 64; ++i) {
    const uint32_t x = s_w[i];
    off += (i < w) ? x : 0u;
    tot += x;
  }
  total = tot;
  __syncthreads();
  return off + inc - v;
}

// Writes `len` units of value (w0) or (w0, w1) from dst on: by this lane
// when the run is short, else queued in chunks for launch_gap_fill (chunks
// beyond the queue's capacity, which its bound never reaches, are written
// here as well).
__device__ __forceinline__ void fill_run(const GapQueue &q, uint64_t *dst, int64_t len,
                                         uint64_t w0, uint64_t w1, int words) {
  if (len <= 0) return;
  int64_t from = 0;  // first unit this lane writes itself
  if (len > GAP_INLINE && q.e) {
    const int64_t chunks = (len + GAP_CHUNK - 1) / GAP_CHUNK;
    const uint64_t at = atomicAdd(q.count, (uint32_t)chunks);
    const int64_t queued = at >= q.cap ? 0 : std::min<int64_t>(chunks, (int64_t)q.cap - (int64_t)at);
    for (int64_t c = 0; c < queued; ++c) {
      GapEntry g;
      g.dst = dst + c * GAP_CHUNK * words;
      g.len = std::min<int64_t>(GAP_CHUNK, len - c * GAP_CHUNK);
      g.w0 = w0;
      g.w1 = w1;
      g.words = words;
      q.e[at + c] = g;
    }
    from = std::min<int64_t>(len, queued * GAP_CHUNK);
  }
  __attribute__((address_space(1))) uint64_t *p = G(dst);
  for (int64_t u = from; u < len; ++u) {
    p[u * words] = w0;
    if (words == 2) p[u * words + 1] = w1;
  }
}

}  // namespace ringo
