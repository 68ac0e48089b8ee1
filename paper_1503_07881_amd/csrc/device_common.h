// Device helpers shared by the kernel files of libringo.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace ringo
