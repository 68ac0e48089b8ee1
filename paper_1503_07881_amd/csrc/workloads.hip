// Seeded synthetic edge-table generators (host and device).
//
// This module produces input rows only; it performs none of the conversion's
// arithmetic, and both the GPU pipeline's tests and the CPU oracle's tests
// draw their inputs from it.
//
// Random numbers: counter-based SplitMix64 (Steele, Lea & Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014).  Draw k of a
// stream with seed s is the SplitMix64 output finaliser applied to
// s + (k + 1) * gamma, so any draw can be computed independently, on the host
// or on the device, with identical results.
//
// R-MAT (Chakrabarti, Zhan & Faloutsos, SDM 2004): one 32-bit draw per level,
// most significant level first, compared against integer quadrant thresholds
// so that host and device generation are bit-identical.
//
// Node identifiers: a dense index i is mapped to mix64(i ^ salt); the
// finaliser is a bijection on 64 bits, so distinct indices give distinct
// identifiers, spread over the whole signed 64-bit range.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <thread>
#include <vector>

#define GEN_GAMMA 0x9E3779B97F4A7C15ull

__host__ __device__ static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ static inline uint64_t draw(uint64_t stream, uint64_t k) {
  return mix64(stream + (k + 1) * GEN_GAMMA);
}

// Uniform integer in [0, m) for m < 2^32 from the top 32 bits of a draw
// (multiply-shift; the bias is below 2^-32 * m).
__host__ __device__ static inline uint64_t below(uint64_t x, uint64_t m) {
  return ((x >> 32) * m) >> 32;
}

// Quadrant thresholds: floor(p * 2^32) for a=0.57, b=0.19, c=0.19, cumulated.
#define RMAT_TA 2448131358ull
#define RMAT_TB (RMAT_TA + 816043786ull)
#define RMAT_TC (RMAT_TB + 816043786ull)

__host__ __device__ static inline void rmat_row(uint64_t stream, uint64_t salt, int scale,
                                                uint64_t r, int64_t *s_out, int64_t *d_out) {
  uint64_t s = 0, d = 0;
  const uint64_t base = r * (uint64_t)scale;
  for (int l = 0; l < scale; ++l) {
    const uint64_t u = draw(stream, base + (uint64_t)l) >> 32;
    const uint64_t sb = u >= RMAT_TB;                       // quadrants (1,0), (1,1)
    const uint64_t db = (u >= RMAT_TA && u < RMAT_TB) || u >= RMAT_TC;  // (0,1), (1,1)
    s = (s << 1) | sb;
    d = (d << 1) | db;
  }
  *s_out = (int64_t)mix64(s ^ salt);
  *d_out = (int64_t)mix64(d ^ salt);
}

template <class F>
static void parallel_for(int64_t n, int threads, F f) {
  if (threads <= 1 || n < (1 << 16)) {
    f(0, n);
    return;
  }
  std::vector<std::thread> pool;
  const int64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    pool.emplace_back([=] { f(lo, hi); });
  }
  for (auto &th : pool) th.join();
}

extern "C" {

uint64_t ringo_gen_mix64(uint64_t x) { return mix64(x); }
uint64_t ringo_gen_draw(uint64_t stream, uint64_t k) { return draw(stream, k); }

// Uniform table: n rows whose first n - ndup rows draw src and dst uniformly
// from a pool of `pool` identifiers mix64(k ^ salt), k < pool; the last ndup
// rows are exact copies of uniformly drawn earlier rows; then, if `shuffle`,
// a Fisher-Yates shuffle of all n rows.  Returns 0, or -1 on bad arguments.
int ringo_gen_uniform(int64_t n, int64_t pool, int64_t ndup, int shuffle, uint64_t s_salt,
                      uint64_t s_src, uint64_t s_dst, uint64_t s_dup, uint64_t s_shuf,
                      int threads, int64_t *src, int64_t *dst) {
  if (n < 0 || pool < 1 || pool >= (1ll << 32) || ndup < 0 || ndup > n) return -1;
  const int64_t nb = n - ndup;
  if (ndup > 0 && (nb < 1 || nb >= (1ll << 32))) return -1;
  const uint64_t salt = mix64(s_salt);
  parallel_for(nb, threads, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      src[r] = (int64_t)mix64(below(draw(s_src, r), pool) ^ salt);
      dst[r] = (int64_t)mix64(below(draw(s_dst, r), pool) ^ salt);
    }
  });
  for (int64_t j = 0; j < ndup; ++j) {
    const int64_t from = (int64_t)below(draw(s_dup, j), nb);
    src[nb + j] = src[from];
    dst[nb + j] = dst[from];
  }
  if (shuffle) {
    for (int64_t i = n - 1; i > 0; --i) {
      // uniform in [0, i]; n < 2^32 is required for the multiply-shift
      const int64_t j = (int64_t)below(draw(s_shuf, i), (uint64_t)i + 1);
      std::swap(src[i], src[j]);
      std::swap(dst[i], dst[j]);
    }
  }
  return 0;
}

// R-MAT table: n rows at the given scale, identifiers mix64(index ^ salt).
int ringo_gen_rmat(int64_t n, int scale, uint64_t s_salt, uint64_t s_rmat, int threads,
                   int64_t *src, int64_t *dst) {
  if (n < 0 || scale < 1 || scale > 62) return -1;
  const uint64_t salt = mix64(s_salt);
  parallel_for(n, threads, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) rmat_row(s_rmat, salt, scale, (uint64_t)r, src + r, dst + r);
  });
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------- device side

__global__ void k_gen_rmat(int64_t n, int scale, uint64_t s_rmat, uint64_t salt, int64_t *src,
                           int64_t *dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride)
    rmat_row(s_rmat, salt, scale, (uint64_t)r, src + r, dst + r);
}

__global__ void k_gen_uniform_base(int64_t nb, int64_t pool, uint64_t s_src, uint64_t s_dst,
                                   uint64_t salt, int64_t *src, int64_t *dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nb; r += stride) {
    src[r] = (int64_t)mix64(below(draw(s_src, r), pool) ^ salt);
    dst[r] = (int64_t)mix64(below(draw(s_dst, r), pool) ^ salt);
  }
}

static int gen_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

extern "C" {

// Device R-MAT into caller-owned device arrays src[n], dst[n] on `stream`.
int ringo_gen_rmat_device(int64_t n, int scale, uint64_t s_salt, uint64_t s_rmat, int64_t *src,
                          int64_t *dst, hipStream_t stream) {
  if (n < 0 || scale < 1 || scale > 62) return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_gen_rmat, dim3(gen_grid(n)), dim3(256), 0, stream, n, scale, s_rmat,
                     mix64(s_salt), src, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Device uniform table without injected duplicates or shuffle (ndup = 0).
int ringo_gen_uniform_device(int64_t n, int64_t pool, uint64_t s_salt, uint64_t s_src,
                             uint64_t s_dst, int64_t *src, int64_t *dst, hipStream_t stream) {
  if (n < 0 || pool < 1 || pool >= (1ll << 32)) return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_gen_uniform_base, dim3(gen_grid(n)), dim3(256), 0, stream, n, pool,
                     s_src, s_dst, mix64(s_salt), src, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"

// ------------------------------------------------------------ calibration
//
// Plain streaming copy of `words` 16-byte words: the reference kernel whose
// bandwidth and HBM counter readings calibrate the measurements of the
// conversion kernels.

__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src,
                                                uint4 *__restrict__ dst, int64_t words) {
  // four 16-byte loads per thread in flight before the stores
  constexpr int U = 4;
  const int64_t stride = (int64_t)gridDim.x * 256 * U;
  for (int64_t i = (int64_t)blockIdx.x * 256 * U + threadIdx.x; i < words; i += stride) {
    uint4 v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = src[std::min<int64_t>(i + j * 256, words - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (i + j * 256 < words) dst[i + j * 256] = v[j];
  }
}

extern "C" int ringo_gen_copy_device(void *dst, const void *src, int64_t bytes,
                                     hipStream_t stream) {
  if (bytes < 0 || (bytes & 15) != 0 || ((uintptr_t)dst & 15) != 0 || ((uintptr_t)src & 15) != 0)
    return -1;
  const int64_t words = bytes / 16;
  if (words == 0) return 0;
  int64_t g = std::min<int64_t>((words + 1023) / 1024, 256 * 8);
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)g), dim3(256), 0, stream, (const uint4 *)src,
                     (uint4 *)dst, words);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
