// Internal types shared by the kernels and the host pipeline of libringo.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ringo {

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int NODE_PASSES = 64 / RADIX_BITS;    // node identifiers are 64-bit keys
constexpr uint64_t SIGN_FLIP = 0x8000000000000000ull;  // unsigned order == signed order

// Tile sizes (elements per tile) of the non-sorting kernels.
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;   // unique / dedupe / in-CSR
constexpr int REMAP_TILE = 256 * 32;                 // rows per remap tile
constexpr int DIR_TILE = 256 * 16;                   // nodes per directory tile

// Element ranges that a tiled kernel walks, per table.
enum RangeKind : int32_t {
  RANGE_NODE_KEYS = 0,  // 2n node keys at 2 * row_off
  RANGE_ROWS = 1,       // n edge keys at row_off
  RANGE_EDGES = 2,      // E unique edges at row_off
  RANGE_NODES = 3,      // V unique nodes at 2 * row_off
};

// Per-table plan, written by the host before each phase.
struct SegPlan {
  const int64_t *src;
  const int64_t *dst;
  int64_t n;        // rows
  int64_t row_off;  // sum of rows of earlier tables
  int64_t V;        // distinct nodes (after the node phase)
  int64_t E;        // distinct edges (after the edge phase)
  int32_t b;        // bits of a dense node index, max(1, ceil(log2 V))
  int32_t dirk;     // log2 of the directory bucket count, ceil(log2 V)
  int64_t dir_off;  // first directory entry of this table
  int64_t *node_ids;
  int64_t *out_off;
  int32_t *out_nbr;
  int64_t *in_off;
  int32_t *in_nbr;
};

__host__ __device__ inline int64_t range_start(const SegPlan &p, int kind) {
  return (kind == RANGE_NODE_KEYS || kind == RANGE_NODES) ? 2 * p.row_off : p.row_off;
}
__host__ __device__ inline int64_t range_count(const SegPlan &p, int kind) {
  switch (kind) {
    case RANGE_NODE_KEYS: return 2 * p.n;
    case RANGE_ROWS: return p.n;
    case RANGE_EDGES: return p.E;
    default: return p.V;
  }
}

// ceil(log2 x) for x >= 1
__host__ __device__ inline int ceil_log2(int64_t x) {
  int k = 0;
  while (((int64_t)1 << k) < x) ++k;
  return k;
}

// ------------------------------------------------------------ kernel launchers

struct Workspace;  // host-side view of the device buffers of one call

struct SortLaunch {
  const uint64_t *in;
  uint64_t *out;
  const SegPlan *plan;
  const int64_t *tmap;        // [S+1] first tile of each table
  int32_t num_segs;
  int32_t range_kind;
  int64_t total_tiles;
  int32_t shift;
  int64_t *digit_base;        // [S][RADIX] first output position of each digit's run
  uint32_t *counts;           // [tiles + 1][RADIX] digit counts, then their prefixes
  uint32_t *bsum;             // [runs][RADIX] counts of runs of tiles, then prefixes
};

enum SortMode : int { SORT_PLAIN = 0, SORT_NODE_FIRST = 1, SORT_IN_FIRST = 2 };

struct TileLaunch {
  const SegPlan *plan;
  const int64_t *tmap;
  int32_t num_segs;
  int32_t range_kind;
  int64_t total_tiles;
};

// Launch helpers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t s);
hipError_t launch_sort_pass(const SortLaunch &a, int mode, int items, hipStream_t s);
int sort_tile(int items);
int sort_resident_blocks(int items);
int64_t sort_runs(int64_t tiles);
hipError_t launch_unique(const TileLaunch &t, const uint64_t *in, uint64_t *out, int64_t *seg_count,
                         uint64_t *status, uint32_t *counter, uint32_t epoch, int grid,
                         hipStream_t s);
// Node directory entry: the bucket's first key and its position range.
struct alignas(16) DirEntry {
  uint64_t key;
  uint32_t start;
  uint32_t next;
};

hipError_t launch_dir(const TileLaunch &t, const uint64_t *nodes, DirEntry *dir, int grid,
                      hipStream_t s);
hipError_t launch_remap(const TileLaunch &t, const uint64_t *nodes, const DirEntry *dir,
                        uint64_t *ekeys, int grid, hipStream_t s);
hipError_t launch_dedupe(const TileLaunch &t, const uint64_t *in, uint64_t *out,
                         int64_t *seg_count, uint64_t *status, uint32_t *counter,
                         uint32_t epoch, int grid, hipStream_t s);
hipError_t launch_in_csr(const TileLaunch &t, const uint64_t *in, int grid, hipStream_t s);
hipError_t launch_empty_offsets(const SegPlan *plan, int32_t S, hipStream_t s);
int device_cu_count();

}  // namespace ringo
