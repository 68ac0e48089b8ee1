// Internal types shared by the kernels and the host pipeline of libringo.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ringo.h"

namespace ringo {

// Radix digits of the LSD passes: 8 to 11 bits, chosen per table size by
// the schedule table.
constexpr int MIN_DIGIT_BITS = 8, MAX_DIGIT_BITS = 11, DEFAULT_DIGIT_BITS = 8;
// LSD passes over the low `bits` bits of the keys with digits of rb bits.
inline int lsd_passes(int bits, int rb) { return (bits + rb - 1) / rb; }
// Digit width of pass p of an LSD sort of `bits`-bit keys in
// lsd_passes(bits, rb) passes: where the passes' total width leaves room,
// passes take 8-bit digits (a quarter or less of the counters per tile of
// the wider ones), and those come first; the rest take rb bits.
inline int lsd_width(int bits, int rb, int p) {
  const int P = lsd_passes(bits, rb);
  const int spare = bits - 8 * P;
  const int wide = rb == 8 || spare <= 0 ? 0 : (spare + rb - 9) / (rb - 8);
  return p < P - wide ? 8 : rb;
}
// Lowest key bit of pass p's digit.
inline int lsd_shift(int bits, int rb, int p) {
  int s = 0;
  for (int q = 0; q < p; ++q) s += lsd_width(bits, rb, q);
  return s;
}
// The remap's fused counts of the first edge pass are for 8-bit digits.
constexpr int FUSED_RADIX_BITS = 8;
constexpr int FUSED_RADIX = 1 << FUSED_RADIX_BITS;
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
  RANGE_SLOTS = 4,      // tab_cap node hash table slots at tab_off
  RANGE_EDGES2 = 5,     // E unique edges at 2 * row_off (undirected graphs)
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
  int64_t tab_off;  // first node hash table slot of this table
  int64_t tab_cap;  // node hash table slots (a power of two, or 0)
  int64_t *node_ids;
  int64_t *out_off;
  int32_t *out_nbr;
  int64_t *in_off;
  int32_t *in_nbr;
  int32_t *out_eid;  // multigraph: row of every out-list entry
  int32_t *in_eid;   // multigraph: row of every in-list entry
};

__host__ __device__ inline int64_t range_start(const SegPlan &p, int kind) {
  if (kind == RANGE_SLOTS) return p.tab_off;
  return (kind == RANGE_NODE_KEYS || kind == RANGE_NODES || kind == RANGE_EDGES2) ? 2 * p.row_off
                                                                                  : p.row_off;
}
__host__ __device__ inline int64_t range_count(const SegPlan &p, int kind) {
  switch (kind) {
    case RANGE_NODE_KEYS: return 2 * p.n;
    case RANGE_ROWS: return p.n;
    case RANGE_EDGES:
    case RANGE_EDGES2: return p.E;
    case RANGE_SLOTS: return p.tab_cap;
    default: return p.V;
  }
}

// ceil(log2 x) for x >= 1
__host__ __device__ inline int ceil_log2(int64_t x) {
  int k = 0;
  while (((int64_t)1 << k) < x) ++k;
  return k;
}

// Runs of equal entries in the offset arrays (and the node directory): the
// positions of a node range without edges, such as the leaves of a star,
// all take the value that follows them.  The lane that finds a run writes
// it when it is short; a long run is queued in chunks of GAP_CHUNK units,
// and launch_gap_fill then writes every queued chunk with the whole grid.
constexpr int64_t GAP_INLINE = 256;       // longest run a lane writes itself
constexpr int64_t GAP_CHUNK = 1 << 16;    // units per queued chunk
struct GapEntry {
  uint64_t *dst;   // first word of the chunk
  int64_t len;     // units
  uint64_t w0, w1; // the unit's value: w0 (8-byte units) or w0, w1 (16-byte)
  int64_t words;   // words per unit: 1 or 2
};
struct GapQueue {
  GapEntry *e = nullptr;     // null: every run is written by its lane
  uint32_t *count = nullptr; // chunks queued (may pass cap; those beyond are not queued)
  uint32_t cap = 0;
};
// Chunks that runs totalling `units` entries of one array can queue.
inline int64_t gap_chunks_bound(int64_t units) {
  return units / (GAP_INLINE + 1) + units / GAP_CHUNK + 2;
}

// ------------------------------------------------------------ kernel launchers


struct SortLaunch {
  const uint64_t *in;
  uint64_t *out;
  const SegPlan *plan;
  const int64_t *tmap;        // [S+1] first tile of each table
  int32_t num_segs;
  int32_t range_kind;
  int64_t total_tiles;
  int32_t shift;
  // R = 2^digit bits of the pass
  int64_t *digit_base;        // [S][R] first output position of each digit's run
  uint32_t *counts;           // [tiles + 1][R] digit counts, then their prefixes
  uint32_t *bsum;             // [runs][R] counts of runs of tiles, then prefixes
  const uint32_t *vin;        // values carried with the keys (key-value modes), else null
  uint32_t *vout;
  int64_t *seg_total;         // if set, the count part writes each table's key total
  GapQueue gaps;              // long runs of the out-offsets (first in-pass with dedupe)
  // partition passes (SORT_PART_ROWS): the destination keys carried beside
  // the source keys
  uint64_t *wout;
};

// Key source of a pass: the two first passes read their keys from elsewhere
// (the node keys from the columns, the in-keys by repacking the out-keys);
// the other values are plain passes, kept apart only so that each use of
// the pass is its own kernel instantiation.
// The _KV modes carry a 32-bit value (the row of a multigraph edge) with
// every key.
enum SortMode : int {
  SORT_PLAIN = 0, SORT_NODE_FIRST = 1, SORT_IN_FIRST = 2,
  SORT_NODE = 3, SORT_VNODE = 4, SORT_EDGE = 5, SORT_IN = 6,
  SORT_EDGE_KV = 7, SORT_IN_FIRST_KV = 8, SORT_IN_KV = 9,
  // first in-pass over the sorted edge keys with their repeats: only the
  // first copy of each key is sorted, and the pass also writes out_nbr and
  // out_off at the de-duplicated positions (dedupe folded into the pass)
  SORT_IN_FIRST_DEDUP = 10,
  // Partition passes of the partitioned hash numbering (PART_BITS-bit
  // digits: the part of the table a key's home slot lies in).  ROWS: the
  // rows' source keys (uint64(id) ^ 2^63, grouped by their part) to out,
  // their destination keys beside them to wout.  DST: the keys of in (the
  // grouped destination keys) by their part.  RANK: the same grouping as
  // DST, which it repeats, carrying the 32-bit values of vin (the source
  // keys' positions), and writes only those (to vout).
  SORT_PART_ROWS = 11, SORT_PART_DST = 12, SORT_PART_RANK = 13
};
enum SortPart : int { SORT_PART_COUNT = 1, SORT_PART_SCATTER = 2, SORT_PART_PREFIX = 4 };

struct TileLaunch {
  const SegPlan *plan;
  const int64_t *tmap;
  int32_t num_segs;
  int32_t range_kind;
  int64_t total_tiles;
  GapQueue gaps;  // long runs of offsets or directory entries the kernel writes
};

// Launch helpers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t s);
// One part of a pass on digits of digit_bits bits (MIN_DIGIT_BITS to
// MAX_DIGIT_BITS; anything else is hipErrorInvalidValue): SORT_PART_COUNT
// (digit counts of every tile and their prefixes) or SORT_PART_SCATTER (the
// stable scatter), or both; SORT_PART_PREFIX instead of SORT_PART_COUNT
// when the tile counts (counts [tile][R]) were written by the kernel that
// produced the keys.
hipError_t launch_sort_part(const SortLaunch &a, int mode, int items, int digit_bits, int parts,
                            hipStream_t s);
// The same for one digit width (lsd.h, instantiated in lsd_d8.hip to
// lsd_d11.hip).
template <int RB>
hipError_t launch_sort_part_rb(const SortLaunch &a, int mode, int items, int parts, hipStream_t s);
// Tiles per upsweep run: the power of two in [4, 32] that gives about 2048
// runs (blocks), so that small inputs still spread over the device.
inline int run_tiles_for(int64_t tiles) {
  const int64_t r = tiles / 2048;
  int rt = 4;
  while (rt < 32 && 2 * rt <= r) rt *= 2;
  return rt;
}
int sort_tile(int items);
// Items code of the plain passes' two-half tiles: 2 x 16 keys per thread,
// sort_tile(PAIR_ITEMS) = 8192 keys per tile.
constexpr int PAIR_ITEMS = 32;
int64_t sort_runs(int64_t tiles);
int64_t sort_runs_bound(int64_t max_tiles);  // >= sort_runs(t) for every t <= max_tiles
// Distinct sorted node keys of every table into out, their count into
// seg_count (tcnt: total_tiles + 1 words of workspace).
hipError_t launch_unique(const TileLaunch &t, const uint64_t *in, uint64_t *out, int64_t *seg_count,
                         uint32_t *tcnt, int grid, hipStream_t s);
// Node directory entry: the bucket's first key and its position range.
struct alignas(16) DirEntry {
  uint64_t key;
  uint32_t start;
  uint32_t next;
};

hipError_t launch_dir(const TileLaunch &t, const uint64_t *nodes, DirEntry *dir, int grid,
                      hipStream_t s);
// sym (undirected graphs): both orientations, 2n keys at 2 * row_off.
hipError_t launch_remap(const TileLaunch &t, const uint64_t *nodes, const DirEntry *dir,
                        uint64_t *ekeys, int sym, int grid, hipStream_t s);
// ------------------------------------------------- node hash table (hash.hip)

constexpr int HLL_BITS = 10;                 // log2 of the count-estimate registers
constexpr int HLL_M = 1 << HLL_BITS;
constexpr int HLL_TILE = 256 * 64;           // rows per estimate tile
constexpr uint64_t EMPTY_KEY = ~0ull;        // free slot (the key ~0 is flagged aside)
constexpr uint32_t HFLAG_MAX_KEY = 1;        // the table holds the key ~0
constexpr uint32_t HFLAG_OVERFLOW = 2;       // a probe sequence exceeded its bound
constexpr int NUM_XCD = 8;                   // accelerator complex dies of the MI355X
constexpr uint32_t MAX_PROBES = 4096;        // probe bound of the insert (and of lookups)
// Parts of a node hash table for the partitioned numbering: keys grouped by
// the part of the table their home slot lies in (top PART_BITS bits of the
// slot index) meet only that part's slots, a slice small enough for L2.
constexpr int PART_BITS = 8;

// regs [S][HLL_M] must start at zero; est[S] receives the distinct-count
// estimate of each table's 2n keys.  pcounts (or null): the source keys'
// part counts per grouping tile of ptile rows (a divisor of HLL_TILE, at
// least 2048; tile map ptmap), pcounts [tile][2^PART_BITS], for the rows'
// grouping pass of the partitioned numbering.
hipError_t launch_hll(const TileLaunch &rows, uint32_t *regs, int64_t *est, uint32_t *pcounts,
                      const int64_t *ptmap, int ptile, int grid, hipStream_t s);
// hkeys (tab_cap slots per table at tab_off) must hold EMPTY_KEY; flags [S]
// and count [S] start at zero.  The insert writes the slot of every key to
// slots [2 * row_off + r] (source) and [2 * row_off + n + r] (destination).
// After launch_hash_compact, seg_V[s] is the number of distinct keys of table
// s, or -1 when its table overflowed, and the keys (unordered) are at
// nodes + 2 * row_off.
// Bucketed node sort (one table): buckets of the top BUCKET_BITS key bits.
// bcnt must start at zero.  With a BucketLaunch, launch_hash_compact counts
// the table's keys per bucket (bcnt), scans the counts (bstart, bcur),
// writes the largest bucket to *max_bucket, and places every key in its
// bucket's range (nodes) with its slot (bslot); launch_bucket_sort, allowed
// when no bucket exceeds BUCKET_CAP, then writes node_ids and hrank.
constexpr int BUCKET_BITS = 12;
constexpr int NBUCKETS = 1 << BUCKET_BITS;
constexpr int BUCKET_CAP = 2048;
struct BucketLaunch {
  uint32_t *bcnt;        // [NBUCKETS]
  uint32_t *bstart;      // [NBUCKETS + 1]
  uint32_t *bcur;        // [NBUCKETS]
  uint32_t *bslot;       // [V]
  int64_t *max_bucket;   // one value
};
hipError_t launch_hash_insert(const TileLaunch &rows, uint64_t *hkeys, uint32_t *slots,
                              uint32_t *flags, int grid, hipStream_t s);
hipError_t launch_hash_compact(const TileLaunch &slot_tiles, const uint64_t *hkeys,
                               uint64_t *nodes, uint64_t *count, const uint32_t *flags,
                               int64_t *seg_V, const BucketLaunch *bk, int grid, hipStream_t s);
hipError_t launch_bucket_sort(const SegPlan *plan, const BucketLaunch &bk, const uint64_t *keys,
                              const uint32_t *flags, uint32_t *hrank, hipStream_t s);
// Writes node_ids from the sorted keys and each key's position into hrank at
// its slot.
hipError_t launch_hash_rank(const TileLaunch &nodes_t, const uint64_t *sorted,
                            const uint64_t *hkeys, uint32_t *hrank, int grid, hipStream_t s);
// Every row's (src, dst) slots -> dense positions, packed edge keys (sym as
// for launch_remap).
// counts0 (directed and multigraph keys, sort tiles of sort_tile rows that
// divide REMAP_TILE, tile map esort_tmap): the remap also writes the digit
// counts of the first edge pass (8-bit digits, bits [0, FUSED_RADIX_BITS))
// of every sort tile, counts0 [tile][FUSED_RADIX]; null otherwise.
hipError_t launch_hash_remap(const TileLaunch &rows, const uint32_t *slots, const uint32_t *hrank,
                             uint64_t *ekeys, int sym, uint32_t *counts0, int sort_tile,
                             const int64_t *esort_tmap, int grid, hipStream_t s);
// Partitioned numbering.  Inserts the n keys of each table at keys +
// row_off (uint64(id) ^ 2^63, grouped by part) into its table and writes
// each key's slot to slots + row_off (NO_SLOT for the key ~0); flags as for
// launch_hash_insert.
hipError_t launch_hash_insert_keys(const TileLaunch &rows, const uint64_t *keys, uint64_t *hkeys,
                                   uint32_t *slots, uint32_t *flags, int grid, hipStream_t s);
// The slots at slot_rank + row_off become the keys' positions among their
// table's distinct keys (gathered from hrank at each table's tab_off), in
// place.
hipError_t launch_hash_rank_slots(const TileLaunch &rows, uint32_t *slot_rank,
                                  const uint32_t *hrank, int grid, hipStream_t s);
// Packed edge keys from the grouped destination keys' slots (dslots +
// row_off) and the source positions at the same places (spos + row_off):
// each destination's position is gathered from hrank; sym and counts0 as
// for launch_hash_remap.
hipError_t launch_hash_pack_parts(const TileLaunch &rows, const uint32_t *dslots,
                                  const uint32_t *spos, const uint32_t *hrank, uint64_t *ekeys, int sym,
                                  uint32_t *counts0, int sort_tile, const int64_t *esort_tmap,
                                  int grid, hipStream_t s);

// Multigraph: out-offsets of the sorted keys (every key its own edge) and
// each table's edge count (its key count) into seg_count.
hipError_t launch_multi_offsets(const TileLaunch &t, const uint64_t *in, int64_t *seg_count,
                                int grid, hipStream_t s);
// Undirected graphs: first copy of every sorted key (compaction into out)
// and the out-offsets, by per-tile head counts and a scan (tcnt:
// total_tiles + 1 words of workspace).
hipError_t launch_dedupe_scan(const TileLaunch &t, const uint64_t *in, uint64_t *out,
                              int64_t *seg_count, uint32_t *tcnt, int grid, hipStream_t s);
// vals (multigraph): the row of every (d, s)-sorted edge, copied to in_eid.
hipError_t launch_in_csr(const TileLaunch &t, const uint64_t *in, const uint32_t *vals, int grid,
                         hipStream_t s);
// Undirected graphs: out-neighbours from the unique keys (E at 2 * row_off).
hipError_t launch_out_nbr(const TileLaunch &t, const uint64_t *in, int grid, hipStream_t s);
// Multigraph: v[row_off + r] = r for every row of every table.
hipError_t launch_iota(const TileLaunch &rows, uint32_t *v, int grid, hipStream_t s);
hipError_t launch_empty_offsets(const SegPlan *plan, int32_t S, hipStream_t s);
// Writes the chunks queued in q (after the kernel that queued them).
hipError_t launch_gap_fill(const GapQueue &q, hipStream_t s);
// Sync-free single table (kernels.hip): the plan and tile maps passed by
// value (at most META_WORDS words) and copied to dst, results[0, nres)
// zeroed; V and E moved from results into the plan on the device (and to
// ve = {V, E}); the outputs of an empty table.
constexpr int META_WORDS = 64;
struct MetaWords {
  uint64_t w[META_WORDS];
};
hipError_t launch_meta_init(const MetaWords &m, int32_t nwords, uint64_t *dst, int64_t *results,
                            int32_t nres, hipStream_t s);
// The metadata kernel itself (its node is found in a captured graph by it).
const void *meta_init_kernel();
hipError_t launch_plan_nodes(SegPlan *plan, const int64_t *results, int32_t dirk_cap,
                             hipStream_t s);
hipError_t launch_plan_edges(SegPlan *plan, const int64_t *results, int64_t *ve, hipStream_t s);
hipError_t launch_fixed_empty(int64_t *out_off, int64_t *in_off, int64_t *ve, hipStream_t s);
int device_cu_count();

// ------------------------------------------------ small tables (small.hip)

constexpr int SMALL_ROWS = 2048;  // tables of at most this many rows fit one workgroup's LDS

// One small table: its columns and worst-case-sized outputs (V <= 2n,
// E <= n): node_ids [2n], out_off and in_off [2n + 1], out_nbr and in_nbr [n].
struct SmallTable {
  const int64_t *src;
  const int64_t *dst;
  int64_t n;
  int64_t *node_ids;
  int64_t *out_off;
  int64_t *in_off;
  int32_t *out_nbr;
  int32_t *in_nbr;
};

// Converts count small tables (directed kind), one workgroup each; V and E
// of table i go to vres[2i] and vres[2i + 1].
hipError_t launch_small(const SmallTable *tabs, int count, int64_t *vres, hipStream_t s);

// The batched conversion (directed) with every table's outputs in device
// blocks of its own, so that its graphs are freed one by one (the served
// form), and the device bytes that a graph's outputs hold: the blocks of
// its owner (all tables' blocks when a batch shares them), as requested from
// the allocator; 0 for a graph that owns nothing.
ringo_status_t convert_separate(int32_t S, const int64_t *const *src, const int64_t *const *dst,
                                const int64_t *num_rows, ringo_graph_t *outs, hipStream_t stream);
size_t graph_bytes(const ringo_graph_t *g);
// ringo_graph_free with the release ordered on `stream` instead of the
// stream that built the graph (whose later work the arrays no longer need),
// so that allocations on `stream` can reuse the memory at once.  Only for a
// graph that no enqueued work reads any more.
void graph_free_on(ringo_graph_t *g, hipStream_t stream);

// Stream-ordered device memory from the library's allocator (the caller's
// hooks when set, else the library's cache of device blocks); used by the
// entry points other than the conversion itself.
void *workspace_alloc(size_t bytes, hipStream_t s);
void workspace_free(void *p, hipStream_t s);

}  // namespace ringo
