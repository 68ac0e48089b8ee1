// Host side of libringo: the C ABI, the memory planner and the pass driver.
//
// One call converts S >= 1 tables.  Every phase runs once for the whole
// batch, each kernel walking the tiles of all tables:
//
//   phase N  node numbering, by one of two methods (same result):
//            sort   8 radix passes over the 2n node keys, unique
//            hash   distinct-count estimate (sync #0 sizes the tables),
//                   node hash table insert, compaction of the V keys (for
//                   one table, grouped by bucket of their top bits)
//   sync #1  read back V of every table, size the node-sized outputs
//   phase E  sort: directory + remap; hash: the V keys sorted bucket by
//            bucket in LDS (one table, no crowded bucket) or by radix
//            passes and ranked, then the remap (which also counts the first
//            edge pass's digits); then radix passes over the packed edge
//            keys, dedupe + out-offsets
//   sync #2  read back E of every table, size the edge-sized outputs
//   phase I  radix passes over the (d, s) keys (the first one also writes
//            the out-neighbours), in-CSR
//
// Everything is enqueued on the caller's stream.  The synchronisations exist
// only to size buffers and outputs exactly: like the paper's conversion
// (Section 2.4), which counts neighbours before it places them, nothing is
// sized by a guess that could fall short.

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "ringo.h"
#include "ringo_internal.h"
#include "tuned_schedule.h"

using namespace ringo;

namespace {

// ----------------------------------------------------------- allocation

struct AllocHooks {
  void *(*alloc)(size_t, hipStream_t, void *) = nullptr;
  void (*free_)(void *, hipStream_t, void *) = nullptr;
  void *ctx = nullptr;
};

std::mutex g_mu;
AllocHooks g_hooks;

AllocHooks hooks() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_hooks;
}

// Device blocks of the built-in allocator.  The runtime's stream-ordered
// pool gives its memory back to the device at synchronisations whatever its
// release threshold, so that repeated large calls map and unmap tens of
// gigabytes each time (freeing the outputs of a 10^9-row batch then took
// over a second).  The library keeps its own cache instead: a freed block
// stays allocated, and a request takes the smallest cached block that holds
// it (up to a quarter, or 64 MB, larger) once the block's last use has
// completed, or at once on the stream that used it last (stream order).
// Cached blocks go back to the device only when hipMalloc fails.
struct CachedBlock {
  void *p;
  size_t size;
  hipStream_t stream;
  hipEvent_t ev;  // recorded on `stream` when the block was freed
};
struct DeviceCache {
  std::mutex mu;
  std::multimap<size_t, CachedBlock> idle;   // by size
  std::unordered_map<void *, size_t> live;   // handed-out blocks and their sizes
  std::vector<hipEvent_t> spare;             // events of reused blocks
};
DeviceCache g_cache[64];

size_t size_class(size_t bytes) {
  const size_t g = bytes <= ((size_t)1 << 20) ? 512 : ((size_t)2 << 20);
  return (bytes + g - 1) / g * g;
}

// Every idle block back to the device (after its last use).  Caller holds C.mu.
void release_idle(DeviceCache &C) {
  for (auto &kv : C.idle) {
    (void)hipEventSynchronize(kv.second.ev);
    (void)hipEventDestroy(kv.second.ev);
    (void)hipFree(kv.second.p);
  }
  C.idle.clear();
  (void)hipGetLastError();
}

void *cache_alloc(size_t bytes, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return nullptr;
  }
  DeviceCache &C = g_cache[dev];
  const size_t want = size_class(bytes);
  const size_t most = std::max(want + want / 4, want + ((size_t)64 << 20));
  std::lock_guard<std::mutex> lk(C.mu);
  for (auto it = C.idle.lower_bound(want); it != C.idle.end() && it->first <= most; ++it) {
    const CachedBlock b = it->second;
    bool ready = b.stream == s;
    if (!ready) {
      const hipError_t q = hipEventQuery(b.ev);
      ready = q == hipSuccess;
      if (q != hipSuccess) (void)hipGetLastError();
    }
    if (ready) {
      C.idle.erase(it);
      C.spare.push_back(b.ev);
      C.live[b.p] = b.size;
      return b.p;
    }
  }
  void *p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    release_idle(C);
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  C.live[p] = want;
  return p;
}

void cache_free(void *p, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    dev = 0;
  }
  // the block's device: the current one, else the one whose cache holds it
  for (int k = 0; k < 64; ++k) {
    std::lock_guard<std::mutex> lk(g_cache[(dev + k) % 64].mu);
    if (g_cache[(dev + k) % 64].live.count(p)) {
      dev = (dev + k) % 64;
      break;
    }
  }
  DeviceCache &C = g_cache[dev];
  std::lock_guard<std::mutex> lk(C.mu);
  auto it = C.live.find(p);
  if (it == C.live.end()) return;  // not a block of the cache
  const size_t size = it->second;
  C.live.erase(it);
  hipEvent_t ev = nullptr;
  if (!C.spare.empty()) {
    ev = C.spare.back();
    C.spare.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);  // no event: the block is idle once the stream is
    (void)hipFree(p);
    return;
  }
  if (hipEventRecord(ev, s) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)hipEventRecord(ev, nullptr);
  }
  C.idle.insert({size, CachedBlock{p, size, s, ev}});
}

void *dev_alloc(const AllocHooks &h, size_t bytes, hipStream_t s) {
  bytes = std::max<size_t>(bytes, 256);
  if (h.alloc) return h.alloc(bytes, s, h.ctx);
  return cache_alloc(bytes, s);
}

void dev_free(const AllocHooks &h, void *p, hipStream_t s) {
  if (!p) return;
  if (h.free_) h.free_(p, s, h.ctx);
  else cache_free(p, s);
}

// Owner of output arrays: of one call (shared by the graphs of a batch), or
// of one table when a batch gives every table blocks of its own.
struct Owner {
  std::atomic<int> refs{0};
  void *blocks[3] = {nullptr, nullptr, nullptr};  // node-sized, edge-sized, small tables
  size_t bytes = 0;  // device bytes of the blocks (as requested from the allocator)
  hipStream_t stream = nullptr;
  AllocHooks hooks;
};

void owner_release(Owner *o) {
  if (!o) return;
  if (o->refs.fetch_sub(1) == 1) {
    for (void *b : o->blocks) dev_free(o->hooks, b, o->stream);
    delete o;
  }
}

// Pinned staging buffers for plan uploads and count read-backs.  A buffer
// returns to the pool with an event recorded after its last copy.
struct Pinned {
  void *p = nullptr;
  size_t size = 0;
  hipEvent_t ev = nullptr;
  bool busy = false;
};
std::vector<Pinned *> g_pinned;

Pinned *pinned_acquire(size_t bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (Pinned *b : g_pinned)
    if (!b->busy && b->size >= bytes && hipEventQuery(b->ev) == hipSuccess) {
      b->busy = true;
      return b;
    }
  Pinned *b = new Pinned();
  bytes = std::max<size_t>(bytes, 1 << 16);
  if (hipHostMalloc(&b->p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return nullptr;
  }
  if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(b->p);
    delete b;
    return nullptr;
  }
  b->size = bytes;
  b->busy = true;
  g_pinned.push_back(b);
  return b;
}

void pinned_release(Pinned *b, hipStream_t s) {
  if (!b) return;
  (void)hipEventRecord(b->ev, s);
  std::lock_guard<std::mutex> lk(g_mu);
  b->busy = false;
}

// ------------------------------------------------------------- schedule

// Items per thread of the scatter tile, digit bits of the radix passes and
// node-numbering method by table size (log2 buckets of rows).  Built-in
// defaults, from measurements on an MI355X (R-MAT tables, 2^10 to 1.5e9
// rows): up to 2^26 rows the autotuner's table (tuned_schedule.h, generated
// from its cache); where it has no entry, the sort numbering up to 2^23 rows
// and the hash numbering above, 8 items per thread and 8-bit digits up to
// 2^26 rows; above, 16 items (full 128-byte digit runs), and from 2^29 rows
// 9-bit digits, which save an edge pass and an in-pass once node indices
// need 25 bits or more (3-4% faster at 2^29 and 1.5e9 rows).
int g_items[64];
int g_bits[64];
int g_method[64];
bool g_items_init = false;
constexpr int HASH_DEFAULT_LOG2 = 24;
constexpr int WIDE_TILE_LOG2 = 27;   // 16 items per thread from 2^27 rows
constexpr int WIDE_DIGIT_LOG2 = 29;  // 9-bit digits from 2^29 rows

void schedule_init_locked() {
  if (g_items_init) return;
  for (int i = 0; i < 64; ++i) {
    g_items[i] = i >= WIDE_TILE_LOG2 ? 16 : 8;
    g_bits[i] = i >= WIDE_DIGIT_LOG2 ? 9 : DEFAULT_DIGIT_BITS;
    g_method[i] = i >= HASH_DEFAULT_LOG2 ? RINGO_NODES_HASH : RINGO_NODES_SORT;
  }
  // the autotuner's measured schedules (tuned_schedule.h) for the buckets
  // up to its largest size: each bucket takes the tuned size at or below it
  // (the smallest tuned size for the buckets below that)
  if (NUM_TUNED > 0) {
    for (int i = 0; i <= TUNED[NUM_TUNED - 1].log2_rows && i < 64; ++i) {
      int t = 0;
      for (int j = 0; j < NUM_TUNED; ++j)
        if (TUNED[j].log2_rows <= i) t = j;
      g_items[i] = TUNED[t].items;
      g_bits[i] = TUNED[t].digit_bits;
      g_method[i] = TUNED[t].node_method;
    }
  }
  g_items_init = true;
}

int items_for(int64_t rows) {
  std::lock_guard<std::mutex> lk(g_mu);
  schedule_init_locked();
  return g_items[ceil_log2(std::max<int64_t>(rows, 1))];
}

int digit_bits_for(int64_t rows) {
  std::lock_guard<std::mutex> lk(g_mu);
  schedule_init_locked();
  return g_bits[ceil_log2(std::max<int64_t>(rows, 1))];
}

int method_for(int64_t rows) {
  std::lock_guard<std::mutex> lk(g_mu);
  schedule_init_locked();
  return g_method[ceil_log2(std::max<int64_t>(rows, 1))];
}

// Slots of a table's node hash table: the smallest power of two holding
// 1.5 times the estimated distinct keys (load <= 2/3 while the estimate
// holds; measured faster than 2x, because the rank gathers of the remap
// then touch a smaller array), never more than a load of 1/2 at V = 2n needs,
// never fewer than 64, at most 2^31.  RINGO_HASH_TEST_CAPACITY (test support)
// caps it, to exercise the overflow fallback.
int64_t table_capacity(int64_t est, int64_t rows) {
  int64_t want = std::max<int64_t>(64, est + est / 2);
  want = std::min<int64_t>(want, 4 * std::max<int64_t>(rows, 16));
  want = std::min<int64_t>(want, (int64_t)1 << 31);  // slot indices stay below 2^32 - 1
  int64_t cap = (int64_t)1 << ceil_log2(want);
  const char *env = std::getenv("RINGO_HASH_TEST_CAPACITY");
  const int64_t test_cap = env ? std::max<int64_t>(1, std::atoll(env)) : 0;
  if (test_cap > 0 && cap > test_cap) cap = (int64_t)1 << (63 - __builtin_clzll((uint64_t)test_cap));
  return cap;
}

// Whether a call's node hash tables (slots in all, for rows in all) are
// filled and read through keys grouped by table part (partitioned
// numbering).  Grouping costs passes over the rows and saves on every probe
// that would miss the caches, so it pays for large tables probed often:
// measured faster on R-MAT tables from 2^24 slots at 16 or more rows per
// slot (2^28 rows 34.6 against 35.9 ms, 2^30 rows 141.8 against 157.0 ms)
// and on uniform ones at 16 rows per slot (2^28 rows over 2^24 slots 41.9
// against 44.0 ms), slower below 2^24 slots (2^27 R-MAT rows 16.8 against
// 16.4 ms) and with fewer rows per slot (2^28 uniform rows over 2^26 slots
// 54.0 against 52.3 ms).  RINGO_HASH_PARTS=0 or 1 (test support) turns it
// off or on for every size.
constexpr int64_t PART_MIN_SLOTS = (int64_t)1 << 24;
constexpr int64_t PART_MIN_ROWS_PER_SLOT = 16;
int parts_env() {  // 0 or 1 when RINGO_HASH_PARTS is set, else -1
  const char *e = std::getenv("RINGO_HASH_PARTS");
  return e && *e ? (std::atoi(e) != 0 ? 1 : 0) : -1;
}
bool parts_for(int64_t slots, int64_t rows) {
  const int e = parts_env();
  if (e >= 0) return e == 1;
  return slots >= PART_MIN_SLOTS && rows >= PART_MIN_ROWS_PER_SLOT * slots;
}
// The items code of the plain edge and in-passes: two-half tiles of 8192
// keys where the schedule has 16 items and digits of at most 9 bits (whose
// two halves' staging leaves room for two blocks per CU).  A 9-bit digit's
// run per tile doubles from 8 to 16 keys, so fewer of the lines it writes
// are shared with a neighbouring tile; 8192 divides the remap tile, so the
// first edge pass still takes its counts from the remap.
// RINGO_TILE_PAIRS=0 (test support) keeps one-half tiles.
int pair_items(int items, int rb) {
  const char *e = std::getenv("RINGO_TILE_PAIRS");
  const bool on = !(e && *e && std::atoi(e) == 0);
  return on && items == 16 && rb <= 9 ? PAIR_ITEMS : items;
}

// Whether a call of this many rows may take the partitioned numbering: its
// distinct-count estimate then also counts the rows' parts.
bool parts_possible(int64_t rows) {
  const int e = parts_env();
  if (e >= 0) return e == 1;
  return rows >= PART_MIN_ROWS_PER_SLOT * PART_MIN_SLOTS;
}

// ----------------------------------------------------------- tile maps

enum TileKind {
  TM_NSORT, TM_UNIQ, TM_DIR, TM_REMAP, TM_ESORT, TM_DEDUP, TM_ISORT, TM_ICSR,
  TM_HLL, TM_HCMP, TM_VSORT, TM_PART, TM_IN0, TM_KINDS
};

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

struct Call {
  int S = 0;
  hipStream_t stream = nullptr;
  AllocHooks hooks;
  int items = 16;
  int sort_tile = 4096;
  int eitems = 16;      // items code of the plain edge and in-passes (PAIR_ITEMS: two-half tiles)
  int esort_tile = 4096;
  int rb = DEFAULT_DIGIT_BITS;  // digit bits of the radix passes
  std::vector<SegPlan> plan;
  std::vector<int64_t> tmap;  // TM_KINDS x (S + 1)

  // device workspace
  uint64_t *A = nullptr, *B = nullptr;
  int64_t *base = nullptr;
  int64_t *results = nullptr;
  uint8_t *meta = nullptr;
  DirEntry *dir = nullptr;
  void *tab = nullptr;    // node hash tables: keys, then ranks
  uint32_t *hslots = nullptr;  // slot of every node key
  uint64_t *px = nullptr;  // partitioned numbering: rows grouped by source part (keys, then dst)
  uint64_t *py = nullptr;  // destination keys grouped by part, then source positions (32-bit)
  void *pcnt = nullptr;    // tile prefixes and digit bases of the destination keys' grouping
  uint32_t *vals = nullptr;    // multigraph: rows carried through the sorts (2 x N)
  int kind = RINGO_GRAPH_DIRECTED;
  // small tables converted in LDS (one workgroup each)
  std::vector<int> small;        // their indices in the call
  void *small_ws = nullptr;      // SmallTable array + V/E results
  Pinned *spin = nullptr;        // staging of the SmallTable array and the results
  std::vector<SmallTable> small_tabs;
  void *hmeta = nullptr;  // estimate registers, slot counts and flags of the hash tables
  uint32_t *counts = nullptr;
  uint32_t *bsum = nullptr;
  size_t meta_bytes = 0;
  Pinned *pin = nullptr;
  int upload_slot = 0;
  // queued long runs of offsets (fill_run): chunks, then one counter per use
  char *gaps = nullptr;
  uint32_t gap_cap = 0;
  GapQueue gapq(int use) const {
    GapQueue q;
    q.e = (GapEntry *)gaps;
    q.count = gaps ? (uint32_t *)(gaps + align_up(sizeof(GapEntry) * gap_cap)) + use : nullptr;
    q.cap = gap_cap;
    return q;
  }
  // Output blocks, until the graphs take them: one Owner for the call, or
  // (separate) one per table.
  bool separate = false;
  std::vector<Owner *> owners;

  ~Call() { release_workspace(); }

  Owner *owner_for(int table) {
    const size_t k = separate ? (size_t)table : 0;
    if (owners.size() <= k) owners.resize(k + 1, nullptr);
    if (!owners[k]) {
      owners[k] = new Owner();
      owners[k]->stream = stream;
      owners[k]->hooks = hooks;
    }
    return owners[k];
  }
  // An output block of a table (slot 0 node-sized, 1 edge-sized, 2 small
  // table), held by the table's Owner; null when the allocator refuses.
  char *out_alloc(int table, int slot, size_t bytes) {
    Owner *o = owner_for(table);
    bytes = std::max<size_t>(bytes, 256);
    void *p = dev_alloc(hooks, bytes, stream);
    if (p) {
      o->blocks[slot] = p;
      o->bytes += bytes;
    }
    return (char *)p;
  }
  // The graphs of the call take their Owners (refs: graphs per Owner).
  void hand_over(int S) {
    for (Owner *o : owners)
      if (o) o->refs.store(separate ? 1 : S);
    owners.clear();
  }
  // Output blocks of a failed call.
  void free_outputs() {
    for (Owner *o : owners) {
      if (!o) continue;
      for (void *b : o->blocks) dev_free(hooks, b, stream);
      delete o;
    }
    owners.clear();
  }

  void release_workspace() {
    void *bufs[] = {A, B, base, results, meta, dir, tab, hslots, hmeta, counts,
                    bsum, vals, small_ws, gaps, px, py, pcnt};
    for (void *b : bufs) dev_free(hooks, b, stream);
    px = py = nullptr;
    pcnt = nullptr;
    small_ws = nullptr;
    gaps = nullptr;
    if (spin) pinned_release(spin, stream);
    spin = nullptr;
    tab = nullptr;
    hslots = nullptr;
    vals = nullptr;
    hmeta = nullptr;
    A = B = nullptr;
    base = nullptr;
    results = nullptr;
    meta = nullptr;
    dir = nullptr;
    counts = nullptr;
    bsum = nullptr;
    if (pin) pinned_release(pin, stream);
    pin = nullptr;
  }

  int64_t *tm(int kind) { return tmap.data() + (size_t)kind * (S + 1); }
  const int64_t *tm_dev(int kind) const {
    return (const int64_t *)(meta + align_up(sizeof(SegPlan) * S)) + (size_t)kind * (S + 1);
  }
  const SegPlan *plan_dev() const { return (const SegPlan *)meta; }

  void set_tiles(int kind, int range, int64_t tile) {
    int64_t *t = tm(kind);
    t[0] = 0;
    for (int i = 0; i < S; ++i) {
      const int64_t c = range_count(plan[i], range);
      t[i + 1] = t[i] + (c + tile - 1) / tile;
    }
  }
  int64_t total(int kind) { return tm(kind)[S]; }

  TileLaunch tiles(int kind, int range) {
    TileLaunch t;
    t.plan = plan_dev();
    t.tmap = tm_dev(kind);
    t.num_segs = S;
    t.range_kind = range;
    t.total_tiles = total(kind);
    return t;
  }

  static constexpr int kUploadSlots = 6;  // at most 5 uploads per call

  hipError_t upload() {
    char *stage = (char *)pin->p + (size_t)upload_slot * meta_bytes;
    ++upload_slot;
    std::memcpy(stage, plan.data(), sizeof(SegPlan) * S);
    std::memcpy(stage + align_up(sizeof(SegPlan) * S), tmap.data(), sizeof(int64_t) * tmap.size());
    return hipMemcpyAsync(meta, stage, meta_bytes, hipMemcpyHostToDevice, stream);
  }

  // Read back S counts from results[off..off+S) and wait for the stream.
  // results [off, off + count) to the host (count <= S + 1), synchronising.
  hipError_t readback(int off, std::vector<int64_t> &v, int count = -1) {
    if (count < 0) count = S;
    int64_t *host = (int64_t *)((char *)pin->p + kUploadSlots * meta_bytes);
    hipError_t e = hipMemcpyAsync(host, results + off, sizeof(int64_t) * count,
                                  hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    v.assign(host, host + count);
    return hipSuccess;
  }

  SortLaunch sort_args(const uint64_t *in, uint64_t *out, int kind, int range, int passes, int pass,
                       int shift) {
    SortLaunch a;
    a.in = in;
    a.out = out;
    a.plan = plan_dev();
    a.tmap = tm_dev(kind);
    a.num_segs = S;
    a.range_kind = range;
    a.total_tiles = total(kind);
    a.shift = shift;
    a.digit_base = base;
    a.counts = counts;
    a.bsum = bsum;
    a.vin = nullptr;
    a.vout = nullptr;
    a.seg_total = nullptr;
    a.wout = nullptr;
    return a;
  }
  // Passes of the partitioned numbering: PART_BITS-bit digits, whatever
  // the schedule's width, so their counts, digit bases and run sums live in
  // a block of their own (pcnt, part_bytes()), which also keeps the
  // destination keys' prefixes for the rank pass that groups them again.
  size_t part_count_bytes() { return align_up(sizeof(uint32_t) * (1 << PART_BITS) * (total(TM_NSORT) + 1)); }
  size_t part_base_bytes() { return align_up(sizeof(int64_t) * S * (1 << PART_BITS)); }
  size_t part_bytes() {
    return part_count_bytes() + part_base_bytes() +
           sizeof(uint32_t) * (1 << PART_BITS) * sort_runs_bound(total(TM_NSORT) + 1);
  }
  SortLaunch part_args(const uint64_t *in, uint64_t *out) {
    SortLaunch a = sort_args(in, out, TM_PART, RANGE_ROWS, 1, 0, 0);
    a.counts = (uint32_t *)pcnt;
    a.digit_base = (int64_t *)((char *)pcnt + part_count_bytes());
    a.bsum = (uint32_t *)((char *)pcnt + part_count_bytes() + part_base_bytes());
    return a;
  }
};


#define HIP_TRY(x)                              \
  do {                                          \
    hipError_t _e = (x);                        \
    if (_e != hipSuccess) return RINGO_ERR_HIP; \
  } while (0)

// --------------------------------------------------------------- tracing
//
// When enabled, every kernel launch of a call is bracketed by two HIP events
// recorded on the call's stream; ringo_trace_read reports per-kernel launch
// counts, summed durations and the algorithmic bytes the launches move.

enum TraceKind {
  TK_NODE_COUNT, TK_NODE_SCATTER, TK_UNIQUE, TK_DIR, TK_REMAP, TK_EDGE_COUNT, TK_EDGE_SCATTER,
  TK_DEDUPE, TK_IN_COUNT, TK_IN_SCATTER, TK_IN_CSR, TK_AUX, TK_HLL, TK_HINSERT, TK_HCOMPACT,
  TK_VNODE_COUNT, TK_VNODE_SCATTER, TK_HRANK, TK_HREMAP, TK_SMALL, TK_HBSORT, TK_PLAN, TK_GRAPH,
  TK_HPART_COUNT, TK_HPART_SCATTER, TK_HPART_RANK, TK_HPACK, TK_HRANK_KEYS, TK_HPART_DST,
  TK_KINDS
};
// "count" entries are the small kernels of a pass's digit counting and
// prefixes (three or four); every other entry is a single kernel.
const char *const kTraceNames[TK_KINDS] = {
    "sort_node_count",   "sort_node_scatter", "unique",          "directory",
    "remap_pack",        "sort_edge_count",   "sort_edge_scatter", "dedupe_out_csr",
    "sort_in_count",     "sort_in_scatter",   "in_csr",          "aux",
    "hash_estimate",     "hash_insert",       "hash_compact",    "sort_vnode_count",
    "sort_vnode_scatter", "hash_rank",        "hash_remap_pack", "small_tables",
    "hash_bucket_sort", "plan_device", "fixed_graph_replay", "hash_part_count",
    "hash_part_scatter", "hash_part_rank", "hash_pack_parts", "hash_rank_slots",
    "hash_part_dst_scatter"};

struct TraceRec {
  int kind;
  hipEvent_t a, b;
  double bytes;
  int64_t units;
};
bool g_trace_on = false;
std::vector<TraceRec> g_trace;
std::vector<hipEvent_t> g_evpool;

hipEvent_t trace_event() {
  if (!g_evpool.empty()) {
    hipEvent_t e = g_evpool.back();
    g_evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

struct TraceMark {
  hipEvent_t a = nullptr;
};

TraceMark trace_begin(hipStream_t s) {
  TraceMark m;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_trace_on) return m;
  m.a = trace_event();
  if (m.a) (void)hipEventRecord(m.a, s);
  return m;
}

// Returns the record index (or -1) so that byte counts known only later
// can be filled in.
long trace_end(const TraceMark &m, int kind, int64_t units, double bytes, hipStream_t s) {
  if (!m.a) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = trace_event();
  if (!b) return -1;
  (void)hipEventRecord(b, s);
  g_trace.push_back(TraceRec{kind, m.a, b, bytes, units});
  return (long)g_trace.size() - 1;
}

void trace_set_bytes(long idx, double bytes) {
  if (idx < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((size_t)idx < g_trace.size()) g_trace[(size_t)idx].bytes = bytes;
}

#define TRACED(kind, units, bytes, expr)                       \
  do {                                                         \
    TraceMark _m = trace_begin(st);                            \
    HIP_TRY(expr);                                             \
    (void)trace_end(_m, (kind), (units), (double)(bytes), st); \
  } while (0)

// One radix pass of w-bit digits as two traced entries: counting (reads
// every key) and scatter (reads and writes every key, plus extra bytes per
// key).
#define TRACED_PASS_N(kcount, kscatter, keys, extra, mode, a, w, items)                         \
  do {                                                                                        \
    TRACED(kcount, keys, 8.0 * (keys),                                                        \
           launch_sort_part(a, mode, (items), (w), SORT_PART_COUNT, st));                     \
    TRACED(kscatter, keys, (16.0 + (extra)) * (keys),                                         \
           launch_sort_part(a, mode, (items), (w), SORT_PART_SCATTER, st));                   \
  } while (0)
#define TRACED_PASS(kcount, kscatter, keys, extra, mode, a, w) \
  TRACED_PASS_N(kcount, kscatter, keys, extra, mode, a, w, c.items)

int grid_for(int64_t tiles, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cap));
}


// Largest V a table may have: RINGO_MAX_NODES (int32 neighbours), or less
// under RINGO_TEST_MAX_NODES (test support: exercises the error path
// without building a graph of 2^31 nodes).
int64_t max_nodes() {
  const char *e = std::getenv("RINGO_TEST_MAX_NODES");
  const int64_t v = e ? std::atoll(e) : 0;
  return v > 0 && v < RINGO_MAX_NODES ? v : (int64_t)RINGO_MAX_NODES;
}

// True when a small table's V exceeds the limit (results read back).
bool small_too_many_nodes(const Call &c) {
  const int K = (int)c.small.size();
  const int64_t *vres = (const int64_t *)((char *)c.spin->p + align_up(sizeof(SmallTable) * K));
  for (int k = 0; k < K; ++k)
    if (vres[2 * k] > max_nodes()) return true;
  return false;
}

// Launches the small tables of a call (c.small): worst-case-sized outputs in
// one block (or one per table when the call separates its outputs), the
// SmallTable array uploaded through pinned memory, one workgroup per table,
// and the V/E results copied back to pinned memory on the same stream (read
// after the call's next synchronisation).
ringo_status_t launch_small_part(Call &c, const int64_t *const *src, const int64_t *const *dst,
                                 const int64_t *num_rows) {
  const int K = (int)c.small.size();
  hipStream_t st = c.stream;
  size_t arena = 0;
  std::vector<size_t> off((size_t)5 * K), first(K), size(K);
  for (int k = 0; k < K; ++k) {
    const int64_t n = num_rows[c.small[k]];
    const size_t sz[5] = {sizeof(int64_t) * 2 * n, sizeof(int64_t) * (2 * n + 1),
                          sizeof(int64_t) * (2 * n + 1), sizeof(int32_t) * n, sizeof(int32_t) * n};
    first[k] = arena;
    for (int f = 0; f < 5; ++f) {
      off[(size_t)5 * k + f] = arena;
      arena = align_up(arena + sz[f]);
    }
    size[k] = arena - first[k];
  }
  const size_t tab_bytes = align_up(sizeof(SmallTable) * K);
  // base[k]: the address that table k's offsets are relative to
  std::vector<char *> base(K, nullptr);
  if (c.separate) {
    for (int k = 0; k < K; ++k) {
      char *blk = c.out_alloc(c.small[k], 2, size[k]);
      if (!blk) return RINGO_ERR_OUT_OF_MEMORY;
      base[k] = blk - first[k];
    }
  } else {
    char *blk = c.out_alloc(0, 2, arena);
    if (!blk) return RINGO_ERR_OUT_OF_MEMORY;
    for (int k = 0; k < K; ++k) base[k] = blk;
  }
  c.small_ws = dev_alloc(c.hooks, tab_bytes + sizeof(int64_t) * 2 * K, st);
  c.spin = pinned_acquire(tab_bytes + sizeof(int64_t) * 2 * K);
  if (!c.small_ws || !c.spin) return RINGO_ERR_OUT_OF_MEMORY;
  c.small_tabs.resize(K);
  for (int k = 0; k < K; ++k) {
    const int i = c.small[k];
    char *a = base[k];
    SmallTable &T = c.small_tabs[k];
    T.src = src[i];
    T.dst = dst[i];
    T.n = num_rows[i];
    T.node_ids = (int64_t *)(a + off[(size_t)5 * k]);
    T.out_off = (int64_t *)(a + off[(size_t)5 * k + 1]);
    T.in_off = (int64_t *)(a + off[(size_t)5 * k + 2]);
    T.out_nbr = (int32_t *)(a + off[(size_t)5 * k + 3]);
    T.in_nbr = (int32_t *)(a + off[(size_t)5 * k + 4]);
  }
  std::memcpy(c.spin->p, c.small_tabs.data(), sizeof(SmallTable) * K);
  int64_t *vres = (int64_t *)((char *)c.small_ws + tab_bytes);
  HIP_TRY(hipMemcpyAsync(c.small_ws, c.spin->p, sizeof(SmallTable) * K, hipMemcpyHostToDevice, st));
  TRACED(TK_SMALL, K, 0.0, launch_small((const SmallTable *)c.small_ws, K, vres, st));
  HIP_TRY(hipMemcpyAsync((char *)c.spin->p + tab_bytes, vres, sizeof(int64_t) * 2 * K,
                         hipMemcpyDeviceToHost, st));
  return RINGO_OK;
}

// Fills the graphs of the small tables (after a synchronisation).
void handoff_small(Call &c, const int64_t *num_rows, ringo_graph_t *outs) {
  const int K = (int)c.small.size();
  const int64_t *vres = (const int64_t *)((char *)c.spin->p + align_up(sizeof(SmallTable) * K));
  for (int k = 0; k < K; ++k) {
    const SmallTable &T = c.small_tabs[k];
    ringo_graph_t &g = outs[c.small[k]];
    std::memset(&g, 0, sizeof(g));
    g.num_rows = num_rows[c.small[k]];
    g.num_nodes = vres[2 * k];
    g.num_edges = vres[2 * k + 1];
    g.node_ids = T.node_ids;
    g.out_offsets = T.out_off;
    g.out_nbrs = T.out_nbr;
    g.in_offsets = T.in_off;
    g.in_nbrs = T.in_nbr;
    g.kind = RINGO_GRAPH_DIRECTED;
    g._alloc = c.owner_for(c.small[k]);
  }
}

ringo_status_t run(Call &c, const int64_t *const *src, const int64_t *const *dst,
                   const int64_t *num_rows, ringo_graph_t *outs) {
  const int S = c.S;
  hipStream_t st = c.stream;
  const int cus = device_cu_count();
  long unique_rec = -1, dedupe_rec = -1;
  int64_t sumV = 0, sumE = 0;

  // ------------------------------------------------------- small tables
  // Directed tables of at most SMALL_ROWS rows: one workgroup each, in LDS,
  // launched first; the pass pipeline below sees them as empty.
  c.small.clear();
  // RINGO_SMALL_TABLES=0 (test support) sends every table through the pipeline
  const char *small_env = std::getenv("RINGO_SMALL_TABLES");
  if (c.kind == RINGO_GRAPH_DIRECTED && !(small_env && small_env[0] == '0'))
    for (int i = 0; i < S; ++i)
      if (num_rows[i] > 0 && num_rows[i] <= SMALL_ROWS) c.small.push_back(i);
  std::vector<char> is_small(S, 0);
  for (int i : c.small) is_small[i] = 1;
  if (!c.small.empty()) {
    const ringo_status_t rs = launch_small_part(c, src, dst, num_rows);
    if (rs != RINGO_OK) return rs;
    if ((int)c.small.size() == S) {  // nothing for the pipeline: one synchronisation
      HIP_TRY(hipStreamSynchronize(st));
      if (small_too_many_nodes(c)) return RINGO_ERR_TOO_MANY_NODES;
      handoff_small(c, num_rows, outs);
      c.hand_over(S);
      return RINGO_OK;
    }
  }

  // ---------------------------------------------------------------- plan N
  c.plan.assign(S, SegPlan{});
  c.tmap.assign((size_t)TM_KINDS * (S + 1), 0);
  int64_t N = 0, max_rows = 0;
  for (int i = 0; i < S; ++i) {
    SegPlan &p = c.plan[i];
    p.src = is_small[i] ? nullptr : src[i];
    p.dst = is_small[i] ? nullptr : dst[i];
    p.n = is_small[i] ? 0 : num_rows[i];
    p.row_off = N;
    N += p.n;
    max_rows = std::max(max_rows, p.n);
  }
  c.items = items_for(S == 1 ? max_rows : N);
  c.rb = digit_bits_for(S == 1 ? max_rows : N);
  const int R = 1 << c.rb;
  const bool want_hash = method_for(S == 1 ? max_rows : N) == RINGO_NODES_HASH;
  c.sort_tile = sort_tile(c.items);
  // the plain edge and in-passes (not the multigraph's key-value passes)
  c.eitems = c.kind == RINGO_GRAPH_MULTI ? c.items : pair_items(c.items, c.rb);
  c.esort_tile = sort_tile(c.eitems);
  c.set_tiles(TM_NSORT, RANGE_NODE_KEYS, c.sort_tile);
  c.set_tiles(TM_UNIQ, RANGE_NODE_KEYS, SCAN_TILE);
  c.set_tiles(TM_HLL, RANGE_ROWS, HLL_TILE);
  c.set_tiles(TM_PART, RANGE_ROWS, c.sort_tile);
  c.set_tiles(TM_REMAP, RANGE_ROWS, REMAP_TILE);

  // the node pass has the most tiles: 2n keys per table
  const int64_t max_tiles = c.total(TM_NSORT) + 1;
  const int64_t max_runs = sort_runs_bound(max_tiles);
  c.meta_bytes = align_up(align_up(sizeof(SegPlan) * S) + sizeof(int64_t) * c.tmap.size());
  c.pin = pinned_acquire(Call::kUploadSlots * c.meta_bytes + sizeof(int64_t) * (S + 1));
  if (!c.pin) return RINGO_ERR_OUT_OF_MEMORY;

  const size_t base_words = (size_t)S * R;
  c.A = (uint64_t *)dev_alloc(c.hooks, sizeof(uint64_t) * 2 * N, st);
  c.B = (uint64_t *)dev_alloc(c.hooks, sizeof(uint64_t) * 2 * N, st);
  c.base = (int64_t *)dev_alloc(c.hooks, sizeof(int64_t) * base_words, st);
  c.results = (int64_t *)dev_alloc(c.hooks, sizeof(int64_t) * (2 * S + 1), st);
  c.meta = (uint8_t *)dev_alloc(c.hooks, c.meta_bytes, st);
  c.counts = (uint32_t *)dev_alloc(c.hooks, sizeof(uint32_t) * R * max_tiles, st);
  c.bsum = (uint32_t *)dev_alloc(c.hooks, sizeof(uint32_t) * R * max_runs, st);
  if (!c.A || !c.B || !c.base || !c.results || !c.meta ||
      !c.counts || !c.bsum)
    return RINGO_ERR_OUT_OF_MEMORY;

  HIP_TRY(c.upload());
  HIP_TRY(launch_fill_u64((uint64_t *)c.results, 0, 2 * S, st));

  // ------------------------------------------------------------- phase N
  // Both methods leave V in results[0, S); the sort method leaves the
  // sorted distinct keys in A, the hash method leaves them unordered in A.
  std::vector<int64_t> V;
  bool hashed = false;
  int64_t slots = 0;
  uint64_t *hkeys = nullptr;
  uint32_t *hrank = nullptr;
  uint32_t *hflags = nullptr;
  bool parted = false;  // partitioned numbering
  bool hll_counts = false;  // the estimate counted the rows' parts
  // one table: its distinct keys are placed by bucket of their top bits, and
  // sorted bucket by bucket in LDS when no bucket exceeds BUCKET_CAP keys
  const bool bucket_place = want_hash && S == 1;
  bool bucketed = bucket_place;
  BucketLaunch bkl{};
  long hcompact_rec = -1;
  if (want_hash) {
    const size_t reg_bytes = align_up(sizeof(uint32_t) * HLL_M * S);
    const size_t cnt_bytes = align_up(sizeof(uint64_t) * S);
    const size_t flag_bytes = align_up(sizeof(uint32_t) * S);
    const size_t bkt_bytes = bucketed ? align_up(sizeof(uint32_t) * (3 * NBUCKETS + 1)) : 0;
    const size_t hm_bytes = reg_bytes + cnt_bytes + flag_bytes + bkt_bytes;
    c.hmeta = dev_alloc(c.hooks, hm_bytes, st);
    if (!c.hmeta) return RINGO_ERR_OUT_OF_MEMORY;
    uint32_t *regs = (uint32_t *)c.hmeta;
    uint64_t *hcount = (uint64_t *)((char *)c.hmeta + reg_bytes);
    hflags = (uint32_t *)((char *)c.hmeta + reg_bytes + cnt_bytes);
    if (bucketed) {
      uint32_t *bk = (uint32_t *)((char *)c.hmeta + reg_bytes + cnt_bytes + flag_bytes);
      bkl.bcnt = bk;
      bkl.bstart = bk + NBUCKETS;
      bkl.bcur = bk + 2 * NBUCKETS + 1;
      bkl.bslot = (uint32_t *)c.B;  // B is free until the distinct keys are sorted
      bkl.max_bucket = c.results + S;
    }
    HIP_TRY(launch_fill_u64((uint64_t *)c.hmeta, 0, (int64_t)(hm_bytes / 8), st));
    // where the rows may be grouped, the estimate also counts their parts
    // (into the counts array, free until the grouping's prefixes)
    hll_counts = c.kind != RINGO_GRAPH_MULTI && HLL_TILE % c.sort_tile == 0 && parts_possible(N);
    TRACED(TK_HLL, 2 * N, 16.0 * N,
           launch_hll(c.tiles(TM_HLL, RANGE_ROWS), regs, c.results, hll_counts ? c.counts : nullptr,
                      c.tm_dev(TM_PART), c.sort_tile, grid_for(c.total(TM_HLL), cus * 4), st));
    // sync #0: size every table's node hash table from its estimate
    std::vector<int64_t> est;
    HIP_TRY(c.readback(0, est));
    // Mostly distinct identifiers (V above half the rows, such as the leaves
    // of a star): sorting all 2n keys is then as cheap as the table, whose
    // probes and compaction grow with V; measured faster at 2^25 rows from
    // V/n = 0.5 on (9.9 against 17.2 ms at V/n = 1.6), slower below (4.1
    // against 7.2 ms at V/n = 0.016).
    int64_t est_sum = 0;
    for (int i = 0; i < S; ++i) est_sum += est[i];
    if (2 * est_sum > N) goto numbering;
    for (int i = 0; i < S; ++i) {
      SegPlan &p = c.plan[i];
      p.tab_off = slots;
      p.tab_cap = p.n > 0 ? table_capacity(est[i], p.n) : 0;
      slots += p.tab_cap;
    }
    // Partitioned numbering (not for multigraphs, whose edges keep their row
    // order): the rows are grouped by the table part of their source key,
    // with the destination keys beside them, and the destination keys again
    // by theirs; both groupings are inserted, so that the probes of the
    // blocks of one XCD meet one part of the table at a time.
    parted = c.kind != RINGO_GRAPH_MULTI && parts_for(slots, N);
    const size_t key_bytes = align_up(sizeof(uint64_t) * std::max<int64_t>(slots, 1));
    const size_t rank_bytes = align_up(sizeof(uint32_t) * std::max<int64_t>(slots, 1));
    c.tab = dev_alloc(c.hooks, key_bytes + rank_bytes, st);
    if (parted) {
      c.px = (uint64_t *)dev_alloc(c.hooks, sizeof(uint64_t) * 2 * std::max<int64_t>(N, 1), st);
      // destination keys, then three 32-bit arrays: source positions grouped
      // as destinations, source slots (then positions) grouped as rows,
      // destination slots
      c.py = (uint64_t *)dev_alloc(c.hooks, (sizeof(uint64_t) + 3 * sizeof(uint32_t)) *
                                                std::max<int64_t>(N, 1), st);
      // the node pass's tile count bounds the grouping's (n keys per table)
      c.pcnt = dev_alloc(c.hooks, c.part_bytes(), st);
      if (!c.tab || !c.px || !c.py || !c.pcnt) return RINGO_ERR_OUT_OF_MEMORY;
    } else {
      c.hslots = (uint32_t *)dev_alloc(c.hooks, sizeof(uint32_t) * 2 * std::max<int64_t>(N, 1), st);
      if (!c.tab || !c.hslots) return RINGO_ERR_OUT_OF_MEMORY;
    }
    hkeys = (uint64_t *)c.tab;
    hrank = (uint32_t *)((char *)c.tab + key_bytes);
    c.set_tiles(TM_HCMP, RANGE_SLOTS, SCAN_TILE);
    HIP_TRY(c.upload());
    HIP_TRY(launch_fill_u64(hkeys, EMPTY_KEY, slots, st));
    if (parted) {
      SortLaunch a = c.part_args(nullptr, c.px);
      a.wout = c.px + N;
      if (hll_counts) {  // tile counts written by the estimate
        a.counts = c.counts;
        TRACED(TK_HPART_COUNT, N, 0.0,
               launch_sort_part(a, SORT_PART_ROWS, c.items, PART_BITS, SORT_PART_PREFIX, st));
        TRACED(TK_HPART_SCATTER, N, 32.0 * N,
               launch_sort_part(a, SORT_PART_ROWS, c.items, PART_BITS, SORT_PART_SCATTER, st));
      } else {
        TRACED_PASS(TK_HPART_COUNT, TK_HPART_SCATTER, N, 16.0, SORT_PART_ROWS, a, PART_BITS);
      }
      // its prefixes are kept for the rank pass, which groups the same keys
      SortLaunch d = c.part_args(c.px + N, c.py);
      TRACED_PASS(TK_HPART_COUNT, TK_HPART_DST, N, 0.0, SORT_PART_DST, d, PART_BITS);
      uint32_t *xslot = (uint32_t *)(c.py + N) + N, *yslot = xslot + N;
      // The grouped kernels' grids set how many keys an XCD has in flight,
      // hence how many parts' table or rank slices share its L2 at once:
      // at 1.5e9 rows 4 blocks per CU suit the inserts (12.7 against 13.2 ms
      // at 8, 15.0 at 2) and the pack (10.35 against 10.6), 2 the position
      // gather (7.3 against 8.3 at 4 and 8.85 at 8).
      TRACED(TK_HINSERT, N, 20.0 * N,
             launch_hash_insert_keys(c.tiles(TM_REMAP, RANGE_ROWS), c.px, hkeys, xslot, hflags,
                                     grid_for(c.total(TM_REMAP), cus * 4), st));
      TRACED(TK_HINSERT, N, 20.0 * N,
             launch_hash_insert_keys(c.tiles(TM_REMAP, RANGE_ROWS), c.py, hkeys, yslot, hflags,
                                     grid_for(c.total(TM_REMAP), cus * 4), st));
    } else {
      TRACED(TK_HINSERT, 2 * N, 24.0 * N,
             launch_hash_insert(c.tiles(TM_REMAP, RANGE_ROWS), hkeys, c.hslots, hflags,
                                grid_for(c.total(TM_REMAP), cus * 8), st));
    }
    {
      TraceMark m = trace_begin(st);
      HIP_TRY(launch_hash_compact(c.tiles(TM_HCMP, RANGE_SLOTS), hkeys, c.A, hcount, hflags,
                                  c.results, bucketed ? &bkl : nullptr,
                                  grid_for(c.total(TM_HCMP), cus * 8), st));
      hcompact_rec = trace_end(m, TK_HCOMPACT, slots, 8.0 * slots, st);
    }
    HIP_TRY(c.readback(0, V, S + 1));  // sync #1 (V, and the largest bucket)
    bucketed = bucketed && V[S] <= BUCKET_CAP;
    V.resize(S);
    hashed = true;
    for (int i = 0; i < S; ++i) hashed = hashed && V[i] >= 0;
    if (!hashed) {
      // a table overflowed its probe bound: number the nodes by sorting
      dev_free(c.hooks, c.tab, st);
      dev_free(c.hooks, c.hslots, st);
      dev_free(c.hooks, c.px, st);
      dev_free(c.hooks, c.py, st);
      c.tab = nullptr;
      c.hslots = nullptr;
      c.px = c.py = nullptr;
      parted = false;
      HIP_TRY(launch_fill_u64((uint64_t *)c.results, 0, 2 * S, st));
    }
  }
numbering:
  uint64_t *buf[2] = {c.A, c.B};
  if (!hashed) {
    const int P_n = lsd_passes(64, c.rb);
    // the passes alternate between A and B so that the last one lands in B
    uint64_t *nbuf[2] = {(P_n & 1) ? c.B : c.A, (P_n & 1) ? c.A : c.B};
    for (int p = 0; p < P_n; ++p) {
      SortLaunch a = c.sort_args(p == 0 ? nullptr : nbuf[(p - 1) & 1], nbuf[p & 1], TM_NSORT,
                                 RANGE_NODE_KEYS, P_n, p, lsd_shift(64, c.rb, p));
      TRACED_PASS(TK_NODE_COUNT, TK_NODE_SCATTER, 2 * N, 0.0, p == 0 ? SORT_NODE_FIRST : SORT_NODE,
                  a, lsd_width(64, c.rb, p));
    }
    // the sorted keys are in B; the distinct keys go to A
    TraceMark m = trace_begin(st);
    HIP_TRY(launch_unique(c.tiles(TM_UNIQ, RANGE_NODE_KEYS), c.B, c.A, c.results, c.counts,
                          grid_for(c.total(TM_UNIQ), cus * 4), st));
    unique_rec = trace_end(m, TK_UNIQUE, 2 * N, 16.0 * N, st);
    HIP_TRY(c.readback(0, V));  // sync #1
  }

  // -------------------------------------------------------------- sync #1
  int b_max = 1;
  int64_t dir_words = 0;
  size_t arena1 = 0;
  std::vector<size_t> off1(3 * (size_t)S);
  if (!c.small.empty() && small_too_many_nodes(c)) return RINGO_ERR_TOO_MANY_NODES;
  for (int i = 0; i < S; ++i) {
    if (V[i] > max_nodes()) return RINGO_ERR_TOO_MANY_NODES;
    SegPlan &p = c.plan[i];
    p.V = V[i];
    p.dirk = p.V > 0 ? ceil_log2(p.V) : 0;
    p.b = std::max(1, p.dirk);
    b_max = std::max(b_max, p.V > 0 ? p.b : 1);
    p.dir_off = dir_words;
    if (!hashed) dir_words += p.V > 0 ? ((int64_t)1 << p.dirk) + 1 : 0;
    off1[3 * i] = arena1;
    arena1 = align_up(arena1 + sizeof(int64_t) * p.V);
    off1[3 * i + 1] = arena1;
    arena1 = align_up(arena1 + sizeof(int64_t) * (p.V + 1));
    off1[3 * i + 2] = arena1;
    arena1 = align_up(arena1 + sizeof(int64_t) * (p.V + 1));
  }
  for (int i = 0; i < S; ++i) sumV += V[i];
  trace_set_bytes(unique_rec, 16.0 * N + 8.0 * sumV);
  // the compaction reads every slot once (bucketed: twice) and writes every
  // key (bucketed: with its slot)
  trace_set_bytes(hcompact_rec, (bucket_place ? 16.0 : 8.0) * slots +
                                    (bucket_place ? 12.0 : 8.0) * sumV);
  // node-sized outputs: one block, or one per table (base1[i]: the address
  // that table i's offsets are relative to)
  std::vector<char *> base1(S, nullptr);
  if (c.separate) {
    for (int i = 0; i < S; ++i) {
      const size_t end = i + 1 < S ? off1[3 * (i + 1)] : arena1;
      char *blk = c.out_alloc(i, 0, end - off1[3 * i]);
      if (!blk) return RINGO_ERR_OUT_OF_MEMORY;
      base1[i] = blk - off1[3 * i];
    }
  } else {
    char *blk = c.out_alloc(0, 0, arena1);
    if (!blk) return RINGO_ERR_OUT_OF_MEMORY;
    for (int i = 0; i < S; ++i) base1[i] = blk;
  }
  if (!hashed) {
    c.dir = (DirEntry *)dev_alloc(c.hooks, sizeof(DirEntry) * std::max<int64_t>(dir_words, 1), st);
    if (!c.dir) return RINGO_ERR_OUT_OF_MEMORY;
  }
  for (int i = 0; i < S; ++i) {
    SegPlan &p = c.plan[i];
    p.node_ids = (int64_t *)(base1[i] + off1[3 * i]);
    p.out_off = (int64_t *)(base1[i] + off1[3 * i + 1]);
    p.in_off = (int64_t *)(base1[i] + off1[3 * i + 2]);
  }
  // Long runs of equal offsets or directory entries go to a queue that a
  // fill kernel writes (uses: 0 directory, 1 out-offsets, 2 in-offsets).
  // Every run lies in one array of at most 2V + 1 entries per table.
  c.gap_cap = (uint32_t)std::min<int64_t>(gap_chunks_bound(2 * sumV + 2 * S) + 2 * S, INT32_MAX);
  c.gaps = (char *)dev_alloc(c.hooks, align_up(sizeof(GapEntry) * c.gap_cap) + 64, st);
  if (!c.gaps) return RINGO_ERR_OUT_OF_MEMORY;
  HIP_TRY(launch_fill_u64((uint64_t *)(c.gaps + align_up(sizeof(GapEntry) * c.gap_cap)), 0, 8, st));
  const int P_e = lsd_passes(2 * b_max, c.rb);
  const int P_in = lsd_passes(b_max, c.rb);
  c.set_tiles(TM_DIR, RANGE_NODES, DIR_TILE);
  c.set_tiles(TM_VSORT, RANGE_NODES, c.sort_tile);
  // edge keys: n per table at row_off, or both orientations (2n at
  // 2 row_off) for undirected graphs
  const bool undirected = c.kind == RINGO_GRAPH_UNDIRECTED, multi = c.kind == RINGO_GRAPH_MULTI;
  const int erange = undirected ? RANGE_NODE_KEYS : RANGE_ROWS;
  const int64_t NE = undirected ? 2 * N : N;
  c.set_tiles(TM_ESORT, erange, c.esort_tile);
  c.set_tiles(TM_IN0, erange, c.sort_tile);
  c.set_tiles(TM_DEDUP, erange, SCAN_TILE);
  HIP_TRY(c.upload());

  // The hash remap also counts the first edge pass's digits of every sort
  // tile (directed and multigraph keys, sort tiles that divide its tiles);
  // that pass then starts from its prefixes.
  uint32_t *counts0 = hashed && !undirected && lsd_width(2 * b_max, c.rb, 0) == FUSED_RADIX_BITS &&
                              REMAP_TILE % c.esort_tile == 0
                          ? c.counts
                          : nullptr;

  // ------------------------------------------------------------- phase E
  // Both methods write the packed edge keys to B; A is free afterwards.
  HIP_TRY(launch_empty_offsets(c.plan_dev(), S, st));
  if (hashed && bucketed) {
    TRACED(TK_HBSORT, sumV, 24.0 * sumV,
           launch_bucket_sort(c.plan_dev(), bkl, c.A, hflags, hrank, st));
  } else if (hashed) {
    const int P_n = lsd_passes(64, c.rb);
    for (int p = 0; p < P_n; ++p) {  // A -> B -> ...; an odd count ends in B
      SortLaunch a = c.sort_args(buf[p & 1], buf[(p + 1) & 1], TM_VSORT, RANGE_NODES, P_n, p,
                                 lsd_shift(64, c.rb, p));
      TRACED_PASS(TK_VNODE_COUNT, TK_VNODE_SCATTER, sumV, 0.0, SORT_VNODE, a, lsd_width(64, c.rb, p));
    }
    TRACED(TK_HRANK, sumV, 20.0 * sumV,
           launch_hash_rank(c.tiles(TM_DIR, RANGE_NODES), buf[P_n & 1], hkeys, hrank,
                            grid_for(c.total(TM_DIR), cus * 8), st));
  }
  if (hashed && parted) {
    // source positions, grouped as the destination keys are (the same
    // stable grouping again), then the destination keys' positions beside
    // them make the edge keys
    uint32_t *spos = (uint32_t *)(c.py + N);  // source positions, grouped as dst keys
    uint32_t *xpos = spos + N;                 // source slots, then positions, grouped as rows
    uint32_t *yslot = xpos + N;                // destination slots, grouped
    TRACED(TK_HRANK_KEYS, N, 12.0 * N,
           launch_hash_rank_slots(c.tiles(TM_REMAP, RANGE_ROWS), xpos, hrank,
                                  grid_for(c.total(TM_REMAP), cus * 2), st));
    SortLaunch a = c.part_args(c.px + N, nullptr);
    a.vin = xpos;
    a.vout = spos;
    TRACED(TK_HPART_RANK, N, 16.0 * N,
           launch_sort_part(a, SORT_PART_RANK, c.items, PART_BITS, SORT_PART_SCATTER, st));
    TRACED(TK_HPACK, N, (undirected ? 28.0 : 20.0) * N,
           launch_hash_pack_parts(c.tiles(TM_REMAP, RANGE_ROWS), yslot, spos, hrank, c.B,
                                  undirected, counts0, c.esort_tile, c.tm_dev(TM_ESORT),
                                  grid_for(c.total(TM_REMAP), cus * 4), st));
    dev_free(c.hooks, c.px, st);
    dev_free(c.hooks, c.py, st);
    c.px = c.py = nullptr;
  } else if (hashed) {
    TRACED(TK_HREMAP, N, 16.0 * N,
           launch_hash_remap(c.tiles(TM_REMAP, RANGE_ROWS), c.hslots, hrank, c.B, undirected,
                             counts0, c.esort_tile, c.tm_dev(TM_ESORT),
                             grid_for(c.total(TM_REMAP), cus * 8), st));
  } else {
    TileLaunch dt = c.tiles(TM_DIR, RANGE_NODES);
    dt.gaps = c.gapq(0);
    TRACED(TK_DIR, sumV, 16.0 * sumV + 16.0 * dir_words,
           launch_dir(dt, c.A, c.dir, grid_for(c.total(TM_DIR), cus * 8), st));
    HIP_TRY(launch_gap_fill(dt.gaps, st));
    TRACED(TK_REMAP, N, 24.0 * N,
           launch_remap(c.tiles(TM_REMAP, RANGE_ROWS), c.A, c.dir, c.B, undirected,
                        grid_for(c.total(TM_REMAP), cus * 8), st));
  }
  uint64_t *ebuf[2] = {c.B, c.A};
  // multigraph: every key carries its row through the sorts
  uint32_t *vbuf[2] = {nullptr, nullptr};
  if (multi) {
    c.vals = (uint32_t *)dev_alloc(c.hooks, sizeof(uint32_t) * 2 * std::max<int64_t>(N, 1), st);
    if (!c.vals) return RINGO_ERR_OUT_OF_MEMORY;
    vbuf[0] = c.vals;
    vbuf[1] = c.vals + N;
    HIP_TRY(launch_iota(c.tiles(TM_REMAP, RANGE_ROWS), vbuf[0], grid_for(c.total(TM_REMAP), cus * 8),
                        st));
  }
  {
    for (int p = 0; p < P_e; ++p) {
      const int w = lsd_width(2 * b_max, c.rb, p);
      SortLaunch a = c.sort_args(ebuf[p & 1], ebuf[(p + 1) & 1], TM_ESORT, erange, P_e, p,
                                 lsd_shift(2 * b_max, c.rb, p));
      if (multi) {
        a.vin = vbuf[p & 1];
        a.vout = vbuf[(p + 1) & 1];
      }
      const int mode = multi ? SORT_EDGE_KV : SORT_EDGE;
      if (p == 0 && counts0) {  // tile counts written by the remap
        TRACED(TK_EDGE_COUNT, NE, 0.0,
               launch_sort_part(a, mode, c.eitems, w, SORT_PART_PREFIX, st));
        TRACED(TK_EDGE_SCATTER, NE, (16.0 + (multi ? 8.0 : 0.0)) * NE,
               launch_sort_part(a, mode, c.eitems, w, SORT_PART_SCATTER, st));
      } else {
        TRACED_PASS_N(TK_EDGE_COUNT, TK_EDGE_SCATTER, NE, multi ? 8.0 : 0.0, mode, a, w, c.eitems);
      }
    }
  }
  uint64_t *sorted_edges = ebuf[P_e & 1];
  uint64_t *ukeys = ebuf[(P_e + 1) & 1];
  uint32_t *uvals = vbuf[P_e & 1];  // rows of the (kept) sorted keys, same positions
  const bool folded = !undirected && !multi;
  SortLaunch in0;  // folded: the first in-pass, counted before sync #2, scattered after
  if (folded) {
    // Directed graphs: dedupe is folded into the first in-pass, which counts
    // only the first copy of every key; its per-table totals are E.
    in0 = c.sort_args(sorted_edges, ukeys, TM_IN0, RANGE_ROWS, P_in, 0, 32);
    in0.seg_total = c.results + S;
    TRACED(TK_IN_COUNT, N, 8.0 * N,
           launch_sort_part(in0, SORT_IN_FIRST_DEDUP, c.items, lsd_width(b_max, c.rb, 0),
                            SORT_PART_COUNT, st));
  } else if (multi) {
    // every row is an edge: offsets only, and the in-sort reads the sorted
    // keys in place
    TileLaunch mt = c.tiles(TM_DEDUP, erange);
    mt.gaps = c.gapq(1);
    TraceMark m = trace_begin(st);
    HIP_TRY(launch_multi_offsets(mt, sorted_edges, c.results + S, grid_for(c.total(TM_DEDUP), cus * 8),
                                 st));
    HIP_TRY(launch_gap_fill(mt.gaps, st));
    dedupe_rec = trace_end(m, TK_DEDUPE, NE, 8.0 * NE, st);
  } else {
    // undirected: compaction by per-tile counts and a scan (the digit counts
    // of the edge sort are free now)
    TileLaunch ut = c.tiles(TM_DEDUP, erange);
    ut.gaps = c.gapq(1);
    TraceMark m = trace_begin(st);
    HIP_TRY(launch_dedupe_scan(ut, sorted_edges, ukeys, c.results + S, c.counts,
                               grid_for(c.total(TM_DEDUP), cus * 4), st));
    HIP_TRY(launch_gap_fill(ut.gaps, st));
    dedupe_rec = trace_end(m, TK_DEDUPE, NE, 8.0 * NE, st);
  }

  // -------------------------------------------------------------- sync #2
  std::vector<int64_t> E;
  HIP_TRY(c.readback(S, E));
  // int32 arrays of E per table: out_nbr, then (directed, multigraph)
  // in_nbr, then (multigraph) out_eid and in_eid
  const int narr = undirected ? 1 : multi ? 4 : 2;
  size_t arena2 = 0;
  std::vector<size_t> off2((size_t)narr * S);
  for (int i = 0; i < S; ++i) {
    c.plan[i].E = E[i];
    for (int k = 0; k < narr; ++k) {
      off2[(size_t)narr * i + k] = arena2;
      arena2 = align_up(arena2 + sizeof(int32_t) * E[i]);
    }
  }
  for (int i = 0; i < S; ++i) sumE += E[i];
  trace_set_bytes(dedupe_rec, 8.0 * NE + (multi ? 0.0 : 8.0 * sumE) + 8.0 * (sumV + S));
  std::vector<char *> base2(S, nullptr);
  if (c.separate) {
    for (int i = 0; i < S; ++i) {
      const size_t end = i + 1 < S ? off2[(size_t)narr * (i + 1)] : arena2;
      char *blk = c.out_alloc(i, 1, end - off2[(size_t)narr * i]);
      if (!blk) return RINGO_ERR_OUT_OF_MEMORY;
      base2[i] = blk - off2[(size_t)narr * i];
    }
  } else {
    char *blk = c.out_alloc(0, 1, arena2);
    if (!blk) return RINGO_ERR_OUT_OF_MEMORY;
    for (int i = 0; i < S; ++i) base2[i] = blk;
  }
  for (int i = 0; i < S; ++i) {
    SegPlan &p = c.plan[i];
    char *a2 = base2[i];
    p.out_nbr = (int32_t *)(a2 + off2[(size_t)narr * i]);
    p.in_nbr = undirected ? p.out_nbr : (int32_t *)(a2 + off2[(size_t)narr * i + 1]);
    p.out_eid = multi ? (int32_t *)(a2 + off2[(size_t)narr * i + 2]) : nullptr;
    p.in_eid = multi ? (int32_t *)(a2 + off2[(size_t)narr * i + 3]) : nullptr;
    if (undirected) p.in_off = p.out_off;  // the adjacency is its own transpose
  }
  c.set_tiles(TM_ISORT, RANGE_EDGES, c.esort_tile);
  c.set_tiles(TM_ICSR, undirected ? RANGE_EDGES2 : RANGE_EDGES, SCAN_TILE);
  HIP_TRY(c.upload());

  // ------------------------------------------------------------- phase I
  if (undirected) {
    TRACED(TK_IN_CSR, sumE, 12.0 * sumE,
           launch_out_nbr(c.tiles(TM_ICSR, RANGE_EDGES2), ukeys,
                          grid_for(c.total(TM_ICSR), cus * 8), st));
  } else if (folded) {
    // first in-pass: sorted edge keys with repeats -> distinct (d, s) keys,
    // out_nbr and out_off at the de-duplicated positions
    in0.gaps = c.gapq(1);
    TRACED(TK_IN_SCATTER, N, 8.0 * N + 12.0 * sumE + 8.0 * (sumV + S),
           launch_sort_part(in0, SORT_IN_FIRST_DEDUP, c.items, lsd_width(b_max, c.rb, 0),
                            SORT_PART_SCATTER, st));
    HIP_TRY(launch_gap_fill(in0.gaps, st));
    uint64_t *ib[2] = {ukeys, sorted_edges};
    for (int p = 1; p < P_in; ++p) {
      SortLaunch a = c.sort_args(ib[(p - 1) & 1], ib[p & 1], TM_ISORT, RANGE_EDGES, P_in, p,
                                 32 + lsd_shift(b_max, c.rb, p));
      TRACED_PASS_N(TK_IN_COUNT, TK_IN_SCATTER, sumE, 0.0, SORT_IN, a, lsd_width(b_max, c.rb, p),
                    c.eitems);
    }
    TileLaunch it = c.tiles(TM_ICSR, RANGE_EDGES);
    it.gaps = c.gapq(2);
    TRACED(TK_IN_CSR, sumE, 12.0 * sumE + 8.0 * (sumV + S),
           launch_in_csr(it, ib[(P_in - 1) & 1], nullptr, grid_for(c.total(TM_ICSR), cus * 8), st));
    HIP_TRY(launch_gap_fill(it.gaps, st));
  } else {
    // the multigraph's first in-pass reads the sorted keys themselves
    uint64_t *ibuf[2] = {multi ? sorted_edges : ukeys, multi ? ukeys : sorted_edges};
    uint32_t *ivb[2] = {uvals, multi ? vbuf[(P_e + 1) & 1] : nullptr};
    for (int p = 0; p < P_in; ++p) {
      SortLaunch a = c.sort_args(ibuf[p & 1], ibuf[(p + 1) & 1], TM_ISORT, RANGE_EDGES, P_in, p,
                                 32 + lsd_shift(b_max, c.rb, p));
      int mode = p == 0 ? SORT_IN_FIRST : SORT_IN;
      if (multi) {
        a.vin = ivb[p & 1];
        a.vout = ivb[(p + 1) & 1];
        mode = p == 0 ? SORT_IN_FIRST_KV : SORT_IN_KV;
      }
      TRACED_PASS(TK_IN_COUNT, TK_IN_SCATTER, sumE, (p == 0 ? 4.0 : 0.0) + (multi ? 8.0 : 0.0),
                  mode, a, lsd_width(b_max, c.rb, p));
    }
    TileLaunch it = c.tiles(TM_ICSR, RANGE_EDGES);
    it.gaps = c.gapq(2);
    TRACED(TK_IN_CSR, sumE, 12.0 * sumE + 8.0 * (sumV + S),
           launch_in_csr(it, ibuf[P_in & 1], multi ? ivb[P_in & 1] : nullptr,
                         grid_for(c.total(TM_ICSR), cus * 8), st));
    HIP_TRY(launch_gap_fill(it.gaps, st));
  }

  // ------------------------------------------------------------- handoff
  for (int i = 0; i < S; ++i) {
    const SegPlan &p = c.plan[i];
    ringo_graph_t &g = outs[i];
    g.num_rows = p.n;
    g.num_nodes = p.V;
    g.num_edges = p.E;
    g.node_ids = p.V > 0 ? p.node_ids : nullptr;
    g.out_offsets = p.out_off;
    g.out_nbrs = p.E > 0 ? p.out_nbr : nullptr;
    g.in_offsets = p.in_off;
    g.in_nbrs = p.E > 0 ? p.in_nbr : nullptr;
    g._alloc = c.owner_for(i);
    g.kind = c.kind;
    g.out_eids = p.E > 0 ? p.out_eid : nullptr;
    g.in_eids = p.E > 0 ? p.in_eid : nullptr;
  }
  if (!c.small.empty()) handoff_small(c, num_rows, outs);
  c.hand_over(S);  // now owned by the graphs
  return RINGO_OK;
}

// ------------------------------------------------ sync-free single table
//
// A directed table of at most FIXED_MAX_ROWS rows, numbered by sorting,
// converted with nothing read back in between: every kernel is enqueued at
// once.  All sizes follow from n.  The tile maps are those of the worst
// case (V = 2n nodes, E = n edges); the kernels that count V and E move
// them into the plan on the device, so the later kernels walk the real
// ranges and their extra tiles are empty.  The packed edge key takes
// b = ceil(log2 2n) bits per index whatever V turns out to be: (s << b) | d
// orders the edges the same way for every b >= ceil(log2 V), so the graph is
// identical (at most one edge pass more than the exact b would need).  The
// outputs are sized for the worst case: node_ids [2n], out_off and in_off
// [2n + 1], out_nbr and in_nbr [n].
constexpr int64_t FIXED_MAX_ROWS = (int64_t)1 << 20;

struct FixedOut {
  int64_t *node_ids;
  int64_t *out_off;
  int32_t *out_nbr;
  int64_t *in_off;
  int32_t *in_nbr;
};

// Workspace of the sync-free path: offsets of its buffers in one block.
// results holds V, E and the counters of the three queues of long runs
// (directory, out-offsets, in-offsets).
constexpr int FIXED_RESULTS = 5;
struct FixedLayout {
  int rb = DEFAULT_DIGIT_BITS, items = 8, sort_tile = 2048, b = 1, dirk_cap = 0;
  uint32_t gap_cap = 0;
  size_t off_A = 0, off_B = 0, off_counts = 0, off_bsum = 0, off_base = 0, off_results = 0,
         off_meta = 0, off_dir = 0, off_gaps = 0, bytes = 0;
};

FixedLayout fixed_layout(int64_t n, int rb, int items) {
  FixedLayout L;
  L.rb = rb;
  L.items = items;
  L.sort_tile = sort_tile(items);
  L.b = std::max(1, ceil_log2(2 * std::max<int64_t>(n, 1)));
  L.dirk_cap = ceil_log2(std::max<int64_t>(n, 1));
  const int64_t R = (int64_t)1 << rb;
  const int64_t node_tiles = (2 * n + L.sort_tile - 1) / L.sort_tile;
  const int64_t row_tiles = (n + L.sort_tile - 1) / L.sort_tile;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 8));
    return o;
  };
  L.off_A = take(sizeof(uint64_t) * 2 * n);
  L.off_B = take(sizeof(uint64_t) * 2 * n);
  // tile counts of the largest pass (also the unique's tile counts, fewer)
  L.off_counts = take(sizeof(uint32_t) * R * (node_tiles + 1));
  L.off_bsum = take(sizeof(uint32_t) * R * std::max(sort_runs(node_tiles), sort_runs(row_tiles)));
  L.off_base = take(sizeof(int64_t) * R);
  L.off_results = take(sizeof(int64_t) * FIXED_RESULTS);
  L.off_meta = take(sizeof(uint64_t) * META_WORDS);
  L.off_dir = take(sizeof(DirEntry) * (((size_t)1 << L.dirk_cap) + 1));
  // runs lie in the directory (2^dirk_cap + 1 entries) or in an offset array
  // (at most 2n + 1 entries)
  L.gap_cap = (uint32_t)gap_chunks_bound(std::max<int64_t>(((int64_t)1 << L.dirk_cap) + 1, 2 * n + 1));
  L.off_gaps = take(sizeof(GapEntry) * L.gap_cap);
  L.bytes = off;
  return L;
}

// The call state of the sync-free path over workspace ws: plan (sizes of
// the worst case), tile maps, buffers, and the metadata words its first
// kernel writes (plan and tile maps, laid out as Call::upload lays them out).
ringo_status_t fixed_setup(Call &c, const int64_t *src, const int64_t *dst, int64_t n,
                           const FixedOut &o, char *ws, const FixedLayout &L, MetaWords &m,
                           int32_t &nwords) {
  c.S = 1;
  c.items = L.items;
  c.rb = L.rb;
  c.sort_tile = L.sort_tile;
  c.plan.assign(1, SegPlan{});
  c.tmap.assign((size_t)TM_KINDS * 2, 0);
  SegPlan &p = c.plan[0];
  p.src = src;
  p.dst = dst;
  p.n = n;
  p.row_off = 0;
  p.V = 2 * n;  // the worst case, for the tile maps; the device sets V and E
  p.E = n;
  p.b = L.b;
  p.dirk = L.dirk_cap;
  p.dir_off = 0;
  p.node_ids = o.node_ids;
  p.out_off = o.out_off;
  p.out_nbr = o.out_nbr;
  p.in_off = o.in_off;
  p.in_nbr = o.in_nbr;
  c.set_tiles(TM_NSORT, RANGE_NODE_KEYS, c.sort_tile);
  c.set_tiles(TM_UNIQ, RANGE_NODE_KEYS, SCAN_TILE);
  c.set_tiles(TM_DIR, RANGE_NODES, DIR_TILE);
  c.set_tiles(TM_REMAP, RANGE_ROWS, REMAP_TILE);
  c.set_tiles(TM_ESORT, RANGE_ROWS, c.sort_tile);
  c.set_tiles(TM_ISORT, RANGE_EDGES, c.sort_tile);
  c.set_tiles(TM_ICSR, RANGE_EDGES, SCAN_TILE);
  c.A = (uint64_t *)(ws + L.off_A);
  c.B = (uint64_t *)(ws + L.off_B);
  c.counts = (uint32_t *)(ws + L.off_counts);
  c.bsum = (uint32_t *)(ws + L.off_bsum);
  c.base = (int64_t *)(ws + L.off_base);
  c.results = (int64_t *)(ws + L.off_results);
  c.meta = (uint8_t *)(ws + L.off_meta);
  c.dir = (DirEntry *)(ws + L.off_dir);
  const size_t tmap_at = align_up(sizeof(SegPlan));
  const size_t meta_bytes = tmap_at + sizeof(int64_t) * c.tmap.size();
  static_assert(sizeof(SegPlan) <= 256, "plan fits its slot of the metadata");
  if (meta_bytes > sizeof(MetaWords)) return RINGO_ERR_INVALID_ARG;
  std::memset(&m, 0, sizeof(m));
  std::memcpy(m.w, &p, sizeof(SegPlan));
  std::memcpy((char *)m.w + tmap_at, c.tmap.data(), sizeof(int64_t) * c.tmap.size());
  c.meta_bytes = meta_bytes;
  nwords = (int32_t)((meta_bytes + 7) / 8);
  return RINGO_OK;
}

// The workspace belongs to the caller of the sync-free path: a Call over it
// must not free it.
struct Detach {
  Call &c;
  ~Detach() {
    c.A = c.B = nullptr;
    c.base = c.results = nullptr;
    c.meta = nullptr;
    c.dir = nullptr;
    c.counts = c.bsum = nullptr;
  }
};

// Enqueues the whole conversion of one table on st, in the workspace ws
// (L.bytes bytes, laid out by L); ve receives {V, E} on the device.  No
// allocation, no synchronisation; traced only when `traced` is set.
ringo_status_t enqueue_fixed(const int64_t *src, const int64_t *dst, int64_t n, const FixedOut &o,
                             int64_t *ve, char *ws, const FixedLayout &L, bool traced,
                             hipStream_t st) {
  if (n == 0) {
    HIP_TRY(launch_fixed_empty(o.out_off, o.in_off, ve, st));
    return RINGO_OK;
  }
  Call c;
  Detach detach{c};
  c.stream = st;
  MetaWords m;
  int32_t nwords = 0;
  const ringo_status_t rs = fixed_setup(c, src, dst, n, o, ws, L, m, nwords);
  if (rs != RINGO_OK) return rs;
  const int cus = device_cu_count();
  SegPlan *plan_dev = (SegPlan *)c.meta;

  // traced entries only when asked (TRACED records events when tracing is on)
#define FX(kind, units, bytes, expr)                             \
  do {                                                           \
    if (traced) TRACED(kind, units, bytes, expr);                \
    else HIP_TRY(expr);                                          \
  } while (0)
#define FX_PASS(kcount, kscatter, keys, mode, a, w)                                             \
  do {                                                                                          \
    FX(kcount, keys, 8.0 * (keys), launch_sort_part(a, mode, c.items, (w), SORT_PART_COUNT, st)); \
    FX(kscatter, keys, 16.0 * (keys),                                                           \
       launch_sort_part(a, mode, c.items, (w), SORT_PART_SCATTER, st));                         \
  } while (0)

  HIP_TRY(launch_meta_init(m, nwords, (uint64_t *)c.meta, c.results, FIXED_RESULTS, st));
  // queues of long runs: one counter per use (results[2..4])
  auto gq = [&](int use) {
    GapQueue q;
    q.e = (GapEntry *)(ws + L.off_gaps);
    q.count = (uint32_t *)(c.results + 2 + use);
    q.cap = L.gap_cap;
    return q;
  };
  // node keys: ceil(64 / d) passes, the last one into B
  const int P_n = lsd_passes(64, c.rb);
  uint64_t *nbuf[2] = {(P_n & 1) ? c.B : c.A, (P_n & 1) ? c.A : c.B};
  for (int q = 0; q < P_n; ++q) {
    SortLaunch a = c.sort_args(q == 0 ? nullptr : nbuf[(q - 1) & 1], nbuf[q & 1], TM_NSORT,
                               RANGE_NODE_KEYS, P_n, q, lsd_shift(64, c.rb, q));
    FX_PASS(TK_NODE_COUNT, TK_NODE_SCATTER, 2 * n, q == 0 ? SORT_NODE_FIRST : SORT_NODE, a,
            lsd_width(64, c.rb, q));
  }
  FX(TK_UNIQUE, 2 * n, 16.0 * n,
     launch_unique(c.tiles(TM_UNIQ, RANGE_NODE_KEYS), c.B, c.A, c.results, c.counts,
                   grid_for(c.total(TM_UNIQ), cus * 4), st));
  FX(TK_PLAN, 1, 0.0, launch_plan_nodes(plan_dev, c.results, L.dirk_cap, st));
  TileLaunch dt = c.tiles(TM_DIR, RANGE_NODES);
  dt.gaps = gq(0);
  FX(TK_DIR, 2 * n, 0.0, launch_dir(dt, c.A, c.dir, grid_for(c.total(TM_DIR), cus * 8), st));
  HIP_TRY(launch_gap_fill(dt.gaps, st));
  FX(TK_REMAP, n, 24.0 * n,
     launch_remap(c.tiles(TM_REMAP, RANGE_ROWS), c.A, c.dir, c.B, 0,
                  grid_for(c.total(TM_REMAP), cus * 8), st));
  // edge keys: ceil(2b / d) passes from B
  uint64_t *ebuf[2] = {c.B, c.A};
  const int P_e = lsd_passes(2 * L.b, c.rb);
  const int P_in = lsd_passes(L.b, c.rb);
  for (int q = 0; q < P_e; ++q) {
    SortLaunch a = c.sort_args(ebuf[q & 1], ebuf[(q + 1) & 1], TM_ESORT, RANGE_ROWS, P_e, q,
                               lsd_shift(2 * L.b, c.rb, q));
    FX_PASS(TK_EDGE_COUNT, TK_EDGE_SCATTER, n, SORT_EDGE, a, lsd_width(2 * L.b, c.rb, q));
  }
  uint64_t *sorted_edges = ebuf[P_e & 1];
  uint64_t *ukeys = ebuf[(P_e + 1) & 1];
  // first in-pass with the dedupe folded in: its count gives E
  SortLaunch in0 = c.sort_args(sorted_edges, ukeys, TM_ESORT, RANGE_ROWS, P_in, 0, 32);
  in0.seg_total = c.results + 1;
  FX(TK_IN_COUNT, n, 8.0 * n,
     launch_sort_part(in0, SORT_IN_FIRST_DEDUP, c.items, lsd_width(L.b, c.rb, 0), SORT_PART_COUNT,
                      st));
  FX(TK_PLAN, 1, 0.0, launch_plan_edges(plan_dev, c.results, ve, st));
  in0.gaps = gq(1);
  FX(TK_IN_SCATTER, n, 20.0 * n,
     launch_sort_part(in0, SORT_IN_FIRST_DEDUP, c.items, lsd_width(L.b, c.rb, 0), SORT_PART_SCATTER,
                      st));
  HIP_TRY(launch_gap_fill(in0.gaps, st));
  uint64_t *ib[2] = {ukeys, sorted_edges};
  for (int q = 1; q < P_in; ++q) {
    SortLaunch a = c.sort_args(ib[(q - 1) & 1], ib[q & 1], TM_ISORT, RANGE_EDGES, P_in, q,
                               32 + lsd_shift(L.b, c.rb, q));
    FX_PASS(TK_IN_COUNT, TK_IN_SCATTER, n, SORT_IN, a, lsd_width(L.b, c.rb, q));
  }
  TileLaunch it = c.tiles(TM_ICSR, RANGE_EDGES);
  it.gaps = gq(2);
  FX(TK_IN_CSR, n, 12.0 * n,
     launch_in_csr(it, ib[(P_in - 1) & 1], nullptr, grid_for(c.total(TM_ICSR), cus * 8), st));
  HIP_TRY(launch_gap_fill(it.gaps, st));
#undef FX_PASS
#undef FX
  return RINGO_OK;
}

// ------------------------------------------------ replay of the sync-free path
//
// The sync-free path's launch sequence depends only on n and the schedule,
// and every pointer of a call (columns, outputs) is in the metadata its first
// kernel writes from its arguments.  So each size's sequence is captured once
// into a HIP graph over a workspace the library keeps per device, and a later
// call of that size sets the first kernel's arguments and replays the graph:
// one launch instead of about 75.  One call at a time per device uses the
// kept workspace; a call that finds it busy, and calls through a caller's
// allocator (which owns all device memory then), enqueue the kernels
// themselves.  RINGO_FIXED_GRAPH=0 (test support) turns the replay off.
constexpr int MAX_FIXED_GRAPHS = 32;

struct FixedGraph {
  int64_t n = 0;
  int rb = 0, items = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t meta_node = nullptr;
  hipKernelNodeParams meta{};
  uint64_t used = 0;
};

// Per device: the kept workspace, the capture stream and the graphs.  Held
// by one call at a time (its mutex); never released (the process owns it).
struct GraphSlot {
  std::mutex mu;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t cap = nullptr;
  bool broken = false;  // capture failed once: calls enqueue their kernels
  uint64_t clock = 0;
  std::vector<FixedGraph> graphs;
  // sizes met since their last capture: a size is captured the second time
  // it comes, so one-off sizes cost no capture and a size whose graph was
  // evicted comes back twice before it is captured again
  std::vector<int64_t> seen;
};
GraphSlot g_graph_slots[64];

bool fixed_graph_enabled() {
  const char *e = std::getenv("RINGO_FIXED_GRAPH");
  return !(e && e[0] == '0');
}

void fixed_graph_destroy(FixedGraph &g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

// The largest workspace of the sync-free path over every schedule.
size_t fixed_ws_max() {
  size_t m = 0;
  for (int rb = MIN_DIGIT_BITS; rb <= MAX_DIGIT_BITS; ++rb)
    for (int it : {8, 12, 16}) m = std::max(m, fixed_layout(FIXED_MAX_ROWS, rb, it).bytes);
  return m;
}

// The slot's graph for n rows under layout L, captured when the size comes
// the second time (the call's own pointers go into the capture; every
// replay sets them anew); null when there is no graph (yet), and the call
// enqueues its kernels.
FixedGraph *fixed_graph_for(GraphSlot &S, const int64_t *src, const int64_t *dst, int64_t n,
                            const FixedOut &o, const FixedLayout &L) {
  for (FixedGraph &g : S.graphs)
    if (g.n == n && g.rb == L.rb && g.items == L.items) {
      g.used = ++S.clock;
      return &g;
    }
  if (S.broken || n == 0) return nullptr;
  // a size is captured the second time it comes (the first call has also
  // set up what the launches query)
  const int64_t key = n * 64 + L.rb * 4 + L.items / 4;
  const auto it = std::find(S.seen.begin(), S.seen.end(), key);
  if (it == S.seen.end()) {
    if (S.seen.size() >= 256) S.seen.erase(S.seen.begin());
    S.seen.push_back(key);
    return nullptr;
  }
  S.seen.erase(it);
  if (!S.ws) {
    const size_t bytes = fixed_ws_max();
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      S.broken = true;
      return nullptr;
    }
    S.ws = (char *)p;
    S.ws_bytes = bytes;
  }
  if (L.bytes > S.ws_bytes) return nullptr;
  if (!S.cap && hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    S.cap = nullptr;
    S.broken = true;
    return nullptr;
  }
  FixedGraph g;
  g.n = n;
  g.rb = L.rb;
  g.items = L.items;
  bool ok = hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const ringo_status_t rc =
        enqueue_fixed(src, dst, n, o, (int64_t *)(S.ws + L.off_results), S.ws, L, false, S.cap);
    const hipError_t ec = hipStreamEndCapture(S.cap, &g.graph);
    ok = rc == RINGO_OK && ec == hipSuccess && g.graph;
  }
  if (ok) ok = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) == hipSuccess;
  if (ok) {
    size_t nn = 0;
    ok = hipGraphGetNodes(g.graph, nullptr, &nn) == hipSuccess && nn > 0;
    std::vector<hipGraphNode_t> nodes(ok ? nn : 0);
    if (ok) ok = hipGraphGetNodes(g.graph, nodes.data(), &nn) == hipSuccess;
    for (size_t i = 0; ok && i < nn && !g.meta_node; ++i) {
      hipGraphNodeType t;
      if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
      hipKernelNodeParams kp{};
      if (hipGraphKernelNodeGetParams(nodes[i], &kp) == hipSuccess && kp.func == meta_init_kernel()) {
        g.meta_node = nodes[i];
        g.meta = kp;
      }
    }
    ok = ok && g.meta_node;
  }
  if (!ok) {
    (void)hipGetLastError();
    fixed_graph_destroy(g);
    S.broken = true;
    return nullptr;
  }
  if ((int)S.graphs.size() >= MAX_FIXED_GRAPHS) {
    size_t lru = 0;
    for (size_t i = 1; i < S.graphs.size(); ++i)
      if (S.graphs[i].used < S.graphs[lru].used) lru = i;
    fixed_graph_destroy(S.graphs[lru]);
    S.graphs.erase(S.graphs.begin() + (long)lru);
  }
  g.used = ++S.clock;
  S.graphs.push_back(g);
  return &S.graphs.back();
}

// One replay: the metadata kernel's arguments set to this call's, then the
// graph launched on st (traced as one entry).
ringo_status_t replay_fixed(GraphSlot &S, FixedGraph &g, const int64_t *src, const int64_t *dst,
                            int64_t n, const FixedOut &o, const FixedLayout &L, hipStream_t st) {
  Call c;
  Detach detach{c};
  c.stream = st;
  MetaWords m;
  int32_t nwords = 0;
  const ringo_status_t rs = fixed_setup(c, src, dst, n, o, S.ws, L, m, nwords);
  if (rs != RINGO_OK) return rs;
  uint64_t *meta_dst = (uint64_t *)(S.ws + L.off_meta);
  int64_t *results = (int64_t *)(S.ws + L.off_results);
  int32_t nres = FIXED_RESULTS;
  void *args[] = {&m, &nwords, &meta_dst, &results, &nres};
  hipKernelNodeParams p = g.meta;
  p.kernelParams = args;
  p.extra = nullptr;
  HIP_TRY(hipGraphExecKernelNodeSetParams(g.exec, g.meta_node, &p));
  TRACED(TK_GRAPH, n, 0.0, hipGraphLaunch(g.exec, st));
  return RINGO_OK;
}

// The single-table call through the sync-free path: outputs sized for the
// worst case in one block, the kept workspace and a graph replay when free
// (else a workspace from the allocator and the kernels enqueued), one
// synchronisation at the end to read V and E.  With `exact`, the arrays are
// then copied into a block of their exact sizes (for graphs that stay
// resident) and the worst-case block is freed.
ringo_status_t convert_fixed(const int64_t *src, const int64_t *dst, int64_t n, ringo_graph_t *out,
                             hipStream_t st, bool exact) {
  const AllocHooks h = hooks();
  const FixedLayout L = fixed_layout(n, digit_bits_for(n), items_for(n));
  size_t offs[5], arena = 0;
  const size_t sz[5] = {sizeof(int64_t) * 2 * n, sizeof(int64_t) * (2 * n + 1),
                        sizeof(int32_t) * n, sizeof(int64_t) * (2 * n + 1), sizeof(int32_t) * n};
  for (int f = 0; f < 5; ++f) {
    offs[f] = arena;
    arena = align_up(arena + sz[f]);
  }
  // the kept workspace, when no caller's allocator is set and it is free
  GraphSlot *slot = nullptr;
  std::unique_lock<std::mutex> slot_lock;
  int dev = -1;
  if (!h.alloc && fixed_graph_enabled() && hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
    std::unique_lock<std::mutex> l(g_graph_slots[dev].mu, std::try_to_lock);
    if (l.owns_lock()) {
      slot = &g_graph_slots[dev];
      slot_lock = std::move(l);
    }
  }
  (void)hipGetLastError();
  char *blk = (char *)dev_alloc(h, arena, st);
  Pinned *pin = pinned_acquire(sizeof(int64_t) * 2);
  ringo_status_t rc = RINGO_OK;
  int64_t V = 0, E = 0;
  char *ws = nullptr, *own_ws = nullptr;
  if (!blk || !pin) {
    rc = RINGO_ERR_OUT_OF_MEMORY;
  } else {
    FixedOut o{(int64_t *)(blk + offs[0]), (int64_t *)(blk + offs[1]), (int32_t *)(blk + offs[2]),
               (int64_t *)(blk + offs[3]), (int32_t *)(blk + offs[4])};
    FixedGraph *g = slot ? fixed_graph_for(*slot, src, dst, n, o, L) : nullptr;
    if (g) {
      ws = slot->ws;
      rc = replay_fixed(*slot, *g, src, dst, n, o, L, st);
    } else {
      ws = own_ws = (char *)dev_alloc(h, L.bytes, st);
      rc = ws ? enqueue_fixed(src, dst, n, o, (int64_t *)(ws + L.off_results), ws, L, true, st)
              : RINGO_ERR_OUT_OF_MEMORY;
    }
    if (rc == RINGO_OK &&
        (hipMemcpyAsync(pin->p, ws + L.off_results, sizeof(int64_t) * 2, hipMemcpyDeviceToHost, st) !=
             hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
      rc = RINGO_ERR_HIP;
    if (rc == RINGO_OK) {
      V = ((const int64_t *)pin->p)[0];
      E = ((const int64_t *)pin->p)[1];
      if (V > max_nodes()) rc = RINGO_ERR_TOO_MANY_NODES;
    }
    size_t kept = std::max<size_t>(arena, 256);
    if (rc == RINGO_OK && exact) {
      // the graph's arrays into a block of their exact sizes
      const size_t esz[5] = {sizeof(int64_t) * V, sizeof(int64_t) * (V + 1), sizeof(int32_t) * E,
                             sizeof(int64_t) * (V + 1), sizeof(int32_t) * E};
      void *const from[5] = {o.node_ids, o.out_off, o.out_nbr, o.in_off, o.in_nbr};
      size_t eoff[5], ebytes = 0;
      for (int f = 0; f < 5; ++f) {
        eoff[f] = ebytes;
        ebytes = align_up(ebytes + esz[f]);
      }
      char *eb = (char *)dev_alloc(h, ebytes, st);
      if (!eb) rc = RINGO_ERR_OUT_OF_MEMORY;
      for (int f = 0; f < 5 && rc == RINGO_OK; ++f)
        if (esz[f] > 0 &&
            hipMemcpyAsync(eb + eoff[f], from[f], esz[f], hipMemcpyDeviceToDevice, st) != hipSuccess)
          rc = RINGO_ERR_HIP;
      if (rc == RINGO_OK) {
        dev_free(h, blk, st);
        blk = eb;
        kept = std::max<size_t>(ebytes, 256);
        o = FixedOut{(int64_t *)(eb + eoff[0]), (int64_t *)(eb + eoff[1]), (int32_t *)(eb + eoff[2]),
                     (int64_t *)(eb + eoff[3]), (int32_t *)(eb + eoff[4])};
      } else {
        dev_free(h, eb, st);
      }
    }
    if (rc == RINGO_OK) {
      std::memset(out, 0, sizeof(*out));
      Owner *owner = new Owner();
      owner->stream = st;
      owner->hooks = h;
      owner->blocks[0] = blk;
      owner->bytes = kept;
      owner->refs.store(1);
      out->num_rows = n;
      out->num_nodes = V;
      out->num_edges = E;
      out->node_ids = o.node_ids;
      out->out_offsets = o.out_off;
      out->out_nbrs = o.out_nbr;
      out->in_offsets = o.in_off;
      out->in_nbrs = o.in_nbr;
      out->kind = RINGO_GRAPH_DIRECTED;
      out->_alloc = owner;
      blk = nullptr;  // now owned by the graph
    }
  }
  if (rc != RINGO_OK) {
    (void)hipStreamSynchronize(st);
    (void)hipGetLastError();
  }
  dev_free(h, own_ws, st);
  dev_free(h, blk, st);
  if (pin) pinned_release(pin, st);
  return rc;
}

// ------------------------------------------- the entry point that allocates nothing
//
// Its workspace is one file-scope device array, the same on every call: the
// sync-free path's layout for RINGO_NOALLOC_MAX_ROWS rows with 8-bit digits
// and 8 items per thread fits in it (checked per call).  Host code never
// passes the array's name to a kernel: its device address is looked up once
// per device and kept.
static __device__ __align__(256) uint8_t scratch[RINGO_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {nullptr};

// The device address of `scratch` on the current device, or null.
void *scratch_address() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// The sync-free path serves directed single tables above the LDS path's
// size and up to FIXED_MAX_ROWS rows whose schedule numbers nodes by
// sorting.  RINGO_FIXED_PATH=0 (test support) sends them through the pass
// pipeline instead.
bool fixed_path_for(int32_t S, int32_t kind, int64_t n) {
  if (S != 1 || kind != RINGO_GRAPH_DIRECTED || n <= SMALL_ROWS || n > FIXED_MAX_ROWS) return false;
  const char *e = std::getenv("RINGO_FIXED_PATH");
  if (e && e[0] == '0') return false;
  return method_for(n) == RINGO_NODES_SORT;
}

// Stable LSD sort of n keys by their low `bits` bits with the conversion's
// radix passes (one table, plain mode, the schedule's digit width for n
// rows); the last pass writes `out`.
ringo_status_t sort_keys(const uint64_t *in, uint64_t *out, int64_t n, int bits, hipStream_t st) {
  Call c;
  c.S = 1;
  c.stream = st;
  c.hooks = hooks();
  c.plan.assign(1, SegPlan{});
  c.plan[0].n = n;
  c.tmap.assign((size_t)TM_KINDS * 2, 0);
  c.rb = digit_bits_for(n);
  c.items = pair_items(items_for(n), c.rb);
  const int R = 1 << c.rb;
  c.sort_tile = sort_tile(c.items);
  c.set_tiles(TM_ESORT, RANGE_ROWS, c.sort_tile);
  const int64_t max_tiles = c.total(TM_ESORT) + 1;
  const int passes = lsd_passes(bits, c.rb);
  c.meta_bytes = align_up(align_up(sizeof(SegPlan)) + sizeof(int64_t) * c.tmap.size());
  c.pin = pinned_acquire(Call::kUploadSlots * c.meta_bytes + sizeof(int64_t));
  c.counts = (uint32_t *)dev_alloc(c.hooks, sizeof(uint32_t) * R * max_tiles, st);
  c.bsum = (uint32_t *)dev_alloc(c.hooks, sizeof(uint32_t) * R * sort_runs_bound(max_tiles), st);
  c.base = (int64_t *)dev_alloc(c.hooks, sizeof(int64_t) * R, st);
  c.meta = (uint8_t *)dev_alloc(c.hooks, c.meta_bytes, st);
  c.A = passes > 1 ? (uint64_t *)dev_alloc(c.hooks, sizeof(uint64_t) * n, st) : nullptr;
  ringo_status_t rc = RINGO_OK;
  if (!c.pin || !c.counts || !c.bsum || !c.base || !c.meta || (passes > 1 && !c.A)) {
    rc = RINGO_ERR_OUT_OF_MEMORY;
  } else if (c.upload() != hipSuccess) {
    rc = RINGO_ERR_HIP;
  } else {
    // destinations alternate so that the last pass lands in `out`
    uint64_t *dst_of[2] = {(passes & 1) ? out : c.A, (passes & 1) ? c.A : out};
    const uint64_t *src_p = in;
    for (int p = 0; p < passes && rc == RINGO_OK; ++p) {
      uint64_t *dst_p = dst_of[p & 1];
      const SortLaunch a = c.sort_args(src_p, dst_p, TM_ESORT, RANGE_ROWS, passes, p, c.rb * p);
      if (launch_sort_part(a, SORT_PLAIN, c.items, c.rb, SORT_PART_COUNT | SORT_PART_SCATTER,
                           st) != hipSuccess)
        rc = RINGO_ERR_HIP;
      src_p = dst_p;
    }
  }
  c.release_workspace();
  return rc;
}

ringo_status_t convert(int32_t S, const int64_t *const *src, const int64_t *const *dst,
                       const int64_t *num_rows, int32_t kind, ringo_graph_t *outs,
                       hipStream_t stream, bool separate = false) {
  if (S < 0 || (S > 0 && (!src || !dst || !num_rows || !outs))) return RINGO_ERR_INVALID_ARG;
  if (kind != RINGO_GRAPH_DIRECTED && kind != RINGO_GRAPH_UNDIRECTED && kind != RINGO_GRAPH_MULTI)
    return RINGO_ERR_INVALID_ARG;
  for (int i = 0; i < S; ++i) std::memset(&outs[i], 0, sizeof(ringo_graph_t));
  for (int i = 0; i < S; ++i) {
    if (num_rows[i] < 0 || num_rows[i] > RINGO_MAX_ROWS) return RINGO_ERR_INVALID_ARG;
    if (num_rows[i] > 0 && (!src[i] || !dst[i])) return RINGO_ERR_INVALID_ARG;
  }
  if (S == 0) return RINGO_OK;
  (void)hipGetLastError();
  if (fixed_path_for(S, kind, num_rows[0])) {
    const ringo_status_t rc = convert_fixed(src[0], dst[0], num_rows[0], &outs[0], stream, separate);
    if (rc != RINGO_OK) std::memset(&outs[0], 0, sizeof(ringo_graph_t));
    return rc;
  }
  Call c;
  c.S = S;
  c.kind = kind;
  c.stream = stream;
  c.hooks = hooks();
  c.separate = separate;
  ringo_status_t rc = run(c, src, dst, num_rows, outs);
  if (rc != RINGO_OK) {
    // drain what was enqueued before releasing anything it may touch
    (void)hipStreamSynchronize(stream);
    (void)hipGetLastError();
    c.free_outputs();
    for (int i = 0; i < S; ++i) std::memset(&outs[i], 0, sizeof(ringo_graph_t));
  }
  c.release_workspace();
  return rc;
}

}  // namespace

namespace ringo {

ringo_status_t convert_separate(int32_t S, const int64_t *const *src, const int64_t *const *dst,
                                const int64_t *num_rows, ringo_graph_t *outs, hipStream_t stream) {
  return convert(S, src, dst, num_rows, RINGO_GRAPH_DIRECTED, outs, stream, true);
}

size_t graph_bytes(const ringo_graph_t *g) {
  const Owner *o = g ? (const Owner *)g->_alloc : nullptr;
  return o ? o->bytes : 0;
}

void graph_free_on(ringo_graph_t *g, hipStream_t stream) {
  if (!g) return;
  Owner *o = (Owner *)g->_alloc;
  if (o) o->stream = stream;
  owner_release(o);
  std::memset(g, 0, sizeof(*g));
}

}  // namespace ringo

extern "C" {

ringo_status_t ringo_table_to_graph(const int64_t *src, const int64_t *dst, int64_t num_rows,
                                    ringo_graph_t *out, hipStream_t stream) {
  if (!out) return RINGO_ERR_INVALID_ARG;
  return convert(1, &src, &dst, &num_rows, RINGO_GRAPH_DIRECTED, out, stream);
}

ringo_status_t ringo_table_to_graph_noalloc(const int64_t *src, const int64_t *dst,
                                            int64_t num_rows, int64_t *node_ids,
                                            int64_t *out_offsets, int32_t *out_nbrs,
                                            int64_t *in_offsets, int32_t *in_nbrs, int64_t *counts,
                                            hipStream_t stream) {
  if (num_rows < 0 || num_rows > RINGO_NOALLOC_MAX_ROWS) return RINGO_ERR_INVALID_ARG;
  if (!out_offsets || !in_offsets || !counts) return RINGO_ERR_INVALID_ARG;
  if (num_rows > 0 && (!src || !dst || !node_ids || !out_nbrs || !in_nbrs))
    return RINGO_ERR_INVALID_ARG;
  (void)hipGetLastError();
  const FixedLayout L = fixed_layout(num_rows, DEFAULT_DIGIT_BITS, 8);
  if (L.bytes > (size_t)RINGO_NOALLOC_SCRATCH_BYTES) return RINGO_ERR_INVALID_ARG;
  char *ws = (char *)scratch_address();
  if (!ws) return RINGO_ERR_HIP;
  const FixedOut o{node_ids, out_offsets, out_nbrs, in_offsets, in_nbrs};
  return enqueue_fixed(src, dst, num_rows, o, counts, ws, L, false, stream);
}

ringo_status_t ringo_table_to_graph_batched(int32_t num_tables, const int64_t *const *src,
                                            const int64_t *const *dst, const int64_t *num_rows,
                                            ringo_graph_t *outs, hipStream_t stream) {
  return convert(num_tables, src, dst, num_rows, RINGO_GRAPH_DIRECTED, outs, stream);
}

ringo_status_t ringo_table_to_graph_ex(const int64_t *src, const int64_t *dst, int64_t num_rows,
                                       int32_t kind, ringo_graph_t *out, hipStream_t stream) {
  if (!out) return RINGO_ERR_INVALID_ARG;
  return convert(1, &src, &dst, &num_rows, kind, out, stream);
}

ringo_status_t ringo_table_to_graph_batched_ex(int32_t num_tables, const int64_t *const *src,
                                               const int64_t *const *dst, const int64_t *num_rows,
                                               int32_t kind, ringo_graph_t *outs,
                                               hipStream_t stream) {
  return convert(num_tables, src, dst, num_rows, kind, outs, stream);
}

ringo_status_t ringo_sort_keys(const uint64_t *in, uint64_t *out, int64_t n, int32_t bits,
                               hipStream_t stream) {
  if (n < 0 || n > 2 * (int64_t)RINGO_MAX_ROWS || bits < 1 || bits > 64) return RINGO_ERR_INVALID_ARG;
  if (n == 0) return RINGO_OK;
  if (!in || !out) return RINGO_ERR_INVALID_ARG;
  // overlapping arrays would be read and written by the same pass
  const uintptr_t a0 = (uintptr_t)in, a1 = a0 + sizeof(uint64_t) * n;
  const uintptr_t b0 = (uintptr_t)out, b1 = b0 + sizeof(uint64_t) * n;
  if (a0 < b1 && b0 < a1) return RINGO_ERR_INVALID_ARG;
  (void)hipGetLastError();
  return sort_keys(in, out, n, bits, stream);
}

void ringo_graph_free(ringo_graph_t *g) {
  if (!g) return;
  owner_release((Owner *)g->_alloc);
  std::memset(g, 0, sizeof(*g));
}

const char *ringo_status_string(ringo_status_t s) {
  switch (s) {
    case RINGO_OK: return "ok";
    case RINGO_ERR_INVALID_ARG: return "invalid argument";
    case RINGO_ERR_TOO_MANY_NODES: return "too many nodes (V > 2^31 - 1)";
    case RINGO_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RINGO_ERR_HIP: return "HIP runtime error";
    case RINGO_ERR_EVICTED: return "result evicted";
    case RINGO_ERR_PENDING: return "request pending";
  }
  return "unknown status";
}

ringo_status_t ringo_set_allocator(void *(*alloc)(size_t, hipStream_t, void *),
                                   void (*free_)(void *, hipStream_t, void *), void *ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) return RINGO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  g_hooks.alloc = alloc;
  g_hooks.free_ = free_;
  g_hooks.ctx = alloc ? ctx : nullptr;
  return RINGO_OK;
}

ringo_status_t ringo_release_cached(int64_t *bytes_released) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return RINGO_ERR_HIP;
  }
  DeviceCache &C = g_cache[dev];
  std::lock_guard<std::mutex> lk(C.mu);
  int64_t total = 0;
  for (const auto &kv : C.idle) total += (int64_t)kv.second.size;
  release_idle(C);
  if (bytes_released) *bytes_released = total;
  return RINGO_OK;
}

ringo_status_t ringo_tune_get(int64_t num_rows, ringo_schedule_t *out) {
  if (!out || num_rows < 0) return RINGO_ERR_INVALID_ARG;
  out->digit_bits = digit_bits_for(num_rows);
  out->items_per_thread = items_for(num_rows);
  out->node_method = method_for(num_rows);
  return RINGO_OK;
}

ringo_status_t ringo_tune_set(int64_t num_rows, const ringo_schedule_t *sched) {
  if (!sched || num_rows < 0 || sched->digit_bits < MIN_DIGIT_BITS ||
      sched->digit_bits > MAX_DIGIT_BITS)
    return RINGO_ERR_INVALID_ARG;
  const int it = sched->items_per_thread;
  if (it != 8 && it != 12 && it != 16) return RINGO_ERR_INVALID_ARG;
  const int m = sched->node_method;
  if (m != RINGO_NODES_SORT && m != RINGO_NODES_HASH) return RINGO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  schedule_init_locked();
  const int k = ceil_log2(std::max<int64_t>(num_rows, 1));
  g_items[k] = it;
  g_bits[k] = sched->digit_bits;
  g_method[k] = m;
  return RINGO_OK;
}


void ringo_trace_enable(int on) {
  std::vector<TraceRec> old;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_trace_on = on != 0;
    old.swap(g_trace);
  }
  for (auto &r : old) {
    (void)hipEventSynchronize(r.b);
    std::lock_guard<std::mutex> lk(g_mu);
    g_evpool.push_back(r.a);
    g_evpool.push_back(r.b);
  }
}

int ringo_trace_read(ringo_trace_entry_t *out, int max_entries) {
  std::vector<TraceRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    recs = g_trace;
  }
  ringo_trace_entry_t acc[TK_KINDS];
  for (int k = 0; k < TK_KINDS; ++k) {
    acc[k].kernel = kTraceNames[k];
    acc[k].launches = 0;
    acc[k].total_ms = 0;
    acc[k].bytes = 0;
    acc[k].units = 0;
  }
  for (auto &r : recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return -1;
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -1;
    ringo_trace_entry_t &e = acc[r.kind];
    e.launches += 1;
    e.total_ms += ms;
    e.bytes += r.bytes;
    e.units += r.units;
  }
  int n = 0;
  for (int k = 0; k < TK_KINDS && n < max_entries; ++k)
    if (acc[k].launches > 0) out[n++] = acc[k];
  return n;
}

const char *ringo_version(void) { return "ringo-mi355x 0.1 (gfx950)"; }

}  // extern "C"

// ------------------------------------------------ workspace for other entry points

namespace ringo {

void *workspace_alloc(size_t bytes, hipStream_t s) {
  return dev_alloc(hooks(), bytes, s);
}

void workspace_free(void *p, hipStream_t s) { dev_free(hooks(), p, s); }

}  // namespace ringo
