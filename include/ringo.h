/*
 * ringo.h -- C ABI of the MI355X table-to-graph conversion library.
 *
 * The operation (Section 2.4, "Conversion of tables to graphs"): an edge
 * table T with a source column S and a destination column D defines the
 * directed graph G = (V, E) whose nodes are the distinct values found in S
 * and D and whose edges are the pairs (r_S, r_D) of its rows.  The paper's
 * graph keeps, for every node, a sorted out-neighbour vector and a sorted
 * in-neighbour vector (Sections 2.2 and 2.4); this library emits the same
 * lists in compressed-sparse-row form (the node vector plus edge vector of
 * Section 2.2), one CSR per direction.
 *
 * Readings fixed by this library:
 *   - E is a set: repeated rows give one edge; self-loops are kept.
 *   - node_ids lists V in ascending signed 64-bit order; every 64-bit value,
 *     INT64_MIN included, is a valid identifier.
 *   - Neighbours are stored as 32-bit dense positions into node_ids, so each
 *     list is strictly increasing by position and by identifier.
 *   - The whole method runs on the GPU ("sort-first", Section 2.4): sort the
 *     column copies, count neighbours, place the neighbour lists.
 *
 * Memory: unless noted otherwise, pointers named src/dst and every array in
 * ringo_graph_t are DEVICE pointers on the current HIP device; counts and
 * arrays of pointers passed by the caller are HOST memory.
 *
 * Errors: every entry point returns a ringo_status_t.  On any error the
 * output structs are zeroed, nothing is leaked and no partial result is
 * returned.
 */
#ifndef RINGO_H
#define RINGO_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RINGO_OK = 0,
  RINGO_ERR_INVALID_ARG = 1,    /* NULL pointer with rows > 0, negative or too many rows */
  RINGO_ERR_TOO_MANY_NODES = 2, /* V > 2^31 - 1: neighbours would not fit 32 bits */
  RINGO_ERR_OUT_OF_MEMORY = 3,  /* workspace or outputs could not be allocated */
  RINGO_ERR_HIP = 4,            /* a HIP runtime call failed */
  RINGO_ERR_EVICTED = 5,        /* served form: the result was evicted under the HBM budget */
  RINGO_ERR_PENDING = 6         /* served form: the request has not finished yet */
} ringo_status_t;

/* Largest row count of one table: 2 * rows must index 32-bit slots. */
#define RINGO_MAX_ROWS ((int64_t)2147483647)
/* Largest node count: neighbours are 32-bit positions. */
#define RINGO_MAX_NODES ((int64_t)2147483647)

/*
 * Graph kinds.  The paper discusses directed graphs (Section 2.4) and
 * defines the conversion for them; the other two kinds apply the same
 * definition with another edge rule:
 *   RINGO_GRAPH_DIRECTED   E is the set of distinct (src, dst) pairs
 *                          (a simple directed graph; self-loops kept).
 *   RINGO_GRAPH_UNDIRECTED the adjacency of v is the set of w with a row
 *                          (v, w) or (w, v), ascending; a self-loop appears
 *                          once.  num_edges is the number of adjacency
 *                          entries (each non-loop pair counts twice), and
 *                          the in-arrays are the out-arrays (same pointers).
 *   RINGO_GRAPH_MULTI      every row is its own edge (num_edges = num_rows),
 *                          identified by its row index: out-lists ascend by
 *                          (destination, row), in-lists by (source, row),
 *                          and out_eids / in_eids give each entry's row.
 */
#define RINGO_GRAPH_DIRECTED 0
#define RINGO_GRAPH_UNDIRECTED 1
#define RINGO_GRAPH_MULTI 2

/*
 * The converted graph (Section 2.4).  Scalars are host values, valid when
 * the call returns; arrays are device memory owned by the library, valid
 * once the stream passed to the call has completed, released with
 * ringo_graph_free.  (Field comments describe the directed kind.)
 */
typedef struct {
  int64_t num_rows;     /* n: rows of the input table                          */
  int64_t num_nodes;    /* V: distinct identifiers in src and dst              */
  int64_t num_edges;    /* E: distinct (src, dst) pairs                        */
  int64_t *node_ids;    /* [V]   strictly increasing, signed order             */
  int64_t *out_offsets; /* [V+1] out_offsets[0] = 0, out_offsets[V] = E        */
  int32_t *out_nbrs;    /* [E]   out-neighbours of v at out_offsets[v]..[v+1], */
                        /*       strictly increasing positions into node_ids   */
  int64_t *in_offsets;  /* [V+1] in_offsets[0] = 0, in_offsets[V] = E          */
  int32_t *in_nbrs;     /* [E]   in-neighbours, strictly increasing            */
  void *_alloc;         /* opaque owner of the arrays                          */
  int32_t kind;         /* RINGO_GRAPH_*                                       */
  int32_t _reserved;
  int32_t *out_eids;    /* [E]   RINGO_GRAPH_MULTI: row of each out-entry      */
  int32_t *in_eids;     /* [E]   RINGO_GRAPH_MULTI: row of each in-entry       */
} ringo_graph_t;

/*
 * Table-to-graph conversion of one edge table (Section 2.4).
 *   src, dst : device arrays of num_rows int64 identifiers, caller-owned,
 *              read-only, and valid until `stream` reaches this work.
 *   num_rows : 0 <= num_rows <= RINGO_MAX_ROWS.  num_rows == 0 is legal:
 *              V = E = 0, both offset arrays hold the single value 0 and
 *              the other arrays are NULL.
 *   out      : host struct filled on success (see ringo_graph_t).
 *   stream   : all device work is ordered on this stream.  The call
 *              synchronises with the stream to size its outputs: after the
 *              node set and after the edge set are known, plus once before
 *              the node hash table is sized (RINGO_NODES_HASH); it returns
 *              with the in-direction still enqueued.  A table of at most
 *              2048 rows is converted by one workgroup in LDS instead (one
 *              launch, one synchronisation); its arrays are then sized for
 *              the worst case (V <= 2n, E <= n), of which the first V,
 *              V + 1 and E entries hold the graph.
 * Errors: RINGO_ERR_INVALID_ARG (NULL out, NULL src/dst with rows > 0,
 * rows out of range), RINGO_ERR_TOO_MANY_NODES, RINGO_ERR_OUT_OF_MEMORY,
 * RINGO_ERR_HIP.
 */
ringo_status_t ringo_table_to_graph(const int64_t *src, const int64_t *dst, int64_t num_rows,
                                    ringo_graph_t *out, hipStream_t stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * conversion as ringo_table_to_graph (the graph is identical) for one table
 * of at most RINGO_NOALLOC_MAX_ROWS rows, into arrays the caller allocates
 * for the worst case, with the library's workspace in one fixed device array
 * of RINGO_NOALLOC_SCRATCH_BYTES per device (held from the library's first
 * use on that device until the process ends).  Nothing is allocated, and
 * nothing is synchronised: the call only enqueues kernels on `stream`.
 *   src, dst    : device arrays of num_rows int64 identifiers (as for
 *                 ringo_table_to_graph).
 *   num_rows    : 0 <= num_rows <= RINGO_NOALLOC_MAX_ROWS.
 *   node_ids    : device int64 [2 * num_rows]      } the first V, V + 1, E
 *   out_offsets : device int64 [2 * num_rows + 1]  } entries hold the graph
 *   out_nbrs    : device int32 [num_rows]          } once the stream reaches
 *   in_offsets  : device int64 [2 * num_rows + 1]  } the end of this work;
 *   in_nbrs     : device int32 [num_rows]          } the rest is untouched
 *   counts      : device int64 [2], receives {V, E}.
 * With num_rows == 0 only out_offsets[0], in_offsets[0] (both 0) and counts
 * ({0, 0}) are written; src, dst, node_ids and the neighbour arrays may then
 * be NULL.
 * Every call on a device uses that device's one workspace: calls that
 * overlap on one device race and give wrong results, so order them (one
 * stream, or events).  Each call writes every part of the workspace it
 * reads, so no clearing is needed between calls.
 * Errors: RINGO_ERR_INVALID_ARG (a NULL array, num_rows out of range),
 * RINGO_ERR_HIP (the workspace's address could not be obtained, or a launch
 * failed).
 */
#define RINGO_NOALLOC_MAX_ROWS ((int64_t)1 << 20)
#define RINGO_NOALLOC_SCRATCH_BYTES ((size_t)50 << 20)
ringo_status_t ringo_table_to_graph_noalloc(const int64_t *src, const int64_t *dst,
                                            int64_t num_rows, int64_t *node_ids,
                                            int64_t *out_offsets, int32_t *out_nbrs,
                                            int64_t *in_offsets, int32_t *in_nbrs, int64_t *counts,
                                            hipStream_t stream);

/*
 * Batched conversion of num_tables independent edge tables (the same
 * operation as ringo_table_to_graph, Section 2.4, applied to each table).
 *   src, dst : HOST arrays of num_tables DEVICE pointers.
 *   num_rows : HOST array of num_tables row counts (each as above).
 *   outs     : HOST array of num_tables structs, filled on success.
 * Every phase of the pipeline runs once for the whole batch: one launch per
 * pass covers all tables, and the batch synchronises with the stream as
 * often as one call does.  Tables of at most 2048 rows (directed kind) are
 * converted by one workgroup each, all in one launch beside the pipeline.
 * outs[i] is bit-identical to ringo_table_to_graph on table i.
 * All-or-nothing: on error every outs[i] is zeroed.
 */
ringo_status_t ringo_table_to_graph_batched(int32_t num_tables, const int64_t *const *src,
                                            const int64_t *const *dst, const int64_t *num_rows,
                                            ringo_graph_t *outs, hipStream_t stream);

/*
 * The conversion for any graph kind (RINGO_GRAPH_*; ringo_table_to_graph and
 * ringo_table_to_graph_batched are the RINGO_GRAPH_DIRECTED cases).  Same
 * arguments, ownership and errors, plus RINGO_ERR_INVALID_ARG for an unknown
 * kind.  Undirected graphs sort both orientations of every row (2n edge
 * keys) and have no separate in-direction; multigraphs carry every row's
 * index through the edge sorts and keep every row.
 */
ringo_status_t ringo_table_to_graph_ex(const int64_t *src, const int64_t *dst, int64_t num_rows,
                                       int32_t kind, ringo_graph_t *out, hipStream_t stream);
ringo_status_t ringo_table_to_graph_batched_ex(int32_t num_tables, const int64_t *const *src,
                                               const int64_t *const *dst, const int64_t *num_rows,
                                               int32_t kind, ringo_graph_t *outs,
                                               hipStream_t stream);

/*
 * Stable least-significant-digit radix sort of uint64 keys: the sort the
 * conversion runs on its column copies (Section 2.4), exposed as a primitive.
 * It takes ceil(bits / d) passes of d-bit digits, d being the digit width of
 * the schedule for n rows (ringo_tune_get), so keys are ordered by their low
 * min(64, d * ceil(bits / d)) bits (all of them for bits = 64); keys equal in
 * those bits keep their input order, and the higher bits travel with the
 * keys.  For keys below 2^b, bits = b gives the full ascending order.
 *   in, out : DEVICE arrays of n keys; they must not overlap.
 *   n       : 0 <= n <= 2 * RINGO_MAX_ROWS.
 *   bits    : 1..64.
 * Enqueued on `stream` with stream-ordered workspace; no synchronisation.
 * Errors: RINGO_ERR_INVALID_ARG, RINGO_ERR_OUT_OF_MEMORY, RINGO_ERR_HIP.
 */
ringo_status_t ringo_sort_keys(const uint64_t *in, uint64_t *out, int64_t n, int32_t bits,
                               hipStream_t stream);

/* Releases the arrays of a graph and zeroes *g.  Idempotent; NULL is a no-op.
 * The caller must make sure no enqueued work still reads the arrays. */
void ringo_graph_free(ringo_graph_t *g);

/*
 * Graph-to-table conversion (Section 2.4, "Conversion of graphs to tables";
 * Table 5 times it for LiveJournal and Twitter2010).
 *
 * ringo_graph_to_edge_table writes the edge table of g: row i is
 * (node_ids[u], node_ids[out_nbrs[i]]) for the i-th edge in out-CSR order,
 * u being the edge's source; rows are therefore in ascending (source,
 * destination) order, signed, with no duplicates.  For a graph made by
 * ringo_table_to_graph this is the sorted distinct rows of the input table.
 *   g                 : a graph (host struct, device arrays); only num_nodes,
 *                       num_edges, node_ids, out_offsets and out_nbrs are read.
 *   src_ids, dst_ids  : caller-allocated DEVICE arrays of g->num_edges int64.
 * ringo_graph_to_node_table writes the node table of g: row v is
 * (node_ids[v], out-degree of v, in-degree of v); each of the three DEVICE
 * arrays of g->num_nodes int64 may be NULL to skip that column.
 * Both are enqueued on `stream` without any synchronisation and allocate
 * nothing.  Errors: RINGO_ERR_INVALID_ARG (NULL g, negative sizes, a needed
 * array NULL), RINGO_ERR_HIP (launch failure).
 */
ringo_status_t ringo_graph_to_edge_table(const ringo_graph_t *g, int64_t *src_ids,
                                         int64_t *dst_ids, hipStream_t stream);
ringo_status_t ringo_graph_to_node_table(const ringo_graph_t *g, int64_t *node_ids,
                                         int64_t *out_degree, int64_t *in_degree,
                                         hipStream_t stream);

/*
 * PageRank of a graph (the paper's workflow computes it on a converted graph,
 * Section 4; Table 3 times ten iterations).  Page, Brin, Motwani & Winograd's
 * definition, in fp64, with the teleport and the rank of nodes without
 * out-edges spread uniformly over all nodes:
 *   r_0[v] = 1/V;  r_{t+1}[v] = (1-d)/V + d * (sum over edges u->v of
 *   r_t[u]/outdeg(u) + (sum of r_t[u] over nodes without out-edges)/V).
 *   g          : a graph; num_nodes, num_edges, out_offsets, in_offsets and
 *                in_nbrs are read (in-CSR pull, out-degrees from out_offsets).
 *   damping    : d in [0, 1] (0.85 is the usual value).
 *   iterations : t >= 0; the result is r_t.
 *   ranks      : caller-allocated DEVICE array of num_nodes doubles.
 * Enqueued on `stream`; stream-ordered workspace from the library's
 * allocator, released in stream order.  Results are deterministic (fixed
 * summation order).  Errors: RINGO_ERR_INVALID_ARG, RINGO_ERR_OUT_OF_MEMORY,
 * RINGO_ERR_HIP.
 */
ringo_status_t ringo_pagerank(const ringo_graph_t *g, double damping, int32_t iterations,
                              double *ranks, hipStream_t stream);

/* Static, human-readable name of a status code. */
const char *ringo_status_string(ringo_status_t s);

/*
 * Optional device allocator for workspaces and outputs (for example a
 * framework's caching allocator).  alloc(bytes, stream, ctx) returns device
 * memory usable in stream order on `stream`, or NULL; free_(ptr, stream, ctx)
 * returns it.  Passing NULL for both restores the built-in allocator: a
 * cache of device blocks per device (hipMalloc), where a freed block stays
 * allocated and is reused by later requests on the stream that freed it at
 * once, on other streams once the work before its release has completed;
 * cached blocks are returned to the device only when hipMalloc fails.  Must
 * not be changed while graphs allocated by the previous allocator are
 * alive.
 */
ringo_status_t ringo_set_allocator(void *(*alloc)(size_t bytes, hipStream_t stream, void *ctx),
                                   void (*free_)(void *ptr, hipStream_t stream, void *ctx),
                                   void *ctx);

/*
 * Returns the built-in allocator's idle cached blocks on the current device
 * to the device (hipFree, once the work before each block's release has
 * completed; it may wait for that work).  Blocks in use (resident graphs,
 * calls in flight) are not touched, and later calls cache blocks again.
 * For callers that share the device with another allocator (a framework's
 * caching allocator) and need the memory back.  *bytes_released (may be
 * NULL) receives the bytes returned.  RINGO_ERR_HIP if there is no current
 * device.
 */
ringo_status_t ringo_release_cached(int64_t *bytes_released);

/*
 * Tuning schedule: digit width (bits per radix pass), items per thread of
 * the scatter tile, and the node-numbering method.  ringo_tune_get returns
 * the schedule the library will use for a table of num_rows rows (for a
 * batch: of the batch's total rows); ringo_tune_set overrides it for the
 * size bucket holding num_rows (powers of two; used by the autotuner).
 * Valid digit widths: 8 to 11 bits (a pass sorts on that many bits, so a
 * key of k bits takes ceil(k / digit_bits) passes); valid items per thread:
 * 8, 12, 16.
 *
 * Node numbering (both give the same graph, bit for bit):
 *   RINGO_NODES_SORT  radix sort of all 2n identifiers, then unique.
 *   RINGO_NODES_HASH  the paper's node hash table (open addressing, linear
 *                     probing; Section 2.5): insert the 2n identifiers, sort
 *                     only the V distinct ones.  One more stream
 *                     synchronisation per call (a distinct-count estimate
 *                     sizes the table).  Should a probe sequence exceed its
 *                     bound (an estimate far too low), the call falls back to
 *                     RINGO_NODES_SORT by itself.
 * Built-in defaults (measured on an MI355X): RINGO_NODES_SORT up to 2^23 rows,
 * RINGO_NODES_HASH above; 8 items per thread and 8-bit digits up to 2^26
 * rows, 16 items above, and 9-bit digits from 2^29 rows.
 */
#define RINGO_NODES_SORT 0
#define RINGO_NODES_HASH 1
typedef struct {
  int32_t digit_bits;
  int32_t items_per_thread;
  int32_t node_method;
} ringo_schedule_t;
ringo_status_t ringo_tune_get(int64_t num_rows, ringo_schedule_t *out);
ringo_status_t ringo_tune_set(int64_t num_rows, const ringo_schedule_t *sched);

/*
 * Kernel tracing (measurement support).  While enabled, every kernel launch
 * of every call is bracketed by two HIP events recorded on the call's
 * stream.  ringo_trace_read waits for the recorded events and fills up to
 * max_entries entries, one per kernel kind that ran, with the launch count,
 * the summed event-measured duration, the algorithmic bytes the launches
 * move (input read once, output written once, per the kernel's definition)
 * and the processed element count.  Returns the number of entries, or -1 on
 * a HIP error.  ringo_trace_enable(0 or 1) discards the records so far.
 */
typedef struct {
  const char *kernel; /* static name: hist_node, sort_pass_node, ...     */
  int64_t launches;
  double total_ms;
  double bytes;
  int64_t units;      /* keys, rows, nodes or edges processed in total    */
} ringo_trace_entry_t;
void ringo_trace_enable(int on);
int ringo_trace_read(ringo_trace_entry_t *out, int max_entries);

/*
 * Served form: an interactive request loop that keeps built graphs resident
 * on the device (the paper's interactive-use goal, Sections 1 and 2.4).
 * Requests are host edge tables; worker threads, each with its own stream,
 * take every queued request that fits into one batch and convert it as
 * ringo_table_to_graph_batched does, so batches started by different workers
 * overlap on the device.  Every graph of a batch holds device blocks of its
 * own, in exact sizes, and counts against the budget by their bytes.  A
 * request is admitted only while the HBM budget holds its estimated
 * footprint on top of the resident graphs; the least recently used resident
 * graph that is not pinned is evicted when it does not.  Each result is
 * bit-identical to ringo_table_to_graph on the same table.
 */
typedef struct ringo_server ringo_server_t;
typedef struct {
  int64_t budget_bytes;     /* device bytes for resident graphs and in-flight work  */
  int32_t num_streams;      /* worker threads / streams, 1..16                       */
  int32_t max_batch_tables; /* requests per batch, >= 1                              */
  int64_t max_batch_rows;   /* rows per batch (a larger single request still runs)   */
} ringo_server_config_t;
typedef struct {
  int64_t submitted, completed, failed, evicted, queued;
  int64_t batches, max_concurrent_batches;
  int64_t rows_completed;
  int64_t resident_bytes, peak_reserved_bytes;
} ringo_server_stats_t;

/* Starts the workers on the current HIP device.  RINGO_ERR_INVALID_ARG on a
 * bad configuration, RINGO_ERR_HIP if no device is current. */
ringo_status_t ringo_server_create(const ringo_server_config_t *cfg, ringo_server_t **out);
/* Queues a conversion of the HOST arrays src[num_rows], dst[num_rows]
 * (pinned memory for full copy speed).  They must stay valid and unchanged
 * until the request leaves RINGO_ERR_PENDING.  *req_id identifies it. */
ringo_status_t ringo_server_submit(ringo_server_t *s, const int64_t *src, const int64_t *dst,
                                   int64_t num_rows, int64_t *req_id);
/* RINGO_OK with *out set to a view of the resident graph (the server keeps
 * ownership: out->_alloc is NULL; the view is valid until the request is
 * released or evicted), RINGO_ERR_PENDING, RINGO_ERR_EVICTED, or the
 * conversion's error.  *latency_s (may be NULL) receives the time from
 * submission to the graph being resident once the request has finished.
 * Polling a resident graph marks it as recently used. */
ringo_status_t ringo_server_poll(ringo_server_t *s, int64_t req_id, ringo_graph_t *out,
                                 double *latency_s);
/* Frees a finished request and its resident graph; RINGO_ERR_PENDING while
 * it is still queued or running, or pinned. */
ringo_status_t ringo_server_release(ringo_server_t *s, int64_t req_id);
/* A view as ringo_server_poll gives it (same results), pinned: the graph is
 * not evicted until ringo_server_unpin.  A client that reads a view on its
 * own stream pins it first and unpins it once that stream has finished the
 * reads (an evicted graph's memory is freed in the order of the server's
 * streams, not the client's).  Pins nest; RINGO_ERR_INVALID_ARG when unpin
 * finds no pin. */
ringo_status_t ringo_server_pin(ringo_server_t *s, int64_t req_id, ringo_graph_t *out);
ringo_status_t ringo_server_unpin(ringo_server_t *s, int64_t req_id);
/* Device times of finished batches (the latest max_entries of them, at most
 * 65536 kept): events recorded on the batch's worker stream before its input
 * copies and after its last kernel, in milliseconds since the server
 * started.  Returns the number of entries written, or -1 (HIP error, bad
 * argument).  Batches on different streams whose intervals intersect ran
 * on the device at the same time. */
typedef struct {
  int64_t first_request; /* id of the batch's first request */
  int64_t rows;          /* rows of its tables                */
  int32_t stream;        /* worker (stream) index             */
  int32_t tables;        /* requests in the batch             */
  double start_ms, end_ms;
} ringo_server_batch_t;
int ringo_server_batches(ringo_server_t *s, ringo_server_batch_t *out, int max_entries);
ringo_status_t ringo_server_stats(ringo_server_t *s, ringo_server_stats_t *out);
/* Finishes the queued requests, frees every resident graph, joins the
 * workers.  NULL is a no-op. */
void ringo_server_destroy(ringo_server_t *s);

/* Version string of the library build. */
const char *ringo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RINGO_H */
