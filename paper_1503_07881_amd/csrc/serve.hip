// Served form of the conversion: an interactive request loop that keeps
// built graphs resident on the device.
//
// The paper aims the conversion at interactive sessions: very large tables
// have to become graphs quickly enough for an analyst to wait on them
// (Section 2.4), and the graphs stay in memory for the analysis that
// follows (Sections 1 and 2.1).  The server here:
//   * queues requests (host edge tables) in arrival order;
//   * runs W worker threads, each with its own HIP stream; a free worker
//     takes every queued request that fits into one batch and converts the
//     batch with ringo_table_to_graph_batched, so requests that arrive while
//     other batches are on the GPU start as soon as a worker is free and
//     their work overlaps on the device (continuous batching);
//   * admits a request only while the HBM budget holds its estimated
//     footprint (input, workspace, outputs) on top of the resident graphs,
//     evicting the least recently used resident graph that no client holds
//     pinned when it does not;
//   * gives every graph of a batch output blocks of its own and counts a
//     resident graph by the bytes those blocks hold, so that evicting a
//     graph frees what it is counted for;
//   * records each request's latency from submission to its graph being
//     resident (the host-to-device copy of its input included), and each
//     batch's device start and end (events on its stream).
// A request's result is bit-identical to a lone ringo_table_to_graph call:
// every table of a batch is converted independently.

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ringo.h"
#include "ringo_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { RS_QUEUED, RS_RUNNING, RS_READY, RS_FAILED, RS_EVICTED, RS_RELEASED };

struct Request {
  int64_t id = 0;
  const int64_t *src = nullptr;
  const int64_t *dst = nullptr;
  int64_t n = 0;
  Clock::time_point submitted, finished;
  ReqState state = RS_QUEUED;
  ringo_status_t status = RINGO_OK;
  ringo_graph_t graph{};
  int64_t reserve = 0;    // bytes held against the budget
  uint64_t last_use = 0;  // LRU clock
  int pins = 0;           // client reads in flight: not evictable while > 0
};

// One batch's device work: events on its worker stream before its input
// copy and after its last kernel.
struct BatchRec {
  hipEvent_t start = nullptr, end = nullptr;
  int32_t stream = 0, tables = 0;
  int64_t rows = 0, first_request = 0;
};

// Bytes a request may need while it is converted: its input columns, the
// workspace (two key buffers of 2n keys, slot indices, per-tile digit counts
// of the schedule's tiles and digit width) and its outputs at their upper
// bound (V <= 2n nodes, E <= n edges).  A table of at most 2^20 rows also
// holds its node directory (up to 2^ceil(log2 n) entries) and, once
// converted into worst-case arrays, the copy in exact sizes.
int64_t footprint(int64_t n) {
  const int64_t input = 16 * n;
  ringo_schedule_t sc;
  if (ringo_tune_get(n, &sc) != RINGO_OK) sc.digit_bits = 11, sc.items_per_thread = 8;
  const int64_t tiles = 2 * n / (256 * sc.items_per_thread) + 2;
  const int64_t counts = 4 * tiles * ((int64_t)1 << sc.digit_bits);
  const int64_t workspace = 32 * n + 8 * n + counts + (int64_t)(1 << 20);
  const int64_t outputs = 8 * (2 * n) + 16 * (2 * n + 1) + 8 * n;
  const int64_t small_extra = n <= ((int64_t)1 << 20) ? 32 * n + outputs : 0;
  return input + workspace + outputs + small_extra;
}

// Batches whose device times are kept (the latest ones).
constexpr size_t MAX_BATCH_RECS = 1 << 16;

}  // namespace

struct ringo_server {
  ringo_server_config_t cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int64_t> queue;
  std::unordered_map<int64_t, Request> reqs;
  int64_t next_id = 1;
  int64_t reserved = 0;  // in-flight footprints + resident graphs
  uint64_t clock = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;  // one per worker; resident graphs free on them
  ringo_server_stats_t stats{};
  int running_batches = 0;
  hipEvent_t t0 = nullptr;  // device time origin of the batch records
  std::vector<BatchRec> batch_recs;
  std::vector<BatchRec> done_recs;  // events of dropped records, freed at the end

  // Evicts least recently used resident graphs that no client has pinned
  // until `need` more bytes fit in the budget.  Returns whether they fit.
  // An evicted graph's memory is released in the order of `stream`, the
  // admitting worker's, so that its next allocations reuse the memory at
  // once (the stream that built the graph may be busy with another batch).
  // Caller holds mu.
  bool make_room(int64_t need, hipStream_t stream) {
    while (reserved + need > cfg.budget_bytes) {
      Request *victim = nullptr;
      for (auto &kv : reqs) {
        Request &r = kv.second;
        if (r.state == RS_READY && r.pins == 0 && (!victim || r.last_use < victim->last_use))
          victim = &r;
      }
      if (!victim) return false;
      ringo::graph_free_on(&victim->graph, stream);
      reserved -= victim->reserve;
      victim->reserve = 0;
      victim->state = RS_EVICTED;
      stats.evicted += 1;
    }
    return true;
  }

  void worker_main(int index) {
    (void)hipSetDevice(device);
    hipStream_t stream = streams[index];
    std::vector<int64_t> batch;
    for (;;) {
      batch.clear();
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !queue.empty(); });
        if (stop && queue.empty()) break;
        int64_t rows = 0;
        while (!queue.empty() && (int)batch.size() < cfg.max_batch_tables) {
          Request &r = reqs[queue.front()];
          if (!batch.empty() && rows + r.n > cfg.max_batch_rows) break;
          const int64_t need = footprint(r.n);
          if (need > cfg.budget_bytes) {  // can never fit
            queue.pop_front();
            r.state = RS_FAILED;
            r.status = RINGO_ERR_OUT_OF_MEMORY;
            r.finished = Clock::now();
            stats.failed += 1;
            continue;
          }
          if (!make_room(need, stream)) break;  // wait for running batches to finish
          queue.pop_front();
          reserved += need;
          r.reserve = need;
          r.state = RS_RUNNING;
          rows += r.n;
          batch.push_back(r.id);
        }
        if (batch.empty()) {
          // the head of the queue does not fit yet: wait for a batch to end
          cv.wait_for(lk, std::chrono::milliseconds(1));
          continue;
        }
        running_batches += 1;
        stats.batches += 1;
        stats.max_concurrent_batches =
            std::max<int64_t>(stats.max_concurrent_batches, running_batches);
        stats.peak_reserved_bytes = std::max<int64_t>(stats.peak_reserved_bytes, reserved);
      }
      run_batch(batch, stream, index);
      {
        std::lock_guard<std::mutex> lk(mu);
        running_batches -= 1;
      }
      cv.notify_all();
    }
  }

  void run_batch(const std::vector<int64_t> &ids, hipStream_t stream, int index) {
    const size_t k = ids.size();
    std::vector<const int64_t *> hsrc(k), hdst(k);
    std::vector<int64_t> n(k), off(k + 1, 0);
    {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t i = 0; i < k; ++i) {
        const Request &r = reqs[ids[i]];
        hsrc[i] = r.src;
        hdst[i] = r.dst;
        n[i] = r.n;
        off[i + 1] = off[i] + r.n;
      }
    }
    ringo_status_t rc = RINGO_OK;
    int64_t *dev = nullptr;
    const int64_t total = off[k];
    BatchRec rec;
    rec.stream = index;
    rec.tables = (int32_t)k;
    rec.rows = total;
    rec.first_request = ids.empty() ? 0 : ids[0];
    if (hipEventCreate(&rec.start) != hipSuccess || hipEventCreate(&rec.end) != hipSuccess ||
        hipEventRecord(rec.start, stream) != hipSuccess) {
      (void)hipGetLastError();
      if (rec.start) (void)hipEventDestroy(rec.start);
      if (rec.end) (void)hipEventDestroy(rec.end);
      rec.start = rec.end = nullptr;
    }
    dev = (int64_t *)ringo::workspace_alloc((size_t)std::max<int64_t>(16 * total, 256), stream);
    if (!dev) rc = RINGO_ERR_OUT_OF_MEMORY;
    std::vector<const int64_t *> dsrc(k), ddst(k);
    std::vector<ringo_graph_t> outs(k);
    if (rc == RINGO_OK) {
      for (size_t i = 0; i < k && rc == RINGO_OK; ++i) {
        dsrc[i] = dev + off[i];
        ddst[i] = dev + total + off[i];
        if (n[i] > 0 &&
            (hipMemcpyAsync((void *)dsrc[i], hsrc[i], 8 * n[i], hipMemcpyHostToDevice, stream) !=
                 hipSuccess ||
             hipMemcpyAsync((void *)ddst[i], hdst[i], 8 * n[i], hipMemcpyHostToDevice, stream) !=
                 hipSuccess))
          rc = RINGO_ERR_HIP;
      }
    }
    // every graph in blocks of its own: evicting one frees what it is counted for
    if (rc == RINGO_OK)
      rc = ringo::convert_separate((int32_t)k, dsrc.data(), ddst.data(), n.data(), outs.data(),
                                   stream);
    if (rc == RINGO_OK && rec.end && hipEventRecord(rec.end, stream) != hipSuccess) {
      (void)hipGetLastError();
      rc = RINGO_ERR_HIP;
    }
    if (rc == RINGO_OK && hipStreamSynchronize(stream) != hipSuccess) rc = RINGO_ERR_HIP;
    if (dev) ringo::workspace_free(dev, stream);
    if (rc != RINGO_OK) {
      (void)hipStreamSynchronize(stream);
      (void)hipGetLastError();
    }
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < k; ++i) {
      Request &r = reqs[ids[i]];
      r.finished = now;
      reserved -= r.reserve;
      if (rc == RINGO_OK) {
        r.graph = outs[i];
        r.reserve = (int64_t)ringo::graph_bytes(&outs[i]);
        reserved += r.reserve;
        r.state = RS_READY;
        r.last_use = ++clock;
        stats.completed += 1;
        stats.rows_completed += r.n;
      } else {
        r.reserve = 0;
        r.state = RS_FAILED;
        r.status = rc;
        stats.failed += 1;
      }
    }
    stats.resident_bytes = reserved;
    if (rec.start && rec.end) {
      if (rc == RINGO_OK) {
        if (batch_recs.size() >= MAX_BATCH_RECS) {
          done_recs.push_back(batch_recs.front());
          batch_recs.erase(batch_recs.begin());
        }
        batch_recs.push_back(rec);
      } else {
        done_recs.push_back(rec);
      }
    }
  }
};

extern "C" {

ringo_status_t ringo_server_create(const ringo_server_config_t *cfg, ringo_server_t **out) {
  if (!cfg || !out || cfg->budget_bytes <= 0 || cfg->num_streams < 1 || cfg->num_streams > 16 ||
      cfg->max_batch_tables < 1 || cfg->max_batch_rows < 1)
    return RINGO_ERR_INVALID_ARG;
  *out = nullptr;
  ringo_server *s = new ringo_server();
  s->cfg = *cfg;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return RINGO_ERR_HIP;
  }
  for (int i = 0; i < cfg->num_streams; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return RINGO_ERR_HIP;
    }
    s->streams.push_back(st);
  }
  if (hipEventCreate(&s->t0) != hipSuccess || hipEventRecord(s->t0, s->streams[0]) != hipSuccess ||
      hipEventSynchronize(s->t0) != hipSuccess) {
    (void)hipGetLastError();
    if (s->t0) (void)hipEventDestroy(s->t0);
    s->t0 = nullptr;
  }
  for (int i = 0; i < cfg->num_streams; ++i)
    s->workers.emplace_back([s, i] { s->worker_main(i); });
  *out = s;
  return RINGO_OK;
}

ringo_status_t ringo_server_submit(ringo_server_t *s, const int64_t *src, const int64_t *dst,
                                   int64_t num_rows, int64_t *req_id) {
  if (!s || !req_id || num_rows < 0 || num_rows > RINGO_MAX_ROWS ||
      (num_rows > 0 && (!src || !dst)))
    return RINGO_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    Request r;
    r.id = s->next_id++;
    r.src = src;
    r.dst = dst;
    r.n = num_rows;
    r.submitted = Clock::now();
    *req_id = r.id;
    s->reqs[r.id] = r;
    s->queue.push_back(r.id);
    s->stats.submitted += 1;
  }
  s->cv.notify_all();
  return RINGO_OK;
}

ringo_status_t ringo_server_poll(ringo_server_t *s, int64_t req_id, ringo_graph_t *out,
                                 double *latency_s) {
  if (!s) return RINGO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return RINGO_ERR_INVALID_ARG;
  Request &r = it->second;
  if (latency_s && r.state != RS_QUEUED && r.state != RS_RUNNING)
    *latency_s = std::chrono::duration<double>(r.finished - r.submitted).count();
  switch (r.state) {
    case RS_QUEUED:
    case RS_RUNNING: return RINGO_ERR_PENDING;
    case RS_EVICTED: return RINGO_ERR_EVICTED;
    case RS_RELEASED: return RINGO_ERR_INVALID_ARG;
    case RS_FAILED: return r.status;
    case RS_READY:
      r.last_use = ++s->clock;
      if (out) {
        *out = r.graph;
        out->_alloc = nullptr;  // a view: the server keeps ownership
      }
      return RINGO_OK;
  }
  return RINGO_ERR_INVALID_ARG;
}

ringo_status_t ringo_server_release(ringo_server_t *s, int64_t req_id) {
  if (!s) return RINGO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return RINGO_ERR_INVALID_ARG;
  Request &r = it->second;
  if (r.state == RS_QUEUED || r.state == RS_RUNNING || r.pins > 0) return RINGO_ERR_PENDING;
  if (r.state == RS_READY) {
    ringo_graph_free(&r.graph);
    s->reserved -= r.reserve;
    s->stats.resident_bytes = s->reserved;
  }
  s->reqs.erase(it);
  return RINGO_OK;
}

ringo_status_t ringo_server_pin(ringo_server_t *s, int64_t req_id, ringo_graph_t *out) {
  if (!s) return RINGO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return RINGO_ERR_INVALID_ARG;
  Request &r = it->second;
  switch (r.state) {
    case RS_QUEUED:
    case RS_RUNNING: return RINGO_ERR_PENDING;
    case RS_EVICTED: return RINGO_ERR_EVICTED;
    case RS_RELEASED: return RINGO_ERR_INVALID_ARG;
    case RS_FAILED: return r.status;
    case RS_READY:
      r.pins += 1;
      r.last_use = ++s->clock;
      if (out) {
        *out = r.graph;
        out->_alloc = nullptr;
      }
      return RINGO_OK;
  }
  return RINGO_ERR_INVALID_ARG;
}

ringo_status_t ringo_server_unpin(ringo_server_t *s, int64_t req_id) {
  if (!s) return RINGO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end() || it->second.pins <= 0) return RINGO_ERR_INVALID_ARG;
  it->second.pins -= 1;
  return RINGO_OK;
}

int ringo_server_batches(ringo_server_t *s, ringo_server_batch_t *out, int max_entries) {
  if (!s || max_entries < 0 || (max_entries > 0 && !out)) return -1;
  std::vector<BatchRec> recs;
  hipEvent_t t0 = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    recs = s->batch_recs;
    t0 = s->t0;
  }
  if (!t0) return -1;
  const size_t first = recs.size() > (size_t)max_entries ? recs.size() - (size_t)max_entries : 0;
  int n = 0;
  for (size_t i = first; i < recs.size(); ++i) {
    const BatchRec &r = recs[i];
    float a = 0, b = 0;
    if (hipEventSynchronize(r.end) != hipSuccess || hipEventElapsedTime(&a, t0, r.start) != hipSuccess ||
        hipEventElapsedTime(&b, t0, r.end) != hipSuccess) {
      (void)hipGetLastError();
      return -1;
    }
    ringo_server_batch_t &o = out[n++];
    o.first_request = r.first_request;
    o.rows = r.rows;
    o.stream = r.stream;
    o.tables = r.tables;
    o.start_ms = a;
    o.end_ms = b;
  }
  return n;
}

ringo_status_t ringo_server_stats(ringo_server_t *s, ringo_server_stats_t *out) {
  if (!s || !out) return RINGO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->resident_bytes = s->reserved;
  out->queued = (int64_t)s->queue.size();
  return RINGO_OK;
}

void ringo_server_destroy(ringo_server_t *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto &t : s->workers) t.join();
  // graphs free in order on the streams that built them, so the streams go last
  for (auto &kv : s->reqs)
    if (kv.second.state == RS_READY) ringo_graph_free(&kv.second.graph);
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto *v : {&s->batch_recs, &s->done_recs})
    for (BatchRec &r : *v) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.end);
    }
  if (s->t0) (void)hipEventDestroy(s->t0);
  delete s;
}

}  // extern "C"
