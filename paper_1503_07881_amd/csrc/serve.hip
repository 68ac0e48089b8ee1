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
//     evicting the least recently used resident graph when it does not;
//   * records each request's latency from submission to its graph being
//     resident (the host-to-device copy of its input included).
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
};

// Bytes a request may need while it is converted: its input columns, the
// workspace (two key buffers of 2n keys, slot indices or directory, per-tile
// digit counts of the schedule's tiles and digit width) and an upper bound
// of its outputs (V <= 2n nodes, E <= n edges).
int64_t footprint(int64_t n) {
  const int64_t input = 16 * n;
  ringo_schedule_t sc;
  if (ringo_tune_get(n, &sc) != RINGO_OK) sc.digit_bits = 11, sc.items_per_thread = 8;
  const int64_t tiles = 2 * n / (256 * sc.items_per_thread) + 2;
  const int64_t counts = 4 * tiles * ((int64_t)1 << sc.digit_bits);
  const int64_t workspace = 32 * n + 8 * n + counts + (int64_t)(1 << 20);
  const int64_t outputs = 8 * (2 * n) + 16 * (2 * n + 1) + 8 * n;
  return input + workspace + outputs;
}

int64_t resident_bytes(const ringo_graph_t &g) {
  return 8 * g.num_nodes + 16 * (g.num_nodes + 1) + 8 * g.num_edges;
}

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

  // Evicts least recently used resident graphs until `need` more bytes fit
  // in the budget.  Returns whether they fit.  Caller holds mu.
  bool make_room(int64_t need) {
    while (reserved + need > cfg.budget_bytes) {
      Request *victim = nullptr;
      for (auto &kv : reqs) {
        Request &r = kv.second;
        if (r.state == RS_READY && (!victim || r.last_use < victim->last_use)) victim = &r;
      }
      if (!victim) return false;
      ringo_graph_free(&victim->graph);
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
          if (!make_room(need)) break;  // wait for running batches to finish
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
      run_batch(batch, stream);
      {
        std::lock_guard<std::mutex> lk(mu);
        running_batches -= 1;
      }
      cv.notify_all();
    }
  }

  void run_batch(const std::vector<int64_t> &ids, hipStream_t stream) {
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
    if (hipMallocAsync((void **)&dev, (size_t)std::max<int64_t>(16 * total, 256), stream) !=
        hipSuccess) {
      (void)hipGetLastError();
      rc = RINGO_ERR_OUT_OF_MEMORY;
    }
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
    if (rc == RINGO_OK)
      rc = ringo_table_to_graph_batched((int32_t)k, dsrc.data(), ddst.data(), n.data(), outs.data(),
                                        stream);
    if (rc == RINGO_OK && hipStreamSynchronize(stream) != hipSuccess) rc = RINGO_ERR_HIP;
    if (dev) (void)hipFreeAsync(dev, stream);
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
        r.reserve = resident_bytes(outs[i]);
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
  if (r.state == RS_QUEUED || r.state == RS_RUNNING) return RINGO_ERR_PENDING;
  if (r.state == RS_READY) {
    ringo_graph_free(&r.graph);
    s->reserved -= r.reserve;
    s->stats.resident_bytes = s->reserved;
  }
  s->reqs.erase(it);
  return RINGO_OK;
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
  delete s;
}

}  // extern "C"
