// serve.cpp -- request loop of the race check: continuous batching of
// trace-check requests over worker threads, admission by device-memory
// footprint, latency statistics (the sim_server_* / sim_submit / sim_poll /
// sim_wait entry points of include/simcheck.h).
//
// Each worker owns a context (grow-only device buffers), a stream and a
// device buffer for records.  A free worker takes pending requests in
// arrival order while they fit its batch limits and the unused part of the
// budget, copies their records straight from the callers' memory into its
// device buffer as one trace list, runs one check over all of them on its
// stream, and splits the result by request.  Workers run
// independently, so the batches of different workers overlap on the GPU
// while new requests queue for the next free worker.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/simcheck.h"
#include "launch.h"

namespace sc {
size_t ctx_device_bytes(const sim_ctx* c);
void ctx_trim(sim_ctx* c);
}  // namespace sc

using namespace sc;
using Clock = std::chrono::steady_clock;

namespace {

thread_local std::string t_err;

int fail(int code, const char* msg) {
  t_err = msg;
  return code;
}

// Device bytes a request needs while it is checked: records (16 B), two key
// buffers (8 B each), the output's first allocation (up to 64 Ki entries of
// 64 B), per-tile tables (histogram row 1 KiB, group rows up to 3 KiB,
// summaries, statistics, crossing entries: under 4.5 KiB) and per-trace
// tables, plus the 1/8 growth headroom of the buffers.
uint64_t footprint(uint64_t n, uint64_t n_traces, uint64_t n_tiles) {
  const uint64_t out0 = (n < 65536 ? n : 65536) * 64;
  const uint64_t raw = 32 * n + out0 + 4608 * n_tiles + 128 * n_traces + 4096;
  return raw + raw / 8;
}

sim_result* new_result(uint64_t n_races, uint32_t n_traces) {
  sim_result* r = (sim_result*)calloc(1, sizeof(sim_result));
  if (!r) return nullptr;
  r->n_races = n_races;
  r->n_traces = n_traces;
  r->races = (sim_race*)malloc(n_races ? n_races * sizeof(sim_race) : 1);
  r->traces = (sim_trace_summary*)calloc(n_traces ? n_traces : 1, sizeof(sim_trace_summary));
  if (!r->races || !r->traces) {
    sim_result_free(r);
    return nullptr;
  }
  return r;
}

struct Request {
  uint64_t ticket = 0;
  const sim_record* records = nullptr;
  std::vector<uint64_t> offsets;  // n_traces + 1
  std::vector<uint32_t> tpb;
  uint64_t n = 0;
  uint32_t n_traces = 0;
  uint64_t bytes = 0;  // footprint
  Clock::time_point t_submit;
  bool done = false;
  int rc = SIM_OK;
  std::string err;
  sim_result* result = nullptr;
};

struct Worker {
  sim_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  void* drec = nullptr;  // the batch's records, device memory
  size_t drec_cap = 0;
  size_t held = 0;  // device bytes of the worker, updated under the server lock
  std::thread th;
};

size_t worker_bytes(const Worker& w) { return ctx_device_bytes(w.ctx) + w.drec_cap; }

void release_records(Worker& w) {
  if (w.drec) (void)hipFree(w.drec);
  w.drec = nullptr;
  w.drec_cap = 0;
}

}  // namespace

struct sim_server {
  int device = 0;
  sim_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work;  // workers: requests pending, budget freed, stop
  std::condition_variable cv_done;  // sim_wait: a request finished
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> live;  // submitted and not yet collected
  uint64_t next_ticket = 1;
  uint64_t inflight = 0;
  bool stop = false;
  std::vector<Worker> workers;

  // statistics
  uint64_t submitted = 0, completed = 0, failed = 0, batches = 0, records = 0, batched_requests = 0;
  uint64_t peak_inflight = 0;
  std::vector<double> lat_ms;
  bool any = false;
  Clock::time_point t_first, t_last;
};

namespace {

// Check a list of requests as one call on worker w's context; fills each
// request's rc / err / result.  A failing batch of several requests is
// checked again request by request, so an error stays with its request.
void check_batch(sim_server* S, Worker& w, const std::vector<Request*>& batch) {
  uint64_t n = 0, nt = 0;
  for (Request* r : batch) {
    n += r->n;
    nt += r->n_traces;
  }
  const size_t need = (size_t)(n ? n : 1) * sizeof(sim_record);
  if (w.drec_cap < need) {
    release_records(w);
    if (hipMalloc(&w.drec, need) != hipSuccess) {
      w.drec = nullptr;
      for (Request* r : batch) {
        r->rc = SIM_ENOMEM;
        r->err = "device allocation for the batch's records failed";
      }
      return;
    }
    w.drec_cap = need;
  }
  std::vector<uint64_t> off(nt + 1, 0);
  std::vector<uint32_t> tpb(nt ? nt : 1, 1);
  uint64_t rb = 0, tb = 0;
  for (Request* r : batch) {
    if (r->n &&
        hipMemcpyAsync((sim_record*)w.drec + rb, r->records, r->n * sizeof(sim_record), hipMemcpyHostToDevice,
                       w.stream) != hipSuccess) {
      for (Request* q : batch) {
        q->rc = SIM_EDEVICE;
        q->err = "record upload failed";
      }
      return;
    }
    for (uint32_t i = 0; i < r->n_traces; i++) {
      off[tb + i + 1] = rb + r->offsets[i + 1];
      tpb[tb + i] = r->tpb[i];
    }
    rb += r->n;
    tb += r->n_traces;
  }
  sim_result* res = nullptr;
  const int rc = sim_check_traces_device(w.ctx, (const sim_record*)w.drec, off.data(), (uint32_t)nt, tpb.data(),
                                         w.stream, &res);
  if (rc != SIM_OK) {
    if (batch.size() == 1) {
      batch[0]->rc = rc;
      batch[0]->err = sim_last_error(w.ctx);
      return;
    }
    for (Request* r : batch) check_batch(S, w, std::vector<Request*>{r});
    return;
  }
  // split: entries are ordered by trace, so each request's entries are one run
  uint64_t k = 0;
  tb = 0;
  for (Request* r : batch) {
    uint64_t k1 = k;
    while (k1 < res->n_races && res->races[k1].trace < tb + r->n_traces) k1++;
    sim_result* mine = new_result(k1 - k, r->n_traces);
    if (!mine) {
      r->rc = SIM_ENOMEM;
      r->err = "host allocation failed";
    } else {
      if (k1 > k) std::memcpy(mine->races, res->races + k, (k1 - k) * sizeof(sim_race));
      for (uint64_t q = 0; q < k1 - k; q++) mine->races[q].trace -= (uint32_t)tb;
      if (r->n_traces) std::memcpy(mine->traces, res->traces + tb, r->n_traces * sizeof(sim_trace_summary));
      r->rc = SIM_OK;
      r->result = mine;
    }
    k = k1;
    tb += r->n_traces;
  }
  sim_result_free(res);
}

void worker_loop(sim_server* S, Worker* w) {
  (void)hipSetDevice(S->device);
  const uint64_t budget = S->cfg.hbm_budget_bytes;
  const uint64_t share = budget / S->cfg.slots;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_work.wait(lk, [&] {
      if (S->pending.empty()) return S->stop;
      return S->pending.front()->bytes <= budget - S->inflight;
    });
    if (S->pending.empty()) return;  // stopping, nothing left
    // the batch: pending requests in arrival order while they fit
    std::vector<Request*> batch;
    uint64_t bytes = 0, recs = 0;
    while (!S->pending.empty()) {
      Request* r = S->pending.front();
      const bool first = batch.empty();
      if (!first && (batch.size() >= S->cfg.max_batch_requests || recs + r->n > S->cfg.max_batch_records ||
                     bytes + r->bytes > budget - S->inflight))
        break;
      batch.push_back(r);
      bytes += r->bytes;
      recs += r->n;
      S->pending.pop_front();
    }
    S->inflight += bytes;
    S->peak_inflight = std::max(S->peak_inflight, S->inflight);
    lk.unlock();

    check_batch(S, *w, batch);

    lk.lock();
    S->inflight -= bytes;
    S->batches++;
    const Clock::time_point now = Clock::now();
    for (Request* r : batch) {
      r->done = true;
      if (r->rc == SIM_OK) {
        S->completed++;
        S->batched_requests++;
        S->records += r->n;
        S->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        S->t_last = now;
      } else {
        S->failed++;
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
    lk.unlock();
    // keep an idle worker's device buffers within its share of the budget
    if (worker_bytes(*w) > share) {
      ctx_trim(w->ctx);
      release_records(*w);
    }
    const size_t held = worker_bytes(*w);
    lk.lock();
    w->held = held;
  }
}

int take(sim_server* S, std::unordered_map<uint64_t, Request*>::iterator it, sim_result** out) {
  Request* r = it->second;
  S->live.erase(it);
  const int rc = r->rc;
  if (rc == SIM_OK) *out = r->result;
  else t_err = r->err;
  delete r;
  return rc;
}

}  // namespace

extern "C" {

int sim_server_create(sim_server** out, int hip_device, const sim_server_config* cfg) {
  if (!out) return fail(SIM_EINVAL, "out is NULL");
  *out = nullptr;
  sim_server* S = new (std::nothrow) sim_server();
  if (!S) return fail(SIM_ENOMEM, "host allocation failed");
  S->device = hip_device;
  if (cfg) S->cfg = *cfg;
  if (!S->cfg.hbm_budget_bytes) S->cfg.hbm_budget_bytes = 8ull << 30;
  if (!S->cfg.max_batch_records) S->cfg.max_batch_records = 1ull << 26;
  if (!S->cfg.slots) S->cfg.slots = 2;
  if (!S->cfg.max_batch_requests) S->cfg.max_batch_requests = 1024;
  if (!S->cfg.max_pending) S->cfg.max_pending = 65536;
  if (S->cfg.slots > 16) {
    delete S;
    return fail(SIM_EINVAL, "at most 16 slots");
  }
  const uint64_t rsv = S->cfg.reserve_records;
  if (rsv) {
    const uint64_t tiles = (rsv + TILE - 1) / TILE + S->cfg.max_batch_requests;
    if (rsv >= (1ull << 32) ||
        footprint(rsv, S->cfg.max_batch_requests, tiles) > S->cfg.hbm_budget_bytes / S->cfg.slots) {
      delete S;
      return fail(SIM_EINVAL, "reserve_records does not fit the budget share of a worker");
    }
  }
  S->workers.resize(S->cfg.slots);
  for (Worker& w : S->workers) {
    const sim_config wc{rsv, 0u, S->cfg.max_batch_requests};
    const int rc = sim_create(&w.ctx, hip_device, &wc);
    if (rc != SIM_OK) {
      sim_server_destroy(S);
      return fail(rc, "sim_create failed (needs a gfx950 device, or the reservation did not fit)");
    }
    (void)hipSetDevice(hip_device);
    if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) {
      w.stream = nullptr;
      sim_server_destroy(S);
      return fail(SIM_EDEVICE, "stream creation failed");
    }
    if (rsv) {
      if (hipMalloc(&w.drec, rsv * sizeof(sim_record)) != hipSuccess) {
        w.drec = nullptr;
        sim_server_destroy(S);
        return fail(SIM_ENOMEM, "device allocation for records failed");
      }
      w.drec_cap = rsv * sizeof(sim_record);
    }
    w.held = worker_bytes(w);
  }
  for (Worker& w : S->workers) w.th = std::thread(worker_loop, S, &w);
  *out = S;
  return SIM_OK;
}

void sim_server_destroy(sim_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (Worker& w : S->workers)
    if (w.th.joinable()) w.th.join();
  for (auto& kv : S->live) {
    sim_result_free(kv.second->result);
    delete kv.second;
  }
  for (Worker& w : S->workers) {
    sim_destroy(w.ctx);
    if (w.drec || w.stream) (void)hipSetDevice(S->device);
    release_records(w);
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  delete S;
}

int sim_submit(sim_server* S, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
               const uint32_t* threads_per_block, uint64_t* ticket) {
  if (!S || !ticket) return fail(SIM_EINVAL, "server or ticket is NULL");
  if (n_traces && (!offsets || !threads_per_block)) return fail(SIM_EINVAL, "offsets or threads_per_block is NULL");
  if (n_traces && offsets[0] != 0) return fail(SIM_EINVAL, "offsets[0] must be 0");
  uint64_t tiles = 0;
  for (uint32_t i = 0; i < n_traces; i++) {
    if (offsets[i + 1] < offsets[i]) return fail(SIM_EINVAL, "offsets decrease");
    if (threads_per_block[i] == 0) return fail(SIM_EINVAL, "threads_per_block is 0");
    tiles += (offsets[i + 1] - offsets[i] + TILE - 1) / TILE;
  }
  const uint64_t n = n_traces ? offsets[n_traces] : 0;
  if (n >= (1ull << 32)) return fail(SIM_EINVAL, "a request holds at most 2^32 - 1 records");
  if (n && !records) return fail(SIM_EINVAL, "records is NULL");
  Request* r = new (std::nothrow) Request();
  if (!r) return fail(SIM_ENOMEM, "host allocation failed");
  r->records = records;
  r->offsets.assign(offsets ? offsets : nullptr, offsets ? offsets + n_traces + 1 : nullptr);
  if (r->offsets.empty()) r->offsets.push_back(0);
  r->tpb.assign(threads_per_block ? threads_per_block : nullptr,
                threads_per_block ? threads_per_block + n_traces : nullptr);
  r->n = n;
  r->n_traces = n_traces;
  r->bytes = footprint(n, n_traces, tiles);
  if (r->bytes > S->cfg.hbm_budget_bytes) {
    delete r;
    return fail(SIM_ENOMEM, "request footprint exceeds the server's HBM budget");
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->pending.size() >= S->cfg.max_pending) {
    delete r;
    return fail(SIM_EAGAIN, "pending queue full");
  }
  r->ticket = S->next_ticket++;
  r->t_submit = Clock::now();
  if (!S->any) {
    S->any = true;
    S->t_first = r->t_submit;
  }
  S->submitted++;
  S->pending.push_back(r);
  S->live[r->ticket] = r;
  *ticket = r->ticket;
  S->cv_work.notify_one();
  return SIM_OK;
}

int sim_poll(sim_server* S, uint64_t ticket, sim_result** out) {
  if (!S || !out) return fail(SIM_EINVAL, "server or out is NULL");
  *out = nullptr;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->live.find(ticket);
  if (it == S->live.end()) return fail(SIM_EINVAL, "unknown ticket");
  if (!it->second->done) return fail(SIM_EAGAIN, "pending");
  return take(S, it, out);
}

int sim_wait(sim_server* S, uint64_t ticket, int64_t timeout_ms, sim_result** out) {
  if (!S || !out) return fail(SIM_EINVAL, "server or out is NULL");
  *out = nullptr;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->live.find(ticket);
  if (it == S->live.end()) return fail(SIM_EINVAL, "unknown ticket");
  Request* r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return fail(SIM_EAGAIN, "timed out");
  }
  return take(S, S->live.find(ticket), out);
}

int sim_server_get_stats(sim_server* S, sim_server_stats* out, int reset) {
  if (!S || !out) return fail(SIM_EINVAL, "server or out is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  sim_server_stats st{};
  st.submitted = S->submitted;
  st.completed = S->completed;
  st.failed = S->failed;
  st.batches = S->batches;
  st.records = S->records;
  std::vector<double> v = S->lat_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      size_t i = (size_t)(p * (double)v.size() + 0.999999);  // nearest rank
      i = i ? i - 1 : 0;
      return v[std::min(i, v.size() - 1)];
    };
    st.p50_ms = pct(0.50);
    st.p99_ms = pct(0.99);
    st.max_ms = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    st.mean_ms = sum / (double)v.size();
    const double span = std::chrono::duration<double>(S->t_last - S->t_first).count();
    st.records_per_s = span > 0 ? (double)S->records / span : 0.0;
  }
  st.mean_batch_requests = S->batches ? (double)S->batched_requests / (double)S->batches : 0.0;
  st.peak_inflight_bytes = S->peak_inflight;
  size_t held = 0;
  for (const Worker& w : S->workers) held += w.held;
  st.device_bytes = held;
  *out = st;
  if (reset) {
    S->submitted = S->completed = S->failed = S->batches = S->records = S->batched_requests = 0;
    S->peak_inflight = S->inflight;
    S->lat_ms.clear();
    S->any = false;
  }
  return SIM_OK;
}

const char* sim_server_last_error(void) { return t_err.c_str(); }

}  // extern "C"
