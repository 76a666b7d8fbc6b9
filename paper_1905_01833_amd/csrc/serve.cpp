// serve.cpp -- request loop of the race check: continuous batching of
// trace-check requests over worker threads, admission by device-memory
// footprint, latency statistics (the sim_server_* / sim_submit* / sim_poll /
// sim_wait entry points of include/simcheck.h).
//
// Each worker owns a context (grow-only device buffers), a stream and a
// device buffer for the records of host requests.  A free worker takes
// pending requests in arrival order while they fit its batch limits and
// the device-memory budget, copies the records of host requests into its
// device buffer (requests whose records already live in device memory are
// read where they are), runs one check over all of them on its stream, and
// splits the result by request.  Workers run independently, so the batches
// of different workers overlap on the GPU while new requests queue for the
// next free worker.
//
// Budget accounting: every worker has a charge, the device bytes it may
// hold.  An idle worker is charged what it holds; a worker checking a batch
// is charged max(held, footprint of the batch), and its context may not
// grow beyond that charge (a context whose buffers would exceed it releases
// them and allocates the batch's sizes afresh).  The charges of all workers
// never exceed the budget.
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
void ctx_set_limit(sim_ctx* c, uint64_t bytes);
uint64_t ctx_call_bytes(uint64_t total, uint32_t n_traces, uint32_t n_tiles, uint32_t key_bytes, uint64_t entries,
                        uint64_t staged);
int ctx_check_gather(sim_ctx* c, const sim_record* const* trace_recs, const uint64_t* offsets, uint32_t n_traces,
                     const uint32_t* tpb, hipStream_t s, sim_result** out);
}  // namespace sc

using namespace sc;
using Clock = std::chrono::steady_clock;

namespace {

thread_local std::string t_err;

int fail(int code, const char* msg) {
  t_err = msg;
  return code;
}

// Device bytes a request (or a batch) of n records in n_traces traces and
// n_tiles tiles may need while it is checked: its records if they come from
// host memory (16 B each), and what a context allocates for the call with
// two-word keys (the keys' width is only known on the device).  The usual
// estimate allows one output allocation (up to 64 Ki entries); the worst
// case allows an entry for every second record, in the output and in the
// staging buffer of a tile overflow (a racing location holds at least two
// records).  A batch whose output outgrows the usual estimate fails with
// SIM_ENOMEM at the worker's limit, and its requests are checked again one
// by one, each charged its worst case.
uint64_t footprint(uint64_t n, uint64_t n_traces, uint64_t n_tiles, bool host_records, bool worst) {
  const uint64_t entries = worst ? n / 2 : (n < 65536 ? n : 65536);
  const uint64_t staged = worst ? n / 2 : 0;
  return (host_records ? 16 * n : 0) + ctx_call_bytes(n, (uint32_t)n_traces, (uint32_t)n_tiles, 16, entries, staged);
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
  const sim_record* records = nullptr;  // host memory (device == false) or device memory
  bool device = false;
  std::vector<uint64_t> offsets;  // n_traces + 1
  std::vector<uint32_t> tpb;
  uint64_t n = 0;
  uint32_t n_traces = 0;
  uint64_t n_tiles = 0;
  uint64_t bytes = 0;  // footprint charged for it
  bool worst = false;  // charged its worst case (after failing within the usual estimate)
  bool retry = false;  // failed for memory within the usual estimate: queue it again, charged its worst case
  Clock::time_point t_submit;
  bool done = false;
  int rc = SIM_OK;
  std::string err;
  sim_result* result = nullptr;
};

struct Worker {
  sim_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  void* drec = nullptr;  // the batch's host records, device memory
  size_t drec_cap = 0;
  uint64_t held = 0;     // device bytes the worker holds (under the server lock)
  uint64_t charge = 0;   // device bytes it may hold: held when idle, max(held, batch) when busy
  bool busy = false;
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
  std::condition_variable cv_work;  // workers: requests pending, memory freed, stop
  std::condition_variable cv_done;  // sim_wait: a request finished
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> live;  // submitted and not yet collected
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<Worker> workers;

  // statistics
  uint64_t submitted = 0, completed = 0, failed = 0, batches = 0, records = 0, batched_requests = 0;
  uint64_t peak_charged = 0, requeued = 0;
  std::vector<double> lat_ms;
  bool any = false;
  Clock::time_point t_first, t_last;
};

namespace {

uint64_t charged_except(const sim_server* S, const Worker* w) {
  uint64_t t = 0;
  for (const Worker& v : S->workers)
    if (&v != w) t += v.charge;
  return t;
}

// Whether worker w can take a batch of footprint `bytes` now.
bool fits(const sim_server* S, const Worker* w, uint64_t bytes) {
  return charged_except(S, w) + std::max<uint64_t>(w->held, bytes) <= S->cfg.hbm_budget_bytes;
}

// Check a list of requests as one call on worker w's context, within the
// worker's charge; fills each request's rc / err / result.  A failing batch
// of several requests is checked again request by request, so an error
// stays with its request.
void check_batch(sim_server* S, Worker& w, const std::vector<Request*>& batch, uint64_t charge) {
  uint64_t n_host = 0, nt = 0;
  for (Request* r : batch) {
    n_host += r->device ? 0 : r->n;
    nt += r->n_traces;
  }
  auto fail_all = [&](int code, const char* msg) {
    for (Request* r : batch) {
      r->rc = code;
      r->err = msg;
      r->retry = code == SIM_ENOMEM && !r->worst;
    }
  };
  // the host requests' records go to the worker's record buffer
  const size_t need = (size_t)n_host * sizeof(sim_record);
  auto records_buffer = [&]() -> bool {
    release_records(w);
    if (!need) return true;
    // the worker holds at most its charge at every moment
    if (ctx_device_bytes(w.ctx) + need > charge) ctx_trim(w.ctx);
    if (hipMalloc(&w.drec, need) != hipSuccess) {
      w.drec = nullptr;
      return false;
    }
    w.drec_cap = need;
    return true;
  };
  if (w.drec_cap < need && !records_buffer()) {
    fail_all(SIM_ENOMEM, "device allocation for the batch's records failed");
    return;
  }
  std::vector<uint64_t> off(nt + 1, 0);
  std::vector<uint32_t> tpb(nt ? nt : 1, 1);
  std::vector<const sim_record*> base(nt ? nt : 1, nullptr);
  sim_result* res = nullptr;
  bool upload_failed = false;
  auto attempt = [&]() -> int {
    ctx_set_limit(w.ctx, charge - std::min<uint64_t>(charge, w.drec_cap));
    uint64_t rb = 0, hb = 0, tb = 0;
    for (Request* r : batch) {
      const sim_record* src = r->records;
      if (!r->device) {
        src = (const sim_record*)w.drec + hb;
        if (r->n && hipMemcpyAsync((sim_record*)w.drec + hb, r->records, r->n * sizeof(sim_record),
                                   hipMemcpyHostToDevice, w.stream) != hipSuccess) {
          upload_failed = true;
          return SIM_EDEVICE;
        }
        hb += r->n;
      }
      for (uint32_t i = 0; i < r->n_traces; i++) {
        off[tb + i + 1] = rb + r->offsets[i + 1];
        tpb[tb + i] = r->tpb[i];
        base[tb + i] = src + r->offsets[i];
      }
      rb += r->n;
      tb += r->n_traces;
    }
    return ctx_check_gather(w.ctx, base.data(), off.data(), (uint32_t)nt, tpb.data(), w.stream, &res);
  };
  int rc = attempt();
  if (rc == SIM_ENOMEM && w.drec_cap > need) {
    // a record buffer larger than this batch needs left the context too
    // little of the charge: shrink it and try again
    if (!records_buffer()) {
      fail_all(SIM_ENOMEM, "device allocation for the batch's records failed");
      return;
    }
    rc = attempt();
  }
  if (upload_failed) {
    fail_all(SIM_EDEVICE, "record upload failed");
    return;
  }
  if (rc != SIM_OK) {
    if (batch.size() == 1) {
      batch[0]->rc = rc;
      batch[0]->err = sim_last_error(w.ctx);
      batch[0]->retry = rc == SIM_ENOMEM && !batch[0]->worst;
      return;
    }
    for (Request* r : batch) check_batch(S, w, std::vector<Request*>{r}, charge);
    return;
  }
  // split: entries are ordered by trace, so each request's entries are one run
  uint64_t k = 0, tb = 0;
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
    // Wake for: stop with nothing pending; a first request that fits; or a
    // first request that fits no idle worker while this one holds memory
    // (it then releases its buffers so that the request can run).
    bool release = false;
    S->cv_work.wait(lk, [&] {
      release = false;
      if (S->pending.empty()) return S->stop;
      const uint64_t f = S->pending.front()->bytes;
      if (fits(S, w, f)) return true;
      if (w->held == 0) return false;
      for (const Worker& v : S->workers)
        if (&v != w && !v.busy && fits(S, &v, f)) return false;
      release = true;
      return true;
    });
    if (S->pending.empty()) return;  // stopping, nothing left
    if (release) {
      w->busy = true;  // its charge stays until the buffers are gone
      lk.unlock();
      ctx_trim(w->ctx);
      release_records(*w);
      lk.lock();
      w->busy = false;
      w->held = w->charge = 0;
      S->cv_work.notify_all();
      continue;
    }
    // the batch: pending requests in arrival order while they fit
    std::vector<Request*> batch;
    uint64_t recs = 0, traces = 0, tiles = 0, host = 0;
    bool worst = false;
    auto batch_bytes = [&](uint64_t n, uint64_t t, uint64_t k, uint64_t h, bool wc) {
      return footprint(n, t, k, false, wc) + 16 * h;
    };
    while (!S->pending.empty()) {
      Request* r = S->pending.front();
      if (!batch.empty()) {
        // a request charged its worst case runs alone
        if (r->worst || worst || batch.size() >= S->cfg.max_batch_requests ||
            recs + r->n > S->cfg.max_batch_records ||
            !fits(S, w, batch_bytes(recs + r->n, traces + r->n_traces, tiles + r->n_tiles,
                                    host + (r->device ? 0 : r->n), false)))
          break;
      }
      batch.push_back(r);
      recs += r->n;
      traces += r->n_traces;
      tiles += r->n_tiles;
      host += r->device ? 0 : r->n;
      worst = worst || r->worst;
      S->pending.pop_front();
    }
    const uint64_t charge = std::max<uint64_t>(
        w->held, batch.size() == 1 ? batch[0]->bytes : batch_bytes(recs, traces, tiles, host, false));
    w->busy = true;
    w->charge = charge;
    S->peak_charged = std::max(S->peak_charged, charged_except(S, nullptr));
    lk.unlock();

    check_batch(S, *w, batch, charge);
    // keep an idle worker's device buffers within its share of the budget
    if (worker_bytes(*w) > share) {
      ctx_trim(w->ctx);
      release_records(*w);
    }
    const uint64_t held = worker_bytes(*w);

    lk.lock();
    w->busy = false;
    w->held = w->charge = held;
    S->batches++;
    const Clock::time_point now = Clock::now();
    for (auto it = batch.rbegin(); it != batch.rend(); ++it) {  // retries go back to the front, in order
      Request* r = *it;
      if (r->retry) {
        r->retry = false;
        r->worst = true;
        r->bytes = footprint(r->n, r->n_traces, r->n_tiles, !r->device, true);
        if (r->bytes <= budget) {
          r->rc = SIM_OK;
          r->err.clear();
          S->pending.push_front(r);
          S->requeued++;
          continue;
        }
        r->rc = SIM_ENOMEM;
        r->err = "the request's worst-case device footprint exceeds the server's budget";
      }
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
  }
}

int take(sim_server* S, std::unordered_map<uint64_t, Request*>::iterator it, sim_result** out) {
  Request* r = it->second;
  S->live.erase(it);
  S->cv_done.notify_all();  // another waiter on this ticket sees it gone
  const int rc = r->rc;
  if (rc == SIM_OK) *out = r->result;
  else t_err = r->err;
  delete r;
  return rc;
}

int submit(sim_server* S, const sim_record* records, bool device, const uint64_t* offsets, uint32_t n_traces,
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
  r->device = device;
  r->offsets.assign(offsets ? offsets : nullptr, offsets ? offsets + n_traces + 1 : nullptr);
  if (r->offsets.empty()) r->offsets.push_back(0);
  r->tpb.assign(threads_per_block ? threads_per_block : nullptr,
                threads_per_block ? threads_per_block + n_traces : nullptr);
  r->n = n;
  r->n_traces = n_traces;
  r->n_tiles = tiles;
  r->bytes = footprint(n, n_traces, tiles, !device, false);
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
  S->cv_work.notify_all();
  return SIM_OK;
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
    // what a worker then holds: its context's buffers for a call of rsv
    // records in max_batch_requests traces (one-word keys, first output
    // allocation) and a record buffer of rsv records
    const uint64_t tiles = (rsv + TILE - 1) / TILE + S->cfg.max_batch_requests;
    if (rsv >= (1ull << 32) ||
        16 * rsv + ctx_call_bytes(rsv, S->cfg.max_batch_requests, (uint32_t)tiles, 8, rsv < 65536 ? rsv : 65536, 0) >
            S->cfg.hbm_budget_bytes / S->cfg.slots) {
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
    w.held = w.charge = worker_bytes(w);
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
  return submit(S, records, false, offsets, n_traces, threads_per_block, ticket);
}

int sim_submit_device(sim_server* S, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                      const uint32_t* threads_per_block, uint64_t* ticket) {
  return submit(S, d_records, true, offsets, n_traces, threads_per_block, ticket);
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
  if (S->live.find(ticket) == S->live.end()) return fail(SIM_EINVAL, "unknown ticket");
  // the request is looked up again at every wake-up: another thread may
  // collect it (sim_poll / sim_wait on the same ticket) while this one waits
  auto ready = [&] {
    auto it = S->live.find(ticket);
    return it == S->live.end() || it->second->done;
  };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return fail(SIM_EAGAIN, "timed out");
  }
  auto it = S->live.find(ticket);
  if (it == S->live.end()) return fail(SIM_EINVAL, "ticket collected by another caller");
  return take(S, it, out);
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
  st.peak_inflight_bytes = S->peak_charged;
  uint64_t held = 0;
  for (const Worker& w : S->workers) held += w.held;
  st.device_bytes = held;
  st.requeued = S->requeued;
  *out = st;
  if (reset) {
    S->submitted = S->completed = S->failed = S->batches = S->records = S->batched_requests = S->requeued = 0;
    S->peak_charged = charged_except(S, nullptr);
    S->lat_ms.clear();
    S->any = false;
  }
  return SIM_OK;
}

const char* sim_server_last_error(void) { return t_err.c_str(); }

}  // extern "C"
