// api.cpp -- host runtime behind the C ABI of include/simcheck.h.
//
// A context owns grow-only device buffers sized by the largest call seen so
// far, a default-priority stream for the host-record entry point, pinned
// host staging for the small per-call tables and results.  A check is one
// ordered sequence of kernel launches on one stream
// and one synchronisation; there is no CPU fallback.  Rare conditions cost
// a second round on the device: a trace needing more radix passes than the
// previous call did, a tile with more racing locations than its staging
// slice holds, or more racing locations than the output buffer holds.
//
// The no-allocation entry point runs the same sequence with every device
// buffer carved out of a fixed scratch array (kernels.hip) and the tables
// in pinned host memory the context allocated at creation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/simcheck.h"
#include "launch.h"

using namespace sc;

static_assert(sizeof(sim_record) == 16, "sim_record is 16 bytes");
static_assert(sizeof(sim_race) == 64, "sim_race is 64 bytes");
static_assert(sizeof(RaceOut) == sizeof(sim_race), "device entry mirrors sim_race");
static_assert(sizeof(sim_barrier) == 24, "sim_barrier is 24 bytes");
static_assert(sizeof(sim_divergence) == sizeof(DivOut), "device divergence entry mirrors sim_divergence");
static_assert(sizeof(sim_fitness) == sizeof(FitOut), "device fitness row mirrors sim_fitness");

namespace {

constexpr int N_STAGE = ST_COUNT;
const char* const kStageNames[N_STAGE] = {"init",      "stats",      "layout",     "keygen",  "upsweep",
                                          "sort_pass", "scan_tiles", "scan_cross", "scan_out", "sort_small"};
constexpr int MAX_EV = 96;

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct sim_ctx {
  int device = 0;
  uint32_t n_cu = 256;           // compute units of the device
  hipStream_t stream = nullptr;  // used by sim_check_traces
  uint32_t flags = 0;
  uint32_t pass_guess = 0;  // radix passes the previous call needed
  bool wide_guess = false;  // the previous call had a trace needing two-word keys
  uint32_t fit_pass_guess = 0;  // the same for the fitness count, whose keys are shorter
  bool fit_wide_guess = false;
  uint32_t warp_pass_guess = 0;  // ... and for the warp-aware check, whose keys are longer
  bool warp_wide_guess = false;
  // per kind as above: the key bits the previous call sorted (0: none yet),
  // and the digit width its passes (the pass guess) were counted in
  uint32_t bits_guess = 0, fit_bits_guess = 0, warp_bits_guess = 0;
  uint32_t db_guess = RADIX_BITS, fit_db_guess = RADIX_BITS, warp_db_guess = RADIX_BITS;
  uint64_t alloc_gen = 0;   // bumped whenever a device buffer is reallocated
  uint64_t meta_gen = 0;    // bumped whenever a call's tables are uploaded
  uint64_t host_gen = 0;    // bumped whenever the host copy's trace and group tables are rebuilt
  // the trace and group tables in the host copy, and what they were built
  // from: a call of the same offsets, threads per block, group bias and
  // LDS-sort limit reuses them while host_gen is unchanged
  struct {
    std::vector<uint64_t> offsets;
    std::vector<uint32_t> tpb;
    int32_t bias = 0;
    uint32_t small_max_tiles = 0;
    uint64_t host_gen = 0;
    bool valid = false;
    uint32_t n_hgroups = 0, max_group_tiles = 1, max_trace_groups = 1, n_small1 = 0, n_small4 = 0;
  } plan;

  // one captured launch sequence, replayed while calls keep the same shape
  struct {
    hipGraphExec_t exec = nullptr;
    const void* records = nullptr;
    hipStream_t stream = nullptr;
    uint64_t total = 0, gen = 0;
    std::vector<uint64_t> offsets;  // the captured call's tables (compared in full)
    std::vector<uint32_t> tpb;
    uint32_t n_traces = 0, n_tiles = 0, guess = 0;
    uint64_t tuning_gen = 0;
    uint64_t meta_gen = 0;  // the table upload the captured launches read
    bool wide = false;
    uint32_t db = 0;  // digit width of the captured passes
  } graph;

  // launch shapes per size class (set by hand or by sim_autotune)
  sim_tuning tuning[SIM_SIZE_CLASSES] = {};
  bool tuned[SIM_SIZE_CLASSES] = {};
  uint64_t tuning_gen = 0;
  const sim_tuning* force = nullptr;  // sim_autotune's candidate
  std::string err;

  DevBuf records, keys0, keys1, meta, stats_part, layout, thist, tcnt, gtot, gbase, agg, tout, cross, cross_flag,
      group_sum, stage, stage_ref, ctrl, out, bar, bar_base;
  // the barrier-divergence check: arrival counts of host calls, chunk table,
  // per-block results, per-chunk counts and offsets, divergent blocks
  DevBuf div_in, div_chunks, div_blocks, div_cnt, div_off, div_out;
  DevBuf fit_out;  // the fitness count's rows
  // the warp-aware check: side words of host calls, removed pairs per entry,
  // refined entries, their number
  DevBuf side, warp_rm, warp_out, warp_n;
  void* h_div = nullptr;  // pinned: the chunk table, then the divergent-block count
  size_t h_div_cap = 0;
  uint64_t dev_limit = 0;  // device bytes the buffers may hold (0: no limit; set by a server's worker)
  void* h_meta = nullptr;  // pinned: the call's tables (the layout of meta), then room for the
                           // per-tile words of a staging overflow (tile counts down, references up)
  size_t h_meta_cap = 0;
  Ctrl* h_ctrl = nullptr;  // pinned
  void* scratch = nullptr; // this device's no-allocation scratch (nullptr: its lookup failed)
  hipError_t scratch_err = hipSuccess;

  hipEvent_t ev[MAX_EV] = {};
  sim_stage_time times[N_STAGE] = {};
};

namespace {

// Every device buffer of a context.
std::vector<DevBuf*> all_bufs(sim_ctx* c) {
  return {&c->records, &c->keys0, &c->keys1, &c->meta, &c->stats_part, &c->layout, &c->thist, &c->tcnt, &c->gtot,
          &c->gbase,   &c->agg,   &c->tout,  &c->cross, &c->cross_flag, &c->group_sum, &c->stage,
          &c->stage_ref, &c->ctrl, &c->out, &c->bar, &c->bar_base, &c->div_in, &c->div_chunks, &c->div_blocks,
          &c->div_cnt, &c->div_off, &c->div_out, &c->fit_out, &c->side, &c->warp_rm, &c->warp_out, &c->warp_n};
}

int fail(sim_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

int hip_fail(sim_ctx* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? SIM_ENOMEM : SIM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Make the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Grow a device buffer to at least `bytes` (contents are not kept); *gen is
// bumped on reallocation (captured launch sequences hold buffer addresses).
hipError_t ensure(DevBuf& b, size_t bytes, bool zero = false, uint64_t* gen = nullptr) {
  if (bytes == 0) bytes = 64;
  if (b.cap >= bytes) return hipSuccess;
  if (gen) ++*gen;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 8;  // headroom against small growth steps
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) return e;
  b.cap = want;
  if (zero) {
    e = hipMemset(b.p, 0, want);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void release(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

int validate(sim_ctx* c, const uint64_t* offsets, uint32_t n_traces, const uint32_t* tpb, sim_result** out,
             uint64_t* total, uint32_t* n_tiles) {
  if (!out) return fail(c, SIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_traces && (!offsets || !tpb)) return fail(c, SIM_EINVAL, "offsets or threads_per_block is NULL");
  if (n_traces && offsets[0] != 0) return fail(c, SIM_EINVAL, "offsets[0] must be 0");
  uint64_t tiles = 0;
  for (uint32_t i = 0; i < n_traces; i++) {
    if (offsets[i + 1] < offsets[i]) return fail(c, SIM_EINVAL, "offsets decrease at trace %u", i);
    if (tpb[i] == 0) return fail(c, SIM_EINVAL, "threads_per_block[%u] is 0", i);
    tiles += (offsets[i + 1] - offsets[i] + TILE - 1) / TILE;
  }
  *total = n_traces ? offsets[n_traces] : 0;
  if (*total >= (1ull << 32)) return fail(c, SIM_EINVAL, "a call holds at most 2^32 - 1 records");
  *n_tiles = (uint32_t)tiles;
  return SIM_OK;
}

// Pinned blocks for large entry lists: their download is one DMA, with no
// host copy (3.35 MB: 0.067 ms, against 0.19 ms into pageable memory).
// sim_result_free hands a block back for reuse; blocks are never released
// (so freeing a result needs no HIP call, whenever it happens), and at most
// POOL_BLOCKS exist: beyond that, entry lists are plain host memory.
struct PinnedPool {
  std::mutex mu;
  std::unordered_set<void*> all;           // every block
  std::vector<std::pair<void*, size_t>> idle;  // blocks not in a result, with their sizes
  std::vector<std::pair<void*, size_t>> busy;  // blocks in a result
};
constexpr size_t POOL_MIN_BYTES = 1u << 20;
constexpr size_t POOL_BLOCKS = 8;

PinnedPool& pinned_pool() {
  static PinnedPool* p = new PinnedPool;  // never destroyed: results may be freed at any time
  return *p;
}

void* pool_take(size_t bytes) {
  if (bytes < POOL_MIN_BYTES) return nullptr;
  PinnedPool& P = pinned_pool();
  std::lock_guard<std::mutex> lk(P.mu);
  size_t best = P.idle.size();
  for (size_t i = 0; i < P.idle.size(); i++)  // the smallest idle block that fits
    if (P.idle[i].second >= bytes && (best == P.idle.size() || P.idle[i].second < P.idle[best].second)) best = i;
  if (best < P.idle.size()) {
    const auto blk = P.idle[best];
    P.idle.erase(P.idle.begin() + (ptrdiff_t)best);
    P.busy.push_back(blk);
    return blk.first;
  }
  if (P.all.size() >= POOL_BLOCKS) return nullptr;
  const size_t cap = bytes + bytes / 8;  // headroom for a slightly larger next result
  void* q = nullptr;
  if (hipHostMalloc(&q, cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  P.all.insert(q);
  P.busy.push_back({q, cap});
  return q;
}

bool pool_give_back(void* q) {
  PinnedPool& P = pinned_pool();
  std::lock_guard<std::mutex> lk(P.mu);
  if (!P.all.count(q)) return false;
  for (size_t i = 0; i < P.busy.size(); i++)
    if (P.busy[i].first == q) {
      P.idle.push_back(P.busy[i]);
      P.busy.erase(P.busy.begin() + (ptrdiff_t)i);
      break;
    }
  return true;
}

sim_result* alloc_result(uint64_t n_races, uint32_t n_traces) {
  sim_result* r = (sim_result*)calloc(1, sizeof(sim_result));
  if (!r) return nullptr;
  r->n_races = n_races;
  r->n_traces = n_traces;
  r->races = (sim_race*)pool_take(n_races * sizeof(sim_race));
  if (!r->races) r->races = (sim_race*)malloc(n_races ? n_races * sizeof(sim_race) : 1);
  r->traces = (sim_trace_summary*)calloc(n_traces ? n_traces : 1, sizeof(sim_trace_summary));
  if (!r->races || !r->traces) {
    if (r->races && !pool_give_back(r->races)) free(r->races);
    free(r->traces);
    free(r);
    return nullptr;
  }
  return r;
}

uint32_t size_class(uint64_t total) {
  uint32_t k = 0;
  while (k < 64 && (total >> k) != 0) k++;
  return k < SIM_SIZE_CLASSES ? k : SIM_SIZE_CLASSES - 1;
}

// Launch shape of a call of `total` records: the forced candidate while
// autotuning, else the shape of its size class, else of the nearest tuned
// class, else one workgroup per tile and no group-size bias.
sim_tuning pick_tuning(const sim_ctx* c, uint64_t total) {
  if (c->force) return *c->force;
  const int k = (int)size_class(total);
  int best = -1;
  for (int d = 0; d < SIM_SIZE_CLASSES && best < 0; d++) {
    if (k - d >= 0 && c->tuned[k - d]) best = k - d;
    else if (k + d < SIM_SIZE_CLASSES && c->tuned[k + d]) best = k + d;
  }
  return best >= 0 ? c->tuning[best] : sim_tuning{0, 0, 0, 0, 0, 0, 0.0};
}

// Threads of a scatter workgroup: the shape's, else by call size -- 512 of
// 8 keys up to 16384 tiles (measured faster on single traces of 2^24
// records), 256 of 16 keys above (faster on calls of 2^29 records).
uint32_t scatter_threads(const sim_tuning& t, uint32_t n_tiles) {
  return t.scatter_threads ? t.scatter_threads : (n_tiles <= 16384 ? 512u : 256u);
}

int group_shift(uint64_t n_tiles, int bias) {
  int gs = 0;
  while (gs < (int)MAX_HGROUP_SHIFT && (1ull << (2 * gs)) < n_tiles) gs++;
  gs += bias;
  return gs < 0 ? 0 : (gs > (int)MAX_HGROUP_SHIFT ? (int)MAX_HGROUP_SHIFT : gs);
}

// The call's tables, one block in host and device memory (one upload):
// trace descriptors, tile references, histogram groups, then the traces
// sorted whole in LDS (at most one entry per trace).
static size_t meta_bytes(uint32_t n_traces, uint32_t n_tiles, uint64_t n_hgroups) {
  return (size_t)n_traces * sizeof(TraceDesc) + (size_t)n_tiles * sizeof(TileRef) +
         (size_t)n_hgroups * sizeof(GroupRef) + (size_t)n_traces * sizeof(uint32_t);
}

// Pinned host bytes of a call: its tables, then two words per tile for a
// staging overflow (the tiles' entry counts, then their staging references).
static size_t host_bytes(uint32_t n_traces, uint32_t n_tiles, uint64_t n_hgroups) {
  return (meta_bytes(n_traces, n_tiles, n_hgroups) + 15) / 16 * 16 + (size_t)n_tiles * 16;
}

// Limits of the no-allocation entry point besides the scratch itself: the
// pinned tables every context allocates at creation hold this many traces
// and tiles (2^23 records in the largest call the scratch can hold, plus one
// partial tile per trace).
constexpr uint32_t NOALLOC_MAX_TRACES = 4096;
constexpr uint32_t NOALLOC_MAX_TILES = (1u << 23) / TILE + NOALLOC_MAX_TRACES;

// The fixed device regions of a call, in one order for both ways of
// providing them (grow-only context buffers, or the scratch).
enum { R_KEYS0, R_KEYS1, R_META, R_STATS, R_LAYOUT, R_THIST, R_TCNT, R_GTOT, R_GBASE, R_AGG, R_TOUT, R_CROSS,
       R_CFLAG, R_GSUM, R_CTRL, N_REGION };

// radix: digits of the call's widest pass (RADIX, or RADIX_MAX with 9-bit digits).
void region_bytes(size_t need[N_REGION], uint64_t total, uint32_t n_traces, uint32_t n_tiles, uint64_t n_hgroups,
                  uint32_t key_bytes, uint32_t radix) {
  const uint32_t n_groups = (n_tiles + GROUP - 1) / GROUP;
  need[R_KEYS0] = total * key_bytes;
  need[R_KEYS1] = total * key_bytes;
  need[R_META] = meta_bytes(n_traces, n_tiles, n_hgroups);
  need[R_STATS] = (size_t)n_tiles * sizeof(TraceStats);
  need[R_LAYOUT] = (size_t)n_traces * sizeof(TraceLayout);
  need[R_THIST] = (size_t)n_tiles * radix * 4;
  need[R_TCNT] = (size_t)n_tiles * radix * 2;
  need[R_GTOT] = (size_t)n_hgroups * radix * 4;
  need[R_GBASE] = (size_t)n_hgroups * radix * 8;
  need[R_AGG] = (size_t)n_tiles * SW * 4;
  need[R_TOUT] = (size_t)n_tiles * sizeof(TileOut);
  need[R_CROSS] = (size_t)n_tiles * sizeof(RaceOut);
  need[R_CFLAG] = (size_t)n_tiles * 4;
  need[R_GSUM] = (size_t)n_groups * 4;
  need[R_CTRL] = sizeof(Ctrl);
}

DevBuf* region_buf(sim_ctx* c, int r) {
  DevBuf* const bufs[N_REGION] = {&c->keys0, &c->keys1, &c->meta,  &c->stats_part, &c->layout,
                                  &c->thist, &c->tcnt,  &c->gtot,  &c->gbase,      &c->agg,
                                  &c->tout,  &c->cross, &c->cross_flag, &c->group_sum, &c->ctrl};
  return bufs[r];
}

// Capacity ensure() gives a buffer asked for `bytes` (its headroom included).
size_t grown(size_t bytes) {
  if (bytes == 0) bytes = 64;
  return bytes + bytes / 8;
}

}  // namespace

namespace sc {
size_t ctx_device_bytes(const sim_ctx* c);
}  // namespace sc

namespace {

// Grow one buffer within the context's device limit.
hipError_t grow(sim_ctx* c, DevBuf& b, size_t bytes) {
  if (b.cap >= bytes) return hipSuccess;
  if (c->dev_limit && ctx_device_bytes(c) - b.cap + grown(bytes) > c->dev_limit) return hipErrorOutOfMemory;
  return ensure(b, bytes, false, &c->alloc_gen);
}

// Grow the context's buffers for a call of `total` records in `n_traces`
// traces, `n_tiles` tiles and `n_hgroups` histogram groups.  Under a device
// limit, a context whose grown buffers would exceed it first releases all of
// them (they are idle between calls) and allocates the call's sizes afresh.
hipError_t size_buffers(sim_ctx* c, uint64_t total, uint32_t n_traces, uint32_t n_tiles, uint64_t n_hgroups,
                        uint32_t key_bytes, uint32_t radix) {
  size_t need[N_REGION];
  region_bytes(need, total, n_traces, n_tiles, n_hgroups, key_bytes, radix);
  const uint64_t cap0 = total < 65536 ? total : 65536;
  const size_t out_need = c->out.cap ? c->out.cap : cap0 * sizeof(RaceOut);
  if (c->dev_limit) {
    auto after = [&]() {
      size_t t = ctx_device_bytes(c);
      for (int r = 0; r < N_REGION; r++) {
        const DevBuf* b = region_buf(c, r);
        if (b->cap < need[r]) t += grown(need[r]) - b->cap;
      }
      if (c->out.cap < out_need) t += grown(out_need) - c->out.cap;
      return t;
    };
    if (after() > c->dev_limit) {
      for (int r = 0; r < N_REGION; r++) release(*region_buf(c, r));
      for (DevBuf* b : {&c->out, &c->stage, &c->stage_ref, &c->bar, &c->bar_base, &c->div_in, &c->div_chunks,
                        &c->div_blocks, &c->div_cnt, &c->div_off, &c->div_out, &c->fit_out})
        release(*b);
      if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
      c->graph.exec = nullptr;
      c->alloc_gen++;
      if (after() > c->dev_limit) return hipErrorOutOfMemory;
    }
  }
  for (int r = 0; r < N_REGION; r++) {
    const hipError_t e = ensure(*region_buf(c, r), need[r], false, &c->alloc_gen);
    if (e != hipSuccess) return e;
  }
  return ensure(c->out, out_need, false, &c->alloc_gen);
}

// Where a call's result goes: a result the library allocates (the ordinary
// entry points), or buffers the caller owns (the no-allocation entry point).
struct Sink {
  sim_result** out = nullptr;
  sim_race* races = nullptr;
  uint64_t races_cap = 0;
  uint64_t* n_races = nullptr;
  sim_trace_summary* traces = nullptr;
  sim_barrier_result** barriers = nullptr;  // also the redundant-barrier check
  sim_fitness* fitness = nullptr;           // instead of the race check: the EP fitness rows (host, n_traces)
  const uint32_t* side = nullptr;           // the warp-aware check: one side word per record (device)
};

void barrier_result_free(sim_barrier_result* r) {
  if (!r) return;
  free(r->barriers);
  free(r);
}

// One call.  Trace i's records start at trace_recs[i] when trace_recs is
// given (device pointers, the traces need not be adjacent), else at
// d_records + offsets[i].  noalloc: every device buffer comes from the
// scratch and nothing is allocated.
int run(sim_ctx* c, const sim_record* d_records, const sim_record* const* trace_recs, const uint64_t* offsets,
        uint32_t n_traces, const uint32_t* tpb, hipStream_t s, const Sink& sink, bool noalloc) {
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  sim_result* dummy = nullptr;
  int rc = validate(c, offsets, n_traces, tpb, sink.out ? sink.out : &dummy, &total, &n_tiles);
  if (rc) return rc;
  if (total && !d_records && !trace_recs) return fail(c, SIM_EINVAL, "records is NULL");
  if (trace_recs)
    for (uint32_t i = 0; i < n_traces; i++)
      if (offsets[i + 1] > offsets[i] && !trace_recs[i]) return fail(c, SIM_EINVAL, "records of trace %u is NULL", i);
  if (noalloc) {
    if (!c->scratch)
      return fail(c, SIM_EDEVICE, "no-allocation scratch unavailable on device %d: %s", c->device,
                  hipGetErrorString(c->scratch_err));
    if (n_traces > NOALLOC_MAX_TRACES)
      return fail(c, SIM_EINVAL, "a no-allocation call holds at most %u traces", NOALLOC_MAX_TRACES);
    if (n_tiles > NOALLOC_MAX_TILES)
      return fail(c, SIM_EINVAL, "a no-allocation call holds at most %u tiles of 4096 records", NOALLOC_MAX_TILES);
  }
  for (auto& t : c->times) t = sim_stage_time{0.0, 0, 0};
  const bool fit = sink.fitness != nullptr;
  if (fit && noalloc) return fail(c, SIM_EINVAL, "the fitness count has no no-allocation form");
  const bool warp = sink.side != nullptr;
  if (warp && (noalloc || trace_recs || fit || sink.barriers))
    return fail(c, SIM_EINVAL, "the warp-aware check runs on its own, on adjacent device records");
  // radix passes and key width the previous call of this kind needed
  uint32_t& pass_guess = fit ? c->fit_pass_guess : (warp ? c->warp_pass_guess : c->pass_guess);
  bool& wide_guess = fit ? c->fit_wide_guess : (warp ? c->warp_wide_guess : c->wide_guess);
  uint32_t& bits_guess = fit ? c->fit_bits_guess : (warp ? c->warp_bits_guess : c->bits_guess);
  uint32_t& db_guess = fit ? c->fit_db_guess : (warp ? c->warp_db_guess : c->db_guess);

  // result delivery: summaries from the entry list, entries downloaded from
  // `dev_out` (n_races of them)
  auto deliver = [&](uint64_t n_races, const void* dev_out) -> int {
    sim_trace_summary* sums = nullptr;
    sim_race* races = nullptr;
    sim_result* r = nullptr;
    if (sink.out) {
      r = alloc_result(n_races, n_traces);
      if (!r) return fail(c, SIM_ENOMEM, "host allocation failed");
      sums = r->traces;
      races = r->races;
    } else {
      *sink.n_races = n_races;
      if (n_races > sink.races_cap)
        return fail(c, SIM_ENOSPC, "%llu racing locations, the output buffer holds %llu",
                    (unsigned long long)n_races, (unsigned long long)sink.races_cap);
      sums = sink.traces;
      races = sink.races;
      for (uint32_t i = 0; i < n_traces; i++) sums[i] = sim_trace_summary{0, 0, 0};
    }
    hipError_t e;
    if (n_races && ((e = hipMemcpyAsync(races, dev_out, n_races * sizeof(sim_race), hipMemcpyDeviceToHost, s)) ||
                    (e = hipStreamSynchronize(s)))) {
      sim_result_free(r);
      return hip_fail(c, e, "result download");
    }
    for (uint32_t i = 0; i < n_traces; i++) sums[i].n_records = offsets[i + 1] - offsets[i];
    for (uint64_t k = 0; k < n_races; k++) {
      const sim_race& x = races[k];
      if (x.trace >= n_traces) {
        sim_result_free(r);
        return fail(c, SIM_EDEVICE, "entry %llu names trace %u", (unsigned long long)k, x.trace);
      }
      sums[x.trace].n_race_locs += 1;
      sums[x.trace].n_pairs += x.pairs_ww + x.pairs_rw + x.pairs_aw + x.pairs_ar;
    }
    if (sink.out) *sink.out = r;
    return SIM_OK;
  };

  if (fit && total == 0) {  // every trace empty: F = 1, no locations
    for (uint32_t i = 0; i < n_traces; i++) sink.fitness[i] = sim_fitness{0, 0, 0, 0, 0, 1.0};
    return SIM_OK;
  }
  if (total == 0) {  // nothing to check: summaries only (and no barrier instances)
    sim_barrier_result* br = nullptr;
    if (sink.barriers) {
      br = (sim_barrier_result*)calloc(1, sizeof(sim_barrier_result));
      if (br) br->barriers = (sim_barrier*)malloc(sizeof(sim_barrier));
      if (!br || !br->barriers) {
        barrier_result_free(br);
        return fail(c, SIM_ENOMEM, "host allocation failed");
      }
    }
    const int rc0 = deliver(0, nullptr);
    if (rc0 != SIM_OK) {
      barrier_result_free(br);
      return rc0;
    }
    if (sink.barriers) *sink.barriers = br;
    return SIM_OK;
  }

  // ---- per-call tables (pinned); histogram groups of about sqrt(ntiles)
  // tiles keep both serial offset loops of the radix kernels short
  hipError_t e;
  const sim_tuning tune = pick_tuning(c, total);
  // digit width of the passes after the first: the tuning's, else 9 bits
  // where the previous call's widest key sorts in fewer passes with them
  // (no-allocation calls: 8, the scratch's tables are sized for it)
  uint32_t db = tune.digit_bits ? tune.digit_bits : RADIX_BITS;
  if (!tune.digit_bits && bits_guess &&
      radix_passes(bits_guess, RADIX_WIDE_BITS) < radix_passes(bits_guess, RADIX_BITS))
    db = RADIX_WIDE_BITS;
  if (noalloc) db = RADIX_BITS;
  // traces sorted whole in LDS: one tile, or up to four with one-word keys
  const bool wide = wide_guess;
  const uint32_t small_max_tiles = wide ? 1u : 4u;
  auto& P = c->plan;
  const bool plan_hit = P.valid && P.host_gen == c->host_gen && P.bias == tune.group_shift_bias &&
                        P.small_max_tiles == small_max_tiles && P.offsets.size() == (size_t)n_traces + 1 &&
                        std::memcmp(P.offsets.data(), offsets, ((size_t)n_traces + 1) * sizeof(uint64_t)) == 0 &&
                        std::memcmp(P.tpb.data(), tpb, (size_t)n_traces * sizeof(uint32_t)) == 0;
  uint64_t n_hgroups64 = plan_hit ? P.n_hgroups : 0;
  if (!plan_hit)
    for (uint32_t i = 0; i < n_traces; i++) {
      const uint64_t nt = (offsets[i + 1] - offsets[i] + TILE - 1) / TILE;
      const int gs = group_shift(nt, tune.group_shift_bias);
      n_hgroups64 += (nt + (1ull << gs) - 1) >> gs;
    }
  const size_t h_bytes = host_bytes(n_traces, n_tiles, n_hgroups64);
  if (c->h_meta_cap < h_bytes) {
    if (noalloc) return fail(c, SIM_EINVAL, "the call's tables exceed the context's pinned tables");
    if (c->h_meta) (void)hipHostFree(c->h_meta);
    c->h_meta = nullptr;
    c->h_meta_cap = 0;
    c->host_gen++;  // (a plan hit never gets here: its tables fitted before)
    e = hipHostMalloc(&c->h_meta, h_bytes + h_bytes / 8, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(c, e, "pinned allocation");
    c->h_meta_cap = h_bytes + h_bytes / 8;
  }
  TraceDesc* hd = (TraceDesc*)c->h_meta;
  TileRef* ht = (TileRef*)(hd + n_traces);
  GroupRef* hg = (GroupRef*)(ht + n_tiles);
  uint32_t* hs = (uint32_t*)(hg + n_hgroups64);
  uint32_t t0 = 0, g0 = 0, max_group_tiles = 1, max_trace_groups = 1, n_small1 = 0, n_small4 = 0;
  if (plan_hit) {  // the host copy holds this call's trace and group tables
    g0 = P.n_hgroups;
    max_group_tiles = P.max_group_tiles;
    max_trace_groups = P.max_trace_groups;
    n_small1 = P.n_small1;
    n_small4 = P.n_small4;
  }
  for (uint32_t i = 0; i < (plan_hit ? 0u : n_traces); i++) {
    const uint64_t n = offsets[i + 1] - offsets[i];
    const uint32_t nt = (uint32_t)((n + TILE - 1) / TILE);
    const uint32_t gs = (uint32_t)group_shift(nt, tune.group_shift_bias);
    const uint32_t ng = (nt + (1u << gs) - 1) >> gs;
    max_group_tiles = std::max(max_group_tiles, std::min(nt, 1u << gs));
    max_trace_groups = std::max(max_trace_groups, ng);
    hd[i] = TraceDesc{offsets[i], n, tpb[i], t0, nt, g0, ng, gs, {0, 0, 0}};
    for (uint32_t k = 0; k < ng; k++)
      hg[g0 + k] = GroupRef{i, t0 + (k << gs), std::min(nt - (k << gs), 1u << gs) | (nt <= small_max_tiles ? TILE_SHORT : 0u),
                            0u};
    if (nt == 1) hs[n_small1++] = i;
    else if (nt >= 2 && nt <= small_max_tiles) hs[n_traces - 1 - n_small4++] = i;  // from the back
    t0 += nt;
    g0 += ng;
  }
  const uint32_t n_hgroups = g0;
  if (!plan_hit) {
    if (n_small4) memmove(hs + n_small1, hs + n_traces - n_small4, (size_t)n_small4 * sizeof(uint32_t));
    c->host_gen++;
    P.offsets.assign(offsets, offsets + n_traces + 1);
    P.tpb.assign(tpb, tpb + n_traces);
    P.bias = tune.group_shift_bias;
    P.small_max_tiles = small_max_tiles;
    P.host_gen = c->host_gen;
    P.valid = true;
    P.n_hgroups = n_hgroups;
    P.max_group_tiles = max_group_tiles;
    P.max_trace_groups = max_trace_groups;
    P.n_small1 = n_small1;
    P.n_small4 = n_small4;
  }
  // the (trace, tile) table: filled only when the tables are uploaded (a
  // graph replay whose upload is still on the device skips both)
  auto fill_tiles = [&]() {
    for (uint32_t i = 0; i < n_traces; i++) {
      const uint32_t nt = hd[i].ntiles, tt = hd[i].tile0;
      const uint32_t short_flag = nt <= small_max_tiles ? TILE_SHORT : 0u;
      const sim_record* base = trace_recs ? trace_recs[i] : d_records + offsets[i];
      for (uint32_t k = 0; k < nt; k++) {
        const uint64_t first = offsets[i] + (uint64_t)k * TILE;
        const uint32_t n_in = (uint32_t)std::min<uint64_t>(TILE, offsets[i + 1] - first);
        ht[tt + k] = TileRef{i, k, (uint32_t)first, n_in | short_flag, base + (uint64_t)k * TILE};
      }
    }
  };
  // host words of a staging overflow, after the tables
  TileOut* h_tout = (TileOut*)((char*)c->h_meta + (meta_bytes(n_traces, n_tiles, n_hgroups) + 15) / 16 * 16);
  uint64_t* h_sref = (uint64_t*)(h_tout + n_tiles);

  // ---- device buffers: the context's (grown as needed) or the scratch's
  const uint32_t key_bytes = wide ? 16u : 8u;
  void* reg[N_REGION];
  RaceOut* out_p = nullptr;
  uint64_t out_cap = 0;
  char* rest = nullptr;  // no-allocation calls: the scratch after the fixed regions
  size_t rest_bytes = 0;
  uint64_t* d_sref = nullptr;
  if (noalloc) {
    size_t need[N_REGION];
    region_bytes(need, total, n_traces, n_tiles, n_hgroups, key_bytes, RADIX);
    size_t off = 0;
    auto carve = [&](size_t bytes) {
      off = (off + 255) / 256 * 256;
      void* p = (char*)c->scratch + off;
      off += bytes;
      return p;
    };
    for (int r = 0; r < N_REGION; r++) reg[r] = carve(need[r]);
    d_sref = (uint64_t*)carve((size_t)n_tiles * 8);
    off = (off + 255) / 256 * 256;
    if (off > SCRATCH_BYTES)
      return fail(c, SIM_EINVAL,
                  "the call needs %llu bytes of device buffers (%u-byte keys), the no-allocation scratch holds %llu",
                  (unsigned long long)off, key_bytes, (unsigned long long)SCRATCH_BYTES);
    rest = (char*)c->scratch + off;
    rest_bytes = SCRATCH_BYTES - off;
    out_p = (RaceOut*)rest;
    out_cap = rest_bytes / sizeof(RaceOut);
  } else {
    if ((e = size_buffers(c, total, n_traces, n_tiles, n_hgroups, key_bytes, 1u << db)) != hipSuccess)
      return hip_fail(c, e, "device allocation");
    for (int r = 0; r < N_REGION; r++) reg[r] = region_buf(c, r)->p;
    out_p = (RaceOut*)c->out.p;
    out_cap = c->out.cap / sizeof(RaceOut);
  }

  Buffers b;
  b.desc = (const TraceDesc*)reg[R_META];
  b.tiles = (const TileRef*)(b.desc + n_traces);
  b.stats_part = (TraceStats*)reg[R_STATS];
  b.layout = (TraceLayout*)reg[R_LAYOUT];
  b.keys[0] = reg[R_KEYS0];
  b.keys[1] = reg[R_KEYS1];
  b.wide = wide ? 1u : 0u;
  b.key_bytes = key_bytes;
  b.fitness = fit ? 1u : 0u;
  b.side = warp ? sink.side : nullptr;
  b.digit_bits = db;
  b.groups = (const GroupRef*)(b.tiles + n_tiles);
  b.small_traces = (const uint32_t*)(b.groups + n_hgroups);
  b.n_small1 = n_small1;
  b.n_small4 = n_small4;
  b.small_max_tiles = small_max_tiles;
  b.thist = (uint32_t*)reg[R_THIST];
  b.tcnt = (uint16_t*)reg[R_TCNT];
  b.gtot = (uint32_t*)reg[R_GTOT];
  b.gbase = (uint64_t*)reg[R_GBASE];
  b.agg = (uint32_t*)reg[R_AGG];
  b.tout = (TileOut*)reg[R_TOUT];
  b.cross = (RaceOut*)reg[R_CROSS];
  b.cross_flag = (uint32_t*)reg[R_CFLAG];
  b.group_sum = (uint32_t*)reg[R_GSUM];
  b.stage = nullptr;
  b.stage_ref = nullptr;
  b.ctrl = (Ctrl*)reg[R_CTRL];
  b.out = out_p;
  b.out_cap = out_cap;
  b.n_traces = n_traces;
  b.n_tiles = n_tiles;
  b.n_groups = n_hgroups;
  b.grid_stream = tile_grid(n_tiles, tune.stream_wgs_per_cu, c->n_cu);
  b.grid_sort = tile_grid(n_tiles, tune.sort_wgs_per_cu, c->n_cu);
  b.scatter_nt = (scatter_threads(tune, n_tiles) == 512 && !wide) ? 512u : 256u;
  b.grid_scan = tile_grid(n_tiles, tune.scan_wgs_per_cu, c->n_cu);
  b.max_group_tiles = max_group_tiles;
  b.max_trace_groups = max_trace_groups;
  // radix digit 0 is tid mod 256 when threads per block is a power of two
  // >= 256 (the local-tid field then fills key bits [2, 10)): stats build
  // its histograms and key generation does pass 0
  // (not with a side field, which takes the key's lowest bits above the action)
  b.fuse0 = warp ? 0 : 1;
  for (uint32_t i = 0; i < n_traces; i++)
    if (tpb[i] < 256 || (tpb[i] & (tpb[i] - 1)) != 0) b.fuse0 = 0;
  // a call of one-tile traces only is sorted in LDS from pass 0 on, with no
  // global pass at all
  uint32_t n_empty = 0;
  for (uint32_t i = 0; i < n_traces; i++) n_empty += offsets[i + 1] == offsets[i] ? 1u : 0u;
  const bool all_small = n_small1 + n_small4 + n_empty == n_traces;
  if (all_small) b.fuse0 = 0;
  const uint32_t first_pass = b.fuse0 ? 1u : 0u;
  b.small_from = first_pass;

  // ---- the pipeline.  Radix passes: the context remembers how many the
  // previous call needed and launches that many; the scan kernels do
  // nothing if some trace needs more, and the host then adds the missing
  // passes and scans again.
  const bool prof = (c->flags & SIM_CFG_PROFILE) != 0;
  int nev = 0;
  int ev_stage[MAX_EV / 2];
  bool ev_counts[MAX_EV / 2];
  auto timed = [&](int stage, bool counts, auto&& launch) -> hipError_t {
    const bool rec = prof && nev + 2 <= MAX_EV;
    if (rec) {
      hipError_t e0 = hipEventRecord(c->ev[nev], s);
      if (e0 != hipSuccess) return e0;
    }
    hipError_t e1 = launch();
    if (e1 != hipSuccess) return e1;
    if (rec) {
      hipError_t e2 = hipEventRecord(c->ev[nev + 1], s);
      if (e2 != hipSuccess) return e2;
      ev_stage[nev / 2] = stage;
      ev_counts[nev / 2] = counts;
      nev += 2;
    }
    return hipSuccess;
  };
  auto sync_ctrl = [&]() -> hipError_t {
    hipError_t e1 = hipMemcpyAsync(c->h_ctrl, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
    return e1 != hipSuccess ? e1 : hipStreamSynchronize(s);
  };
  auto sort_passes = [&](uint32_t from, uint32_t to) -> hipError_t {
    if (all_small) return hipSuccess;  // k_sort_small did every pass
    for (uint32_t p = from; p < to; p++) {
      hipError_t e1 = timed(ST_UPSWEEP, true, [&] { return launch_upsweep(b, p, s); });
      if (e1 == hipSuccess) e1 = timed(ST_SORT, true, [&] { return launch_scatter(b, p, s); });
      if (e1 != hipSuccess) return e1;
    }
    return hipSuccess;
  };
  // counts: whether the launches are real work (a scan before missing
  // passes, or a rescan after an overflow, is left out of the stage times)
  FitOut* fit_out = nullptr;
  if (fit) {
    if ((e = grow(c, c->fit_out, (size_t)n_traces * sizeof(FitOut)))) return hip_fail(c, e, "device allocation");
    fit_out = (FitOut*)c->fit_out.p;
  }
  auto scan = [&](uint32_t passes_done, bool counts) -> hipError_t {
    if (fit) return timed(ST_SCAN, counts, [&] { return launch_fitness(b, passes_done, fit_out, s); });
    hipError_t e1 = timed(ST_SCAN, counts, [&] { return launch_scan_tiles(b, passes_done, s); });
    if (e1 == hipSuccess) e1 = timed(ST_CROSS, counts, [&] { return launch_scan_cross(b, passes_done, s); });
    if (e1 == hipSuccess) e1 = timed(ST_OUT, counts, [&] { return launch_scan_out(b, passes_done, s); });
    return e1;
  };

  // (a call of one-tile traces has all its passes done before the scan)
  // (a guess counted in another width is recounted from the key bits)
  const uint32_t prev_guess = db == db_guess || !bits_guess ? pass_guess : radix_passes(bits_guess, db);
  const uint32_t guess = all_small ? MAX_PASSES : (prev_guess < MAX_PASSES ? prev_guess : MAX_PASSES);
  int first_scan_ev = 0;  // events of the first round before its scan
  auto first_round = [&]() -> hipError_t {
    hipError_t e1;
    if ((e1 = timed(ST_INIT, true, [&] { return launch_init(b, s); })) ||
        (e1 = timed(ST_STATS, true, [&] { return launch_stats(b, s); })) ||
        (e1 = timed(ST_LAYOUT, true, [&] { return launch_layout(b, s); })))
      return e1;
    if (b.fuse0 && (e1 = timed(ST_UPSWEEP, true, [&] { return launch_upsweep(b, 0, s); }))) return e1;
    if ((e1 = timed(ST_KEYGEN, true, [&] { return launch_keygen(b, s); })) ||
        (b.n_small1 + b.n_small4 &&
         (e1 = timed(ST_SORT_SMALL, true, [&] { return launch_sort_small(b, s); }))) ||
        (e1 = sort_passes(first_pass, guess)))
      return e1;
    first_scan_ev = nev / 2;
    if (guess && (e1 = scan(guess, true))) return e1;
    return hipMemcpyAsync(c->h_ctrl, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
  };
  // Graph mode: the first round (every launch up to the control download)
  // is captured once per call shape and replayed while the shape, the
  // buffers, the pass count and the digit width stay the same.  (Not for gathered traces,
  // whose record addresses are not part of the shape, nor for calls that
  // may not allocate: instantiating a graph does.)
  const bool use_graph =
      (c->flags & SIM_CFG_GRAPHS) && !prof && s != nullptr && guess > 0 && !trace_recs && !noalloc && !fit && !warp;
  auto& G = c->graph;
  const bool replay = use_graph && G.exec && G.records == d_records && G.stream == s && G.total == total &&
                      G.n_traces == n_traces && G.n_tiles == n_tiles && G.gen == c->alloc_gen && G.guess == guess &&
                      G.tuning_gen == c->tuning_gen && G.wide == wide && G.db == db &&
                      std::memcmp(G.offsets.data(), offsets, (size_t)(n_traces + 1) * sizeof(uint64_t)) == 0 &&
                      std::memcmp(G.tpb.data(), tpb, (size_t)n_traces * sizeof(uint32_t)) == 0;
  // The tables: a replay finds them on the device when no other call
  // uploaded tables since the captured one (same shape, same buffers, same
  // records: the same tables); otherwise they are built and uploaded.
  if (!(replay && G.meta_gen == c->meta_gen)) {
    fill_tiles();
    if ((e = hipMemcpyAsync(reg[R_META], c->h_meta, meta_bytes(n_traces, n_tiles, n_hgroups), hipMemcpyHostToDevice,
                            s)))
      return hip_fail(c, e, "table upload");
    c->meta_gen++;
  }
  if (replay) {
    e = hipGraphLaunch(G.exec, s);
  } else if (use_graph) {
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t e_cap = first_round();
      e = hipStreamEndCapture(s, &graph);
      if (e_cap != hipSuccess) e = e_cap;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) {
      G.records = d_records;
      G.stream = s;
      G.total = total;
      G.n_traces = n_traces;
      G.n_tiles = n_tiles;
      G.offsets.assign(offsets, offsets + n_traces + 1);
      G.tpb.assign(tpb, tpb + n_traces);
      G.gen = c->alloc_gen;
      G.guess = guess;
      G.tuning_gen = c->tuning_gen;
      G.meta_gen = c->meta_gen;
      G.wide = wide;
      G.db = db;
      e = hipGraphLaunch(G.exec, s);
    } else {  // capture not possible here: run the launches directly
      (void)hipGetLastError();
      if (G.exec) (void)hipGraphExecDestroy(G.exec);
      G.exec = nullptr;
      e = first_round();
    }
  } else {
    e = first_round();
  }
  if (e != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "pipeline");

  Ctrl ctl = *c->h_ctrl;
  if (ctl.error_flags & LAYOUT_ERR_RECORD)
    return fail(c, SIM_ERECORD, "invalid record at index %llu (action > 2 or space > 1)",
                (unsigned long long)ctl.first_bad);
  if (ctl.error_flags & LAYOUT_ERR_WIDE) return fail(c, SIM_ERANGE, "a trace's sort key needs more than 128 bits");
  if (ctl.error_flags & ERR_NEEDS_WIDE) {
    // a trace needs two-word keys: run the whole call again in that mode
    // (the next call starts in it while its traces keep needing it)
    wide_guess = true;
    return run(c, d_records, trace_recs, offsets, n_traces, tpb, s, sink, noalloc);
  }
  const uint32_t needed = ctrl_passes(ctl.pass_bits);
  if (needed > guess) {
    // too few passes ran: the scan kernels above returned at once
    for (int k = first_scan_ev; k < nev / 2; k++) ev_counts[k] = false;
    if ((e = sort_passes(guess > first_pass ? guess : first_pass, needed)) || (e = scan(needed, true)) ||
        (e = sync_ctrl()))
      return hip_fail(c, e, "pipeline");
    ctl = *c->h_ctrl;
  }
  if (!all_small) {  // an LDS-sorted call tells nothing about global passes
    pass_guess = needed;
    db_guess = db;
    bits_guess = ctl.pass_bits & 0xFFFFu;
  }
  wide_guess = ctl.wide_traces > 0;
  if (fit) {
    if (ctl.error_flags) return fail(c, SIM_EDEVICE, "internal kernel check failed (flags 0x%x)", ctl.error_flags);
    if ((e = hipMemcpyAsync(sink.fitness, fit_out, (size_t)n_traces * sizeof(FitOut), hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
      return hip_fail(c, e, "fitness download");
    if (prof)
      for (int k = 0; k < nev / 2; k++) {
        if (!ev_counts[k]) continue;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]);
        c->times[ev_stage[k]].ms += ms;
        c->times[ev_stage[k]].launches += 1;
      }
    return SIM_OK;
  }
  if (ctl.error_flags & ERR_STAGE_OVERFLOW) {
    // Some tile holds more racing locations than its slice of the idle key
    // buffer: give each such tile a range of a dedicated staging buffer, as
    // large as the entry count this scan found for it, and scan again.
    if ((e = hipMemcpyAsync(h_tout, b.tout, (size_t)n_tiles * sizeof(TileOut), hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
      return hip_fail(c, e, "tile counts download");
    uint64_t staged = 0;
    for (uint32_t t = 0; t < n_tiles; t++) {
      const uint32_t n_in = ht[t].n_flags & ~TILE_SHORT;
      const uint32_t cnt = h_tout[t].in_count;
      if (cnt > n_in * key_bytes / (uint32_t)sizeof(RaceOut)) {
        h_sref[t] = (staged << STAGE_CAP_BITS) | cnt;
        staged += cnt;
      } else {
        h_sref[t] = 0;
      }
    }
    RaceOut* stage = nullptr;
    if (noalloc) {  // from the end of the scratch's free part; the output keeps the rest
      const size_t sbytes = (size_t)staged * sizeof(RaceOut);
      if (sbytes > rest_bytes)
        return fail(c, SIM_ENOSPC, "the call stages %llu entries, more than the no-allocation scratch holds",
                    (unsigned long long)staged);
      stage = (RaceOut*)(rest + (rest_bytes - sbytes) / 256 * 256);
      b.out_cap = (size_t)((char*)stage - rest) / sizeof(RaceOut);
    } else {
      if ((e = grow(c, c->stage, (size_t)staged * sizeof(RaceOut))) ||
          (e = grow(c, c->stage_ref, (size_t)n_tiles * sizeof(uint64_t))))
        return hip_fail(c, e, "device allocation");
      stage = (RaceOut*)c->stage.p;
      d_sref = (uint64_t*)c->stage_ref.p;
    }
    if ((e = hipMemcpyAsync(d_sref, h_sref, (size_t)n_tiles * sizeof(uint64_t), hipMemcpyHostToDevice, s)))
      return hip_fail(c, e, "staging table upload");
    b.stage = stage;
    b.stage_ref = d_sref;
    if ((e = launch_reset_errors(b, ERR_STAGE_OVERFLOW, s)) || (e = scan(needed, false)) || (e = sync_ctrl()))
      return hip_fail(c, e, "rescan");
    ctl = *c->h_ctrl;
  }
  if (ctl.error_flags)
    return fail(c, SIM_EDEVICE, "internal kernel check failed (flags 0x%x)", ctl.error_flags);

  uint64_t n_races = ctl.total_entries;
  if (n_races > b.out_cap) {  // more racing locations than the output buffer holds
    if (noalloc) {
      if (sink.n_races) *sink.n_races = n_races;
      return fail(c, SIM_ENOSPC, "%llu racing locations, the no-allocation scratch holds %llu",
                  (unsigned long long)n_races, (unsigned long long)b.out_cap);
    }
    if ((e = grow(c, c->out, n_races * sizeof(RaceOut)))) return hip_fail(c, e, "device allocation");
    b.out = (RaceOut*)c->out.p;
    b.out_cap = c->out.cap / sizeof(RaceOut);
    if ((e = timed(ST_OUT, false, [&] { return launch_scan_out(b, needed, s); })) || (e = sync_ctrl()))
      return hip_fail(c, e, "rescan");
    if (c->h_ctrl->total_entries != n_races) return fail(c, SIM_EDEVICE, "entry count changed between scans");
  }

  if (prof) {
    for (int k = 0; k < nev / 2; k++) {
      if (!ev_counts[k]) continue;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]);
      c->times[ev_stage[k]].ms += ms;
      c->times[ev_stage[k]].launches += 1;
    }
  }
  if (warp) {
    // Theorem 1's warp clauses: subtract the pairs lockstep orders, keep
    // the entries left with a pair
    if ((e = grow(c, c->warp_rm, (size_t)(n_races ? n_races : 1) * 4 * sizeof(uint64_t))) ||
        (e = grow(c, c->warp_out, (size_t)(n_races ? n_races : 1) * sizeof(RaceOut))) ||
        (e = grow(c, c->warp_n, sizeof(uint64_t))))
      return hip_fail(c, e, "device allocation");
    uint64_t n_ref = 0;
    if ((e = launch_warp_refine(b, b.out, n_races, (unsigned long long*)c->warp_rm.p, (RaceOut*)c->warp_out.p,
                                (unsigned long long*)c->warp_n.p, s)) ||
        (e = hipMemcpyAsync(&n_ref, c->warp_n.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s)) ||
        (e = sync_ctrl()))
      return hip_fail(c, e, "warp refinement");
    if (c->h_ctrl->error_flags)
      return fail(c, SIM_EDEVICE, "internal kernel check failed (flags 0x%x)", c->h_ctrl->error_flags);
    return deliver(n_ref, c->warp_out.p);
  }
  if (!sink.barriers) return deliver(n_races, b.out);

  // ---- the redundant-barrier check over the same sorted keys: every
  // trace's boundaries (0 .. its largest epoch - 1) get a pair of counters
  std::vector<TraceLayout> lay(n_traces);
  if ((e = hipMemcpyAsync(lay.data(), b.layout, (size_t)n_traces * sizeof(TraceLayout), hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(c, e, "layout download");
  std::vector<uint64_t> base(n_traces + 1, 0);
  for (uint32_t i = 0; i < n_traces; i++)
    base[i + 1] = base[i] + (offsets[i + 1] > offsets[i] ? lay[i].max_epoch : 0u);
  const uint64_t nb = base[n_traces];
  const uint32_t copies = nb <= 4096 ? 16u : (nb <= 65536 ? 4u : 1u);
  if ((e = grow(c, c->bar, (size_t)(nb ? nb : 1) * copies * sizeof(BarrierCount))) ||
      (e = grow(c, c->bar_base, (size_t)n_traces * sizeof(uint64_t))))
    return hip_fail(c, e, "device allocation");
  std::vector<BarrierCount> counts((size_t)nb * copies);
  if ((e = hipMemcpyAsync(c->bar_base.p, base.data(), (size_t)n_traces * sizeof(uint64_t), hipMemcpyHostToDevice, s)) ||
      (e = launch_barriers(b, (const uint64_t*)c->bar_base.p, (BarrierCount*)c->bar.p, nb * copies, copies, s)) ||
      (nb && (e = hipMemcpyAsync(counts.data(), c->bar.p, counts.size() * sizeof(BarrierCount), hipMemcpyDeviceToHost,
                                 s))) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(c, e, "barrier check");
  uint64_t n_bar = 0;
  for (uint64_t k = 0; k < nb; k++) {
    uint64_t inst = 0;
    for (uint32_t q = 0; q < copies; q++) inst += counts[k * copies + q].instances;
    n_bar += inst ? 1 : 0;
  }
  sim_barrier_result* br = (sim_barrier_result*)calloc(1, sizeof(sim_barrier_result));
  if (br) br->barriers = (sim_barrier*)malloc((n_bar ? n_bar : 1) * sizeof(sim_barrier));
  if (!br || !br->barriers) {
    barrier_result_free(br);
    return fail(c, SIM_ENOMEM, "host allocation failed");
  }
  for (uint32_t i = 0; i < n_traces; i++)
    for (uint64_t k = base[i]; k < base[i + 1]; k++) {
      sim_barrier x{i, (uint32_t)(k - base[i]), 0, 0};
      for (uint32_t q = 0; q < copies; q++) {
        x.instances += counts[k * copies + q].instances;
        x.racing += counts[k * copies + q].racing;
      }
      if (x.instances) br->barriers[br->n_barriers++] = x;
    }
  const int rc2 = deliver(n_races, b.out);
  if (rc2 != SIM_OK) {
    barrier_result_free(br);
    return rc2;
  }
  *sink.barriers = br;
  return SIM_OK;
}

void divergence_result_free(sim_divergence_result* r) {
  if (!r) return;
  free(r->blocks);
  free(r);
}

// The barrier-divergence check of one call (arrival counts in device
// memory): chunk table on the host, then per-block reductions, the chunk
// offsets and the ordered output on the device.
// Checks the tables of a divergence call; *total threads, *n_chunks chunks.
int div_tables(sim_ctx* c, const uint64_t* offsets, uint32_t n_traces, const uint32_t* tpb, uint64_t* total,
               uint32_t* n_chunks) {
  if (n_traces && (!offsets || !tpb)) return fail(c, SIM_EINVAL, "offsets or threads_per_block is NULL");
  if (n_traces && offsets[0] != 0) return fail(c, SIM_EINVAL, "offsets[0] must be 0");
  uint64_t n_chunks64 = 0;
  for (uint32_t i = 0; i < n_traces; i++) {
    if (offsets[i + 1] < offsets[i]) return fail(c, SIM_EINVAL, "offsets decrease at trace %u", i);
    if (tpb[i] == 0) return fail(c, SIM_EINVAL, "threads_per_block[%u] is 0", i);
    const uint64_t n = offsets[i + 1] - offsets[i];
    if (n % tpb[i]) return fail(c, SIM_EINVAL, "trace %u holds %llu threads, not whole blocks of %u", i,
                                (unsigned long long)n, tpb[i]);
    const uint64_t per = std::max<uint64_t>(1, DIV_CHUNK_THREADS / tpb[i]);
    n_chunks64 += (n / tpb[i] + per - 1) / per;
  }
  *total = n_traces ? offsets[n_traces] : 0;
  if (*total >= (1ull << 32)) return fail(c, SIM_EINVAL, "a call holds at most 2^32 - 1 threads");
  *n_chunks = (uint32_t)n_chunks64;
  return SIM_OK;
}

int divergence(sim_ctx* c, const uint32_t* d_arr, const uint64_t* offsets, uint32_t n_traces, const uint32_t* tpb,
               hipStream_t s, sim_divergence_result** out) {
  if (!out) return fail(c, SIM_EINVAL, "out is NULL");
  *out = nullptr;
  uint64_t total = 0;
  uint32_t n_chunks = 0;
  const int rc = div_tables(c, offsets, n_traces, tpb, &total, &n_chunks);
  if (rc) return rc;
  if (total && !d_arr) return fail(c, SIM_EINVAL, "arrival counts are NULL");
  sim_divergence_result* r = (sim_divergence_result*)calloc(1, sizeof(sim_divergence_result));
  if (!r) return fail(c, SIM_ENOMEM, "host allocation failed");
  if (total == 0) {
    r->blocks = (sim_divergence*)malloc(sizeof(sim_divergence));
    if (!r->blocks) {
      divergence_result_free(r);
      return fail(c, SIM_ENOMEM, "host allocation failed");
    }
    *out = r;
    return SIM_OK;
  }
  // chunk table (pinned), the count word after it
  const size_t tab = ((size_t)n_chunks * sizeof(DivChunk) + 15) / 16 * 16;
  hipError_t e;
  if (c->h_div_cap < tab + 16) {
    if (c->h_div) (void)hipHostFree(c->h_div);
    c->h_div = nullptr;
    c->h_div_cap = 0;
    if ((e = hipHostMalloc(&c->h_div, tab + 16 + tab / 8, hipHostMallocDefault)) != hipSuccess) {
      divergence_result_free(r);
      return hip_fail(c, e, "pinned allocation");
    }
    c->h_div_cap = tab + 16 + tab / 8;
  }
  DivChunk* hc = (DivChunk*)c->h_div;
  uint64_t* h_total = (uint64_t*)((char*)c->h_div + tab);
  uint32_t k = 0, block0 = 0;
  for (uint32_t i = 0; i < n_traces; i++) {
    const uint64_t nb = (offsets[i + 1] - offsets[i]) / tpb[i];
    const uint64_t per = std::max<uint64_t>(1, DIV_CHUNK_THREADS / tpb[i]);
    for (uint64_t b = 0; b < nb; b += per) {
      const uint32_t m = (uint32_t)std::min<uint64_t>(per, nb - b);
      hc[k++] = DivChunk{offsets[i] + b * tpb[i], i, (uint32_t)b, m, tpb[i], block0, 0};
      block0 += m;
    }
  }
  const uint64_t n_blocks = block0;
  if ((e = grow(c, c->div_chunks, (size_t)n_chunks * sizeof(DivChunk))) ||
      (e = grow(c, c->div_blocks, (size_t)n_blocks * sizeof(DivBlock))) ||
      (e = grow(c, c->div_cnt, (size_t)n_chunks * 4)) || (e = grow(c, c->div_off, ((size_t)n_chunks + 1) * 8))) {
    divergence_result_free(r);
    return hip_fail(c, e, "device allocation");
  }
  DivChunk* d_chunks = (DivChunk*)c->div_chunks.p;
  uint64_t* d_off = (uint64_t*)c->div_off.p;
  if ((e = hipMemcpyAsync(d_chunks, hc, (size_t)n_chunks * sizeof(DivChunk), hipMemcpyHostToDevice, s)) ||
      (e = launch_divergence(d_chunks, n_chunks, d_arr, (DivBlock*)c->div_blocks.p, (uint32_t*)c->div_cnt.p, d_off,
                             d_off + n_chunks, s)) ||
      (e = hipMemcpyAsync(h_total, d_off + n_chunks, 8, hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s))) {
    divergence_result_free(r);
    return hip_fail(c, e, "divergence check");
  }
  const uint64_t n_div = *h_total;
  if (n_div > n_blocks) {
    divergence_result_free(r);
    return fail(c, SIM_EDEVICE, "divergent block count %llu exceeds the %llu blocks", (unsigned long long)n_div,
                (unsigned long long)n_blocks);
  }
  r->blocks = (sim_divergence*)malloc((n_div ? n_div : 1) * sizeof(sim_divergence));
  if (!r->blocks) {
    divergence_result_free(r);
    return fail(c, SIM_ENOMEM, "host allocation failed");
  }
  r->n_blocks = n_div;
  if (n_div) {
    if ((e = grow(c, c->div_out, (size_t)n_div * sizeof(DivOut))) ||
        (e = launch_divergence_emit(d_chunks, n_chunks, (const DivBlock*)c->div_blocks.p, d_off,
                                    (DivOut*)c->div_out.p, s)) ||
        (e = hipMemcpyAsync(r->blocks, c->div_out.p, (size_t)n_div * sizeof(DivOut), hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s))) {
      divergence_result_free(r);
      return hip_fail(c, e, "divergence output");
    }
  }
  *out = r;
  return SIM_OK;
}

}  // namespace

// ---- internal hooks for the serving runtime (serve.cpp)
namespace sc {

size_t ctx_device_bytes(const sim_ctx* c) {
  size_t t = 0;
  for (const DevBuf* b : all_bufs(const_cast<sim_ctx*>(c))) t += b->cap;
  return t;
}

// Release every device buffer of an idle context (they grow again on use).
void ctx_trim(sim_ctx* c) {
  DeviceGuard g(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : all_bufs(c)) release(*b);
  if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
  c->graph.exec = nullptr;
  c->alloc_gen++;
}

// Device bytes the context's buffers may hold from now on (0: no limit).  A
// call that would need more fails with SIM_ENOMEM.
void ctx_set_limit(sim_ctx* c, uint64_t bytes) { c->dev_limit = bytes; }

// Device bytes a call of this shape holds at most in an empty context with
// one-word (8) or two-word (16) keys and 9-bit digits: every fixed buffer
// with its growth headroom, the output's first allocation, and a staging
// overflow of `staged` entries with the output grown to `entries`.
uint64_t ctx_call_bytes(uint64_t total, uint32_t n_traces, uint32_t n_tiles, uint32_t key_bytes, uint64_t entries,
                        uint64_t staged) {
  size_t need[N_REGION];  // histogram groups: at most one per tile
  region_bytes(need, total, n_traces, n_tiles, n_tiles, key_bytes, RADIX_MAX);
  uint64_t t = 0;
  for (int r = 0; r < N_REGION; r++) t += grown(need[r]);
  const uint64_t cap0 = total < 65536 ? total : 65536;
  t += grown((entries > cap0 ? entries : cap0) * sizeof(RaceOut));
  if (staged) t += grown(staged * sizeof(RaceOut)) + grown((uint64_t)n_tiles * 8);
  return t;
}

// sim_check_traces_device for traces whose records lie anywhere in device
// memory: trace i's records start at trace_recs[i]; offsets are the call's
// CSR offsets as usual (they number the records of the call).
int ctx_check_gather(sim_ctx* c, const sim_record* const* trace_recs, const uint64_t* offsets, uint32_t n_traces,
                     const uint32_t* tpb, hipStream_t s, sim_result** out) {
  c->err.clear();
  DeviceGuard g(c->device);
  Sink sink;
  sink.out = out;
  return run(c, nullptr, trace_recs, offsets, n_traces, tpb, s, sink, false);
}

}  // namespace sc

extern "C" {

int sim_create(sim_ctx** out, int hip_device, const sim_config* cfg) {
  if (!out) return SIM_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return SIM_EDEVICE;
  if (hip_device < 0 || hip_device >= n) return SIM_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return SIM_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SIM_EDEVICE;
  sim_ctx* c = new (std::nothrow) sim_ctx();
  if (!c) return SIM_ENOMEM;
  c->device = hip_device;
  c->flags = cfg ? cfg->flags : 0;
  c->n_cu = prop.multiProcessorCount > 0 ? (uint32_t)prop.multiProcessorCount : 256u;
  DeviceGuard g(hip_device);
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void**)&c->h_ctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) {
    sim_destroy(c);
    return SIM_EDEVICE;
  }
  for (auto& ev : c->ev)
    if (hipEventCreate(&ev) != hipSuccess) {
      sim_destroy(c);
      return SIM_EDEVICE;
    }
  // the no-allocation entry point: this device's scratch address (looked up
  // once per device, with the device current), pinned tables for its
  // largest call, and room for error texts
  c->scratch_err = scratch_address(hip_device, &c->scratch);
  {
    const size_t hb = host_bytes(NOALLOC_MAX_TRACES, NOALLOC_MAX_TILES, NOALLOC_MAX_TILES);
    if (hipHostMalloc(&c->h_meta, hb, hipHostMallocDefault) != hipSuccess) {
      c->h_meta = nullptr;
      sim_destroy(c);
      return SIM_ENOMEM;
    }
    c->h_meta_cap = hb;
  }
  c->err.reserve(512);
  if (cfg && cfg->reserve_records) {  // every buffer of a call this large, allocated now
    const uint64_t n_rec = cfg->reserve_records;
    const uint32_t n_tr = cfg->reserve_traces ? cfg->reserve_traces : 1;
    const uint64_t tiles = (n_rec + TILE - 1) / TILE + n_tr;
    if (n_rec >= (1ull << 32) || tiles >= (1ull << 32) || ensure(c->records, n_rec * 16) ||
        size_buffers(c, n_rec, n_tr, (uint32_t)tiles, tiles, 8, RADIX_MAX) != hipSuccess) {
      sim_destroy(c);
      return SIM_ENOMEM;
    }
  }
  *out = c;
  return SIM_OK;
}

void sim_destroy(sim_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : all_bufs(c)) release(*b);
  if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
  if (c->h_meta) (void)hipHostFree(c->h_meta);
  if (c->h_div) (void)hipHostFree(c->h_div);
  if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
  for (auto& ev : c->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* sim_last_error(const sim_ctx* c) { return c ? c->err.c_str() : "no context"; }

int sim_check_traces_device(sim_ctx* c, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                            const uint32_t* threads_per_block, void* stream, sim_result** out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  DeviceGuard g(c->device);
  Sink sink;
  sink.out = out;
  return run(c, d_records, nullptr, offsets, n_traces, threads_per_block, (hipStream_t)stream, sink, false);
}

int sim_check_traces_device_noalloc(sim_ctx* c, const sim_record* d_records, const uint64_t* offsets,
                                    uint32_t n_traces, const uint32_t* threads_per_block, void* stream,
                                    sim_race* races, uint64_t races_cap, uint64_t* n_races,
                                    sim_trace_summary* traces) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (!n_races) return fail(c, SIM_EINVAL, "n_races is NULL");
  *n_races = 0;
  if (n_traces && !traces) return fail(c, SIM_EINVAL, "traces is NULL");
  if (races_cap && !races) return fail(c, SIM_EINVAL, "races is NULL with a nonzero capacity");
  DeviceGuard g(c->device);
  Sink sink;
  sink.races = races;
  sink.races_cap = races_cap;
  sink.n_races = n_races;
  sink.traces = traces;
  return run(c, d_records, nullptr, offsets, n_traces, threads_per_block, (hipStream_t)stream, sink, true);
}

int sim_check_traces(sim_ctx* c, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
                     const uint32_t* threads_per_block, sim_result** out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (out) *out = nullptr;
  DeviceGuard g(c->device);
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  int rc = validate(c, offsets, n_traces, threads_per_block, out, &total, &n_tiles);
  if (rc) return rc;
  if (total && !records) return fail(c, SIM_EINVAL, "records is NULL");
  if (total) {
    hipError_t e = ensure(c->records, total * sizeof(sim_record));
    if (e != hipSuccess) return hip_fail(c, e, "device allocation");
    e = hipMemcpyAsync(c->records.p, records, total * sizeof(sim_record), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "record upload");
  }
  Sink sink;
  sink.out = out;
  return run(c, (const sim_record*)c->records.p, nullptr, offsets, n_traces, threads_per_block, c->stream, sink,
             false);
}

int sim_check_traces_warp_device(sim_ctx* c, const sim_record* d_records, const uint32_t* d_side,
                                 const uint64_t* offsets, uint32_t n_traces, const uint32_t* threads_per_block,
                                 void* stream, sim_result** out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (out) *out = nullptr;
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  int rc = validate(c, offsets, n_traces, threads_per_block, out, &total, &n_tiles);
  if (rc) return rc;
  if (total && !d_side) return fail(c, SIM_EINVAL, "side is NULL");
  if (!total) {  // no records: the plain check's empty result
    Sink sink;
    sink.out = out;
    DeviceGuard g(c->device);
    return run(c, d_records, nullptr, offsets, n_traces, threads_per_block, (hipStream_t)stream, sink, false);
  }
  DeviceGuard g(c->device);
  Sink sink;
  sink.out = out;
  sink.side = d_side;
  return run(c, d_records, nullptr, offsets, n_traces, threads_per_block, (hipStream_t)stream, sink, false);
}

int sim_check_traces_warp(sim_ctx* c, const sim_record* records, const uint32_t* side, const uint64_t* offsets,
                          uint32_t n_traces, const uint32_t* threads_per_block, sim_result** out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (out) *out = nullptr;
  DeviceGuard g(c->device);
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  int rc = validate(c, offsets, n_traces, threads_per_block, out, &total, &n_tiles);
  if (rc) return rc;
  if (total && (!records || !side)) return fail(c, SIM_EINVAL, "records or side is NULL");
  if (total) {
    hipError_t e = ensure(c->records, total * sizeof(sim_record));
    if (e == hipSuccess) e = ensure(c->side, total * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(c, e, "device allocation");
    e = hipMemcpyAsync(c->records.p, records, total * sizeof(sim_record), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->side.p, side, total * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "record upload");
  }
  Sink sink;
  sink.out = out;
  sink.side = total ? (const uint32_t*)c->side.p : nullptr;
  return run(c, (const sim_record*)c->records.p, nullptr, offsets, n_traces, threads_per_block, c->stream, sink,
             false);
}

int sim_check_sync_device(sim_ctx* c, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                          const uint32_t* threads_per_block, void* stream, sim_result** races,
                          sim_barrier_result** barriers) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (barriers) *barriers = nullptr;
  if (!races) return fail(c, SIM_EINVAL, "races is NULL");
  DeviceGuard g(c->device);
  Sink sink;
  sink.out = races;
  sink.barriers = barriers;
  return run(c, d_records, nullptr, offsets, n_traces, threads_per_block, (hipStream_t)stream, sink, false);
}

int sim_check_sync(sim_ctx* c, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
                   const uint32_t* threads_per_block, sim_result** races, sim_barrier_result** barriers) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (races) *races = nullptr;
  if (barriers) *barriers = nullptr;
  DeviceGuard g(c->device);
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  int rc = validate(c, offsets, n_traces, threads_per_block, races, &total, &n_tiles);
  if (rc) return rc;
  if (total && !records) return fail(c, SIM_EINVAL, "records is NULL");
  if (total) {
    hipError_t e = ensure(c->records, total * sizeof(sim_record));
    if (e != hipSuccess) return hip_fail(c, e, "device allocation");
    e = hipMemcpyAsync(c->records.p, records, total * sizeof(sim_record), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "record upload");
  }
  Sink sink;
  sink.out = races;
  sink.barriers = barriers;
  return run(c, (const sim_record*)c->records.p, nullptr, offsets, n_traces, threads_per_block, c->stream, sink,
             false);
}

void sim_barrier_result_free(sim_barrier_result* r) { barrier_result_free(r); }

int sim_eval_fitness_device(sim_ctx* c, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                            const uint32_t* threads_per_block, void* stream, sim_fitness* out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (!out && n_traces) return fail(c, SIM_EINVAL, "out is NULL");
  DeviceGuard g(c->device);
  Sink sink;
  sink.fitness = out;
  sim_fitness dummy;
  if (!n_traces) sink.fitness = &dummy;
  return run(c, d_records, nullptr, offsets, n_traces, threads_per_block, (hipStream_t)stream, sink, false);
}

int sim_eval_fitness(sim_ctx* c, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
                     const uint32_t* threads_per_block, sim_fitness* out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (!out && n_traces) return fail(c, SIM_EINVAL, "out is NULL");
  DeviceGuard g(c->device);
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  sim_result* dummy_r = nullptr;
  int rc = validate(c, offsets, n_traces, threads_per_block, &dummy_r, &total, &n_tiles);
  if (rc) return rc;
  if (total && !records) return fail(c, SIM_EINVAL, "records is NULL");
  if (total) {
    hipError_t e = ensure(c->records, total * sizeof(sim_record));
    if (e != hipSuccess) return hip_fail(c, e, "device allocation");
    e = hipMemcpyAsync(c->records.p, records, total * sizeof(sim_record), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "record upload");
  }
  Sink sink;
  sink.fitness = out;
  sim_fitness dummy;
  if (!n_traces) sink.fitness = &dummy;
  return run(c, (const sim_record*)c->records.p, nullptr, offsets, n_traces, threads_per_block, c->stream, sink,
             false);
}

int sim_check_divergence_device(sim_ctx* c, const uint32_t* d_arrivals, const uint64_t* offsets, uint32_t n_traces,
                                const uint32_t* threads_per_block, void* stream, sim_divergence_result** out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  DeviceGuard g(c->device);
  return divergence(c, d_arrivals, offsets, n_traces, threads_per_block, (hipStream_t)stream, out);
}

int sim_check_divergence(sim_ctx* c, const uint32_t* arrivals, const uint64_t* offsets, uint32_t n_traces,
                         const uint32_t* threads_per_block, sim_divergence_result** out) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (out) *out = nullptr;
  if (!out) return fail(c, SIM_EINVAL, "out is NULL");
  DeviceGuard g(c->device);
  uint64_t total = 0;
  uint32_t n_chunks = 0;
  const int rc = div_tables(c, offsets, n_traces, threads_per_block, &total, &n_chunks);
  if (rc) return rc;
  if (total && !arrivals) return fail(c, SIM_EINVAL, "arrival counts are NULL");
  if (total) {
    hipError_t e = grow(c, c->div_in, total * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(c, e, "device allocation");
    e = hipMemcpyAsync(c->div_in.p, arrivals, total * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "arrival upload");
  }
  return divergence(c, (const uint32_t*)c->div_in.p, offsets, n_traces, threads_per_block, c->stream, out);
}

void sim_divergence_result_free(sim_divergence_result* r) { divergence_result_free(r); }

void sim_result_free(sim_result* r) {
  if (!r) return;
  if (!pool_give_back(r->races)) free(r->races);
  free(r->traces);
  free(r);
}

int sim_stage_times(const sim_ctx* c, sim_stage_time* out, int cap) {
  if (!c || !out) return 0;
  int n = cap < N_STAGE ? cap : N_STAGE;
  for (int i = 0; i < n; i++) out[i] = c->times[i];
  return n;
}

const char* sim_stage_name(int stage) { return (stage >= 0 && stage < N_STAGE) ? kStageNames[stage] : ""; }

uint32_t sim_size_class(uint64_t total_records) { return size_class(total_records); }

int sim_set_tuning(sim_ctx* c, uint32_t cls, const sim_tuning* t) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (cls >= SIM_SIZE_CLASSES) return fail(c, SIM_EINVAL, "size class %u out of range", cls);
  if (t && (t->stream_wgs_per_cu > 64 || t->sort_wgs_per_cu > 64 || t->scan_wgs_per_cu > 64 ||
            t->group_shift_bias < -12 || t->group_shift_bias > 12 ||
            (t->scatter_threads != 0 && t->scatter_threads != 256 && t->scatter_threads != 512) ||
            (t->digit_bits != 0 && t->digit_bits != RADIX_BITS && t->digit_bits != RADIX_WIDE_BITS)))
    return fail(c, SIM_EINVAL,
                "tuning out of range (workgroups per CU <= 64, |bias| <= 12, scatter threads 0, 256 or 512, "
                "digit bits 0, 8 or 9)");
  c->tuned[cls] = t != nullptr;
  c->tuning[cls] = t ? *t : sim_tuning{0, 0, 0, 0, 0, 0, 0.0};
  c->tuning_gen++;
  return SIM_OK;
}

int sim_get_tuning(const sim_ctx* c, uint32_t cls, sim_tuning* t) {
  if (!c || !t || cls >= SIM_SIZE_CLASSES) return SIM_EINVAL;
  *t = c->tuning[cls];
  return c->tuned[cls] ? 1 : 0;
}

int sim_autotune(sim_ctx* c, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                 const uint32_t* threads_per_block, void* stream, uint32_t reps, sim_tuning* best) {
  if (!c) return SIM_EINVAL;
  c->err.clear();
  if (!best) return fail(c, SIM_EINVAL, "best is NULL");
  DeviceGuard g(c->device);
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  sim_result* scratch = nullptr;
  int rc = validate(c, offsets, n_traces, threads_per_block, &scratch, &total, &n_tiles);
  if (rc) return rc;
  if (reps == 0) reps = 3;
  const uint32_t saved_flags = c->flags;
  c->flags &= ~(uint32_t)(SIM_CFG_GRAPHS | SIM_CFG_PROFILE);  // plain launches, timed on the host
  hipStream_t s = (hipStream_t)stream;
  // wall time of one complete call with shape t
  auto one_call = [&](const sim_tuning& t, double* ms) -> int {
    c->force = &t;
    sim_result* res = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    Sink sink;
    sink.out = &res;
    const int rc1 = run(c, d_records, nullptr, offsets, n_traces, threads_per_block, s, sink, false);
    const auto t1 = std::chrono::steady_clock::now();
    c->force = nullptr;
    sim_result_free(res);
    *ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return rc1;
  };
  // the fastest of `reps` calls of each shape, the two shapes' calls taking
  // turns (so that a drift of the GPU's speed during tuning, from clocks or
  // caches, reaches both alike); the work is deterministic: noise only adds
  // time
  auto measure_pair = [&](const sim_tuning& a, const sim_tuning& b2, double* ms_a, double* ms_b) -> int {
    *ms_a = *ms_b = 1e300;
    for (uint32_t r = 0; r < reps; r++) {
      double x = 0;
      int rc1 = one_call((r & 1) ? b2 : a, &x);
      if (rc1) return rc1;
      double& first = (r & 1) ? *ms_b : *ms_a;
      first = std::min(first, x);
      rc1 = one_call((r & 1) ? a : b2, &x);
      if (rc1) return rc1;
      double& second = (r & 1) ? *ms_a : *ms_b;
      second = std::min(second, x);
    }
    return SIM_OK;
  };
  sim_tuning cur{0, 0, 0, 0, 0, 0, 0.0};
  double cur_ms = 0;
  double warm = 0;
  rc = one_call(cur, &warm);  // buffers, pass count, digit width
  if (!rc) rc = one_call(cur, &warm);
  // short calls are noisier: at least 5 repetitions below 10 ms
  if (!rc && warm < 10.0 && reps < 5) reps = 5;
  // coordinate descent over the five knobs, one at a time
  static const uint32_t kWgs[] = {0, 1, 2, 4, 8};
  static const int32_t kBias[] = {-2, -1, 1, 2};
  for (int knob = 0; knob < 5 && !rc; knob++) {
    const int nval = knob == 3 ? 4 : (knob == 4 ? 1 : 5);
    const int32_t bias0 = cur.group_shift_bias;
    for (int q = 0; q < nval && !rc; q++) {
      sim_tuning t = cur;
      if (knob == 0) { if (t.sort_wgs_per_cu == kWgs[q]) continue; t.sort_wgs_per_cu = kWgs[q]; }
      if (knob == 1) { if (t.scan_wgs_per_cu == kWgs[q]) continue; t.scan_wgs_per_cu = kWgs[q]; }
      if (knob == 2) { if (t.stream_wgs_per_cu == kWgs[q]) continue; t.stream_wgs_per_cu = kWgs[q]; }
      if (knob == 3) t.group_shift_bias = bias0 + kBias[q];
      if (knob == 4) t.scatter_threads = scatter_threads(cur, n_tiles) == 512 ? 256 : 512;  // the other shape
      double ms = 0, base = 0;
      rc = measure_pair(cur, t, &base, &ms);
      if (!rc && ms < base * 0.995) {  // a shape must win beyond the noise to replace the current one
        cur = t;
        cur_ms = ms;
      } else if (!rc) {
        cur_ms = base;
      }
    }
  }
  c->flags = saved_flags;
  if (rc) return rc;
  cur.ms = cur_ms;
  const uint32_t cls = size_class(total);
  c->tuning[cls] = cur;
  c->tuned[cls] = true;
  c->tuning_gen++;
  *best = cur;
  return SIM_OK;
}

}  // extern "C"
