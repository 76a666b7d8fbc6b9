// api.cpp -- host runtime behind the C ABI of include/simcheck.h.
//
// A context owns grow-only device buffers sized by the largest call seen so
// far, a default-priority stream for the host-record entry point, pinned
// host staging for the small per-call tables and the results, and the
// launch-tag counter that keeps look-back status words of different
// launches apart.  Every check runs as one ordered sequence of kernel
// launches on one stream followed by a single synchronisation; there is no
// CPU fallback.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/simcheck.h"
#include "launch.h"

using namespace sc;

static_assert(sizeof(sim_record) == 16, "sim_record is 16 bytes");
static_assert(sizeof(sim_race) == 64, "sim_race is 64 bytes");
static_assert(sizeof(RaceOut) == sizeof(sim_race), "device entry mirrors sim_race");
static_assert(sizeof(Summary) == sizeof(sim_trace_summary), "device summary mirrors sim_trace_summary");

namespace {

constexpr int N_STAGE = ST_COUNT;
const char* const kStageNames[N_STAGE] = {"init", "stats", "layout", "keygen", "digits", "sort_pass", "scan"};

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct sim_ctx {
  int device = 0;
  hipStream_t stream = nullptr;  // used by sim_check_traces
  uint32_t flags = 0;
  uint32_t tag = 0;
  std::string err;

  DevBuf records, keys0, keys1, desc, tiles, stats, layout, hist, sort_status, seg_status, cnt_status, ctrl, summary,
      out;
  void* h_meta = nullptr;  // pinned: TraceDesc[] then TileRef[]
  size_t h_meta_cap = 0;
  Ctrl* h_ctrl = nullptr;  // pinned

  hipEvent_t ev[2 * 16] = {};
  sim_stage_time times[N_STAGE] = {};
};

namespace {

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

// Grow a device buffer to at least `bytes` (contents are not kept).  Status
// buffers are zeroed so that no stale word carries a live tag.
hipError_t ensure(DevBuf& b, size_t bytes, bool zero = false) {
  if (bytes == 0) bytes = 64;
  if (b.cap >= bytes) return hipSuccess;
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

// Next launch tag; when the 24-bit space is used up the status buffers are
// cleared and numbering restarts.
hipError_t next_tag(sim_ctx* c, hipStream_t s, uint32_t* tag) {
  if (c->tag >= TAG_MAX) {
    for (DevBuf* b : {&c->sort_status, &c->seg_status, &c->cnt_status}) {
      if (b->p) {
        hipError_t e = hipMemsetAsync(b->p, 0, b->cap, s);
        if (e != hipSuccess) return e;
      }
    }
    c->tag = 0;
  }
  *tag = ++c->tag;
  return hipSuccess;
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
    const uint64_t n = offsets[i + 1] - offsets[i];
    if (n >= (1ull << 32)) return fail(c, SIM_EINVAL, "trace %u has 2^32 or more records", i);
    tiles += (n + TILE - 1) / TILE;
  }
  if (tiles >= (1ull << 31)) return fail(c, SIM_EINVAL, "too many records in one call");
  *total = n_traces ? offsets[n_traces] : 0;
  *n_tiles = (uint32_t)tiles;
  return SIM_OK;
}

sim_result* alloc_result(uint64_t n_races, uint32_t n_traces) {
  sim_result* r = (sim_result*)calloc(1, sizeof(sim_result));
  if (!r) return nullptr;
  r->n_races = n_races;
  r->n_traces = n_traces;
  r->races = (sim_race*)malloc(n_races ? n_races * sizeof(sim_race) : 1);
  r->traces = (sim_trace_summary*)malloc(n_traces ? n_traces * sizeof(sim_trace_summary) : 1);
  if (!r->races || !r->traces) {
    free(r->races);
    free(r->traces);
    free(r);
    return nullptr;
  }
  return r;
}

int run(sim_ctx* c, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces, const uint32_t* tpb,
        hipStream_t s, sim_result** out) {
  uint64_t total = 0;
  uint32_t n_tiles = 0;
  int rc = validate(c, offsets, n_traces, tpb, out, &total, &n_tiles);
  if (rc) return rc;
  if (total && !d_records) return fail(c, SIM_EINVAL, "records is NULL");
  for (auto& t : c->times) t = sim_stage_time{0.0, 0, 0};

  if (total == 0) {  // nothing to check: summaries only
    sim_result* r = alloc_result(0, n_traces);
    if (!r) return fail(c, SIM_ENOMEM, "host allocation failed");
    for (uint32_t i = 0; i < n_traces; i++) r->traces[i] = sim_trace_summary{0, 0, 0};
    *out = r;
    return SIM_OK;
  }

  // ---- buffers
  hipError_t e;
  const size_t meta_bytes = (size_t)n_traces * sizeof(TraceDesc) + (size_t)n_tiles * sizeof(TileRef);
  if (c->h_meta_cap < meta_bytes) {
    if (c->h_meta) (void)hipHostFree(c->h_meta);
    c->h_meta = nullptr;
    c->h_meta_cap = 0;
    e = hipHostMalloc(&c->h_meta, meta_bytes + meta_bytes / 8, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(c, e, "pinned allocation");
    c->h_meta_cap = meta_bytes + meta_bytes / 8;
  }
  const uint64_t cap0 = total < 65536 ? total : 65536;
  struct {
    DevBuf* b;
    size_t bytes;
    bool zero;
  } need[] = {
      {&c->keys0, total * 8, false},
      {&c->keys1, total * 8, false},
      {&c->desc, (size_t)n_traces * sizeof(TraceDesc), false},
      {&c->tiles, (size_t)n_tiles * sizeof(TileRef), false},
      {&c->stats, (size_t)n_traces * sizeof(TraceStats), false},
      {&c->layout, (size_t)n_traces * sizeof(TraceLayout), false},
      {&c->hist, (size_t)n_traces * MAX_PASSES * RADIX * 4, false},
      {&c->sort_status, (size_t)n_tiles * RADIX * 8, true},
      {&c->seg_status, (size_t)n_tiles * 2 * SW * 8, true},
      {&c->cnt_status, (size_t)n_tiles * 8, true},
      {&c->ctrl, sizeof(Ctrl), false},
      {&c->summary, (size_t)n_traces * sizeof(Summary), false},
      {&c->out, (size_t)(c->out.cap ? c->out.cap : cap0 * sizeof(RaceOut)), false},
  };
  for (auto& nb : need) {
    e = ensure(*nb.b, nb.bytes, nb.zero);
    if (e != hipSuccess) return hip_fail(c, e, "device allocation");
  }

  // ---- per-call tables
  TraceDesc* hd = (TraceDesc*)c->h_meta;
  TileRef* ht = (TileRef*)(hd + n_traces);
  uint32_t t0 = 0;
  for (uint32_t i = 0; i < n_traces; i++) {
    const uint64_t n = offsets[i + 1] - offsets[i];
    const uint32_t nt = (uint32_t)((n + TILE - 1) / TILE);
    hd[i] = TraceDesc{offsets[i], n, tpb[i], t0, nt, 0};
    for (uint32_t k = 0; k < nt; k++) ht[t0 + k] = TileRef{i, k};
    t0 += nt;
  }
  if ((e = hipMemcpyAsync(c->desc.p, hd, (size_t)n_traces * sizeof(TraceDesc), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(c->tiles.p, ht, (size_t)n_tiles * sizeof(TileRef), hipMemcpyHostToDevice, s)))
    return hip_fail(c, e, "table upload");

  Buffers b;
  b.records = d_records;
  b.desc = (const TraceDesc*)c->desc.p;
  b.tiles = (const TileRef*)c->tiles.p;
  b.stats = (TraceStats*)c->stats.p;
  b.layout = (TraceLayout*)c->layout.p;
  b.hist = (uint32_t*)c->hist.p;
  b.keys[0] = (uint64_t*)c->keys0.p;
  b.keys[1] = (uint64_t*)c->keys1.p;
  b.sort_status = (uint64_t*)c->sort_status.p;
  b.seg_status = (uint64_t*)c->seg_status.p;
  b.cnt_status = (uint64_t*)c->cnt_status.p;
  b.ctrl = (Ctrl*)c->ctrl.p;
  b.summary = (Summary*)c->summary.p;
  b.out = (RaceOut*)c->out.p;
  b.out_cap = c->out.cap / sizeof(RaceOut);
  b.n_traces = n_traces;
  b.n_tiles = n_tiles;

  const bool prof = (c->flags & SIM_CFG_PROFILE) != 0;
  int evn = 0;
  auto mark = [&]() -> hipError_t { return prof ? hipEventRecord(c->ev[evn++], s) : hipSuccess; };

  // ---- the pipeline (stage events: init, stats, layout, keygen, digits, pass 0..7, scan)
  uint32_t tags[MAX_PASSES + 1];
  for (uint32_t p = 0; p <= MAX_PASSES; p++)
    if ((e = next_tag(c, s, &tags[p]))) return hip_fail(c, e, "status reset");
  if ((e = mark()) || (e = launch_init(b, s)) || (e = mark()) || (e = launch_stats(b, s)) || (e = mark()) ||
      (e = launch_layout(b, s)) || (e = mark()) || (e = launch_keygen(b, s)) || (e = mark()) ||
      (e = launch_digits(b, s)) || (e = mark()))
    return hip_fail(c, e, "launch");
  for (uint32_t p = 0; p < MAX_PASSES; p++)
    if ((e = launch_sort_pass(b, p, tags[p], s)) || (e = mark())) return hip_fail(c, e, "launch");
  if ((e = launch_scan(b, tags[MAX_PASSES], s)) || (e = mark())) return hip_fail(c, e, "launch");
  if ((e = hipMemcpyAsync(c->h_ctrl, c->ctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(c, e, "pipeline");

  const Ctrl ctl = *c->h_ctrl;
  if (ctl.error_flags & LAYOUT_ERR_RECORD)
    return fail(c, SIM_ERECORD, "invalid record at index %llu (action > 2 or space > 1)",
                (unsigned long long)ctl.first_bad);
  if (ctl.error_flags & LAYOUT_ERR_WIDE) return fail(c, SIM_ERANGE, "a trace's sort key needs more than 64 bits");
  if (ctl.error_flags & (ERR_INTERNAL_BOUNDS | ERR_INTERNAL_SPIN))
    return fail(c, SIM_EDEVICE, "internal kernel check failed (flags 0x%x)", ctl.error_flags);

  if (prof) {
    const int stage_of_event[] = {ST_INIT, ST_STATS, ST_LAYOUT, ST_KEYGEN, ST_DIGITS};
    int k = 0;
    for (; k < 5; k++) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]);
      c->times[stage_of_event[k]].ms += ms;
      c->times[stage_of_event[k]].launches += 1;
    }
    for (uint32_t p = 0; p < MAX_PASSES; p++, k++) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]);
      c->times[ST_SORT].ms += ms;
      if (p < ctl.max_passes) c->times[ST_SORT].launches += 1;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]);
    c->times[ST_SCAN].ms += ms;
    c->times[ST_SCAN].launches += 1;
  }

  uint64_t n_races = ctl.total_entries;
  if (n_races > b.out_cap) {  // more racing locations than the output buffer holds: grow and rescan
    if ((e = ensure(c->out, n_races * sizeof(RaceOut)))) return hip_fail(c, e, "device allocation");
    b.out = (RaceOut*)c->out.p;
    b.out_cap = c->out.cap / sizeof(RaceOut);
    uint32_t tag;
    if ((e = next_tag(c, s, &tag)) || (e = launch_scan_reset(b, s)) || (e = launch_scan(b, tag, s)) ||
        (e = hipMemcpyAsync(c->h_ctrl, c->ctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
      return hip_fail(c, e, "rescan");
    n_races = c->h_ctrl->total_entries;
    if (c->h_ctrl->error_flags) return fail(c, SIM_EDEVICE, "internal kernel check failed on rescan");
    if (n_races > b.out_cap) return fail(c, SIM_EDEVICE, "entry count changed between scans");
  }

  sim_result* r = alloc_result(n_races, n_traces);
  if (!r) return fail(c, SIM_ENOMEM, "host allocation failed");
  if ((n_races && (e = hipMemcpyAsync(r->races, c->out.p, n_races * sizeof(sim_race), hipMemcpyDeviceToHost, s))) ||
      (e = hipMemcpyAsync(r->traces, c->summary.p, (size_t)n_traces * sizeof(sim_trace_summary),
                          hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s))) {
    sim_result_free(r);
    return hip_fail(c, e, "result download");
  }
  *out = r;
  return SIM_OK;
}

}  // namespace

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
  if (cfg && cfg->reserve_records) {
    const uint64_t n_rec = cfg->reserve_records;
    if (ensure(c->records, n_rec * 16) || ensure(c->keys0, n_rec * 8) || ensure(c->keys1, n_rec * 8)) {
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
  for (DevBuf* b : {&c->records, &c->keys0, &c->keys1, &c->desc, &c->tiles, &c->stats, &c->layout, &c->hist,
                    &c->sort_status, &c->seg_status, &c->cnt_status, &c->ctrl, &c->summary, &c->out})
    release(*b);
  if (c->h_meta) (void)hipHostFree(c->h_meta);
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
  return run(c, d_records, offsets, n_traces, threads_per_block, (hipStream_t)stream, out);
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
  return run(c, (const sim_record*)c->records.p, offsets, n_traces, threads_per_block, c->stream, out);
}

void sim_result_free(sim_result* r) {
  if (!r) return;
  free(r->races);
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

}  // extern "C"
