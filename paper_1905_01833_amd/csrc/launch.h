// launch.h -- device data structures and kernel launch wrappers of the race
// check, shared by the kernels (kernels.hip) and the host runtime (api.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "keys.h"

namespace sc {

constexpr int NT = 256;            // threads per workgroup
constexpr int ITEMS = 16;          // keys per thread
constexpr int TILE = NT * ITEMS;   // keys per tile (sort and scan)
constexpr int SW = 45;             // 32-bit words of a serialised segment State
constexpr uint32_t TAG_MAX = (1u << 24) - 1;

struct TraceDesc {   // one trace of a call (host-filled)
  uint64_t off;      // first record
  uint64_t n;        // records
  uint32_t tpb;      // threads per block
  uint32_t tile0;    // first tile
  uint32_t ntiles;
  uint32_t pad;
};

struct TileRef {     // tile -> (trace, tile within trace)
  uint32_t trace;
  uint32_t local;
};

struct Ctrl {               // per-call control block (device)
  uint32_t ticket[16];      // dynamic tile tickets: [p] sort pass p, [8] scan
  uint32_t max_passes;      // max radix passes over the call's traces
  uint32_t error_flags;     // LAYOUT_ERR_* of any trace
  uint64_t first_bad;       // smallest global index of an invalid record
  uint64_t total_entries;   // racing locations of the call
};

struct Summary {            // mirrors sim_trace_summary
  uint64_t n_records, n_race_locs, n_pairs;
};

struct RaceOut {            // mirrors sim_race (64 bytes)
  uint32_t trace;
  uint8_t space, kinds;
  uint16_t reserved16;
  uint32_t block, reserved32;
  uint64_t unit, ww, rw, aw, ar, xb;
};

struct Buffers {            // device pointers of one call
  const void* records;      // sim_record[n_total]
  const TraceDesc* desc;
  const TileRef* tiles;
  TraceStats* stats;
  TraceLayout* layout;
  uint32_t* hist;           // [trace][MAX_PASSES][RADIX]
  uint64_t* keys[2];
  uint64_t* sort_status;    // [tile][RADIX]
  uint64_t* seg_status;     // [tile][2][SW]
  uint64_t* cnt_status;     // [tile]
  Ctrl* ctrl;
  Summary* summary;
  RaceOut* out;
  uint64_t out_cap;
  uint32_t n_traces;
  uint32_t n_tiles;
};

// Kernel stages, in launch order.
enum Stage { ST_INIT = 0, ST_STATS, ST_LAYOUT, ST_KEYGEN, ST_DIGITS, ST_SORT, ST_SCAN, ST_COUNT };

hipError_t launch_init(const Buffers& b, hipStream_t s);
hipError_t launch_stats(const Buffers& b, hipStream_t s);
hipError_t launch_layout(const Buffers& b, hipStream_t s);
hipError_t launch_keygen(const Buffers& b, hipStream_t s);
hipError_t launch_digits(const Buffers& b, hipStream_t s);
hipError_t launch_sort_pass(const Buffers& b, uint32_t pass, uint32_t tag, hipStream_t s);
hipError_t launch_scan(const Buffers& b, uint32_t tag, hipStream_t s);
hipError_t launch_scan_reset(const Buffers& b, hipStream_t s);

}  // namespace sc
