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
constexpr int GROUP = 256;         // tiles per group of the output prefix
constexpr uint32_t TAG_MAX = (1u << 24) - 1;
constexpr uint32_t REP_TILES = 256; // tiles sharing one histogram replica

// kernel-side error flags beyond the per-trace layout errors of keys.h
enum : uint32_t { ERR_STAGE_OVERFLOW = 16 };

struct TraceDesc {   // one trace of a call (host-filled)
  uint64_t off;      // first record
  uint64_t n;        // records
  uint32_t tpb;      // threads per block
  uint32_t tile0;    // first tile
  uint32_t ntiles;
  uint32_t rep0;     // first histogram replica
  uint32_t nrep;     // histogram replicas (ceil(ntiles / REP_TILES))
  uint32_t pad;
};

struct TileRef {     // tile -> (trace, tile within trace)
  uint32_t trace;
  uint32_t local;
};

struct TileOut {     // per tile, from the tile scan
  uint32_t in_count; // racing locations that start and end inside the tile
  uint32_t owns;     // 1: the tile's last location continues into the next tile
};

struct Ctrl {               // per-call control block (device)
  uint32_t max_passes;      // max radix passes over the call's traces
  uint32_t error_flags;     // LAYOUT_ERR_* / ERR_* of any trace or kernel
  uint64_t first_bad;       // smallest global index of an invalid record
  uint64_t total_entries;   // racing locations of the call
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
  TraceStats* stats_part;   // [tile]
  TraceLayout* layout;      // [trace]
  uint32_t* hist;           // [replica][MAX_PASSES][RADIX]; replica rep0 of a trace ends up holding digit bases
  uint64_t* keys[2];
  uint64_t* sort_status;    // [tile][RADIX]
  uint32_t* agg;            // [tile][SW]
  TileOut* tout;            // [tile]
  RaceOut* cross;           // [tile]
  uint32_t* cross_flag;     // [tile]
  uint32_t* group_sum;      // [group]
  uint64_t* group_off;      // [group]
  RaceOut* stage;           // dedicated staging ([tile][TILE/2 + 1]) or nullptr: the idle key buffer
  Ctrl* ctrl;
  RaceOut* out;
  uint64_t out_cap;
  uint32_t n_traces;
  uint32_t n_tiles;
  uint32_t n_reps;
  uint32_t sort_grid;       // co-resident workgroups of the cooperative radix pass
};

// Kernel stages, in launch order.
enum Stage { ST_INIT = 0, ST_STATS, ST_LAYOUT, ST_KEYGEN, ST_DIGITS, ST_SORT, ST_SCAN, ST_CROSS, ST_OUT, ST_COUNT };

hipError_t launch_init(const Buffers& b, hipStream_t s);
hipError_t launch_stats(const Buffers& b, hipStream_t s);
hipError_t launch_layout(const Buffers& b, hipStream_t s);
hipError_t launch_keygen(const Buffers& b, hipStream_t s);
hipError_t launch_digits(const Buffers& b, hipStream_t s);
hipError_t launch_sort_pass(const Buffers& b, uint32_t pass, uint32_t tag, hipStream_t s);
hipError_t launch_scan_tiles(const Buffers& b, uint32_t passes_done, hipStream_t s);
hipError_t launch_scan_cross(const Buffers& b, uint32_t passes_done, hipStream_t s);
hipError_t launch_scan_out(const Buffers& b, uint32_t passes_done, hipStream_t s);
hipError_t launch_reset_errors(const Buffers& b, uint32_t mask, hipStream_t s);
int sort_pass_blocks_per_cu();

}  // namespace sc
