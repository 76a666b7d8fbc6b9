// launch.h -- device data structures and kernel launch wrappers of the race
// check, shared by the kernels (kernels.hip) and the host runtime (api.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "keys.h"
#include "tilewalk.h"

namespace sc {

constexpr int NT = 256;            // threads per workgroup
constexpr int ITEMS = 16;          // keys per thread
constexpr int TILE = NT * ITEMS;   // keys per tile (sort and scan)
constexpr int SW = 45;             // 32-bit words of a serialised segment State
constexpr int GROUP = 256;         // tiles per group of the output prefix
constexpr uint32_t MAX_HGROUP_SHIFT = 12; // histogram groups hold at most 4096 tiles

// kernel-side error flags beyond the per-trace layout errors of keys.h
enum : uint32_t { ERR_STAGE_OVERFLOW = 16, ERR_NEEDS_WIDE = 32 };

struct TraceDesc {   // one trace of a call (host-filled)
  uint64_t off;      // first record
  uint64_t n;        // records
  uint32_t tpb;      // threads per block
  uint32_t tile0;    // first tile
  uint32_t ntiles;
  uint32_t group0;   // first histogram group (runs of 2^gshift tiles of this trace)
  uint32_t ngroups;
  uint32_t gshift;   // log2 of the tiles per histogram group (about sqrt(ntiles))
  uint32_t pad[3];
};

struct TileRef {     // tile -> (trace, tile within trace), and where its records are
  uint32_t trace;
  uint32_t local;
  uint32_t first;    // call index of the tile's first record: its keys (a call holds < 2^32 records)
  uint32_t n_flags;  // records in the tile (bits 0..30); bit 31: the trace is sorted whole in LDS
  const void* rec;   // the tile's first record (device memory; the traces of a call need not be adjacent)
};
constexpr uint32_t TILE_SHORT = 1u << 31;

// Dedicated staging of a tile whose racing locations outgrow its slice of
// the idle key buffer: stage_ref[tile] = (first entry in `stage` <<
// STAGE_CAP_BITS) | capacity, or 0 for a tile that stages in its slice.
constexpr uint32_t STAGE_CAP_BITS = 16;
constexpr uint64_t STAGE_CAP_MASK = (1ull << STAGE_CAP_BITS) - 1;

struct GroupRef {    // histogram group -> trace, and its tiles
  uint32_t trace;
  uint32_t first;    // call index of the group's first tile
  uint32_t n_flags;  // tiles in the group (bits 0..30); bit 31 (TILE_SHORT): the trace is sorted whole in LDS
  uint32_t pad;
};

struct TileOut {     // per tile, from the tile scan
  uint32_t in_count; // racing locations that start and end inside the tile
  uint32_t owns;     // 1: the tile's last location continues into the next tile
};

struct Ctrl {               // per-call control block (device)
  uint32_t pass_bits;       // (most radix passes of a trace << 16) | the key bits that trace sorts
  uint32_t error_flags;     // LAYOUT_ERR_* / ERR_* of any trace or kernel
  uint64_t first_bad;       // smallest global index of an invalid record
  uint64_t total_entries;   // racing locations of the call
  uint32_t wide_traces;     // traces whose key needs two words
  uint32_t pad;
};
// Radix passes the call's traces need (all of them done: the scan may run).
SC_HD uint32_t ctrl_passes(uint32_t pass_bits) { return pass_bits >> 16; }

struct RaceOut {            // mirrors sim_race (64 bytes)
  uint32_t trace;
  uint8_t space, kinds;
  uint16_t reserved16;
  uint32_t block, reserved32;
  uint64_t unit, ww, rw, aw, ar, xb;
};

struct Buffers {            // device pointers of one call
  const TraceDesc* desc;
  const TileRef* tiles;
  TraceStats* stats_part;   // [tile]
  TraceLayout* layout;      // [trace]
  void* keys[2];             // uint64_t[] (one-word keys) or u128[] (two-word keys, `wide`)
  const GroupRef* groups;   // [group]
  uint32_t* thist;          // [tile][radix] the current pass's digit offsets within the tile's group
                            // (uint16_t when no group has more than 16 tiles, see kernels.hip)
  uint16_t* tcnt;           // [tile][radix] the current pass's digit counts (a tile holds 4096 keys)
  uint32_t* gtot;           // [group][radix] group totals
  uint64_t* gbase;          // [group][radix] absolute digit bases of the group
                            // (radix: 2^8 in pass 0, 2^digit_bits after it; rows of RADIX_MAX words at most)
  uint32_t* agg;            // [tile][SW]
  TileOut* tout;            // [tile]
  RaceOut* cross;           // [tile]
  uint32_t* cross_flag;     // [tile]
  uint32_t* group_sum;      // [group]
  RaceOut* stage;           // dedicated staging of the tiles stage_ref names (see STAGE_CAP_BITS)
  const uint64_t* stage_ref;// [tile], or nullptr: every tile stages in its slice of the idle key buffer
  Ctrl* ctrl;
  RaceOut* out;
  uint64_t out_cap;
  uint32_t n_traces;
  uint32_t n_tiles;
  uint32_t n_groups;        // histogram groups
  uint32_t grid_stream;     // workgroups of k_stats / k_keygen / k_upsweep (multiple of 8)
  uint32_t grid_sort;       // workgroups of k_scatter
  uint32_t scatter_nt;      // threads of a k_scatter workgroup: 256, or 512 (one-word keys)
  uint32_t grid_scan;       // workgroups of k_scan_tiles
  uint32_t max_group_tiles; // most tiles in one histogram group of the call
  uint32_t max_trace_groups;// most histogram groups in one trace of the call
  uint32_t fuse0;           // 1: digit 0 is tid mod 256 in every trace; k_stats builds its histograms
                            // and k_keygen_scatter does radix pass 0 (see kernels.hip)
  uint32_t wide;            // 1: two-word keys for every trace of the call
  const uint32_t* small_traces; // traces sorted whole in LDS: n_small1 of one tile, then
                            // n_small4 of two to four tiles (one-word keys only)
  uint32_t n_small1, n_small4;
  uint32_t small_max_tiles; // 4 with one-word keys, 1 with two-word keys
  uint32_t small_from;      // first radix pass done in LDS for those traces (pass 0 is
                            // k_keygen_scatter's when fuse0)
  uint32_t key_bytes;       // 8 or 16
  uint32_t fitness;         // 1: fitness keys (epoch and action dropped), for the EP fitness count
  const uint32_t* side;     // warp-aware check: one side word per record (call index), else nullptr
  uint32_t digit_bits;      // digit width of the radix passes after pass 0: RADIX_BITS or RADIX_WIDE_BITS
};

// Barrier instances (per trace and boundary) of the redundant-barrier check:
// `copies` copies of every counter pair, spread over cache lines, summed by
// the host.  Trace i's boundaries start at bar_base[i].
struct BarrierCount {
  unsigned long long instances;
  unsigned long long racing;
};

// Kernel stages, in launch order.
enum Stage { ST_INIT = 0, ST_STATS, ST_LAYOUT, ST_KEYGEN, ST_UPSWEEP, ST_SORT, ST_SCAN, ST_CROSS, ST_OUT,
             ST_SORT_SMALL, ST_COUNT };

hipError_t launch_init(const Buffers& b, hipStream_t s);
hipError_t launch_stats(const Buffers& b, hipStream_t s);
hipError_t launch_layout(const Buffers& b, hipStream_t s);
hipError_t launch_keygen(const Buffers& b, hipStream_t s);  // with fuse0: keys + radix pass 0
hipError_t launch_upsweep(const Buffers& b, uint32_t pass, hipStream_t s);  // histograms and offsets
hipError_t launch_scatter(const Buffers& b, uint32_t pass, hipStream_t s);
hipError_t launch_sort_small(const Buffers& b, hipStream_t s);
hipError_t launch_scan_tiles(const Buffers& b, uint32_t passes_done, hipStream_t s);
hipError_t launch_scan_cross(const Buffers& b, uint32_t passes_done, hipStream_t s);
hipError_t launch_scan_out(const Buffers& b, uint32_t passes_done, hipStream_t s);
hipError_t launch_reset_errors(const Buffers& b, uint32_t mask, hipStream_t s);
// Redundant-barrier check over the sorted keys of a finished call: clears
// `table` (n_counts entries) and counts every trace's barrier instances.
hipError_t launch_barriers(const Buffers& b, const uint64_t* bar_base, BarrierCount* table, uint64_t n_counts,
                           uint32_t copies, hipStream_t s);

// EP fitness of one trace (mirrors sim_fitness, 48 bytes).
struct FitOut {
  uint64_t n_records, n_locations, n_location_threads, global_range, shared_range;
  double fitness;
};
// Over the sorted fitness keys of a finished call: every trace's row to out
// (device memory, n_traces rows).  Does nothing while fewer than the needed
// radix passes ran (the host runs them and launches again).
hipError_t launch_fitness(const Buffers& b, uint32_t passes_done, FitOut* out, hipStream_t s);

// Barrier divergence (Alg. 4): whole blocks of one trace per chunk.
struct DivChunk {
  uint64_t thread0;  // the chunk's first thread (index into the arrival counts)
  uint32_t trace;
  uint32_t block;    // the chunk's first block within its trace
  uint32_t n_blocks;
  uint32_t tpb;      // threads per block
  uint32_t block0;   // the chunk's first block among the call's blocks (dense results)
  uint32_t pad;
};
struct DivBlock {    // one block: fewest and most arrivals, threads below the most
  uint32_t lo, hi, early, pad;
};
struct DivOut {      // mirrors sim_divergence (24 bytes)
  uint32_t trace, block, lo, hi;
  uint64_t early;
};
constexpr uint32_t DIV_CHUNK_THREADS = TILE;  // threads per chunk (whole blocks, at least one)

// Per-block results and per-chunk counts, then the chunks' output offsets
// and the number of divergent blocks (*total, device memory).
hipError_t launch_divergence(const DivChunk* chunks, uint32_t n_chunks, const uint32_t* arrivals, DivBlock* blocks,
                             uint32_t* chunk_cnt, uint64_t* chunk_off, uint64_t* total, hipStream_t s);
// The divergent blocks, in (trace, block) order, to out.
hipError_t launch_divergence_emit(const DivChunk* chunks, uint32_t n_chunks, const DivBlock* blocks,
                                  const uint64_t* chunk_off, DivOut* out, hipStream_t s);

// Warp-aware check (Theorem 1's warp clauses) after the plain check of a
// call whose keys carry the side field: the pairs lockstep execution
// orders are subtracted from the plain entries (n_entries of them, device
// memory, in key order; `removed` holds 4 counters per entry), and the
// entries left with a pair go to `out`, their number to *n_out (device).
hipError_t launch_warp_refine(const Buffers& b, const RaceOut* entries, uint64_t n_entries, unsigned long long* removed,
                              RaceOut* out, unsigned long long* n_out, hipStream_t s);

// Device memory of the no-allocation entry point: a file-scope array of
// SCRATCH_BYTES in the library's device code, one copy per GPU.
constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;
// The array's address on `device` (which must be the current device), looked
// up once per device and remembered; the error of that lookup otherwise.
hipError_t scratch_address(int device, void** out);

}  // namespace sc
