// kernels.hip -- gfx950 kernels of the Memory-Model data-race check.
//
// Pipeline for a call over one or more traces (records of a trace are
// contiguous; kernels work on 4096-record tiles and a tile never spans two
// traces):
//   k_stats       per-call state reset (k_init instead for a call without
//                 records), per-tile unit ranges, largest tid and epoch,
//                 record checks (and the digit-0 histograms when digit 0 is
//                 tid mod 256)
//   k_layout      per-trace reduction of the tile statistics, key layout
//   k_keygen      records -> keys, tile histograms of radix digit 0;
//                 or k_keygen_scatter: records -> keys in their places after
//                 radix pass 0 (when k_stats built the digit-0 histograms)
//   k_upsweep     tile histograms of radix digit p (p >= 1)
//   k_group_offsets / k_trace_offsets  histograms -> scatter offsets
//   k_scatter     one stable LSD radix pass, 8-bit digits (x passes)
// Every tile kernel walks the call's (trace, tile) queue (tilewalk.h), one
// tile per workgroup or several per workgroup of a persistent grid.
//   k_scan_tiles  racing-pair counts of every location inside a tile, and
//                 the tile's summary for locations that cross tiles
//   k_scan_cross  pair counts of the locations that cross tiles
//   k_group_sums / k_scan_out  ordered output (two-level prefix over tiles;
//                 calls of at most 32 groups of 256 tiles skip k_group_sums)
//
// No kernel waits on another workgroup.  Radix offsets are computed
// reduce-then-scan style: every tile stores its digit histogram, two small
// kernels turn the histograms into offsets, and the scatter of a pass reads
// finished offsets.  Device-scope atomics that many workgroups aim at one
// address serialise (about 11 ns each on MI355X) and an agent-scope fence
// writes back the whole L2, so neither appears on a hot path: statistics are
// per-tile partials and hand-offs between workgroups go through kernel
// boundaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "barrier.h"
#include "launch.h"
#include "segstate.h"

namespace sc {

constexpr int NWAVE = NT / 64;
static_assert(NT == (int)RADIX, "one thread per digit in the radix kernels");
static_assert(GROUP == NT, "one thread per tile in the output kernels");
constexpr uint64_t SEGF = 1ull << 63;   // head flag of packed segmented values
constexpr uint32_t CLS_NONE = 3;        // padding element past the end of a trace

// ------------------------------------------------------------- utilities

// record fields from its two 64-bit halves (little-endian sim_record)
struct Rec {
  uint64_t unit;
  uint32_t tid, epoch, action, space;
};
__device__ __forceinline__ Rec unpack_rec(ulonglong2 v) {
  Rec r;
  r.unit = v.x;
  r.tid = (uint32_t)v.y;
  r.epoch = (uint32_t)(v.y >> 32) & 0xFFFFu;
  r.action = (uint32_t)(v.y >> 48) & 0xFFu;
  r.space = (uint32_t)(v.y >> 56);
  return r;
}


// Cross-lane moves of the wave's data-parallel primitives (DPP): the value
// of another lane, or 0 where that lane is outside the pattern or the row
// is masked off.  Row = 16 lanes.
enum : int {
  DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118,
  DPP_WAVE_SHR1 = 0x138,   // lane i gets lane i - 1
  DPP_ROW_BCAST15 = 0x142, // last lane of each row to the next row
  DPP_ROW_BCAST31 = 0x143  // lane 31 to rows 2 and 3
};
// (`old` instead of 0 where the source lane is outside the pattern.)
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t v, uint32_t old = 0u) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint64_t dpp(uint64_t v, uint64_t old = 0ull) {
  return ((uint64_t)dpp<CTRL, ROWS>((uint32_t)(v >> 32), (uint32_t)(old >> 32)) << 32) |
         dpp<CTRL, ROWS>((uint32_t)v, (uint32_t)old);
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ uint64_t readlane(uint64_t v, int lane) {
  return ((uint64_t)readlane((uint32_t)(v >> 32), lane) << 32) | readlane((uint32_t)v, lane);
}
__device__ __forceinline__ uint64_t readfirstlane(uint64_t v) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
}

// Reduction over the 64 lanes with an associative, commutative operator
// whose identity is `id`: the scan pattern below ends with the total in
// lane 63, which every lane then reads.
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, T id, Op op) {
  v = op(dpp<DPP_ROW_SHR1>(v, id), v);
  v = op(dpp<DPP_ROW_SHR2>(v, id), v);
  v = op(dpp<DPP_ROW_SHR4>(v, id), v);
  v = op(dpp<DPP_ROW_SHR8>(v, id), v);
  v = op(dpp<DPP_ROW_BCAST15, 0xa>(v, id), v);
  v = op(dpp<DPP_ROW_BCAST31, 0xc>(v, id), v);
  return readlane(v, 63);
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
  return wave_reduce(v, (T)~(T)0, [](T a, T b) { return a < b ? a : b; });
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  return wave_reduce(v, (T)0, [](T a, T b) { return a > b ? a : b; });
}

// Inclusive scan over the 64 lanes of a wave with an associative operator
// whose identity is 0: within rows (shifts 1, 2, 4, 8), then across rows
// (row 0's total into row 1 and row 2's into row 3, then lane 31's into
// rows 2 and 3).
template <typename T, typename Op>
__device__ __forceinline__ T wave_incl_scan(T v, Op op) {
  v = op(dpp<DPP_ROW_SHR1>(v), v);
  v = op(dpp<DPP_ROW_SHR2>(v), v);
  v = op(dpp<DPP_ROW_SHR4>(v), v);
  v = op(dpp<DPP_ROW_SHR8>(v), v);
  v = op(dpp<DPP_ROW_BCAST15, 0xa>(v), v);
  v = op(dpp<DPP_ROW_BCAST31, 0xc>(v), v);
  return v;
}

// Exclusive sum over a workgroup of NW waves; *total receives the sum of all
// values.  Every thread of the workgroup must call it (it holds barriers).
template <int NW>
__device__ uint32_t block_excl_sum_n(uint32_t v, uint32_t* lds /* NW */, uint32_t* total) {
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v, [](uint32_t a, uint32_t b) { return a + b; });
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; w++) {
    const uint32_t x = lds[w];
    if (w < (int)wave) pre += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* lds /* NWAVE */, uint32_t* total) {
  return block_excl_sum_n<NWAVE>(v, lds, total);
}

// Segmented exclusive scan over the workgroup of three packed words that
// share one head flag (SEGF in bit 63 of the first: the thread holds a
// head; the words then hold its sums after its last head).  The value a
// segmented scan gives thread t is flagged when some earlier thread h holds
// a head, and then sums the words of h .. t - 1, which is C(t) - C(h) for
// the plain exclusive prefix C of the words; otherwise it is C(t).  So one
// add scan per word, one max scan of (thread + 1) over the head holders and
// one look-up of C(h) in a table of the thread prefixes give it.
// v: the thread's words; ex: its exclusive values; tot: the workgroup's
// inclusive values (uniform); P: an [NT][3] table of LDS free for the call;
// C, H: the waves' totals.
struct HeadScanLds {
  uint64_t C[NWAVE][3];
  uint32_t H[NWAVE];
};
__device__ void block_head_scan3(const uint64_t (&v)[3], uint64_t (&ex)[3], uint64_t (&tot)[3], uint64_t (*P)[3],
                                 HeadScanLds& S) {
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6, tid = threadIdx.x;
  uint64_t c[3];
#pragma unroll
  for (int q = 0; q < 3; q++) c[q] = wave_incl_scan(v[q] & ~SEGF, [](uint64_t a, uint64_t b) { return a + b; });
  const uint32_t hinc = wave_incl_scan((v[0] & SEGF) ? tid + 1u : 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
  if (lane == 63) {
#pragma unroll
    for (int q = 0; q < 3; q++) S.C[wave][q] = c[q];
    S.H[wave] = hinc;
  }
#pragma unroll
  for (int q = 0; q < 3; q++) c[q] = dpp<DPP_WAVE_SHR1>(c[q]);
  uint32_t h = dpp<DPP_WAVE_SHR1>(hinc);
  __syncthreads();
  uint64_t call[3] = {0, 0, 0};
  uint32_t hall = 0;
#pragma unroll
  for (int w = 0; w < NWAVE; w++) {
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const uint64_t x = S.C[w][q];
      if (w < (int)wave) c[q] += x;
      call[q] += x;
    }
    const uint32_t xh = S.H[w];
    if (w < (int)wave) h = max(h, xh);
    hall = max(hall, xh);
  }
#pragma unroll
  for (int q = 0; q < 3; q++) P[tid][q] = c[q];
  __syncthreads();
  hall = (uint32_t)__builtin_amdgcn_readfirstlane((int)hall);
#pragma unroll
  for (int q = 0; q < 3; q++) {
    ex[q] = h ? ((c[q] - P[h - 1][q]) | SEGF) : c[q];
    tot[q] = readfirstlane(hall ? ((call[q] - P[hall - 1][q]) | SEGF) : call[q]);  // uniform
  }
  __syncthreads();
}

// Per 16-bit field maximum of two words of four fields.
__device__ __forceinline__ uint32_t max_u16x2(uint32_t a, uint32_t b) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_max(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint64_t max_u16x4(uint64_t a, uint64_t b) {
  return ((uint64_t)max_u16x2((uint32_t)(a >> 32), (uint32_t)(b >> 32)) << 32) | max_u16x2((uint32_t)a, (uint32_t)b);
}

// LDS of block_nested_scan: each thread's prefix before its last head per
// level, and the waves' totals.
struct NestedLds {
  uint64_t P[NT][4];
  uint64_t C[NWAVE];
  uint64_t H[NWAVE];
};

// The nested segmented scan of the tile scan's class counts, over the NT
// threads of a workgroup, in the value a segmented scan of the per-level
// aggregates (SEGF if the thread holds a head at level l or
// coarser) | (its counts after the last such head) gives.  The levels nest
// (a head at level l is one at every finer level too), so the segment of
// level l before thread t starts after the last head at level l or coarser
// of h, the last earlier thread that holds one: its counts are C(t) - P_l(h),
// with C the plain exclusive prefix of the counts and P_l(h) = C(h) + the
// counts of h's elements before that head (P_l(h) <= C(t) field by field:
// no borrows).  One plain add scan, one max scan of (thread + 1) per level
// in 16-bit fields, and one LDS look-up per level replace four segmented
// 64-bit scans.
// cnt: the thread's class counts (16-bit fields); snap[l]: its counts before
// its last head at level l or coarser; mn: its smallest head level.  ex: the
// exclusive value per level (SEGF: some earlier thread holds a head at that
// level or coarser); tot: the workgroup's inclusive value per level.
__device__ void block_nested_scan(uint64_t cnt, const uint64_t (&snap)[4], uint32_t mn, uint64_t (&ex)[4],
                                  uint64_t (&tot)[4], NestedLds& S) {
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6, tid = threadIdx.x;
  const uint64_t cinc = wave_incl_scan(cnt, [](uint64_t a, uint64_t b) { return a + b; });
  uint64_t hv = 0;
#pragma unroll
  for (int l = 0; l < 4; l++) hv |= mn <= (uint32_t)l ? (uint64_t)(tid + 1) << (16 * l) : 0ull;
  const uint64_t hinc = wave_incl_scan(hv, max_u16x4);
  if (lane == 63) {
    S.C[wave] = cinc;
    S.H[wave] = hinc;
  }
  uint64_t c = dpp<DPP_WAVE_SHR1>(cinc), h = dpp<DPP_WAVE_SHR1>(hinc);
  __syncthreads();
  uint64_t call = 0, hall = 0;
#pragma unroll
  for (int w = 0; w < NWAVE; w++) {
    const uint64_t xc = S.C[w], xh = S.H[w];
    if (w < (int)wave) {
      c += xc;
      h = max_u16x4(h, xh);
    }
    call += xc;
    hall = max_u16x4(hall, xh);
  }
#pragma unroll
  for (int l = 0; l < 4; l++) S.P[tid][l] = c + snap[l];
  __syncthreads();
#pragma unroll
  for (int l = 0; l < 4; l++) {
    const uint32_t hl = (uint32_t)(h >> (16 * l)) & 0xFFFFu;
    ex[l] = hl ? ((c - S.P[hl - 1][l]) | SEGF) : c;
    const uint32_t tl = (uint32_t)readfirstlane((uint32_t)(hall >> (16 * l)) & 0xFFFFu);
    tot[l] = readfirstlane(tl ? ((call - S.P[tl - 1][l]) | SEGF) : call);  // uniform
  }
  __syncthreads();
}

// --------------------------------------------------------------- k_init

// The call's control words start clear.  k_stats does this in its first
// workgroup (no kernel before k_layout reads them); k_init serves calls
// without tiles.
__device__ __forceinline__ void ctrl_reset(Ctrl* ctrl) {
  ctrl->pass_bits = 0;
  ctrl->error_flags = 0;
  ctrl->first_bad = ~0ull;
  ctrl->total_entries = 0;
  ctrl->wide_traces = 0;
}

__global__ void k_init(Ctrl* ctrl) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl_reset(ctrl);
}

// Add one digit per lane of the wave to an LDS histogram.  When every live
// lane holds the same digit (a skewed digit: the top key bits often take a
// handful of values) the first live lane adds the count once; otherwise
// each lane adds 1, which rarely conflicts for a spread digit.
__device__ __forceinline__ void wave_hist_add(uint32_t* h, uint32_t dg, bool valid) {
  const uint64_t live = __ballot(valid);
  if (!live) return;
  const uint32_t lead = (uint32_t)__ffsll((unsigned long long)live) - 1u;  // uniform
  const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)dg, (int)lead);
  if (__ballot(valid && dg == d0) == live) {
    if (__lane_id() == lead) atomicAdd(&h[d0], (uint32_t)__popcll(live));
  } else if (valid) {
    atomicAdd(&h[dg], 1u);
  }
}

// -------------------------------------------------------------- k_stats
// A tile's records, read through the pointer its table entry holds.  To the
// compiler that pointer is generic, so it would load through flat
// instructions, and a flat load also holds up every wait for an LDS
// operation.  Records are always in memory the GPU addresses as global, so
// they are read as global memory.
typedef uint64_t rec_words __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) rec_words* GRecords;
__device__ __forceinline__ GRecords global_records(const void* p) { return (GRecords)p; }
__device__ __forceinline__ ulonglong2 load_record(GRecords p, uint32_t j) {
  const rec_words v = p[j];
  return ulonglong2{v.x, v.y};
}

// Per-tile partial statistics; k_layout reduces them per trace.

// HIST: also the tile histogram of radix digit 0 for calls whose digit 0 is
// tid mod 256 (see k_keygen_scatter).
// NTH threads of TILE / NTH records each.
template <bool LOOP, bool HIST, int NTH = NT>
__global__ __launch_bounds__(NTH) void k_stats(const TileRef* __restrict__ tiles, uint32_t n_tiles,
                                               TraceStats* __restrict__ part, uint16_t* __restrict__ tcnt,
                                               Ctrl* ctrl, const uint32_t* __restrict__ side) {
  constexpr int IT = TILE / NTH, NW = NTH / 64;
  static_assert(NTH >= (int)RADIX, "one thread per histogram bin");
  __shared__ uint64_t s64[5][NW];
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl_reset(ctrl);
  __shared__ uint32_t s32[3][NW];
  __shared__ uint32_t h[RADIX];
  const TileWalk tw = tile_walk(n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    const TileRef tr = tiles[tile];
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = tr.n_flags & ~TILE_SHORT;
    const GRecords p = global_records(tr.rec);
    uint64_t gmin = ~0ull, gmax = 0, smin = ~0ull, smax = 0, bad = ~0ull;
    uint32_t mt = 0, me = 0, ms = 0;
    if (side)  // warp-aware check: the largest statement id sizes the key's side field
      for (uint32_t j = tx; j < n_in; j += NTH) ms = max(ms, side[tr.first + j] & ~SIDE_DIVERGED);
    if (HIST) {
      if (tx < RADIX) h[tx] = 0;
      __syncthreads();
    }
    // all loads first: every record of the thread in flight
    ulonglong2 vr[IT];
#pragma unroll
    for (int r = 0; r < IT; r++) vr[r] = tx + r * NTH < n_in ? load_record(p, tx + r * NTH) : ulonglong2{0ull, 0ull};
#pragma unroll
    for (int r = 0; r < IT; r++) {
      const uint32_t j = tx + r * NTH;
      const bool valid = j < n_in;
      const ulonglong2 v = vr[r];
      // tid mod 256: neighbouring records mostly belong to different threads,
      // so plain LDS atomics rarely conflict here
      if (HIST && valid) atomicAdd(&h[(uint32_t)v.y & (RADIX - 1)], 1u);
      if (valid) {
        const Rec x = unpack_rec(v);
        if (x.action > 2 || x.space > 1) {
          bad = min<uint64_t>(bad, start + j);
        } else {
          if (x.space == 0) {
            gmin = min(gmin, x.unit);
            gmax = max(gmax, x.unit);
          } else {
            smin = min(smin, x.unit);
            smax = max(smax, x.unit);
          }
          mt = max(mt, x.tid);
          me = max(me, x.epoch);
        }
      }
    }
    gmin = wave_min(gmin); smin = wave_min(smin); bad = wave_min(bad);
    gmax = wave_max(gmax); smax = wave_max(smax);
    mt = wave_max(mt); me = wave_max(me); ms = wave_max(ms);
    const uint32_t lane = tx & 63u, wave = tx >> 6;
    if (lane == 0) {
      s64[0][wave] = gmin; s64[1][wave] = gmax; s64[2][wave] = smin; s64[3][wave] = smax; s64[4][wave] = bad;
      s32[0][wave] = mt; s32[1][wave] = me; s32[2][wave] = ms;
    }
    __syncthreads();
    if (tx == 0) {
      for (int w = 1; w < NW; w++) {
        gmin = min(gmin, s64[0][w]); gmax = max(gmax, s64[1][w]);
        smin = min(smin, s64[2][w]); smax = max(smax, s64[3][w]);
        bad = min(bad, s64[4][w]);
        mt = max(mt, s32[0][w]); me = max(me, s32[1][w]); ms = max(ms, s32[2][w]);
      }
      TraceStats S;
      S.gmin = gmin; S.gmax = gmax; S.smin = smin; S.smax = smax; S.bad_index = bad;
      S.max_tid = mt; S.max_epoch = me; S.max_stmt = ms; S.pad = 0;
      part[tile] = S;
    }
    if (HIST && tx < RADIX) tcnt[(uint64_t)tile * RADIX + tx] = (uint16_t)h[tx];
  }
}

// ------------------------------------------------------------- k_layout
// One workgroup per trace: reduce the trace's tile statistics, derive the
// key layout.  Global atomics only on rare events (an error, a new maximum
// pass count).

// wide_call: the call runs with two-word keys.  Otherwise a trace whose key
// needs two words raises ERR_NEEDS_WIDE, which stops the call's later
// kernels; the host then runs the call again with two-word keys.
// NTH threads per trace: 256, or 1024 for calls of a few long traces (more
// partial loads in flight per trace; with thousands of traces the wider
// workgroups only cost launch capacity).
template <int NTH = NT>
__global__ __launch_bounds__(NTH) void k_layout(const TraceDesc* __restrict__ desc,
                                                const TraceStats* __restrict__ part, TraceLayout* lay, Ctrl* ctrl,
                                                uint32_t wide_call, uint32_t fitness, uint32_t warp,
                                                uint32_t digit_bits) {
  constexpr int NW = NTH / 64;
  __shared__ uint64_t s64[5][NW];
  __shared__ uint32_t s32[3][NW];
  const uint32_t t = blockIdx.x;
  const TraceDesc T = desc[t];
  TraceStats S;
  stats_init(S);
  for (uint32_t i = threadIdx.x; i < T.ntiles; i += NTH) {
    const TraceStats P = part[T.tile0 + i];
    S.gmin = min(S.gmin, P.gmin); S.gmax = max(S.gmax, P.gmax);
    S.smin = min(S.smin, P.smin); S.smax = max(S.smax, P.smax);
    S.bad_index = min(S.bad_index, P.bad_index);
    S.max_tid = max(S.max_tid, P.max_tid); S.max_epoch = max(S.max_epoch, P.max_epoch);
    S.max_stmt = max(S.max_stmt, P.max_stmt);
  }
  S.gmin = wave_min(S.gmin); S.smin = wave_min(S.smin); S.bad_index = wave_min(S.bad_index);
  S.gmax = wave_max(S.gmax); S.smax = wave_max(S.smax);
  S.max_tid = wave_max(S.max_tid); S.max_epoch = wave_max(S.max_epoch); S.max_stmt = wave_max(S.max_stmt);
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  if (lane == 0) {
    s64[0][wave] = S.gmin; s64[1][wave] = S.gmax; s64[2][wave] = S.smin; s64[3][wave] = S.smax;
    s64[4][wave] = S.bad_index; s32[0][wave] = S.max_tid; s32[1][wave] = S.max_epoch; s32[2][wave] = S.max_stmt;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < NW; w++) {
    S.gmin = min(S.gmin, s64[0][w]); S.gmax = max(S.gmax, s64[1][w]);
    S.smin = min(S.smin, s64[2][w]); S.smax = max(S.smax, s64[3][w]);
    S.bad_index = min(S.bad_index, s64[4][w]);
    S.max_tid = max(S.max_tid, s32[0][w]); S.max_epoch = max(S.max_epoch, s32[1][w]);
    S.max_stmt = max(S.max_stmt, s32[2][w]);
  }
  if (fitness) S.max_epoch = 0;  // fitness keys hold no epoch (and no action)
  TraceLayout L = make_layout(S, T.tpb, warp != 0, digit_bits);
  if (T.n == 0) {
    L.error = 0;
    L.npasses = 0;
  }
  if (L.wide && !L.error) {
    atomicAdd(&ctrl->wide_traces, 1u);
    if (!wide_call) {
      atomicOr(&ctrl->error_flags, ERR_NEEDS_WIDE);
      L.npasses = 0;
    }
  }
  lay[t] = L;
  if (L.error) {
    atomicOr(&ctrl->error_flags, L.error);
    if (L.error & LAYOUT_ERR_RECORD)
      atomicMin((unsigned long long*)&ctrl->first_bad, (unsigned long long)(T.off + S.bad_index));
  }
  // one atomic for the call's pass count and widest key (the host picks the
  // next call's digit width from it): with one digit width per call a
  // trace's passes grow with its sorted bits, so the largest packed word
  // holds the largest of each; traces without passes add nothing.  (The
  // workgroups of all traces run at once and mostly read zero here, so
  // each atomic on this one word costs the whole launch time.)
  const uint32_t pb = L.npasses ? (L.npasses << 16) | (L.key_bits - 2) : 0u;
  if (pb > __hip_atomic_load(&ctrl->pass_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(&ctrl->pass_bits, pb);
}

// A trace of at most b.small_max_tiles tiles is sorted whole in one
// workgroup's LDS (k_sort_small) from pass b.small_from on; the global pass
// kernels leave it alone.
__device__ __forceinline__ bool sorted_in_lds(const Buffers& b, const TraceDesc& T, uint32_t pass) {
  return T.ntiles <= b.small_max_tiles && pass >= b.small_from;
}

// ----------------------------------------------------- radix offsets
//
// Each tile stores the digit histogram of the current pass in tcnt[tile]
// (16-bit counts: half the bytes of the offsets they become).
// k_group_offsets turns the rows of each histogram group (2^gshift
// consecutive tiles of one trace, about sqrt(ntiles) of them) into
// exclusive offsets within the group, in thist, and stores the group totals;
// k_trace_offsets turns a trace's group totals into absolute bases (trace
// offset + digit base + earlier groups).  Separate launches make the
// previous kernel's stores visible to plain, cached loads; no workgroup
// waits on another.

constexpr uint32_t CHUNK = 16;   // rows loaded ahead in the serial offset loops

// In-group offsets are 16-bit when no group of the call has more than 16
// tiles (an offset then sums at most 15 tiles of 4096 keys): half the bytes
// of the rows k_group_offsets writes and k_scatter reads.
constexpr uint32_t THIST16_TILES = 65536u / TILE;
template <uint32_t R>
__device__ __forceinline__ uint32_t d_of() { return threadIdx.x % R; }  // the digit column of a thread
__device__ __forceinline__ bool thist16(const Buffers& b) { return b.max_group_tiles <= THIST16_TILES; }
constexpr int MAX_PARTS = 4;     // offset kernels: up to 4 row ranges per digit (1024 threads)

// Exclusive prefix over `n` rows (stride R, the pass's digit count) of one
// digit column, split over PARTS row ranges handled by the threads d,
// d + R, ... .  Returns the column total; rows are rewritten with `base` +
// prefix.  DIGIT_BASE: `base` is the trace's first record and every digit's
// column starts at base + (totals of the smaller digits) -- the digit bases
// of a radix pass -- computed here from the same reads.  s_sc holds one word
// per wave of the workgroup and s_base one 64-bit word per digit.  narrow
// (uniform): `out` holds 16-bit words instead (32-bit Out only).
template <int PARTS, bool DIGIT_BASE, uint32_t R, typename In, typename Out>
__device__ uint64_t column_prefix(const In* in, Out* out, uint32_t n, uint64_t base, uint64_t (*s_part)[R],
                                  uint32_t* s_sc = nullptr, uint64_t* s_base = nullptr, bool skip = false,
                                  bool narrow = false) {
  auto put = [&](uint32_t row, uint64_t v) {
    if (sizeof(Out) == 4 && narrow) ((uint16_t*)out)[(uint64_t)row * R + d_of<R>()] = (uint16_t)v;
    else out[(uint64_t)row * R + d_of<R>()] = (Out)v;
  };
  const uint32_t d = threadIdx.x % R, part = threadIdx.x / R;
  const uint32_t per = (n + PARTS - 1) / PARTS;
  const uint32_t r0 = min(n, part * per), r1 = min(n, r0 + per);
  // the first chunk stays in registers for the write loop (a range of at
  // most CHUNK rows is read once).  Row indices are clamped to the column's
  // last row (a column has at least one), so every load is issued without a
  // branch; rows past the range count zero.
  const uint32_t last = n ? n - 1 : 0;
  uint64_t first[CHUNK];
#pragma unroll
  for (uint32_t k = 0; k < CHUNK; k++) {
    const uint64_t v = in[(uint64_t)min(r0 + k, last) * R + d];
    first[k] = (r0 + k < r1) ? v : 0ull;
  }
  // skip (uniform over the workgroup): the column needs no offsets in this
  // pass; decided by the caller from loads that went out with these
  if (skip) return 0;
  uint64_t sum = 0;
#pragma unroll
  for (uint32_t k = 0; k < CHUNK; k++) sum += first[k];
  for (uint32_t k0 = r0 + CHUNK; k0 < r1; k0 += CHUNK) {
#pragma unroll
    for (uint32_t k = 0; k < CHUNK; k++) {
      const uint64_t v = in[(uint64_t)min(k0 + k, last) * R + d];
      sum += (k0 + k < r1) ? v : 0ull;
    }
  }
  s_part[part][d] = sum;
  __syncthreads();
  uint64_t total = 0, within = 0;
#pragma unroll
  for (int q = 0; q < PARTS; q++) {
    const uint64_t x = s_part[q][d];
    if (q < (int)part) within += x;
    total += x;
  }
  if (DIGIT_BASE) {
    // every thread takes part in the scan (it holds barriers); threads past
    // the first R contribute 0 and come after them
    uint32_t all;
    const uint32_t ex = block_excl_sum_n<PARTS * R / 64>(part == 0 ? (uint32_t)total : 0u, s_sc, &all);
    if (part == 0) s_base[d] = base + ex;
    __syncthreads();
    base = s_base[d];
  }
  uint64_t run = base + within;
#pragma unroll
  for (uint32_t k = 0; k < CHUNK; k++)
    if (r0 + k < r1) {
      put(r0 + k, run);
      run += first[k];
    }
  for (uint32_t k0 = r0 + CHUNK; k0 < r1; k0 += CHUNK) {
    uint64_t c[CHUNK];
#pragma unroll
    for (uint32_t k = 0; k < CHUNK; k++) {
      const uint64_t v = in[(uint64_t)min(k0 + k, last) * R + d];
      c[k] = (k0 + k < r1) ? v : 0ull;
    }
#pragma unroll
    for (uint32_t k = 0; k < CHUNK; k++)
      if (k0 + k < r1) {
        put(k0 + k, run);
        run += c[k];
      }
  }
  __syncthreads();
  return total;
}

// Row ranges per digit for a column of n rows: one range per CHUNK rows, at
// most MAX_PARTS (short columns need no more than one 256-thread workgroup),
// and at most 1024 threads with R digits.
SC_HD uint32_t offset_parts(uint32_t max_rows, uint32_t R) {
  const uint32_t p = max_rows <= CHUNK ? 1u : (max_rows <= 2 * CHUNK ? 2u : 4u);
  return p * R <= 1024u ? p : 1024u / R;
}

template <int PARTS, uint32_t R>
__global__ __launch_bounds__(R * PARTS) void k_group_offsets(Buffers b, uint32_t pass) {
  __shared__ uint64_t s_part[PARTS][R];
  const uint32_t g = blockIdx.x;
  // the group's rows are read together with the trace's pass count (one
  // round trip after the group reference); a group that needs no offsets in
  // this pass writes nothing
  const GroupRef gr = b.groups[g];
  const bool skip = pass >= b.layout[gr.trace].npasses || ((gr.n_flags & TILE_SHORT) && pass >= b.small_from);
  const uint16_t* counts = b.tcnt + (uint64_t)gr.first * R;
  const uint32_t rows = gr.n_flags & ~TILE_SHORT;
  uint32_t* offsets = b.thist + (uint64_t)gr.first * R;  // 32-bit rows, or 16-bit ones from the same start
  if (thist16(b)) offsets = (uint32_t*)((uint16_t*)b.thist + (uint64_t)gr.first * R);
  const uint64_t total = column_prefix<PARTS, false, R>(counts, offsets, rows, 0, s_part, nullptr, nullptr, skip,
                                                        thist16(b));
  if (skip) return;
  if (threadIdx.x < R) b.gtot[(uint64_t)g * R + threadIdx.x] = (uint32_t)total;
}

template <int PARTS, uint32_t R>
__global__ __launch_bounds__(R * PARTS) void k_trace_offsets(Buffers b, uint32_t pass) {
  __shared__ uint64_t s_part[PARTS][R];
  __shared__ uint64_t s_base[R];
  __shared__ uint32_t s_sc[PARTS * R / 64];
  const uint32_t t = blockIdx.x;
  const TraceDesc T = b.desc[t];
  if (pass >= b.layout[t].npasses || sorted_in_lds(b, T, pass)) return;  // uniform over the workgroup
  // group rows of the trace -> digit bases (from the column totals) and the
  // absolute base of every group (digit base + earlier groups)
  (void)column_prefix<PARTS, true, R>(b.gtot + (uint64_t)T.group0 * R, b.gbase + (uint64_t)T.group0 * R, T.ngroups,
                                       T.off, s_part, s_sc, s_base);
}


// ------------------------------------------------------------- k_keygen
// Records -> keys, and the tile histogram of radix digit 0.

template <typename K, bool LOOP>
__global__ __launch_bounds__(NT) void k_keygen(Buffers b) {
  __shared__ uint32_t h[RADIX];
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    const TileRef tr = b.tiles[tile];
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    if (L.npasses == 0) continue;
    const uint32_t keep = b.fitness ? 0u : ~0u;  // fitness keys: epoch and action dropped
    h[tx] = 0;
    __syncthreads();
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
    const GRecords p = global_records(tr.rec);
    K* kout = (K*)b.keys[0] + T.off + start;
    ulonglong2 vr[ITEMS];  // all loads first
#pragma unroll
    for (int r = 0; r < ITEMS; r++) vr[r] = tx + r * NT < n_in ? load_record(p, tx + r * NT) : ulonglong2{0ull, 0ull};
    // the block size's form is uniform over the tile: one branch, and each
    // side computes the block index one way
    auto keys_of = [&](auto blk_form) {
#pragma unroll
      for (int r = 0; r < ITEMS; r++) {
        const uint32_t j = tx + r * NT;
        const bool valid = j < n_in;
        K k = 0;
        if (valid) {
          const Rec x = unpack_rec(vr[r]);
          k = make_key_t<K, decltype(blk_form)::value>(L, x.unit, x.tid, x.epoch & keep, x.action & keep, x.space,
                                                        T.tpb, b.side ? b.side[tr.first + j] : 0u);
          kout[j] = k;
        }
        wave_hist_add(h, (uint32_t)(k >> 2) & (RADIX - 1), valid);
      }
    };
    if ((T.tpb & (T.tpb - 1)) == 0) keys_of(std::integral_constant<int, BLK_POW2>{});
    else keys_of(std::integral_constant<int, BLK_DIV>{});
    __syncthreads();
    b.tcnt[(uint64_t)tile * RADIX + tx] = (uint16_t)h[tx];
  }
}

// ------------------------------------------------------------ k_upsweep
constexpr int HIST_SPREAD = 8;

// Tile histogram of radix digit `pass` (keys in the buffer that pass reads),
// a digit of DB bits (the call's width; passes after the first).

template <typename K, bool LOOP, uint32_t DB>
__global__ __launch_bounds__(NT) void k_upsweep(Buffers b, uint32_t pass) {
  // HIST_SPREAD copies of every bin, one per group of lanes (lane mod
  // HIST_SPREAD): the lanes of one atomic instruction that share a digit
  // mostly hit different copies.  High digits often take a handful of
  // values, and with one copy their atomics serialised up to 64 deep.
  constexpr uint32_t R = 1u << DB, DPT = R / NT;  // digits per thread
  static_assert(R % NT == 0, "whole digits per thread");
  __shared__ uint32_t h[R * HIST_SPREAD];
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    // the tile reference locates the keys: their loads go out together
    // with the layout's, one round trip after it
    const TileRef tr = b.tiles[tile];
    const uint32_t n_in = tr.n_flags & ~TILE_SHORT;
    const K* src = (const K*)b.keys[pass & 1] + tr.first;
    K k[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
      const uint32_t j = tx + r * NT;
      k[r] = j < n_in ? src[j] : (K)0;
    }
    const uint32_t npasses = b.layout[tr.trace].npasses;
    if (pass >= npasses || ((tr.n_flags & TILE_SHORT) && pass >= b.small_from)) continue;
#pragma unroll
    for (uint32_t q = 0; q < HIST_SPREAD * DPT; q++) h[q * NT + tx] = 0;
    __syncthreads();
    const uint32_t shift = pass_shift(pass, DB);
    const uint32_t copy = tx & (HIST_SPREAD - 1);
#pragma unroll
    for (int r = 0; r < ITEMS; r++)
      if (tx + r * NT < n_in) atomicAdd(&h[((uint32_t)(k[r] >> shift) & (R - 1)) * HIST_SPREAD + copy], 1u);
    __syncthreads();
#pragma unroll
    for (uint32_t e = 0; e < DPT; e++) {
      const uint32_t d = e * NT + tx;
      uint32_t sum = 0;
#pragma unroll
      for (int q = 0; q < HIST_SPREAD; q++) sum += h[d * HIST_SPREAD + q];
      b.tcnt[(uint64_t)tile * R + d] = (uint16_t)sum;
    }
  }
}

// ------------------------------------------------------------ k_scatter
//
// One stable LSD pass on the digit of DB bits at bits [shift, shift + DB)
// (pass_shift).  Keys are loaded wave-striped (key index = wave * 64 * items
// + item * 64 + lane) so that lane order within an item is key order.  Each
// item's digit is matched across the wave with one ballot per digit bit;
// the lowest matching lane advances the wave's per-digit counter, which
// gives every key a stable rank within its wave.  Per-digit wave offsets,
// the tile's digit starts and the offsets left by the upsweep give each key
// its destination; keys are staged in LDS in destination order and written
// out in runs per digit.

// LDS of one scatter workgroup of NTH threads over 2^DB digits; per-wave
// digit counters of type C (16 bits suffice: a tile holds 4096 keys).
// Destinations are call indices, below 2^32: 32-bit digit bases.
template <typename K, int NTH, typename C, uint32_t DB>
struct ScatterLds {
  K keys[TILE];
  C wh[NTH / 64][1u << DB];
  uint32_t gbase[1u << DB];
  uint32_t scan[NTH / 64];
  uint32_t bad;  // some digit's destination range leaves the trace
};

// Counter type of a scatter workgroup: 32 bits for 256 threads over 8-bit
// digits, else 16 (the LDS of four workgroups per CU).
template <int NTH, uint32_t DB>
using ScatterCount = typename std::conditional<NTH == NT && DB == RADIX_BITS, uint32_t, uint16_t>::type;

// Lanes of the wave whose digit equals this lane's: one ballot per digit
// bit; a lane keeps the ballot where its own bit is set and the complement
// where it is clear.  The bit is taken as 0 or all ones (a signed one-bit
// field), so keeping is an XNOR with the ballot's halves.
template <uint32_t DB>
__device__ __forceinline__ uint64_t peer_mask(uint32_t dg) {
  uint32_t lo = ~0u, hi = ~0u;
#pragma unroll
  for (int bt = 0; bt < (int)DB; bt++) {
    const uint32_t all = (uint32_t)__builtin_amdgcn_sbfe((int)dg, bt, 1);  // 0 or ~0
    const uint64_t bal = __builtin_amdgcn_uicmp(all, 0u, 33);  // lanes whose bit is set (33: not equal)
    lo &= ~((uint32_t)bal ^ all);
    hi &= ~((uint32_t)(bal >> 32) ^ all);
  }
  return ((uint64_t)hi << 32) | lo;
}

// Stable rank of every key of the wave among the wave's keys of its digit
// (the DB bits at `shift`), items in order: the lowest lane of each group of
// equal digits advances the wave's counter wh[wave][digit] (zero on entry)
// by the group's size.  On return wh[wave][d] counts the wave's keys of
// digit d.
template <uint32_t DB, typename K, int IT, typename C>
__device__ __forceinline__ void wave_rank(const K (&key)[IT], uint32_t shift, uint32_t tx, C (*wh)[1u << DB],
                                          uint32_t (&rank)[IT]) {
  const uint32_t lane = tx & 63u, wave = tx >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < IT; i++) {
    const uint32_t dg = (uint32_t)(key[i] >> shift) & ((1u << DB) - 1);
    const uint64_t m = peer_mask<DB>(dg);
    const uint32_t before = (uint32_t)__popcll(m & lt_mask);
    const uint32_t old = wh[wave][dg];
    if (before == 0) wh[wave][dg] = (C)(old + (uint32_t)__popcll(m));
    rank[i] = old + before;
  }
}

// One stable pass over one tile: key[] holds the tile's keys wave-striped
// (key index = wave * 64 * items + item * 64 + lane; ~0 past the end, which
// sorts last); they go to their places in `kout`.  The per-digit steps give
// each thread DPT consecutive digits (threads past the last digit idle).
template <typename K, int NTH, typename C, uint32_t DB>
__device__ __forceinline__ void scatter_tile(const Buffers& b, uint32_t pass, uint32_t tile, uint32_t tx,
                                             const TileRef& tr, const TraceDesc& T, uint32_t n_in,
                                             K (&key)[TILE / NTH], K* kout, ScatterLds<K, NTH, C, DB>& S) {
  constexpr int IT = TILE / NTH, NW = NTH / 64;
  constexpr uint32_t R = 1u << DB, DPT = R >= (uint32_t)NTH ? R / NTH : 1u;
  const uint32_t wave = tx >> 6;
  const uint32_t d0 = tx * DPT;  // first digit of the per-digit steps
  const bool dig = d0 < R;
  const uint32_t shift = pass_shift(pass, DB);
  uint32_t rank[IT];
  wave_rank<DB>(key, shift, tx, S.wh, rank);
  // destination base of each digit: group base + offset within the group
  uint64_t gb[DPT];
  if (dig) {
    const uint64_t* grow = b.gbase + (uint64_t)(T.group0 + (tr.local >> T.gshift)) * R;
    const uint64_t row = (uint64_t)tile * R + d0;
    if (thist16(b)) {
      const uint16_t* trow = (const uint16_t*)b.thist + row;
#pragma unroll
      for (uint32_t e = 0; e < DPT; e++) gb[e] = grow[d0 + e] + trow[e];
    } else {
      const uint32_t* trow = b.thist + row;
#pragma unroll
      for (uint32_t e = 0; e < DPT; e++) gb[e] = grow[d0 + e] + trow[e];
    }
  }
  __syncthreads();

  // per digit: tile count, tile-local start, and each wave's first slot
  // (the digit's start + the counts of the earlier waves); only the thread
  // of digit d touches column d of S.wh, which holds the earlier waves'
  // count in between
  uint32_t cnt[DPT], csum = 0;
  if (dig) {
#pragma unroll
    for (uint32_t e = 0; e < DPT; e++) {
      uint32_t c = 0;
#pragma unroll
      for (int w = 0; w < NW; w++) {
        const uint32_t x = S.wh[w][d0 + e];
        S.wh[w][d0 + e] = (C)c;
        c += x;
      }
      cnt[e] = c;
      csum += c;
    }
  }
  if (tx == 0) S.bad = 0;
  uint32_t tot;
  uint32_t dstart = block_excl_sum_n<NW>(csum, S.scan, &tot);
  if (dig) {
    // (padding past the trace's end ranks last, in the digit of an all-ones
    // key: all ones, or fewer in the top pass of a 64- or 128-bit key)
    const uint32_t pad_digit = (uint32_t)(~(K)0 >> shift) & (R - 1);
#pragma unroll
    for (uint32_t e = 0; e < DPT; e++) {
      const uint32_t d = d0 + e;
#pragma unroll
      for (int w = 0; w < NW; w++) S.wh[w][d] = (C)(S.wh[w][d] + dstart);
      S.gbase[d] = (uint32_t)(gb[e] - dstart);
      // bounds, once per digit: the tile's keys of digit d go to [gb, gb + real)
      const uint32_t real = d == pad_digit ? cnt[e] - (uint32_t)(TILE - n_in) : cnt[e];
      if (real && (gb[e] < T.off || gb[e] + real > T.off + T.n)) S.bad = 1;
      dstart += cnt[e];
    }
  }
  __syncthreads();

#pragma unroll
  for (int i = 0; i < IT; i++) {
    const uint32_t dd = (uint32_t)(key[i] >> shift) & (R - 1);
    S.keys[S.wh[wave][dd] + rank[i]] = key[i];
  }
  __syncthreads();
  if (S.bad) {  // uniform: nothing of the tile is written
    if (tx == 0) atomicOr(&b.ctrl->error_flags, ERR_INTERNAL_BOUNDS);
    return;
  }
#pragma unroll 4
  for (int r = 0; r < IT; r++) {
    const uint32_t j = tx + r * NTH;
    if (j < n_in) {
      const K k = S.keys[j];
      kout[(uint32_t)(S.gbase[(uint32_t)(k >> shift) & (R - 1)] + j)] = k;  // a call index (< 2^32)
    }
  }
}

// NTH threads of TILE / NTH keys each: 256 x 16, or 512 x 8 (more waves per
// CU for the same LDS; one-word keys, chosen by the launch shape); digits of
// DB bits (8 in pass 0, the call's width after it).
template <typename K, bool LOOP, int NTH, uint32_t DB>
__global__ __launch_bounds__(NTH) void k_scatter(Buffers b, uint32_t pass) {
  constexpr int IT = TILE / NTH;
  using C = ScatterCount<NTH, DB>;
  __shared__ ScatterLds<K, NTH, C, DB> S;
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    // the tile reference locates the keys: their loads go out together
    // with the trace's descriptor and layout, one round trip after it
    const TileRef tr = b.tiles[tile];
    const uint32_t lane = tx & 63u, wave = tx >> 6;
    const uint32_t n_in = tr.n_flags & ~TILE_SHORT;
    const K* src = (const K*)b.keys[pass & 1] + tr.first;
    K key[IT];
#pragma unroll
    for (int i = 0; i < IT; i++) {
      const uint32_t j = wave * (IT * 64) + i * 64 + lane;
      key[i] = (j < n_in) ? src[j] : ~(K)0;  // padding sorts last (the largest digit, after every real key)
    }
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    if (pass >= L.npasses || sorted_in_lds(b, T, pass)) continue;  // uniform over the workgroup
    for (uint32_t k = tx; k < ((uint32_t)(NTH / 64) << DB); k += NTH) (&S.wh[0][0])[k] = 0;
    __syncthreads();
    scatter_tile<K, NTH, C, DB>(b, pass, tile, tx, tr, T, n_in, key, (K*)b.keys[(pass + 1) & 1], S);
  }
}

// ------------------------------------------------- k_keygen_scatter
// Key generation fused with radix pass 0, for calls whose digit 0 is the
// low byte of the thread id (threads per block a power of two >= 256, so
// bits [2, 10) of the key are tid mod 256): k_stats has built the tile
// histograms of that digit and the offset kernels have turned them into
// scatter offsets, so keys go straight from the records to their places
// after pass 0, in the buffer pass 1 reads.  The ranking is stable in record
// order (as k_scatter's, for any thread count), so the result is identical
// to k_keygen followed by k_scatter(pass 0).

template <typename K, bool LOOP, int NTH = NT>
__global__ __launch_bounds__(NTH) void k_keygen_scatter(Buffers b) {
  constexpr int IT = TILE / NTH;
  using C = ScatterCount<NTH, RADIX_BITS>;
  __shared__ ScatterLds<K, NTH, C, RADIX_BITS> S;
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    // the tile reference locates the records: their loads go out together
    // with the trace's descriptor and layout, one round trip after it
    const TileRef tr = b.tiles[tile];
    const uint32_t lane = tx & 63u, wave = tx >> 6;
    const uint32_t n_in = tr.n_flags & ~TILE_SHORT;
    const GRecords p = global_records(tr.rec);
    ulonglong2 vr[IT];  // all loads first: every record of the thread in flight
#pragma unroll
    for (int i = 0; i < IT; i++) {
      const uint32_t j = wave * (IT * 64) + i * 64 + lane;
      vr[i] = j < n_in ? load_record(p, j) : ulonglong2{0ull, 0ull};
    }
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    if (L.npasses == 0) continue;  // uniform over the workgroup
    for (uint32_t k = tx; k < (uint32_t)(NTH / 64 * RADIX); k += NTH) (&S.wh[0][0])[k] = 0;
    const uint32_t keep = b.fitness ? 0u : ~0u;  // fitness keys: epoch and action dropped
    K key[IT];
#pragma unroll
    for (int i = 0; i < IT; i++) {
      const uint32_t j = wave * (IT * 64) + i * 64 + lane;
      const Rec x = unpack_rec(vr[i]);
      key[i] = j < n_in ? make_key_t<K, BLK_POW2>(L, x.unit, x.tid, x.epoch & keep, x.action & keep, x.space, T.tpb)
                        : ~(K)0;
    }
    __syncthreads();
    scatter_tile<K, NTH, C, RADIX_BITS>(b, 0, tile, tx, tr, T, n_in, key, (K*)b.keys[1], S);
  }
}

// ------------------------------------------------------- k_sort_small
// A short trace (one tile, or up to four with one-word keys): the key bits
// from pass small_from's digit on, sorted all in LDS with 8-bit digits, one
// workgroup of NTH threads (16 keys each) per trace, with the same stable
// wave ranking as k_scatter (a stable LSD sort of the same bits gives the
// order of the global passes, whatever their digit width); the sorted keys
// go to the buffer the scan reads.  Padding past the trace's end holds
// all-ones keys, which rank after every real key in every pass.

template <typename K, int NTH>
struct SortLds {
  K keys[NTH * ITEMS];
  uint32_t wh[NTH / 64][RADIX];
  uint32_t scan[NTH / 64];
};

template <typename K, int NTH>
__global__ __launch_bounds__(NTH) void k_sort_small(Buffers b, const uint32_t* __restrict__ traces) {
  constexpr int NW = NTH / 64, CAP = NTH * ITEMS;
  __shared__ SortLds<K, NTH> S;
  const uint32_t tx = threadIdx.x, lane = tx & 63u, wave = tx >> 6;
  const uint32_t t = traces[blockIdx.x];
  const TraceDesc T = b.desc[t];
  const TraceLayout L = b.layout[t];
  if (L.npasses <= b.small_from || T.n > (uint64_t)CAP) return;  // uniform over the workgroup
  const uint32_t n_in = (uint32_t)T.n;
  const K* src = (const K*)b.keys[b.small_from & 1] + T.off;
  K key[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const uint32_t j = wave * (ITEMS * 64) + i * 64 + lane;
    key[i] = (j < n_in) ? src[j] : ~(K)0;
  }
  // pass small_from's first bit is 2 + 8 small_from whatever the call's
  // width (small_from is 0 or 1)
  const uint32_t n8 = radix_passes(L.key_bits - 2, RADIX_BITS);
  for (uint32_t pass = b.small_from; pass < n8; pass++) {
    const uint32_t shift = pass_shift(pass, RADIX_BITS);
    for (uint32_t k = tx; k < (uint32_t)(NW * RADIX); k += NTH) (&S.wh[0][0])[k] = 0;
    __syncthreads();
    uint32_t rank[ITEMS];
    wave_rank<RADIX_BITS>(key, shift, tx, S.wh, rank);
    __syncthreads();
    // thread d < 256: digit d's count, then each wave's first slot (the
    // digit's start + the counts of the earlier waves); only thread d
    // touches column d of S.wh
    uint32_t cnt = 0;
    if (tx < RADIX) {
      for (int w = 0; w < NW; w++) {
        const uint32_t c = S.wh[w][tx];
        S.wh[w][tx] = cnt;
        cnt += c;
      }
    }
    uint32_t tot;
    const uint32_t dstart = block_excl_sum_n<NW>(cnt, S.scan, &tot);
    if (tx < RADIX) {
      for (int w = 0; w < NW; w++) S.wh[w][tx] += dstart;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t dd = (uint32_t)(key[i] >> shift) & (RADIX - 1);
      S.keys[S.wh[wave][dd] + rank[i]] = key[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) key[i] = S.keys[wave * (ITEMS * 64) + i * 64 + lane];
    __syncthreads();  // S.wh and S.keys are reused by the next pass
  }
  K* dst = (K*)b.keys[L.npasses & 1u] + T.off;  // the real keys are the first n_in
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const uint32_t j = wave * (ITEMS * 64) + i * 64 + lane;
    if (j < n_in) dst[j] = key[i];
  }
}

// --------------------------------------------------------- k_scan_tiles
//
// Racing pairs per location over one tile of sorted keys, without any
// information from other tiles.  Thread t holds keys 16 t .. 16 t + 15.
//   A  segmented class counts per level (location, block, epoch, thread):
//      for every element, the counts of earlier elements of its open runs;
//   B  each element's pairs with earlier partners (segstate.h), summed per
//      location run.
// Locations that start and end in the tile are complete here and are
// staged for output.  The tile's summary (a State) is stored for
// k_scan_cross, which finishes the locations that cross tile boundaries.
// Counts inside a tile fit 16 bits and pair sums 32 bits.

// Two one-word keys, 8-byte aligned (a trace's keys start at any record).
typedef uint64_t u64x2_a8 __attribute__((ext_vector_type(2), aligned(8)));

// Per-item metadata of a thread's sixteen elements, packed: the head level
// (0..4) of item i in bits 3 i of a 64-bit word (levels), its class (0..3)
// in bits 2 i of a 32-bit word (classes).  The rolled loops walk them by
// shifting, one item per step; bits 48..50 of the levels word can carry
// the level of the element after the thread's last (see next_levels).
__device__ __forceinline__ uint32_t lv_of(uint64_t lvs, int i) { return (uint32_t)(lvs >> (3 * i)) & 7u; }
__device__ __forceinline__ uint32_t cls_of(uint32_t cls, int i) { return (cls >> (2 * i)) & 3u; }

__device__ __forceinline__ uint32_t cnt16(uint64_t packed, uint32_t q) { return (uint32_t)(packed >> (16 * q)) & 0xFFFFu; }

// A value uniform over the wave that the compiler may not look through
// (moved to scalar registers).
__device__ __forceinline__ void opaque_sgpr(uint64_t& v) {
  v = readfirstlane(v);
  asm volatile("" : "+s"(v));
}
__device__ __forceinline__ void opaque_sgpr(u128& v) {
  uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
  opaque_sgpr(lo);
  opaque_sgpr(hi);
  v = ((u128)hi << 64) | lo;
}

// Classes with a nonzero count among three 16-bit class fields (bits 0..47;
// nothing else set), as a 3-bit set; tested on the 32-bit halves.
__device__ __forceinline__ uint32_t class_set(uint64_t x) {
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  return ((lo & 0xFFFFu) ? 1u : 0u) | (lo > 0xFFFFu ? 2u : 0u) | (hi ? 4u : 0u);
}

// Three 8-bit class fields (read, write, atomic) to three 16-bit fields;
// the top field (padding) is dropped.
__device__ __forceinline__ uint64_t widen8(uint32_t x) {
  return (uint64_t)(x & 0xFFu) | ((uint64_t)(x & 0xFF00u) << 8) | ((uint64_t)(x & 0xFF0000u) << 16);
}

// Whether some item of a levels word has head level 0 (a location head):
// bit 3 i of the result is set where item i's level is 0.
__device__ __forceinline__ uint64_t loc_heads(uint64_t lvs) {
  return ~(lvs | (lvs >> 1) | (lvs >> 2)) & 0x249249249249ull;
}

// Pairs of one element of class c against the open-run counts run[] (the
// counts of earlier elements of its location / block / epoch / thread runs
// inside the tile, three 16-bit class fields per word).  The runs are
// nested, so the field-wise differences location - block and epoch - thread
// are plain 64-bit subtractions without borrows.
__device__ __forceinline__ void tile_pairs(uint32_t c, const uint64_t run[4], uint32_t v[5]) {
  const uint64_t xbp = run[0] - run[1];          // other blocks of the location
  const uint64_t tot = xbp + (run[2] - run[3]);  // + other threads of the block and epoch
  const uint32_t tR = (uint32_t)tot & 0xFFFFu, tW = (uint32_t)(tot >> 16) & 0xFFFFu;
  const uint32_t tA = (uint32_t)(tot >> 32) & 0xFFFFu;
  const uint32_t xR = (uint32_t)xbp & 0xFFFFu, xW = (uint32_t)(xbp >> 16) & 0xFFFFu;
  const uint32_t xA = (uint32_t)(xbp >> 32) & 0xFFFFu;
  const bool r = c == CLS_R, w = c == CLS_W, a = c == CLS_A;
  v[K_WW] = w ? tW : 0u;
  v[K_RW] = r ? tW : (w ? tR : 0u);
  v[K_AW] = w ? tA : (a ? tW : 0u);
  v[K_AR] = r ? tA : (a ? tR : 0u);
  v[K_XB] = (r ? 0u : xR) + xW + (a ? 0u : xA);
}

__device__ __forceinline__ uint32_t state_word(const State& s, int i) {
  if (i == 0) return s.m;
  if (i < 13) return s.lead[(i - 1) / 3][(i - 1) % 3];
  if (i < 25) return s.trail[(i - 13) / 3][(i - 13) % 3];
  if (i < 35) return (uint32_t)(s.leadsum[(i - 25) / 2] >> (32 * ((i - 25) % 2)));
  return (uint32_t)(s.trailsum[(i - 35) / 2] >> (32 * ((i - 35) % 2)));
}

__device__ __forceinline__ State load_state(const uint32_t* w) {
  State s;
  s.m = w[0];
#pragma unroll
  for (int l = 0; l < 4; l++)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      s.lead[l][q] = w[1 + l * 3 + q];
      s.trail[l][q] = w[13 + l * 3 + q];
    }
#pragma unroll
  for (int k = 0; k < 5; k++) {
    s.leadsum[k] = (uint64_t)w[25 + 2 * k] | ((uint64_t)w[26 + 2 * k] << 32);
    s.trailsum[k] = (uint64_t)w[35 + 2 * k] | ((uint64_t)w[36 + 2 * k] << 32);
  }
  return s;
}

template <typename K>
__device__ __forceinline__ void write_entry(RaceOut* dst, uint32_t trace, const TraceLayout& L, K key,
                                            const uint64_t S[5]) {
  RaceOut e;
  uint32_t sp, blk;
  uint64_t unit;
  key_location_t<K>(L, key, sp, blk, unit);
  e.trace = trace;
  e.space = (uint8_t)sp;
  e.kinds = (uint8_t)((S[K_WW] ? 1 : 0) | (S[K_RW] ? 2 : 0) | (S[K_AW] ? 4 : 0) | (S[K_AR] ? 8 : 0) |
                      (S[K_XB] ? 16 : 0));
  e.reserved16 = 0;
  e.block = blk;
  e.reserved32 = 0;
  e.unit = unit;
  e.ww = S[K_WW]; e.rw = S[K_RW]; e.aw = S[K_AW]; e.ar = S[K_AR]; e.xb = S[K_XB];
  *dst = e;
}

// Staging area of a tile's complete locations: the tile's slice of the key
// buffer that no longer holds live keys, or, for a tile whose locations
// outgrew that slice in an earlier scan of the call, its own range of the
// dedicated buffer (sized by the host from that scan's counts).
__device__ __forceinline__ RaceOut* stage_of(const Buffers& b, uint32_t tile, const TraceDesc& T,
                                             const TraceLayout& L, uint64_t start, uint32_t n_in, uint32_t* cap) {
  if (b.stage_ref) {
    const uint64_t ref = b.stage_ref[tile];
    if (ref & STAGE_CAP_MASK) {
      *cap = (uint32_t)(ref & STAGE_CAP_MASK);
      return b.stage + (ref >> STAGE_CAP_BITS);
    }
  }
  *cap = n_in * b.key_bytes / (uint32_t)sizeof(RaceOut);
  return (RaceOut*)((char*)b.keys[(L.npasses & 1u) ^ 1u] + (T.off + start) * b.key_bytes);
}

// Occupancy of the tile scan: with no LDS copy of the tile its registers
// alone set the waves per SIMD.  The one-tile kernels ask for 8 waves with
// one-word keys (64 VGPRs, no spill) and 5 with two-word keys; the looping
// variants keep their natural counts.
template <typename K, bool LOOP>
constexpr int scan_min_waves() { return LOOP ? 1 : (sizeof(K) == 8 ? 8 : 5); }

template <typename K, bool LOOP>
__global__ __launch_bounds__(NT, (scan_min_waves<K, LOOP>())) void k_scan_tiles(Buffers b, uint32_t passes_done) {
  __shared__ NestedLds s_nest;
  __shared__ HeadScanLds s_scanB;
  __shared__ uint32_t s_scan32[NWAVE];
  __shared__ uint8_t s_firstlv[NT];
  __shared__ uint32_t s_lead[17];  // lead counts [l][c] (12), lead pair sums (5)
  __shared__ uint32_t s_taillast;
  __shared__ uint32_t s_hit;  // some thread of the tile has an element with an in-tile racing partner
  __shared__ uint64_t s_pend[NT][3];  // sums of the location a thread's first element belongs to, when it is emitted there

  // nothing to do on an error, or when fewer radix passes ran than some
  // trace needs (the host then runs the missing passes and scans again)
  if (b.ctrl->error_flags) return;
  if (ctrl_passes(b.ctrl->pass_bits) > passes_done) return;
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    const uint32_t tid = tx, lane = tx & 63u, wave = tx >> 6;
    if (tid < 17) s_lead[tid] = 0;
    if (tid == 0) s_hit = 0;
    const TileRef tr = b.tiles[tile];
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    const K* keys = (const K*)b.keys[L.npasses & 1u];
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
    const K* src = keys + T.off + start;
    const bool trace_end = start + n_in == T.n;

    // each thread's sixteen consecutive keys come straight from memory
    // (with the key before them), with no LDS copy of the tile: the
    // kernel's LDS stays under 15 KiB, so registers alone bound occupancy.
    // Indices past the tile's end are clamped to its last key (a tile holds
    // at least one), so every load is issued without a branch; those items
    // are padding below.
    const uint32_t j0 = ITEMS * tid, jl = n_in - 1;
    K kk[ITEMS];
    if (sizeof(K) == 8 && n_in == (uint32_t)TILE) {
      // a whole tile of one-word keys: two keys per load (a lane's sixteen
      // keys are one 128-byte line, so each load instruction touches 64
      // lines whatever its width; half the instructions, half the touches)
      const u64x2_a8* p2 = (const u64x2_a8*)(src + j0);
#pragma unroll
      for (int i = 0; i < ITEMS / 2; i++) {
        const u64x2_a8 v = p2[i];
        kk[2 * i] = (K)v.x;
        kk[2 * i + 1] = (K)v.y;
      }
    } else {
      // a partial tile: items past its end repeat its last key with the
      // action bits set to the padding class; they differ from the key before
      // them below the thread field only, so they start no run
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const K v = src[min(j0 + (uint32_t)i, jl)];
        kk[i] = j0 + (uint32_t)i < n_in ? v : (v | (K)CLS_NONE);
      }
    }
    // the key before the thread's first (the previous tile's last for
    // thread 0; not read at a trace's first key)
    const K prev0 = src[(j0 == 0 && tr.local == 0) ? 0 : (int64_t)min(j0, n_in) - 1];
    K prev = (j0 == 0 && tr.local == 0) ? (K)0 : prev0;
    if (tid == 0) {  // whether the tile's last location ends with the tile
      const K next = trace_end ? (K)0 : src[n_in];
      s_taillast = trace_end ? 1u : (head_level_t<K>(L, src[n_in - 1], next) == 0 ? 1u : 0u);
    }

    // ---- element metadata and pass A, in one loop.  Metadata: head level
    //      (3 bits) and class (2 bits) of item i, in the words lvs and cls.
    //      The head level comes from four threshold tests on the bits where
    //      the key differs from its predecessor (keys.h: a location, block,
    //      epoch or thread field differs; the thresholds are the fields'
    //      lowest bits, the location's being the block's for shared keys),
    //      and those tests, "a head at level l or coarser", also drive pass
    //      A.  Pass A: segmented class counts per level, inside the thread as
    //      8-bit fields of one word (a thread holds 16 elements): the running
    //      count, and per level its value before the thread's last head at
    //      that level or coarser, both widened to the 16-bit fields of the
    //      block scan (their difference is the thread's aggregate).
    uint64_t lvs = 0;
    uint32_t cls = 0;
    uint64_t cntA, snapA[4];  // the thread's class counts, and before its last head per level (16-bit fields)
    uint32_t mn = NO_HEAD;  // the thread's smallest head level
    {
      const bool trace_first = j0 == 0 && tr.local == 0;  // item 0 is the trace's first key
      // the thresholds stay opaque: compared as they are, not rewritten as
      // shifts of the difference
      HeadThresholds<K> hth = head_thresholds_t<K>(L);
      opaque_sgpr(hth.thread);
      opaque_sgpr(hth.space);
      opaque_sgpr(hth.unit_g);
      opaque_sgpr(hth.block);
      opaque_sgpr(hth.epoch);
      uint32_t cnt = 0, snap[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const K k = kk[i];
        const bool first = i == 0 && trace_first;
        const HeadTests<K> ht = head_tests_t<K>(hth, prev, k);
        const bool h0 = first || ht.h[0];
        const bool h1 = first || ht.h[1];
        const bool h2 = first || ht.h[2];
        const bool h3 = first || ht.h[3];
        const uint32_t lv = h0 ? 0u : h1 ? 1u : h2 ? 2u : h3 ? 3u : 4u;
        const uint32_t c = action_class(k);  // padding: CLS_NONE
        snap[0] = h0 ? cnt : snap[0];
        snap[1] = h1 ? cnt : snap[1];
        snap[2] = h2 ? cnt : snap[2];
        snap[3] = h3 ? cnt : snap[3];
        cnt += 1u << (8 * c);  // padding (class 3) counts in the unused top field
        mn = min(mn, lv);
        lvs |= (uint64_t)lv << (3 * i);
        cls |= c << (2 * i);
        prev = k;
      }
      // the snapshots are formed here, not kept as per-item conditions
      // across the block scan
#pragma unroll
      for (int l = 0; l < 4; l++) asm volatile("" : "+v"(snap[l]));
      cntA = widen8(cnt);
#pragma unroll
      for (int l = 0; l < 4; l++) snapA[l] = widen8(snap[l]);
    }
    s_firstlv[tid] = (uint8_t)(lvs & 7u);

    // the packed metadata is decoded again per pass, not kept decoded
    asm volatile("" : "+v"(lvs));
    asm volatile("" : "+v"(cls));
    uint64_t exA[4], totA[4];
    block_nested_scan(cntA, snapA, mn, exA, totA, s_nest);

    // ---- pass B, test: whether an element of this thread has a racing
    //      partner among the earlier elements of its location in the tile.
    //      The counts an element's pairs are drawn from are (location run -
    //      block run) + (epoch run - thread run); both differences change
    //      only at heads, and only which classes they hold matters here, so
    //      the thread keeps them as 3-bit class sets (d01, d23) beside the
    //      class sets of the open location and epoch runs (r0, r2).  Most
    //      threads find nothing and skip the pair sums below.
    uint32_t hit = 0;
    {
      uint32_t r0 = class_set(exA[0] & ~SEGF), r2 = class_set(exA[2] & ~SEGF);
      uint32_t d01 = class_set((exA[0] & ~SEGF) - (exA[1] & ~SEGF));
      uint32_t d23 = class_set((exA[2] & ~SEGF) - (exA[3] & ~SEGF));
#pragma unroll
      for (int i = 0; i < ITEMS; i++) {
        const uint32_t lv = lv_of(lvs, i), c = cls_of(cls, i);
        // selects, not branches (branches here cost registers)
        const bool z0 = lv == 0, z1 = lv == 1, z2 = lv <= 2, z3 = lv == 3;
        d01 = z0 ? 0u : (z1 ? r0 : d01);
        r0 = z0 ? 0u : r0;
        d23 = z2 ? 0u : (z3 ? r2 : d23);
        r2 = z2 ? 0u : r2;
        // conflicting classes: a read's are writes and atomics (110b), a
        // write's all three (111b), an atomic's reads and writes (011b);
        // padding (class 3) has none and adds none (both from 4-bit tables)
        const uint32_t c4 = 4 * c;
        hit |= (d01 | d23) & ((0x376u >> c4) & 7u);
        const uint32_t bit = (0x0421u >> c4) & 7u;
        r0 |= bit;
        r2 |= bit;
      }
    }
    // ---- lead counts: per level, the class counts of the tile's elements
    //      before its first head at that level or coarser.  The thread that
    //      holds that head adds the counts carried into it (exA) and those of
    //      its own elements before the head; a level without a head in the
    //      tile takes the tile's totals (in the summary).  The pair sums of
    //      those elements are added by the pair pass below: only threads
    //      with an in-tile racing partner have any.  The thread's own
    //      counts come from masks, not a walk: per class a mask of its
    //      items (bit 2 i), per level a mask of the items with a head at
    //      that level or coarser (bit 3 i, from the level's bits: 0, at most
    //      1, at most 2, at most 3 of 0..4), and bit counts below the first
    //      such head.
    {
      const uint32_t cx = cls, cy = cls >> 1;  // padding (class 3) is in no mask
      const uint32_t mR = ~(cx | cy) & 0x55555555u, mW = cx & ~cy & 0x55555555u, mA = ~cx & cy & 0x55555555u;
      const uint64_t M = 0x249249249249ull;
      const uint64_t f0 = lvs & M, f1 = (lvs >> 1) & M, f2 = (lvs >> 2) & M;
      const uint64_t le[4] = {~(f0 | f1 | f2) & M, ~(f1 | f2) & M, ~f2 & ~(f1 & f0) & M, ~f2 & M};
#pragma unroll
      for (int l = 0; l < 4; l++) {
        if ((exA[l] & SEGF) == 0 && mn <= (uint32_t)l) {  // mn <= l: le[l] has a bit
          const uint32_t p = (uint32_t)__builtin_ctzll(le[l]) / 3;  // the first such head
          const uint32_t below = (1u << (2 * p)) - 1u;
          s_lead[l * 3 + CLS_R] = cnt16(exA[l], CLS_R) + __builtin_popcount(mR & below);
          s_lead[l * 3 + CLS_W] = cnt16(exA[l], CLS_W) + __builtin_popcount(mW & below);
          s_lead[l * 3 + CLS_A] = cnt16(exA[l], CLS_A) + __builtin_popcount(mA & below);
        }
      }
    }
    if (hit) s_hit = 1u;
    __syncthreads();  // s_hit and s_lead are complete after it
    const bool tile_hit = s_hit != 0;

    // ---- pass B, sums (tiles with a racing pair only): pairs per element,
    //      summed per location run.  Locations that end in this thread are
    //      counted here when they also start in it; the thread's first
    //      location (it may start in an earlier thread) is settled after the
    //      scan.
    uint64_t exB[3] = {0, 0, 0}, totB[3] = {0, 0, 0};
    uint32_t n_emit = 0;      // complete locations emitted by this thread
    bool pend_emit = false;   // one of them is its first location (sums in s_pend)
    // the levels word with the level of the element after the thread's last
    // in bits 48..50 (the next thread's first), and where the tile ends in
    // this thread, 0 or 4 after its last element by whether the location
    // ends with the tile: an element ends its location where the next
    // level is 0
    auto next_levels = [&]() {
      uint64_t x = lvs | ((uint64_t)(tid + 1 < (uint32_t)NT ? s_firstlv[tid + 1] : 4u) << 48);
      const uint32_t tail_i = n_in - 1 - ITEMS * tid;  // the tile's last element, when it is this thread's
      if (tail_i < (uint32_t)ITEMS) {
        const uint32_t sh = 3 * (tail_i + 1);
        x = (x & ~(7ull << sh)) | ((uint64_t)(s_taillast ? 0u : 4u) << sh);
      }
      return x;
    };
    if (tile_hit) {  // uniform over the workgroup
      uint64_t aggB[3] = {0, 0, 0};
      bool pend = false;
      uint64_t pend0 = 0, pend1 = 0, pend2 = 0;
      uint32_t leads[5] = {0u, 0u, 0u, 0u, 0u};
      if (hit) {
        uint64_t run[4];
#pragma unroll
        for (int l = 0; l < 4; l++) run[l] = exA[l] & ~SEGF;
        bool lead = (exA[0] & SEGF) == 0;  // before the tile's first location head
        uint64_t lw = next_levels();
        uint32_t cw_ = cls;
#pragma unroll 1
        for (uint32_t i = 0; i < (uint32_t)ITEMS; i++) {
          const uint32_t lv = (uint32_t)lw & 7u, c = cw_ & 3u;
          lw >>= 3;
          cw_ >>= 2;
#pragma unroll
          for (int l = 0; l < 4; l++)
            if (lv <= (uint32_t)l) run[l] = 0;
          if (c == CLS_NONE) continue;
          uint32_t v[5];
          tile_pairs(c, run, v);
          if (lv == 0) lead = false;
          if (lead) {
#pragma unroll
            for (int k = 0; k < 5; k++) leads[k] += v[k];
          }
          if (lv == 0) aggB[0] = aggB[1] = aggB[2] = SEGF;
          aggB[0] += (uint64_t)v[K_WW] | ((uint64_t)v[K_RW] << 32);
          aggB[1] += (uint64_t)v[K_AW] | ((uint64_t)v[K_AR] << 32);
          aggB[2] += (uint64_t)v[K_XB];
#pragma unroll
          for (int l = 0; l < 4; l++) run[l] += 1ull << (16 * c);
          if (((uint32_t)lw & 7u) != 0) continue;  // the location does not end here
          if (aggB[0] & SEGF) {  // the location started in this thread
            if (((aggB[0] | aggB[1]) & ~SEGF) != 0) {
              // the first such location's sums and last element wait in
              // LDS (the nested scan's table is free by now) for the output
              if (n_emit == 0) {
                s_nest.P[tid][0] = aggB[0] & ~SEGF;
                s_nest.P[tid][1] = aggB[1] & ~SEGF;
                s_nest.P[tid][2] = (aggB[2] & ~SEGF) | ((uint64_t)i << 48);
              }
              n_emit++;
            }
          } else {
            pend = true;
            pend0 = aggB[0];
            pend1 = aggB[1];
            pend2 = aggB[2];
          }
        }
      } else if (ITEMS * tid < n_in) {
        // every pair sum of this thread is zero: only its location heads
        // and whether its first location ends in it matter
        if (loc_heads(lvs)) {
          aggB[0] = aggB[1] = aggB[2] = SEGF;
          pend = (lvs & 7u) != 0;  // the first location ends before the thread's first head
        } else {
          const uint32_t jl = min(ITEMS * tid + (uint32_t)ITEMS, n_in) - 1;  // last element of the thread
          pend = jl + 1 == n_in ? s_taillast != 0 : s_firstlv[tid + 1] == 0;
        }
      }
      // the lead pair sums: one sum per wave, added by one lane (a lane
      // per thread would make the atomics a loop over the wave's lanes)
      if (__builtin_amdgcn_ballot_w64((leads[0] | leads[1] | leads[2] | leads[3] | leads[4]) != 0)) {
#pragma unroll
        for (int k = 0; k < 5; k++) {
          const uint32_t t = wave_reduce(leads[k], 0u, [](uint32_t a, uint32_t b) { return a + b; });
          if (lane == 0 && t) atomicAdd(&s_lead[12 + k], t);
        }
      }
      block_head_scan3(aggB, exB, totB, s_pend, s_scanB);  // s_pend is free until after it
      // the thread's first location: complete here only if it started in
      // the tile (a location head in an earlier thread); otherwise it belongs
      // to an earlier tile and is finished by k_scan_cross
      if (pend && (exB[0] & SEGF)) {
        const uint64_t f0 = (exB[0] & ~SEGF) + pend0, f1 = (exB[1] & ~SEGF) + pend1;
        if ((f0 | f1) != 0) {
          s_pend[tid][0] = f0;
          s_pend[tid][1] = f1;
          s_pend[tid][2] = (exB[2] & ~SEGF) + pend2;
          pend_emit = true;
          n_emit++;
        }
      }
    }

    // ---- the tile summary (lanes of wave 0 write its words)
    if (wave == 0) {
      State agg;
      // the smallest head level of the tile: the coarsest level whose
      // scan total carries a head flag (every tile holds an element, so
      // the level is at most 4)
      agg.m = (totA[0] & SEGF) ? 0u : (totA[1] & SEGF) ? 1u : (totA[2] & SEGF) ? 2u : (totA[3] & SEGF) ? 3u : 4u;
#pragma unroll
      for (int l = 0; l < 4; l++)
#pragma unroll
        for (int q = 0; q < 3; q++) {
          agg.lead[l][q] = (totA[l] & SEGF) ? s_lead[l * 3 + q] : cnt16(totA[l], q);
          agg.trail[l][q] = cnt16(totA[l], q);
        }
#pragma unroll
      for (int k = 0; k < 5; k++) agg.leadsum[k] = s_lead[12 + k];
      if (agg.m == 0) {
        agg.trailsum[K_WW] = (uint32_t)totB[0];
        agg.trailsum[K_RW] = (uint32_t)(totB[0] >> 32) & 0x7FFFFFFFu;
        agg.trailsum[K_AW] = (uint32_t)totB[1];
        agg.trailsum[K_AR] = (uint32_t)(totB[1] >> 32) & 0x7FFFFFFFu;
        agg.trailsum[K_XB] = (uint32_t)totB[2];
      } else {
#pragma unroll
        for (int k = 0; k < 5; k++) agg.trailsum[k] = 0;
      }
      uint32_t w = 0;
#pragma unroll
      for (int i = 0; i < SW; i++)
        if ((int)lane == i) w = state_word(agg, i);
      if (lane < (uint32_t)SW) b.agg[(uint64_t)tile * SW + lane] = w;
      if (lane == 0) b.tout[tile].owns = (agg.m == 0 && !s_taillast) ? 1u : 0u;
    }

    // ---- complete locations: started after the tile's first location head
    //      and ended inside the tile, written by the thread holding their
    //      last element.  This walk recomputes a thread's sums element by
    //      element; it serves only the rare thread with more than one
    //      complete location of its own (the others write from the sums the
    //      pair pass kept, below).
    auto walk_emit = [&](RaceOut* dst, uint32_t cap, uint32_t pos) {
      uint64_t run[4];
#pragma unroll
      for (int l = 0; l < 4; l++) run[l] = exA[l] & ~SEGF;
      uint64_t s0 = exB[0] & ~SEGF, s1 = exB[1] & ~SEGF, s2 = exB[2] & ~SEGF;
      bool seen0 = (exB[0] & SEGF) != 0;
      uint64_t lw = next_levels();
      uint32_t cw_ = cls;
#pragma unroll 1
      for (uint32_t i = 0; i < (uint32_t)ITEMS; i++) {
        const uint32_t lv = (uint32_t)lw & 7u, c = cw_ & 3u;
        lw >>= 3;
        cw_ >>= 2;
#pragma unroll
        for (int l = 0; l < 4; l++)
          if (lv <= (uint32_t)l) run[l] = 0;
        if (c == CLS_NONE) continue;
        if (lv == 0) {
          s0 = s1 = s2 = 0;
          seen0 = true;
        }
        uint32_t v[5];
        tile_pairs(c, run, v);
        s0 += (uint64_t)v[K_WW] | ((uint64_t)v[K_RW] << 32);
        s1 += (uint64_t)v[K_AW] | ((uint64_t)v[K_AR] << 32);
        s2 += (uint64_t)v[K_XB];
#pragma unroll
        for (int l = 0; l < 4; l++) run[l] += 1ull << (16 * c);
        if (!seen0) continue;  // the location entering the tile belongs to an earlier tile
        if (((uint32_t)lw & 7u) != 0) continue;  // the location does not end here
        uint64_t S[5];
        S[K_WW] = (uint32_t)s0; S[K_RW] = (uint32_t)(s0 >> 32);
        S[K_AW] = (uint32_t)s1; S[K_AR] = (uint32_t)(s1 >> 32);
        S[K_XB] = (uint32_t)s2;
        if (S[K_WW] + S[K_RW] + S[K_AW] + S[K_AR] == 0) continue;
        if (pos < cap) write_entry<K>(dst + pos, tr.trace, L, src[ITEMS * tid + i], S);
        pos++;
      }
    };
    uint32_t tile_emit;
    const uint32_t my_off = block_excl_sum(n_emit, s_scan32, &tile_emit);
    uint32_t cap;
    RaceOut* stage = stage_of(b, tile, T, L, start, n_in, &cap);
    // a thread with at most one complete location besides its first writes
    // them from the sums kept above; one with more walks its elements again
    if (n_emit) {
      const uint32_t own = n_emit - (pend_emit ? 1u : 0u);
      if (own <= 1) {
        uint32_t pos = my_off;
        auto put = [&](uint64_t s0, uint64_t s1, uint64_t s2, uint32_t i) {
          uint64_t S[5];
          S[K_WW] = (uint32_t)s0; S[K_RW] = (uint32_t)(s0 >> 32);
          S[K_AW] = (uint32_t)s1; S[K_AR] = (uint32_t)(s1 >> 32);
          S[K_XB] = (uint32_t)s2;
          if (pos < cap) write_entry<K>(stage + pos, tr.trace, L, src[ITEMS * tid + i], S);
          pos++;
        };
        if (pend_emit) put(s_pend[tid][0], s_pend[tid][1], s_pend[tid][2], 0);
        if (own) put(s_nest.P[tid][0], s_nest.P[tid][1], s_nest.P[tid][2], (uint32_t)(s_nest.P[tid][2] >> 48));
      } else {
        walk_emit(stage, cap, my_off);
      }
    }
    if (tid == 0) {
      b.tout[tile].in_count = tile_emit;
      if (tile_emit > cap) atomicOr(&b.ctrl->error_flags, ERR_STAGE_OVERFLOW);
    }
  }
}

// --------------------------------------------------------- k_scan_cross
//
// A location that starts in tile j and continues into later tiles is
// finished here.  It covers tile j's trailing run, the following tiles
// without a location head, and the part of the next tile before its first
// head (or it runs to the end of the trace).  One wave per owning tile
// combines the tile summaries in order: 64 lanes hold one summary each and
// reduce them as a tree, chunk by chunk.

__device__ __forceinline__ State shfl_down_state(const State& s, uint32_t dlt) {
  State r;
  r.m = __shfl_down(s.m, dlt, 64);
#pragma unroll
  for (int l = 0; l < 4; l++)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      r.lead[l][q] = __shfl_down(s.lead[l][q], dlt, 64);
      r.trail[l][q] = __shfl_down(s.trail[l][q], dlt, 64);
    }
#pragma unroll
  for (int k = 0; k < 5; k++) {
    r.leadsum[k] = __shfl_down(s.leadsum[k], dlt, 64);
    r.trailsum[k] = __shfl_down(s.trailsum[k], dlt, 64);
  }
  return r;
}

__device__ __forceinline__ State readlane_state(const State& s, int src) {
  State r;
  r.m = __shfl(s.m, src, 64);
#pragma unroll
  for (int l = 0; l < 4; l++)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      r.lead[l][q] = __shfl(s.lead[l][q], src, 64);
      r.trail[l][q] = __shfl(s.trail[l][q], src, 64);
    }
#pragma unroll
  for (int k = 0; k < 5; k++) {
    r.leadsum[k] = __shfl(s.leadsum[k], src, 64);
    r.trailsum[k] = __shfl(s.trailsum[k], src, 64);
  }
  return r;
}

template <typename K>
__global__ __launch_bounds__(NT) void k_scan_cross(Buffers b, uint32_t passes_done) {
  if (b.ctrl->error_flags) return;
  if (ctrl_passes(b.ctrl->pass_bits) > passes_done) return;
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint32_t j = blockIdx.x * NWAVE + wave;
  if (j >= b.n_tiles) return;
  // one round of loads: the ownership flag, and for the common span (the
  // location ends in the next tile) that tile's head level and both
  // summaries; a tile that owns a crossing location is not its trace's last
  const bool has_next = j + 1 < b.n_tiles;
  const uint32_t owns = b.tout[j].owns;
  const uint32_t next_m = has_next ? b.agg[(uint64_t)(j + 1) * SW] : 1u;
  State S = load_state(b.agg + (uint64_t)j * SW);
  const State S1 = has_next ? load_state(b.agg + (uint64_t)(j + 1) * SW) : identity();
  if (!owns) {
    if (lane == 0) b.cross_flag[j] = 0;
    return;
  }
  uint64_t fin[5];
  if (next_m == 0) {  // tile j + 1 holds a location head: the span is tile j
    open_sums(S, S1, fin);
  } else {
    const TraceDesc T = b.desc[b.tiles[j].trace];
    const uint32_t last = T.tile0 + T.ntiles - 1;  // last tile of the trace
    // end of the span: the first later tile of the trace with a location
    // head (tile j + 1 has none)
    uint32_t k = j + 2;  // candidate
    bool to_end = false;
    while (true) {
      if (k > last) {
        to_end = true;
        break;
      }
      const uint32_t c = k + lane;
      const bool head = c <= last && b.agg[(uint64_t)c * SW] == 0;
      const uint64_t bal = __ballot(head);
      if (bal) {
        k += (uint32_t)__ffsll((unsigned long long)bal) - 1;
        break;
      }
      k += 64;
    }
    // combine summaries of tiles j + 1 .. end - 1 into S (end = k, or last +
    // 1 when the location runs to the end of the trace)
    const uint32_t end = to_end ? last + 1 : k;
    for (uint32_t c0 = j + 1; c0 < end; c0 += 64) {
      const uint32_t c = c0 + lane;
      State s = c < end ? load_state(b.agg + (uint64_t)c * SW) : identity();
#pragma unroll
      for (uint32_t dlt = 1; dlt < 64; dlt <<= 1) {
        const State o = shfl_down_state(s, dlt);
        if ((lane & (2 * dlt - 1)) == 0) s = combine(s, o);
      }
      S = combine(S, readlane_state(s, 0));
    }
    if (to_end) {
      const uint64_t* t = tail_sums(S);
#pragma unroll
      for (int q = 0; q < 5; q++) fin[q] = t[q];
    } else {
      open_sums(S, load_state(b.agg + (uint64_t)k * SW), fin);
    }
  }
  const bool racing = fin[K_WW] + fin[K_RW] + fin[K_AW] + fin[K_AR] > 0;
  if (lane == 0) {
    b.cross_flag[j] = racing ? 1u : 0u;
    if (racing) {
      const TileRef tr = b.tiles[j];
      const TraceDesc T = b.desc[tr.trace];
      const TraceLayout L = b.layout[tr.trace];
      const uint64_t start = (uint64_t)tr.local * TILE;
      const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
      const K key = ((const K*)b.keys[L.npasses & 1u])[T.off + start + n_in - 1];
      write_entry<K>(&b.cross[j], tr.trace, L, key, fin);
    }
  }
}

// ------------------------------------------------------- ordered output
// Entries of tile j: its complete locations, then (if racing) the location
// it owns that crosses into later tiles.  Groups of 256 tiles.

__global__ __launch_bounds__(NT) void k_group_sums(Buffers b, uint32_t passes_done) {
  __shared__ uint32_t sc[NWAVE];
  if (b.ctrl->error_flags || ctrl_passes(b.ctrl->pass_bits) > passes_done) return;
  const uint32_t t = blockIdx.x * GROUP + threadIdx.x;
  const uint32_t c = t < b.n_tiles ? b.tout[t].in_count + b.cross_flag[t] : 0u;
  uint32_t tot;
  (void)block_excl_sum(c, sc, &tot);
  if (threadIdx.x == 0) b.group_sum[blockIdx.x] = tot;
}

// DIRECT (calls of at most DIRECT_GROUPS groups): each workgroup sums the
// entry counts of the tiles before its group itself, and k_group_sums is
// not launched.  Otherwise it sums the group totals k_group_sums left.
constexpr uint32_t DIRECT_GROUPS = 32;

template <bool DIRECT>
__global__ __launch_bounds__(NT) void k_scan_out(Buffers b, uint32_t passes_done) {
  __shared__ uint32_t sc[NWAVE];
  if (b.ctrl->error_flags || ctrl_passes(b.ctrl->pass_bits) > passes_done) return;
  // entries of the earlier groups
  uint64_t before = 0;
  if (DIRECT) {
#pragma unroll 8
    for (uint32_t t0 = threadIdx.x; t0 < blockIdx.x * GROUP; t0 += NT) before += b.tout[t0].in_count + b.cross_flag[t0];
  } else {
    for (uint32_t g = threadIdx.x; g < blockIdx.x; g += NT) before += b.group_sum[g];
  }
  uint32_t all;
  (void)block_excl_sum((uint32_t)before, sc, &all);
  const uint64_t group_base = all;
  const uint32_t t = blockIdx.x * GROUP + threadIdx.x;
  const bool valid = t < b.n_tiles;
  const uint32_t inc = valid ? b.tout[t].in_count : 0u;
  const uint32_t cf = valid ? b.cross_flag[t] : 0u;
  uint32_t tot;
  const uint32_t ex = block_excl_sum(inc + cf, sc, &tot);
  // the last workgroup publishes the call's total
  if (blockIdx.x + 1 == gridDim.x && threadIdx.x == 0) b.ctrl->total_entries = group_base + tot;
  if (!valid || inc + cf == 0) return;
  uint64_t pos = group_base + ex;
  if (inc) {
    const TileRef tr = b.tiles[t];
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
    uint32_t cap;
    const RaceOut* st = stage_of(b, t, T, L, start, n_in, &cap);
    for (uint32_t e = 0; e < inc && e < cap; e++, pos++)
      if (pos < b.out_cap) b.out[pos] = st[e];
  }
  if (cf && pos < b.out_cap) b.out[pos] = b.cross[t];
}

__global__ void k_reset_errors(Ctrl* ctrl, uint32_t mask) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->error_flags &= ~mask;
}

// ---------------------------------------------------------- k_barriers
//
// Redundant-barrier check (Alg. 5, second loop) over the sorted keys of a
// finished call: one thread per element; an element that heads a barrier
// instance (barrier.h) reads the two epoch runs around it straight from the
// key buffer (they are short except on the hottest locations) and counts
// the instance, racing or not, under its trace and boundary.
//
// Counts are summed per tile in LDS (boundaries below 256; later ones go to
// global memory directly) and added to one of `copies` copies of the
// trace's counters, chosen by tile, so that the atomics of many workgroups
// spread over several cache lines.

template <typename K, bool LOOP>
__global__ __launch_bounds__(NT) void k_barriers(Buffers b, const uint64_t* __restrict__ bar_base,
                                                 BarrierCount* table, uint32_t copies) {
  constexpr uint32_t NBIN = 256;
  __shared__ uint32_t s_inst[NBIN], s_race[NBIN];
  if (b.ctrl->error_flags) return;
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    s_inst[tx] = 0;
    s_race[tx] = 0;
    const TileRef tr = b.tiles[tile];
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    const K* keys = (const K*)b.keys[L.npasses & 1u] + T.off;  // the trace's sorted keys
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = tr.n_flags & ~TILE_SHORT;
    BarrierCount* counts = table + bar_base[tr.trace] * copies;
    __syncthreads();
#pragma unroll 1
    for (int r = 0; r < ITEMS; r++) {
      const uint32_t j = tx + r * NT;
      if (j >= n_in) break;
      uint32_t e0;
      bool racing;
      if (!barrier_instance<K>(L, keys, T.n, start + j, &e0, &racing)) continue;
      if (e0 < NBIN) {
        atomicAdd(&s_inst[e0], 1u);
        if (racing) atomicAdd(&s_race[e0], 1u);
      } else {
        BarrierCount* cnt = counts + (uint64_t)e0 * copies + tile % copies;
        atomicAdd(&cnt->instances, 1ull);
        if (racing) atomicAdd(&cnt->racing, 1ull);
      }
    }
    __syncthreads();
    const uint32_t ni = s_inst[tx];
    if (ni) {  // bins of boundaries the trace has (an instance's boundary is below its max epoch)
      BarrierCount* cnt = counts + (uint64_t)tx * copies + tile % copies;
      atomicAdd(&cnt->instances, (unsigned long long)ni);
      const uint32_t nr = s_race[tx];
      if (nr) atomicAdd(&cnt->racing, (unsigned long long)nr);
    }
  }
}

__global__ void k_fill_zero(unsigned long long* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ------------------------------------------------------------ EP fitness
//
// Eq. 1 (Sec. 4.1.1): for one candidate input, g(i) = 1 for every address i
// the trace touches and f(i) the number of threads touching it; the fitness
// is F = sum g / sum f, and the secondary score the access range.  With
// fitness keys (location, then thread; epoch and action dropped) the sorted
// keys of a trace hold one run per location, split into one run per
// (location, thread): sum g counts location heads and sum f counts heads at
// any level.  k_fit_tiles counts them per tile (the first key of a trace is
// a head of both), k_fit_traces sums a trace's tiles and writes its row.

template <typename K, bool LOOP>
__global__ __launch_bounds__(NT) void k_fit_tiles(Buffers b, uint32_t passes_done) {
  __shared__ uint32_t s_g[NWAVE], s_f[NWAVE];
  if (b.ctrl->error_flags) return;
  if (ctrl_passes(b.ctrl->pass_bits) > passes_done) return;  // the host runs the missing passes first
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    __syncthreads();  // LDS of the previous tile is free
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));
    const TileRef tr = b.tiles[tile];
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    const K* keys = (const K*)b.keys[L.npasses & 1u] + T.off;
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = tr.n_flags & ~TILE_SHORT;
    uint32_t g = 0, f = 0;
    // coalesced: key j of the tile is read by thread j mod NT, with its predecessor
#pragma unroll 4
    for (int r = 0; r < ITEMS; r++) {
      const uint32_t j = tx + r * NT;
      if (j >= n_in) break;
      const uint64_t p = start + j;
      const uint32_t lv = p == 0 ? 0u : head_level_t<K>(L, keys[p - 1], keys[p]);
      g += lv == 0 ? 1u : 0u;
      f += lv < 4 ? 1u : 0u;
    }
    g = wave_reduce(g, 0u, [](uint32_t a, uint32_t c) { return a + c; });
    f = wave_reduce(f, 0u, [](uint32_t a, uint32_t c) { return a + c; });
    if ((tx & 63u) == 0) {
      s_g[tx >> 6] = g;
      s_f[tx >> 6] = f;
    }
    __syncthreads();
    if (tx == 0) {
      uint32_t tg = 0, tf = 0;
#pragma unroll
      for (int w = 0; w < NWAVE; w++) {
        tg += s_g[w];
        tf += s_f[w];
      }
      b.tout[tile] = TileOut{tg, tf};
    }
  }
}

// One thread per trace.
__global__ __launch_bounds__(NT) void k_fit_traces(Buffers b, FitOut* __restrict__ out) {
  const uint32_t t = blockIdx.x * NT + threadIdx.x;
  if (t >= b.n_traces) return;
  const TraceDesc T = b.desc[t];
  const TraceLayout L = b.layout[t];
  uint64_t g = 0, f = 0;
  for (uint32_t k = 0; k < T.ntiles; k++) {
    const TileOut o = b.tout[T.tile0 + k];
    g += o.in_count;
    f += o.owns;
  }
  FitOut r;
  r.n_records = T.n;
  r.n_locations = g;
  r.n_location_threads = f;
  r.global_range = T.n ? L.grange : 0;
  r.shared_range = T.n ? L.srange : 0;
  r.fitness = f ? (double)g / (double)f : 1.0;
  out[t] = r;
}

// ------------------------------------------------- barrier divergence
//
// Alg. 4 (Sec. 4.2.2): a thread that reaches the end of the kernel while
// another thread of its block waits at a barrier is a barrier divergence.
// Input: for every thread the number of barriers it arrived at before it
// finished, block by block.  A block diverges when those numbers are not
// all equal; its entry gives the fewest and most arrivals and how many of
// its threads arrived at fewer than the most.
//
// k_div_blocks: one workgroup per chunk (whole blocks of one trace, about a
// tile of threads).  A block of up to 64 threads takes a segment of
// pow2ceil(tpb) lanes (several blocks per wave, reduced with xor shuffles
// inside the segment); a larger block takes a whole wave, its lanes
// striding over the threads.  Dense per-block results and per-chunk counts
// of divergent blocks go to global memory.  k_div_scan turns the counts
// into offsets (one workgroup), and k_div_emit writes the divergent blocks
// in (trace, block) order.

__device__ __forceinline__ uint32_t seg_lanes(uint32_t tpb) {
  if (tpb >= 64) return 64u;
  uint32_t s = 1;
  while (s < tpb) s <<= 1;
  return s;
}

__global__ __launch_bounds__(NT) void k_div_blocks(const DivChunk* __restrict__ chunks,
                                                   const uint32_t* __restrict__ arrivals, DivBlock* __restrict__ blocks,
                                                   uint32_t* __restrict__ chunk_cnt) {
  __shared__ uint32_t s_cnt;
  const DivChunk ch = chunks[blockIdx.x];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const uint32_t S = seg_lanes(ch.tpb);  // lanes per block (uniform over the workgroup)
  const uint32_t per_wave = 64u / S, sub = lane / S, sl = lane % S;
  uint32_t n_div = 0;
  for (uint32_t b0 = wave * per_wave; b0 < ch.n_blocks; b0 += NWAVE * per_wave) {
    const uint32_t blk = b0 + sub;
    const bool live = blk < ch.n_blocks;
    const uint32_t* c = arrivals + ch.thread0 + (uint64_t)blk * ch.tpb;
    uint32_t lo = ~0u, hi = 0u;
    if (live)
      for (uint32_t i = sl; i < ch.tpb; i += S) {
        const uint32_t v = c[i];
        lo = min(lo, v);
        hi = max(hi, v);
      }
    for (uint32_t d = 1; d < S; d <<= 1) {
      lo = min(lo, (uint32_t)__shfl_xor((int)lo, (int)d, 64));
      hi = max(hi, (uint32_t)__shfl_xor((int)hi, (int)d, 64));
    }
    uint32_t early = 0;
    if (live && lo != hi)  // the same in every lane of the segment
      for (uint32_t i = sl; i < ch.tpb; i += S) early += c[i] < hi ? 1u : 0u;
    for (uint32_t d = 1; d < S; d <<= 1) early += (uint32_t)__shfl_xor((int)early, (int)d, 64);
    if (live && sl == 0) {
      blocks[(uint64_t)ch.block0 + blk] = DivBlock{lo, hi, early, 0u};
      n_div += lo != hi ? 1u : 0u;
    }
  }
  n_div = wave_reduce(n_div, 0u, [](uint32_t a, uint32_t b) { return a + b; });
  if (lane == 0 && n_div) atomicAdd(&s_cnt, n_div);
  __syncthreads();
  if (threadIdx.x == 0) chunk_cnt[blockIdx.x] = s_cnt;
}

// One workgroup: exclusive offsets of the chunks' counts, and the total.
__global__ __launch_bounds__(NT) void k_div_scan(const uint32_t* __restrict__ chunk_cnt, uint64_t* __restrict__ chunk_off,
                                                 uint32_t n_chunks, uint64_t* __restrict__ total) {
  __shared__ uint32_t s_sc[NWAVE];
  uint64_t base = 0;
  for (uint32_t i0 = 0; i0 < n_chunks; i0 += NT) {
    const uint32_t i = i0 + threadIdx.x;
    const uint32_t v = i < n_chunks ? chunk_cnt[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_sum(v, s_sc, &tot);
    if (i < n_chunks) chunk_off[i] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) *total = base;
}

__global__ __launch_bounds__(NT) void k_div_emit(const DivChunk* __restrict__ chunks,
                                                 const DivBlock* __restrict__ blocks,
                                                 const uint64_t* __restrict__ chunk_off, DivOut* __restrict__ out) {
  __shared__ uint32_t s_sc[NWAVE];
  const DivChunk ch = chunks[blockIdx.x];
  uint64_t base = chunk_off[blockIdx.x];
  for (uint32_t b0 = 0; b0 < ch.n_blocks; b0 += NT) {
    const uint32_t blk = b0 + threadIdx.x;
    DivBlock r{0u, 0u, 0u, 0u};
    if (blk < ch.n_blocks) r = blocks[(uint64_t)ch.block0 + blk];
    const uint32_t flag = (blk < ch.n_blocks && r.lo != r.hi) ? 1u : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_sum(flag, s_sc, &tot);
    if (flag) out[base + ex] = DivOut{ch.trace, ch.block + blk, r.lo, r.hi, (uint64_t)r.early};
    base += tot;
  }
}

// ------------------------------------------------- warp refinement
//
// Theorem 1's warp clauses (and the race loop of Alg. 5): two accesses by
// threads of one warp (32 threads of a block, by block-local id) are
// ordered by lockstep execution, and so do not race, unless one of them ran
// diverged or both are writes by one statement.  The plain count over the
// sorted keys includes such pairs.  The keys of a warp-aware call carry the
// side field (keys.h), so the records of one (location, block, epoch, warp)
// -- a warp group -- are adjacent, and every element without the divergence
// bit counts, against the earlier elements of its warp group, the pairs the
// plain count has and lockstep removes: another thread, no divergence bit, a
// conflicting action, and not two writes of one statement.  An element with
// such pairs finds its location's entry in the plain result (entries are in
// key order) and subtracts them there.  Warp groups are short, a few records
// each, except where a warp hammers one word within one barrier interval.

__device__ __forceinline__ int entry_cmp(const RaceOut& e, uint32_t trace, uint32_t space, uint32_t block,
                                         uint64_t unit) {
  if (e.trace != trace) return e.trace < trace ? -1 : 1;
  if (e.space != space) return e.space < space ? -1 : 1;
  if (e.block != block) return e.block < block ? -1 : 1;
  if (e.unit != unit) return e.unit < unit ? -1 : 1;
  return 0;
}

// Kind of a conflicting pair of classes (K_WW .. K_AR), or 4 if they do not
// conflict (two reads, two atomics).
__device__ __forceinline__ uint32_t pair_kind(uint32_t c1, uint32_t c2) {
  const uint32_t lo = min(c1, c2), hi = max(c1, c2);
  if (lo == CLS_W) return hi == CLS_W ? (uint32_t)K_WW : (uint32_t)K_AW;
  if (lo == CLS_R) return hi == CLS_W ? (uint32_t)K_RW : (hi == CLS_A ? (uint32_t)K_AR : 4u);
  return 4u;
}

template <typename K, bool LOOP>
__global__ __launch_bounds__(NT) void k_warp_removed(Buffers b, const RaceOut* __restrict__ entries,
                                                     uint64_t n_entries, unsigned long long* __restrict__ removed) {
  if (b.ctrl->error_flags) return;
  const TileWalk tw = tile_walk(b.n_tiles, gridDim.x, blockIdx.x);
  for (uint32_t tile = tw.first; tile < tw.end; tile = LOOP ? tile + tw.step : tw.end) {
    uint32_t tx = threadIdx.x;
    if (LOOP) asm volatile("" : "+v"(tx));  // per tile: keeps per-item offsets from being hoisted
    const TileRef tr = b.tiles[tile];
    const TraceDesc T = b.desc[tr.trace];
    const TraceLayout L = b.layout[tr.trace];
    const K* keys = (const K*)b.keys[L.npasses & 1u] + T.off;  // the trace's sorted keys
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = tr.n_flags & ~TILE_SHORT;
    const uint32_t wshift = 2 + L.sb + min(L.tb, 5u);  // the bits above: location, block, epoch, warp
#pragma unroll 1
    for (int r = 0; r < ITEMS; r++) {
      const uint32_t j = tx + r * NT;
      if (j >= n_in) break;
      const uint64_t p = start + j;
      const K x = keys[p];
      if (key_diverged_t<K>(L, x)) continue;
      const uint32_t cx = action_class(x), lx = key_ltid_t<K>(L, x), sx = key_stmt_t<K>(L, x);
      const K gx = x >> wshift;
      uint64_t rm[4] = {0, 0, 0, 0};
      for (uint64_t q = p; q > 0; q--) {
        const K y = keys[q - 1];
        if ((y >> wshift) != gx) break;  // the start of x's warp group
        if (key_diverged_t<K>(L, y) || key_ltid_t<K>(L, y) == lx) continue;
        const uint32_t cy = action_class(y), kd = pair_kind(cx, cy);
        if (kd == 4u) continue;
        if (kd == (uint32_t)K_WW && key_stmt_t<K>(L, y) == sx) continue;  // one statement's writes still race
        rm[kd]++;
      }
      if ((rm[0] | rm[1] | rm[2] | rm[3]) == 0) continue;
      uint32_t sp, blk;
      uint64_t unit;
      key_location_t<K>(L, x, sp, blk, unit);
      uint64_t lo = 0, hi = n_entries;  // first entry not below x's location
      while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (entry_cmp(entries[mid], tr.trace, sp, blk, unit) < 0) lo = mid + 1;
        else hi = mid;
      }
      if (lo == n_entries || entry_cmp(entries[lo], tr.trace, sp, blk, unit) != 0) {
        atomicOr(&b.ctrl->error_flags, ERR_INTERNAL_BOUNDS);  // lockstep only removes pairs the plain count has
        continue;
      }
#pragma unroll
      for (int k = 0; k < 4; k++)
        if (rm[k]) atomicAdd(&removed[lo * 4 + k], (unsigned long long)rm[k]);
    }
  }
}

// One workgroup: every entry minus its removed pairs; entries left with a
// pair are written to `out` in order, with their kinds bits; *n_out gets
// their number.
__global__ __launch_bounds__(4 * NT) void k_warp_finish(const RaceOut* __restrict__ in, uint64_t n,
                                                        const unsigned long long* __restrict__ removed,
                                                        RaceOut* __restrict__ out, unsigned long long* __restrict__ n_out,
                                                        Ctrl* ctrl) {
  __shared__ uint32_t s_sc[4 * NWAVE];
  uint64_t base = 0;
  for (uint64_t i0 = 0; i0 < n; i0 += 4 * NT) {
    const uint64_t i = i0 + threadIdx.x;
    RaceOut e;
    uint32_t keep = 0;
    if (i < n) {
      e = in[i];
      const unsigned long long* rm = removed + i * 4;
      if (rm[K_WW] > e.ww || rm[K_RW] > e.rw || rm[K_AW] > e.aw || rm[K_AR] > e.ar)
        atomicOr(&ctrl->error_flags, ERR_INTERNAL_BOUNDS);
      e.ww -= rm[K_WW];
      e.rw -= rm[K_RW];
      e.aw -= rm[K_AW];
      e.ar -= rm[K_AR];
      keep = (e.ww | e.rw | e.aw | e.ar) != 0 ? 1u : 0u;
      e.kinds = (uint8_t)((e.ww ? 1 : 0) | (e.rw ? 2 : 0) | (e.aw ? 4 : 0) | (e.ar ? 8 : 0) | (e.xb ? 16 : 0));
    }
    uint32_t tot;
    const uint32_t ex = block_excl_sum_n<4 * NWAVE>(keep, s_sc, &tot);
    if (keep) out[base + ex] = e;
    base += tot;
  }
  if (threadIdx.x == 0) *n_out = base;
}

// -------------------------------------------------------- launch wrappers

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// The tile walk needs grids that are non-zero multiples of the XCD count.
static inline bool grids_ok(const Buffers& b) {
  for (uint32_t g : {b.grid_stream, b.grid_sort, b.grid_scan})
    if (g == 0 || g % N_XCD != 0) return false;
  return true;
}

// Whether a grid leaves some workgroup more than one tile (the looping
// variant of a tile kernel), or at most one each (the one-tile variant).
static inline bool loops(const Buffers& b, uint32_t grid) { return grid / N_XCD < cdiv(b.n_tiles, N_XCD); }

hipError_t launch_init(const Buffers& b, hipStream_t s) {
  if (b.n_tiles) return hipSuccess;  // k_stats clears the control words
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, b.ctrl);
  return hipGetLastError();
}
hipError_t launch_stats(const Buffers& b, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  if (!grids_ok(b)) return hipErrorInvalidConfiguration;
  const bool lp = loops(b, b.grid_stream);
  auto kern = b.fuse0 ? (lp ? k_stats<true, true> : k_stats<false, true>)
                      : (lp ? k_stats<true, false> : k_stats<false, false>);
  hipLaunchKernelGGL(kern, dim3(b.grid_stream), dim3(NT), 0, s, b.tiles, b.n_tiles, b.stats_part, b.tcnt,
                     b.ctrl, b.side);
  return hipGetLastError();
}
hipError_t launch_layout(const Buffers& b, hipStream_t s) {
  if (!b.n_traces) return hipSuccess;
  if (b.n_traces <= 64 && b.n_tiles >= 64 * b.n_traces)  // a few long traces
    hipLaunchKernelGGL(k_layout<4 * NT>, dim3(b.n_traces), dim3(4 * NT), 0, s, b.desc, b.stats_part, b.layout, b.ctrl,
                       b.wide, b.fitness, b.side ? 1u : 0u, b.digit_bits);
  else
    hipLaunchKernelGGL(k_layout<NT>, dim3(b.n_traces), dim3(NT), 0, s, b.desc, b.stats_part, b.layout, b.ctrl, b.wide,
                       b.fitness, b.side ? 1u : 0u, b.digit_bits);
  return hipGetLastError();
}
hipError_t launch_keygen(const Buffers& b, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  if (!grids_ok(b)) return hipErrorInvalidConfiguration;
  if (b.fuse0) {  // pass 0's offsets come first (launch_upsweep(b, 0)); the keys go straight to pass 1's buffer
    const bool lp = loops(b, b.grid_sort);
    if (b.wide) {
      auto kern = lp ? k_keygen_scatter<u128, true> : k_keygen_scatter<u128, false>;
      hipLaunchKernelGGL(kern, dim3(b.grid_sort), dim3(NT), 0, s, b);
    } else {  // one-word keys: 512 threads of 8 records (7 waves per SIMD instead of 4)
      auto kern = lp ? k_keygen_scatter<uint64_t, true, 2 * NT> : k_keygen_scatter<uint64_t, false, 2 * NT>;
      hipLaunchKernelGGL(kern, dim3(b.grid_sort), dim3(2 * NT), 0, s, b);
    }
  } else {
    const bool lp = loops(b, b.grid_stream);
    auto kern = b.wide ? (lp ? k_keygen<u128, true> : k_keygen<u128, false>)
                       : (lp ? k_keygen<uint64_t, true> : k_keygen<uint64_t, false>);
    hipLaunchKernelGGL(kern, dim3(b.grid_stream), dim3(NT), 0, s, b);
  }
  return hipGetLastError();
}
template <uint32_t R>
static hipError_t launch_offsets(const Buffers& b, uint32_t pass, hipStream_t s) {
  switch (offset_parts(b.max_group_tiles, R)) {
    case 1: hipLaunchKernelGGL((k_group_offsets<1, R>), dim3(b.n_groups), dim3(R), 0, s, b, pass); break;
    case 2: hipLaunchKernelGGL((k_group_offsets<2, R>), dim3(b.n_groups), dim3(2 * R), 0, s, b, pass); break;
    default: hipLaunchKernelGGL((k_group_offsets<4, R>), dim3(b.n_groups), dim3(4 * R), 0, s, b, pass); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (offset_parts(b.max_trace_groups, R)) {
    case 1: hipLaunchKernelGGL((k_trace_offsets<1, R>), dim3(b.n_traces), dim3(R), 0, s, b, pass); break;
    case 2: hipLaunchKernelGGL((k_trace_offsets<2, R>), dim3(b.n_traces), dim3(2 * R), 0, s, b, pass); break;
    default: hipLaunchKernelGGL((k_trace_offsets<4, R>), dim3(b.n_traces), dim3(4 * R), 0, s, b, pass); break;
  }
  return hipGetLastError();
}

// A pass's digit width: 8 bits in pass 0, the call's after it.
static bool wide_digit(const Buffers& b, uint32_t pass) { return pass > 0 && b.digit_bits == RADIX_WIDE_BITS; }

hipError_t launch_upsweep(const Buffers& b, uint32_t pass, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  if (!grids_ok(b)) return hipErrorInvalidConfiguration;
  if (b.digit_bits != RADIX_BITS && b.digit_bits != RADIX_WIDE_BITS) return hipErrorInvalidValue;
  const bool w9 = wide_digit(b, pass);
  if (pass > 0) {  // digit 0's histograms come from k_keygen
    const bool lp = loops(b, b.grid_stream);
    auto kern = w9 ? (b.wide ? (lp ? k_upsweep<u128, true, RADIX_WIDE_BITS> : k_upsweep<u128, false, RADIX_WIDE_BITS>)
                             : (lp ? k_upsweep<uint64_t, true, RADIX_WIDE_BITS>
                                   : k_upsweep<uint64_t, false, RADIX_WIDE_BITS>))
                   : (b.wide ? (lp ? k_upsweep<u128, true, RADIX_BITS> : k_upsweep<u128, false, RADIX_BITS>)
                             : (lp ? k_upsweep<uint64_t, true, RADIX_BITS> : k_upsweep<uint64_t, false, RADIX_BITS>));
    hipLaunchKernelGGL(kern, dim3(b.grid_stream), dim3(NT), 0, s, b, pass);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return w9 ? launch_offsets<RADIX_MAX>(b, pass, s) : launch_offsets<RADIX>(b, pass, s);
}

template <uint32_t DB>
static hipError_t launch_scatter_db(const Buffers& b, uint32_t pass, hipStream_t s) {
  const bool lp = loops(b, b.grid_sort);
  if (b.wide) {
    auto kern = lp ? k_scatter<u128, true, NT, DB> : k_scatter<u128, false, NT, DB>;
    hipLaunchKernelGGL(kern, dim3(b.grid_sort), dim3(NT), 0, s, b, pass);
  } else if (b.scatter_nt == 2 * NT) {
    auto kern = lp ? k_scatter<uint64_t, true, 2 * NT, DB> : k_scatter<uint64_t, false, 2 * NT, DB>;
    hipLaunchKernelGGL(kern, dim3(b.grid_sort), dim3(2 * NT), 0, s, b, pass);
  } else {
    auto kern = lp ? k_scatter<uint64_t, true, NT, DB> : k_scatter<uint64_t, false, NT, DB>;
    hipLaunchKernelGGL(kern, dim3(b.grid_sort), dim3(NT), 0, s, b, pass);
  }
  return hipGetLastError();
}

hipError_t launch_scatter(const Buffers& b, uint32_t pass, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  if (!grids_ok(b)) return hipErrorInvalidConfiguration;
  if (b.digit_bits != RADIX_BITS && b.digit_bits != RADIX_WIDE_BITS) return hipErrorInvalidValue;
  return wide_digit(b, pass) ? launch_scatter_db<RADIX_WIDE_BITS>(b, pass, s) : launch_scatter_db<RADIX_BITS>(b, pass, s);
}
hipError_t launch_sort_small(const Buffers& b, hipStream_t s) {
  if (b.n_small1) {
    auto kern = b.wide ? k_sort_small<u128, NT> : k_sort_small<uint64_t, NT>;
    hipLaunchKernelGGL(kern, dim3(b.n_small1), dim3(NT), 0, s, b, b.small_traces);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.n_small4) {  // one-word keys only (the two-word LDS image would not fit)
    if (b.wide) return hipErrorInvalidValue;
    auto kern = k_sort_small<uint64_t, 4 * NT>;
    hipLaunchKernelGGL(kern, dim3(b.n_small4), dim3(4 * NT), 0, s, b, b.small_traces + b.n_small1);
    return hipGetLastError();
  }
  return hipSuccess;
}
hipError_t launch_scan_tiles(const Buffers& b, uint32_t passes_done, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  if (!grids_ok(b)) return hipErrorInvalidConfiguration;
  const bool lp = loops(b, b.grid_scan);
  auto kern = b.wide ? (lp ? k_scan_tiles<u128, true> : k_scan_tiles<u128, false>)
                     : (lp ? k_scan_tiles<uint64_t, true> : k_scan_tiles<uint64_t, false>);
  hipLaunchKernelGGL(kern, dim3(b.grid_scan), dim3(NT), 0, s, b, passes_done);
  return hipGetLastError();
}
hipError_t launch_scan_cross(const Buffers& b, uint32_t passes_done, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(b.wide ? k_scan_cross<u128> : k_scan_cross<uint64_t>, dim3(cdiv(b.n_tiles, NWAVE)), dim3(NT), 0,
                     s, b, passes_done);
  return hipGetLastError();
}
hipError_t launch_scan_out(const Buffers& b, uint32_t passes_done, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  const uint32_t n_groups = cdiv(b.n_tiles, GROUP);
  if (n_groups <= DIRECT_GROUPS) {
    hipLaunchKernelGGL(k_scan_out<true>, dim3(n_groups), dim3(NT), 0, s, b, passes_done);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_group_sums, dim3(n_groups), dim3(NT), 0, s, b, passes_done);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_out<false>, dim3(n_groups), dim3(NT), 0, s, b, passes_done);
  return hipGetLastError();
}
hipError_t launch_reset_errors(const Buffers& b, uint32_t mask, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_errors, dim3(1), dim3(64), 0, s, b.ctrl, mask);
  return hipGetLastError();
}

hipError_t launch_barriers(const Buffers& b, const uint64_t* bar_base, BarrierCount* table, uint64_t n_counts,
                           uint32_t copies, hipStream_t s) {
  if (n_counts) {
    const uint64_t words = 2 * n_counts;
    hipLaunchKernelGGL(k_fill_zero, dim3((uint32_t)std::min<uint64_t>(4096, (words + NT - 1) / NT)), dim3(NT), 0, s,
                       (unsigned long long*)table, words);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!b.n_tiles || !n_counts) return hipSuccess;
  if (!grids_ok(b) || copies == 0) return hipErrorInvalidConfiguration;
  const bool lp = loops(b, b.grid_scan);
  auto kern = b.wide ? (lp ? k_barriers<u128, true> : k_barriers<u128, false>)
                     : (lp ? k_barriers<uint64_t, true> : k_barriers<uint64_t, false>);
  hipLaunchKernelGGL(kern, dim3(b.grid_scan), dim3(NT), 0, s, b, bar_base, table, copies);
  return hipGetLastError();
}

hipError_t launch_fitness(const Buffers& b, uint32_t passes_done, FitOut* out, hipStream_t s) {
  if (b.n_tiles) {
    if (!grids_ok(b)) return hipErrorInvalidConfiguration;
    const bool lp = loops(b, b.grid_scan);
    auto kern = b.wide ? (lp ? k_fit_tiles<u128, true> : k_fit_tiles<u128, false>)
                       : (lp ? k_fit_tiles<uint64_t, true> : k_fit_tiles<uint64_t, false>);
    hipLaunchKernelGGL(kern, dim3(b.grid_scan), dim3(NT), 0, s, b, passes_done);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!b.n_traces) return hipSuccess;
  hipLaunchKernelGGL(k_fit_traces, dim3(cdiv(b.n_traces, NT)), dim3(NT), 0, s, b, out);
  return hipGetLastError();
}

hipError_t launch_divergence(const DivChunk* chunks, uint32_t n_chunks, const uint32_t* arrivals, DivBlock* blocks,
                             uint32_t* chunk_cnt, uint64_t* chunk_off, uint64_t* total, hipStream_t s) {
  if (n_chunks) {
    hipLaunchKernelGGL(k_div_blocks, dim3(n_chunks), dim3(NT), 0, s, chunks, arrivals, blocks, chunk_cnt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_div_scan, dim3(1), dim3(NT), 0, s, chunk_cnt, chunk_off, n_chunks, total);
  return hipGetLastError();
}

hipError_t launch_divergence_emit(const DivChunk* chunks, uint32_t n_chunks, const DivBlock* blocks,
                                  const uint64_t* chunk_off, DivOut* out, hipStream_t s) {
  if (!n_chunks) return hipSuccess;
  hipLaunchKernelGGL(k_div_emit, dim3(n_chunks), dim3(NT), 0, s, chunks, blocks, chunk_off, out);
  return hipGetLastError();
}

hipError_t launch_warp_refine(const Buffers& b, const RaceOut* entries, uint64_t n_entries, unsigned long long* removed,
                              RaceOut* out, unsigned long long* n_out, hipStream_t s) {
  if (n_entries) {
    hipLaunchKernelGGL(k_fill_zero, dim3(cdiv(4 * n_entries, NT) < 4096 ? cdiv(4 * n_entries, NT) : 4096), dim3(NT),
                       0, s, removed, 4 * n_entries);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.n_tiles) {
      if (!grids_ok(b)) return hipErrorInvalidConfiguration;
      const bool lp = loops(b, b.grid_scan);
      auto kern = b.wide ? (lp ? k_warp_removed<u128, true> : k_warp_removed<u128, false>)
                         : (lp ? k_warp_removed<uint64_t, true> : k_warp_removed<uint64_t, false>);
      hipLaunchKernelGGL(kern, dim3(b.grid_scan), dim3(NT), 0, s, b, entries, n_entries, removed);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_warp_finish, dim3(1), dim3(4 * NT), 0, s, entries, n_entries, removed, out, n_out, b.ctrl);
  return hipGetLastError();
}

// ---------------------------------------------------- no-allocation scratch
//
// Every buffer of a sim_check_traces_device_noalloc call is carved out of
// this array.  Each GPU that loads the library holds its own copy (at its
// own address) until the process ends.  In host code the name `scratch` is
// only a host-side stand-in for the symbol: passing it to a kernel would
// fault.  Host code uses the address scratch_address() returns instead.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_SCRATCH_DEVICES = 64;

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[MAX_SCRATCH_DEVICES];
  static hipError_t err[MAX_SCRATCH_DEVICES];
  static bool looked_up[MAX_SCRATCH_DEVICES];
  *out = nullptr;
  if (device < 0 || device >= MAX_SCRATCH_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!looked_up[device]) {  // once per device, with that device current (the caller's guarantee)
    void* p = nullptr;
    err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    addr[device] = err[device] == hipSuccess ? p : nullptr;
    looked_up[device] = true;
  }
  *out = addr[device];
  return err[device];
}

}  // namespace sc
