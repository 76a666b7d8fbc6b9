// kernels.hip -- gfx950 kernels of the Memory-Model data-race check.
//
// Pipeline for a call over one or more traces (records of a trace are
// contiguous; kernels work on 4096-record tiles and a tile never spans two
// traces):
//   k_init        reset per-call state
//   k_stats       per-tile unit ranges, largest tid and epoch, record checks
//   k_layout      per-trace reduction of the tile statistics, key layout
//   k_keygen      records -> 64-bit keys, digit histograms of every pass
//   k_digits      digit bases (exclusive scan of the histograms)
//   k_sort_pass   one stable LSD radix pass, 8-bit digits (x passes)
//   k_scan_tiles  racing-pair counts of every location inside a tile, and
//                 the tile's summary for locations that cross tiles
//   k_scan_cross  pair counts of the locations that cross tiles
//   k_group_*     ordered output: two-level prefix of per-tile entry counts
//
// Device-scope atomics that many workgroups aim at one address serialise
// (about 11 ns each on MI355X), so no kernel here funnels per-tile work
// through one counter: statistics are per-tile partials, histograms are
// spread over replicas, and the radix pass runs as a cooperative grid whose
// workgroups are all resident, taking tiles in a fixed order instead of
// from a ticket counter.  Only the radix pass chains tiles (decoupled
// look-back); its status words carry a 24-bit tag unique to the launch and
// are accessed with agent-scope atomics, coherent across the XCDs.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "segstate.h"

namespace sc {

constexpr int NWAVE = NT / 64;
static_assert(NT == (int)RADIX, "one thread per digit in k_sort_pass");
static_assert(GROUP == NT, "one thread per tile in the output kernels");
constexpr uint64_t SEGF = 1ull << 63;   // head flag of packed segmented values
constexpr uint32_t CLS_NONE = 3;        // padding element past the end of a trace
constexpr uint32_t LOOKBACK = 8;        // predecessors read per look-back round trip

// ------------------------------------------------------------- utilities

__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_word(uint32_t tag, uint32_t flag, uint32_t val) {
  return ((uint64_t)tag << 40) | ((uint64_t)(flag & 0xFF) << 32) | (uint64_t)val;
}
__device__ __forceinline__ uint32_t status_tag(uint64_t w) { return (uint32_t)(w >> 40); }
__device__ __forceinline__ uint32_t status_flag(uint64_t w) { return (uint32_t)(w >> 32) & 0xFF; }

enum : uint32_t { FLAG_AGG = 1, FLAG_INCL = 2 };

// A look-back wait polls at most this many times (each poll sleeps ~128
// cycles, about 1 s in total) before it gives up and flags an error, so a
// wait can never hang the device.
constexpr uint32_t SPIN_LIMIT = 1u << 24;

__device__ __forceinline__ bool spin_exhausted(uint32_t& spins, Ctrl* ctrl) {
  if (++spins < SPIN_LIMIT) {
    __builtin_amdgcn_s_sleep(2);
    return false;
  }
  atomicOr(&ctrl->error_flags, ERR_INTERNAL_SPIN);
  return true;
}

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

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    T o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    T o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Exclusive sum over the workgroup; *total receives the sum of all values.
__device__ uint32_t block_excl_sum(uint32_t v, uint32_t* lds /* NWAVE */, uint32_t* total) {
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(inc, d, 64);
    if (lane >= (uint32_t)d) inc += o;
  }
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NWAVE; w++) {
    const uint32_t x = lds[w];
    if (w < (int)wave) pre += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

// Segmented scan operator on packed values: a head flag in bit 63 restarts
// the sum.
__device__ __forceinline__ uint64_t seg_op(uint64_t a, uint64_t b) { return (b & SEGF) ? b : a + b; }

// Exclusive segmented scan of K packed words over the workgroup; tot[]
// receives the inclusive value at the last thread.
template <int K>
__device__ void block_seg_scan(const uint64_t (&v)[K], uint64_t (&ex)[K], uint64_t (&tot)[K],
                               uint64_t (*lds)[K] /* [NWAVE][K] */) {
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  uint64_t inc[K];
#pragma unroll
  for (int k = 0; k < K; k++) inc[k] = v[k];
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
    for (int k = 0; k < K; k++) {
      const uint64_t o = __shfl_up(inc[k], d, 64);
      if (lane >= (uint32_t)d) inc[k] = seg_op(o, inc[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    uint64_t e = __shfl_up(inc[k], 1, 64);
    ex[k] = lane == 0 ? 0ull : e;
  }
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < K; k++) lds[wave][k] = inc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    uint64_t pre = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; w++) {
      const uint64_t x = lds[w][k];
      if (w < (int)wave) pre = seg_op(pre, x);
      all = seg_op(all, x);
    }
    ex[k] = seg_op(pre, ex[k]);
    tot[k] = all;
  }
  __syncthreads();
}

// --------------------------------------------------------------- k_init

__global__ void k_init(uint32_t* hist, uint64_t n_hist, Ctrl* ctrl) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctrl->max_passes = 0;
    ctrl->error_flags = 0;
    ctrl->first_bad = ~0ull;
    ctrl->total_entries = 0;
  }
  for (uint64_t j = i; j < n_hist; j += (uint64_t)gridDim.x * blockDim.x) hist[j] = 0;
}

// -------------------------------------------------------------- k_stats
// Per-tile partial statistics; k_layout reduces them per trace.

__global__ __launch_bounds__(NT) void k_stats(const ulonglong2* __restrict__ recs, const TraceDesc* __restrict__ desc,
                                              const TileRef* __restrict__ tiles, TraceStats* __restrict__ part) {
  __shared__ uint64_t s64[5][NWAVE];
  __shared__ uint32_t s32[2][NWAVE];
  const TileRef tr = tiles[blockIdx.x];
  const TraceDesc T = desc[tr.trace];
  const uint64_t start = (uint64_t)tr.local * TILE;
  const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
  const ulonglong2* p = recs + T.off + start;
  uint64_t gmin = ~0ull, gmax = 0, smin = ~0ull, smax = 0, bad = ~0ull;
  uint32_t mt = 0, me = 0;
#pragma unroll 4
  for (int r = 0; r < ITEMS; r++) {
    const uint32_t j = threadIdx.x + r * NT;
    if (j < n_in) {
      const Rec x = unpack_rec(p[j]);
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
  mt = wave_max(mt); me = wave_max(me);
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  if (lane == 0) {
    s64[0][wave] = gmin; s64[1][wave] = gmax; s64[2][wave] = smin; s64[3][wave] = smax; s64[4][wave] = bad;
    s32[0][wave] = mt; s32[1][wave] = me;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NWAVE; w++) {
      gmin = min(gmin, s64[0][w]); gmax = max(gmax, s64[1][w]);
      smin = min(smin, s64[2][w]); smax = max(smax, s64[3][w]);
      bad = min(bad, s64[4][w]);
      mt = max(mt, s32[0][w]); me = max(me, s32[1][w]);
    }
    TraceStats S;
    S.gmin = gmin; S.gmax = gmax; S.smin = smin; S.smax = smax; S.bad_index = bad;
    S.max_tid = mt; S.max_epoch = me;
    part[blockIdx.x] = S;
  }
}

// ------------------------------------------------------------- k_layout
// One workgroup per trace: reduce the trace's tile statistics, derive the
// key layout.  Global atomics only on rare events (an error, a new maximum
// pass count).

__global__ __launch_bounds__(NT) void k_layout(const TraceDesc* __restrict__ desc,
                                               const TraceStats* __restrict__ part, TraceLayout* lay, Ctrl* ctrl) {
  __shared__ uint64_t s64[5][NWAVE];
  __shared__ uint32_t s32[2][NWAVE];
  const uint32_t t = blockIdx.x;
  const TraceDesc T = desc[t];
  TraceStats S;
  stats_init(S);
  for (uint32_t i = threadIdx.x; i < T.ntiles; i += NT) {
    const TraceStats P = part[T.tile0 + i];
    S.gmin = min(S.gmin, P.gmin); S.gmax = max(S.gmax, P.gmax);
    S.smin = min(S.smin, P.smin); S.smax = max(S.smax, P.smax);
    S.bad_index = min(S.bad_index, P.bad_index);
    S.max_tid = max(S.max_tid, P.max_tid); S.max_epoch = max(S.max_epoch, P.max_epoch);
  }
  S.gmin = wave_min(S.gmin); S.smin = wave_min(S.smin); S.bad_index = wave_min(S.bad_index);
  S.gmax = wave_max(S.gmax); S.smax = wave_max(S.smax);
  S.max_tid = wave_max(S.max_tid); S.max_epoch = wave_max(S.max_epoch);
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  if (lane == 0) {
    s64[0][wave] = S.gmin; s64[1][wave] = S.gmax; s64[2][wave] = S.smin; s64[3][wave] = S.smax;
    s64[4][wave] = S.bad_index; s32[0][wave] = S.max_tid; s32[1][wave] = S.max_epoch;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < NWAVE; w++) {
    S.gmin = min(S.gmin, s64[0][w]); S.gmax = max(S.gmax, s64[1][w]);
    S.smin = min(S.smin, s64[2][w]); S.smax = max(S.smax, s64[3][w]);
    S.bad_index = min(S.bad_index, s64[4][w]);
    S.max_tid = max(S.max_tid, s32[0][w]); S.max_epoch = max(S.max_epoch, s32[1][w]);
  }
  TraceLayout L = make_layout(S, T.tpb);
  if (T.n == 0) {
    L.error = 0;
    L.npasses = 0;
  }
  lay[t] = L;
  if (L.error) {
    atomicOr(&ctrl->error_flags, L.error);
    if (L.error & LAYOUT_ERR_RECORD)
      atomicMin((unsigned long long*)&ctrl->first_bad, (unsigned long long)(T.off + S.bad_index));
  }
  if (L.npasses > __hip_atomic_load(&ctrl->max_passes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(&ctrl->max_passes, L.npasses);
}

// ------------------------------------------------------------- k_keygen
// Records -> keys, plus the digit histogram of every radix pass.  A trace's
// tiles add their histograms into one of ceil(ntiles / 256) replicas, so no
// histogram counter takes more than 256 atomic adds.

__global__ __launch_bounds__(NT) void k_keygen(const ulonglong2* __restrict__ recs, const TraceDesc* __restrict__ desc,
                                               const TileRef* __restrict__ tiles, const TraceLayout* __restrict__ lay,
                                               uint64_t* __restrict__ keys, uint32_t* hist) {
  __shared__ uint32_t h[MAX_PASSES * RADIX];
  const TileRef tr = tiles[blockIdx.x];
  const TraceDesc T = desc[tr.trace];
  const TraceLayout L = lay[tr.trace];
  if (L.npasses == 0) return;
  const uint32_t np = L.npasses;
  for (uint32_t i = threadIdx.x; i < np * RADIX; i += NT) h[i] = 0;
  __syncthreads();
  const uint64_t start = (uint64_t)tr.local * TILE;
  const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
  const ulonglong2* p = recs + T.off + start;
  uint64_t* kout = keys + T.off + start;
#pragma unroll 4
  for (int r = 0; r < ITEMS; r++) {
    const uint32_t j = threadIdx.x + r * NT;
    if (j < n_in) {
      const Rec x = unpack_rec(p[j]);
      const uint64_t k = make_key(L, x.unit, x.tid, x.epoch, x.action, x.space, T.tpb);
      kout[j] = k;
      for (uint32_t q = 0; q < np; q++) atomicAdd(&h[q * RADIX + ((k >> (2 + RADIX_BITS * q)) & (RADIX - 1))], 1u);
    }
  }
  __syncthreads();
  uint32_t* gh = hist + (uint64_t)(T.rep0 + tr.local % T.nrep) * MAX_PASSES * RADIX;
  for (uint32_t i = threadIdx.x; i < np * RADIX; i += NT) {
    const uint32_t c = h[i];
    if (c) atomicAdd(&gh[i], c);
  }
}

// ------------------------------------------------------------- k_digits
// Sum a trace's histogram replicas and scan them into digit bases, written
// over the trace's first replica.

__global__ __launch_bounds__(NT) void k_digits(const TraceDesc* __restrict__ desc, const TraceLayout* __restrict__ lay,
                                               uint32_t* hist) {
  __shared__ uint32_t sc[NWAVE];
  const uint32_t trace = blockIdx.x;
  const TraceDesc T = desc[trace];
  const uint32_t np = lay[trace].npasses;
  uint32_t* gh = hist + (uint64_t)T.rep0 * MAX_PASSES * RADIX;
  for (uint32_t q = 0; q < np; q++) {
    uint32_t v = 0;
    for (uint32_t r = 0; r < T.nrep; r++) v += gh[(uint64_t)r * MAX_PASSES * RADIX + q * RADIX + threadIdx.x];
    uint32_t tot;
    const uint32_t ex = block_excl_sum(v, sc, &tot);
    gh[q * RADIX + threadIdx.x] = ex;
  }
}

// ---------------------------------------------------------- k_sort_pass
//
// One stable LSD pass on the 8-bit digit at bits [2 + 8 pass, 10 + 8 pass).
// Launched cooperatively: every workgroup is resident, and workgroup b
// handles tiles b, b + G, b + 2G, ... in order, so the lowest unfinished
// tile never waits on an unfinished one and the look-back always ends.
// Keys are loaded wave-striped (key index = wave * 1024 + item * 64 + lane)
// so that lane order within an item is key order.  Each item's digit is
// matched across the wave with eight ballots; the lowest matching lane
// advances the wave's per-digit counter, which gives every key a stable
// rank within its wave.  Per-digit wave offsets, the tile's digit counts
// and the look-back over earlier tiles of the trace (eight predecessors per
// round trip) give each key its destination; keys are staged in LDS in
// destination order and written out in runs per digit.

__global__ __launch_bounds__(NT) void k_sort_pass(const uint64_t* __restrict__ kin, uint64_t* __restrict__ kout,
                                                  const TraceDesc* __restrict__ desc, const TileRef* __restrict__ tiles,
                                                  const TraceLayout* __restrict__ lay, const uint32_t* __restrict__ hist,
                                                  uint64_t* status, Ctrl* ctrl, uint32_t n_tiles, uint32_t pass,
                                                  uint32_t tag) {
  __shared__ uint64_t s_keys[TILE];
  __shared__ uint32_t s_wh[NWAVE][RADIX];
  __shared__ uint32_t s_dstart[RADIX];
  __shared__ uint64_t s_gbase[RADIX];
  __shared__ uint32_t s_scan[NWAVE];

  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  const uint32_t d = threadIdx.x;

  for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const TileRef tr = tiles[tile];
    const TraceDesc T = desc[tr.trace];
    const TraceLayout L = lay[tr.trace];
    if (pass >= L.npasses) continue;  // uniform over the workgroup
    const uint32_t shift = 2 + RADIX_BITS * pass;
    const uint64_t start = (uint64_t)tr.local * TILE;
    const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
    const uint64_t* src = kin + T.off + start;

    for (uint32_t i = threadIdx.x; i < NWAVE * RADIX; i += NT) (&s_wh[0][0])[i] = 0;
    __syncthreads();

    uint64_t key[ITEMS];
    uint32_t rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t j = wave * (ITEMS * 64) + i * 64 + lane;
      key[i] = (j < n_in) ? src[j] : ~0ull;  // padding sorts last (digit 255, after every real key)
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t dg = (uint32_t)(key[i] >> shift) & (RADIX - 1);
      uint64_t m = ~0ull;
#pragma unroll
      for (int b = 0; b < (int)RADIX_BITS; b++) {
        const uint64_t bal = __ballot((dg >> b) & 1u);
        m &= ((dg >> b) & 1u) ? bal : ~bal;
      }
      const uint32_t before = (uint32_t)__popcll(m & lt_mask);
      const uint32_t old = s_wh[wave][dg];
      if (before == 0) s_wh[wave][dg] = old + (uint32_t)__popcll(m);
      rank[i] = old + before;
    }
    __syncthreads();

    // per digit: offsets of the waves, tile count, tile-local start
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; w++) {
      const uint32_t c = s_wh[w][d];
      s_wh[w][d] = cnt;
      cnt += c;
    }
    uint32_t tot;
    const uint32_t dstart = block_excl_sum(cnt, s_scan, &tot);
    s_dstart[d] = dstart;
    const uint32_t pub = (d == RADIX - 1) ? cnt - (TILE - n_in) : cnt;  // padding is not published

    uint64_t* st = status + (uint64_t)tile * RADIX;
    uint32_t excl = 0;
    if (tr.local == 0) {
      st_agent(&st[d], status_word(tag, FLAG_INCL, pub));
    } else {
      st_agent(&st[d], status_word(tag, FLAG_AGG, pub));
      // Look back over earlier tiles of this trace, LOOKBACK at a time.  The
      // first tile of a trace always publishes an inclusive count.
      int64_t p = (int64_t)tile - 1;
      const int64_t first = (int64_t)T.tile0;
      uint32_t spins = 0;
      bool done = false;
      while (!done) {
        uint64_t w[LOOKBACK];
#pragma unroll
        for (uint32_t k = 0; k < LOOKBACK; k++)
          w[k] = (p - (int64_t)k >= first) ? ld_agent(&status[(uint64_t)(p - k) * RADIX + d]) : 0ull;
        uint32_t k = 0;
        for (; k < LOOKBACK && p - (int64_t)k >= first; k++) {
          if (status_tag(w[k]) != tag || status_flag(w[k]) == 0) break;
          excl += (uint32_t)w[k];
          if (status_flag(w[k]) == FLAG_INCL) {
            done = true;
            break;
          }
        }
        if (done) break;
        p -= k;
        if (k < LOOKBACK && spin_exhausted(spins, ctrl)) break;
      }
      st_agent(&st[d], status_word(tag, FLAG_INCL, excl + pub));
    }
    const uint32_t* base = hist + (uint64_t)T.rep0 * MAX_PASSES * RADIX + (uint64_t)pass * RADIX;
    s_gbase[d] = T.off + (uint64_t)base[d] + excl - dstart;
    __syncthreads();

#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t dd = (uint32_t)(key[i] >> shift) & (RADIX - 1);
      s_keys[s_dstart[dd] + s_wh[wave][dd] + rank[i]] = key[i];
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < ITEMS; r++) {
      const uint32_t j = threadIdx.x + r * NT;
      if (j < n_in) {
        const uint64_t k = s_keys[j];
        const uint32_t dd = (uint32_t)(k >> shift) & (RADIX - 1);
        const uint64_t dst = s_gbase[dd] + j;
        if (dst - T.off < T.n) kout[dst] = k;
        else atomicOr(&ctrl->error_flags, ERR_INTERNAL_BOUNDS);
      }
    }
    __syncthreads();  // LDS is reused by the next tile
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

constexpr uint32_t LDS_PAD(uint32_t j) { return j + (j >> 4); }

__device__ __forceinline__ uint32_t cnt16(uint64_t packed, uint32_t q) { return (uint32_t)(packed >> (16 * q)) & 0xFFFFu; }

// Pairs of one element of class c against the open-run counts run[] (the
// counts of earlier elements of its location / block / epoch / thread runs
// inside the tile).
__device__ __forceinline__ void tile_pairs(uint32_t c, const uint64_t run[4], uint32_t v[5]) {
  uint32_t xb[3], in[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    xb[q] = cnt16(run[0], q) - cnt16(run[1], q);
    in[q] = cnt16(run[2], q) - cnt16(run[3], q);
  }
  element_pairs<uint32_t>(c, xb, in, v);
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

__device__ __forceinline__ void write_entry(RaceOut* dst, uint32_t trace, const TraceLayout& L, uint64_t key,
                                            const uint64_t S[5]) {
  RaceOut e;
  uint32_t sp, blk;
  uint64_t unit;
  key_location(L, key, sp, blk, unit);
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

// Staging area of a tile's complete locations: a dedicated buffer, or the
// tile's slice of the key buffer that no longer holds live keys.
__device__ __forceinline__ RaceOut* stage_of(const Buffers& b, uint32_t tile, const TraceDesc& T,
                                             const TraceLayout& L, uint64_t start, uint32_t n_in, uint32_t* cap) {
  if (b.stage) {
    *cap = TILE / 2 + 1;
    return b.stage + (uint64_t)tile * (TILE / 2 + 1);
  }
  *cap = n_in / 8;
  return (RaceOut*)(b.keys[(L.npasses & 1u) ^ 1u] + T.off + start);
}

__global__ __launch_bounds__(NT) void k_scan_tiles(Buffers b, uint32_t passes_done) {
  __shared__ uint64_t s_keys[LDS_PAD(TILE) + 1];
  __shared__ uint64_t s_scanA[NWAVE][4];
  __shared__ uint64_t s_scanB[NWAVE][3];
  __shared__ uint32_t s_scan32[NWAVE];
  __shared__ uint8_t s_firstlv[NT];
  __shared__ uint32_t s_lead[17];  // lead counts [l][c] (12), lead pair sums (5)
  __shared__ uint32_t s_min;
  __shared__ uint64_t s_prev, s_next;
  __shared__ uint32_t s_taillast;

  // nothing to do on an error, or when fewer radix passes ran than some
  // trace needs (the host then runs the missing passes and scans again)
  if (b.ctrl->error_flags) return;
  if (b.ctrl->max_passes > passes_done) return;
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  const uint32_t tile = blockIdx.x;
  if (tid < 17) s_lead[tid] = 0;
  if (tid == 0) s_min = NO_HEAD;
  const TileRef tr = b.tiles[tile];
  const TraceDesc T = b.desc[tr.trace];
  const TraceLayout L = b.layout[tr.trace];
  const uint64_t* keys = b.keys[L.npasses & 1u];
  const uint64_t start = (uint64_t)tr.local * TILE;
  const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
  const uint64_t* src = keys + T.off + start;
  const bool trace_end = start + n_in == T.n;

  for (uint32_t j = tid; j < (uint32_t)TILE; j += NT) s_keys[LDS_PAD(j)] = (j < n_in) ? src[j] : 0ull;
  if (tid == 0) {
    s_prev = tr.local > 0 ? src[-1] : 0ull;
    s_next = trace_end ? 0ull : src[n_in];
  }
  __syncthreads();
  if (tid == 0) s_taillast = trace_end ? 1u : (head_level(L, s_keys[LDS_PAD(n_in - 1)], s_next) == 0 ? 1u : 0u);

  // ---- element metadata: head level (3 bits) and class (2 bits)
  uint64_t key[ITEMS];
  uint32_t meta[ITEMS];
  uint32_t local_min = NO_HEAD;
  {
    uint64_t prev = tid > 0 ? s_keys[LDS_PAD(ITEMS * tid - 1)] : s_prev;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t j = ITEMS * tid + i;
      const uint64_t k = s_keys[LDS_PAD(j)];
      key[i] = k;
      uint32_t lv, c;
      if (j < n_in) {
        lv = (j == 0 && tr.local == 0) ? 0u : head_level(L, prev, k);
        c = action_class(k);
        local_min = min(local_min, lv);
      } else {
        lv = 4;
        c = CLS_NONE;
      }
      meta[i] = lv | (c << 3);
      prev = k;
    }
    s_firstlv[tid] = (uint8_t)(meta[0] & 7u);
  }
  local_min = wave_min(local_min);
  if (lane == 0 && local_min < NO_HEAD) atomicMin(&s_min, local_min);

  // ---- pass A: segmented class counts per level
  uint64_t aggA[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const uint32_t lv = meta[i] & 7u, c = meta[i] >> 3;
#pragma unroll
    for (int l = 0; l < 4; l++)
      if (lv <= (uint32_t)l) aggA[l] = SEGF;
    if (c != CLS_NONE) {
#pragma unroll
      for (int l = 0; l < 4; l++) aggA[l] += 1ull << (16 * c);
    }
  }
  uint64_t exA[4], totA[4];
  block_seg_scan<4>(aggA, exA, totA, s_scanA);

  // ---- pass B: pairs per element, summed per location run; lead data
  uint64_t aggB[3] = {0, 0, 0};
  {
    uint64_t run[4];
    bool seen[4];
#pragma unroll
    for (int l = 0; l < 4; l++) {
      run[l] = exA[l] & ~SEGF;
      seen[l] = (exA[l] & SEGF) != 0;
    }
    uint32_t leadc[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    uint32_t leads[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t lv = meta[i] & 7u, c = meta[i] >> 3;
#pragma unroll
      for (int l = 0; l < 4; l++)
        if (lv <= (uint32_t)l) {
          run[l] = 0;
          seen[l] = true;
        }
      if (c == CLS_NONE) continue;
      uint32_t v[5];
      tile_pairs(c, run, v);
      if (lv == 0) aggB[0] = aggB[1] = aggB[2] = SEGF;
      aggB[0] += (uint64_t)v[K_WW] | ((uint64_t)v[K_RW] << 32);
      aggB[1] += (uint64_t)v[K_AW] | ((uint64_t)v[K_AR] << 32);
      aggB[2] += (uint64_t)v[K_XB];
#pragma unroll
      for (int l = 0; l < 4; l++) {
        if (!seen[l]) leadc[l][c]++;
        run[l] += 1ull << (16 * c);
      }
      if (!seen[0]) {
#pragma unroll
        for (int k = 0; k < 5; k++) leads[k] += v[k];
      }
    }
#pragma unroll
    for (int l = 0; l < 4; l++)
#pragma unroll
      for (int q = 0; q < 3; q++)
        if (leadc[l][q]) atomicAdd(&s_lead[l * 3 + q], leadc[l][q]);
#pragma unroll
    for (int k = 0; k < 5; k++)
      if (leads[k]) atomicAdd(&s_lead[12 + k], leads[k]);
  }
  uint64_t exB[3], totB[3];
  block_seg_scan<3>(aggB, exB, totB, s_scanB);  // contains a barrier: s_lead and s_min are complete after it

  // ---- the tile summary (lanes of wave 0 write its words)
  if (wave == 0) {
    State agg;
    agg.m = s_min;
#pragma unroll
    for (int l = 0; l < 4; l++)
#pragma unroll
      for (int q = 0; q < 3; q++) {
        agg.lead[l][q] = s_lead[l * 3 + q];
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
  //      and ended inside the tile.  Reported at their last element.
  uint32_t n_emit = 0;
  auto walk_emit = [&](RaceOut* dst, uint32_t cap, uint32_t pos) {
    uint64_t run[4];
#pragma unroll
    for (int l = 0; l < 4; l++) run[l] = exA[l] & ~SEGF;
    uint64_t s0 = exB[0] & ~SEGF, s1 = exB[1] & ~SEGF, s2 = exB[2] & ~SEGF;
    bool seen0 = (exB[0] & SEGF) != 0;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      const uint32_t lv = meta[i] & 7u, c = meta[i] >> 3;
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
      const uint32_t j = ITEMS * tid + i;
      bool last;
      if (j + 1 == n_in) last = s_taillast != 0;
      else if (i + 1 < ITEMS) last = (meta[i + 1] & 7u) == 0;
      else last = s_firstlv[tid + 1] == 0;
      if (!last) continue;
      uint64_t S[5];
      S[K_WW] = (uint32_t)s0; S[K_RW] = (uint32_t)(s0 >> 32);
      S[K_AW] = (uint32_t)s1; S[K_AR] = (uint32_t)(s1 >> 32);
      S[K_XB] = (uint32_t)s2;
      if (S[K_WW] + S[K_RW] + S[K_AW] + S[K_AR] == 0) continue;
      if (dst) {
        if (pos < cap) write_entry(dst + pos, tr.trace, L, key[i], S);
        pos++;
      } else {
        n_emit++;
      }
    }
  };
  walk_emit(nullptr, 0, 0);
  uint32_t tile_emit;
  const uint32_t my_off = block_excl_sum(n_emit, s_scan32, &tile_emit);
  uint32_t cap;
  RaceOut* stage = stage_of(b, tile, T, L, start, n_in, &cap);
  if (n_emit) walk_emit(stage, cap, my_off);
  if (tid == 0) {
    b.tout[tile].in_count = tile_emit;
    if (tile_emit > cap) atomicOr(&b.ctrl->error_flags, ERR_STAGE_OVERFLOW);
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

__global__ __launch_bounds__(NT) void k_scan_cross(Buffers b, uint32_t passes_done) {
  if (b.ctrl->error_flags) return;
  if (b.ctrl->max_passes > passes_done) return;
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint32_t j = blockIdx.x * NWAVE + wave;
  if (j >= b.n_tiles) return;
  if (!b.tout[j].owns) {
    if (lane == 0) b.cross_flag[j] = 0;
    return;
  }
  const TileRef tr = b.tiles[j];
  const TraceDesc T = b.desc[tr.trace];
  const TraceLayout L = b.layout[tr.trace];
  const uint32_t last = T.tile0 + T.ntiles - 1;  // last tile of the trace

  // end of the span: the first later tile of the trace with a location head
  uint32_t k = j + 1;  // candidate
  bool to_end = false;
  while (true) {
    const uint32_t c = k + lane;
    const bool head = c <= last && b.agg[(uint64_t)c * SW] == 0;
    const uint64_t bal = __ballot(head);
    if (bal) {
      k += (uint32_t)__ffsll((unsigned long long)bal) - 1;
      break;
    }
    if (k + 64 > last) {
      to_end = true;
      break;
    }
    k += 64;
  }
  // combine summaries of tiles j .. end-1 (end = k, or last + 1 when the
  // location runs to the end of the trace)
  const uint32_t end = to_end ? last + 1 : k;
  State S = identity();
  for (uint32_t c0 = j; c0 < end; c0 += 64) {
    const uint32_t c = c0 + lane;
    State s = c < end ? load_state(b.agg + (uint64_t)c * SW) : identity();
#pragma unroll
    for (uint32_t dlt = 1; dlt < 64; dlt <<= 1) {
      const State o = shfl_down_state(s, dlt);
      if ((lane & (2 * dlt - 1)) == 0) s = combine(s, o);
    }
    S = combine(S, readlane_state(s, 0));
  }
  uint64_t fin[5];
  if (to_end) {
    const uint64_t* t = tail_sums(S);
#pragma unroll
    for (int q = 0; q < 5; q++) fin[q] = t[q];
  } else {
    open_sums(S, load_state(b.agg + (uint64_t)k * SW), fin);
  }
  const bool racing = fin[K_WW] + fin[K_RW] + fin[K_AW] + fin[K_AR] > 0;
  if (lane == 0) {
    b.cross_flag[j] = racing ? 1u : 0u;
    if (racing) {
      const uint64_t start = (uint64_t)tr.local * TILE;
      const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
      const uint64_t key = b.keys[L.npasses & 1u][T.off + start + n_in - 1];
      write_entry(&b.cross[j], tr.trace, L, key, fin);
    }
  }
}

// ------------------------------------------------------- ordered output
// Entries of tile j: its complete locations, then (if racing) the location
// it owns that crosses into later tiles.  Groups of 256 tiles.

__global__ __launch_bounds__(NT) void k_group_sums(Buffers b, uint32_t passes_done) {
  __shared__ uint32_t sc[NWAVE];
  if (b.ctrl->error_flags || b.ctrl->max_passes > passes_done) return;
  const uint32_t t = blockIdx.x * GROUP + threadIdx.x;
  const uint32_t c = t < b.n_tiles ? b.tout[t].in_count + b.cross_flag[t] : 0u;
  uint32_t tot;
  (void)block_excl_sum(c, sc, &tot);
  if (threadIdx.x == 0) b.group_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(NT) void k_group_scan(Buffers b, uint32_t n_groups, uint32_t passes_done) {
  __shared__ uint32_t sc[NWAVE];
  if (b.ctrl->error_flags || b.ctrl->max_passes > passes_done) return;
  const uint32_t per = (n_groups + NT - 1) / NT;
  const uint32_t g0 = threadIdx.x * per;
  uint64_t mine = 0;
  for (uint32_t g = g0; g < min(n_groups, g0 + per); g++) mine += b.group_sum[g];
  uint32_t tot;
  const uint32_t ex = block_excl_sum((uint32_t)mine, sc, &tot);
  uint64_t run = ex;
  for (uint32_t g = g0; g < min(n_groups, g0 + per); g++) {
    b.group_off[g] = run;
    run += b.group_sum[g];
  }
  if (threadIdx.x == 0) b.ctrl->total_entries = tot;
}

__global__ __launch_bounds__(NT) void k_scan_out(Buffers b, uint32_t passes_done) {
  __shared__ uint32_t sc[NWAVE];
  if (b.ctrl->error_flags || b.ctrl->max_passes > passes_done) return;
  const uint32_t t = blockIdx.x * GROUP + threadIdx.x;
  const bool valid = t < b.n_tiles;
  const uint32_t inc = valid ? b.tout[t].in_count : 0u;
  const uint32_t cf = valid ? b.cross_flag[t] : 0u;
  uint32_t tot;
  const uint32_t ex = block_excl_sum(inc + cf, sc, &tot);
  if (!valid || inc + cf == 0) return;
  uint64_t pos = b.group_off[blockIdx.x] + ex;
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

// -------------------------------------------------------- launch wrappers

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_init(const Buffers& b, hipStream_t s) {
  const uint64_t nh = (uint64_t)b.n_reps * MAX_PASSES * RADIX;
  const uint32_t grid = max(1u, min(2048u, cdiv(nh, NT)));
  hipLaunchKernelGGL(k_init, dim3(grid), dim3(NT), 0, s, b.hist, nh, b.ctrl);
  return hipGetLastError();
}
hipError_t launch_stats(const Buffers& b, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_stats, dim3(b.n_tiles), dim3(NT), 0, s, (const ulonglong2*)b.records, b.desc, b.tiles,
                     b.stats_part);
  return hipGetLastError();
}
hipError_t launch_layout(const Buffers& b, hipStream_t s) {
  if (!b.n_traces) return hipSuccess;
  hipLaunchKernelGGL(k_layout, dim3(b.n_traces), dim3(NT), 0, s, b.desc, b.stats_part, b.layout, b.ctrl);
  return hipGetLastError();
}
hipError_t launch_keygen(const Buffers& b, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_keygen, dim3(b.n_tiles), dim3(NT), 0, s, (const ulonglong2*)b.records, b.desc, b.tiles,
                     b.layout, b.keys[0], b.hist);
  return hipGetLastError();
}
hipError_t launch_digits(const Buffers& b, hipStream_t s) {
  if (!b.n_traces) return hipSuccess;
  hipLaunchKernelGGL(k_digits, dim3(b.n_traces), dim3(NT), 0, s, b.desc, b.layout, b.hist);
  return hipGetLastError();
}
hipError_t launch_sort_pass(const Buffers& b, uint32_t pass, uint32_t tag, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  const uint64_t* kin = b.keys[pass & 1];
  uint64_t* kout = b.keys[(pass + 1) & 1];
  const TraceDesc* desc = b.desc;
  const TileRef* tiles = b.tiles;
  const TraceLayout* lay = b.layout;
  const uint32_t* hist = b.hist;
  uint64_t* status = b.sort_status;
  Ctrl* ctrl = b.ctrl;
  uint32_t n_tiles = b.n_tiles;
  void* args[] = {&kin, &kout, &desc, &tiles, &lay, &hist, &status, &ctrl, &n_tiles, &pass, &tag};
  const uint32_t grid = min(b.n_tiles, b.sort_grid);
  return hipLaunchCooperativeKernel((const void*)k_sort_pass, dim3(grid), dim3(NT), args, 0, s);
}
hipError_t launch_scan_tiles(const Buffers& b, uint32_t passes_done, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_scan_tiles, dim3(b.n_tiles), dim3(NT), 0, s, b, passes_done);
  return hipGetLastError();
}
hipError_t launch_scan_cross(const Buffers& b, uint32_t passes_done, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_scan_cross, dim3(cdiv(b.n_tiles, NWAVE)), dim3(NT), 0, s, b, passes_done);
  return hipGetLastError();
}
hipError_t launch_scan_out(const Buffers& b, uint32_t passes_done, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  const uint32_t n_groups = cdiv(b.n_tiles, GROUP);
  hipLaunchKernelGGL(k_group_sums, dim3(n_groups), dim3(NT), 0, s, b, passes_done);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(NT), 0, s, b, n_groups, passes_done);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_out, dim3(n_groups), dim3(NT), 0, s, b, passes_done);
  return hipGetLastError();
}
hipError_t launch_reset_errors(const Buffers& b, uint32_t mask, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_errors, dim3(1), dim3(64), 0, s, b.ctrl, mask);
  return hipGetLastError();
}

int sort_pass_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_sort_pass, NT, 0) != hipSuccess) return 0;
  return nb;
}

}  // namespace sc
