// kernels.hip -- gfx950 kernels of the Memory-Model data-race check.
//
// Pipeline for a call over one or more traces (records of a trace are
// contiguous; every kernel works on 4096-record tiles, a tile never spans
// two traces):
//   k_init       reset per-call state
//   k_stats      per-trace unit ranges, largest tid and epoch, record checks
//   k_layout     per-trace key layout (keys.h)
//   k_keygen     records -> 64-bit keys, digit histograms of every radix pass
//   k_digits     exclusive scan of the histograms (digit bases)
//   k_sort_pass  one stable LSD radix pass, 8-bit digits (x passes)
//   k_scan       racing-pair counts per location over the sorted keys
//                (segstate.h), ordered emission of racing locations
//
// k_sort_pass and k_scan take tiles from a ticket counter in launch order,
// so every tile they wait on has already started, and chain tiles with a
// decoupled look-back: each tile publishes its own summary first, then its
// inclusive prefix once the predecessors' summaries are in.  Status words
// carry a 24-bit tag unique to the launch, so no status memory is cleared
// between launches; every status word is written and read with agent-scope
// atomics, which keeps them coherent across the XCDs' L2 caches.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "segstate.h"

namespace sc {

constexpr int NWAVE = NT / 64;
static_assert(NT == (int)RADIX, "one thread per digit in k_sort_pass");
constexpr uint64_t SEGF = 1ull << 63;   // head flag of packed segmented values
constexpr uint32_t CLS_NONE = 3;        // padding element past the end of a trace

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

__global__ void k_init(const TraceDesc* __restrict__ desc, uint32_t n_traces, TraceStats* stats,
                       Summary* summ, uint32_t* hist, Ctrl* ctrl) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    for (int t = 0; t < 16; t++) ctrl->ticket[t] = 0;
    ctrl->max_passes = 0;
    ctrl->error_flags = 0;
    ctrl->first_bad = ~0ull;
    ctrl->total_entries = 0;
  }
  if (i < n_traces) {
    stats_init(stats[i]);
    summ[i].n_records = desc[i].n;
    summ[i].n_race_locs = 0;
    summ[i].n_pairs = 0;
  }
  const uint64_t nh = (uint64_t)n_traces * MAX_PASSES * RADIX;
  for (uint64_t j = i; j < nh; j += (uint64_t)gridDim.x * blockDim.x) hist[j] = 0;
}

// -------------------------------------------------------------- k_stats

__global__ __launch_bounds__(NT) void k_stats(const ulonglong2* __restrict__ recs, const TraceDesc* __restrict__ desc,
                                              const TileRef* __restrict__ tiles, TraceStats* stats) {
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
    TraceStats* S = &stats[tr.trace];
    if (gmin <= gmax) {
      atomicMin((unsigned long long*)&S->gmin, (unsigned long long)gmin);
      atomicMax((unsigned long long*)&S->gmax, (unsigned long long)gmax);
    }
    if (smin <= smax) {
      atomicMin((unsigned long long*)&S->smin, (unsigned long long)smin);
      atomicMax((unsigned long long*)&S->smax, (unsigned long long)smax);
    }
    if (bad != ~0ull) atomicMin((unsigned long long*)&S->bad_index, (unsigned long long)bad);
    atomicMax(&S->max_tid, mt);
    atomicMax(&S->max_epoch, me);
  }
}

// ------------------------------------------------------------- k_layout

__global__ void k_layout(const TraceDesc* __restrict__ desc, uint32_t n_traces, const TraceStats* __restrict__ stats,
                         TraceLayout* lay, Ctrl* ctrl) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_traces) return;
  TraceLayout L = make_layout(stats[i], desc[i].tpb);
  if (desc[i].n == 0) {
    L.error = 0;
    L.npasses = 0;
  }
  lay[i] = L;
  if (L.error) {
    atomicOr(&ctrl->error_flags, L.error);
    if (L.error & LAYOUT_ERR_RECORD)
      atomicMin((unsigned long long*)&ctrl->first_bad, (unsigned long long)(desc[i].off + stats[i].bad_index));
  }
  atomicMax(&ctrl->max_passes, L.npasses);
}

// ------------------------------------------------------------- k_keygen

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
  uint32_t* gh = hist + (uint64_t)tr.trace * MAX_PASSES * RADIX;
  for (uint32_t i = threadIdx.x; i < np * RADIX; i += NT) {
    const uint32_t c = h[i];
    if (c) atomicAdd(&gh[i], c);
  }
}

// ------------------------------------------------------------- k_digits

__global__ __launch_bounds__(NT) void k_digits(const TraceLayout* __restrict__ lay, uint32_t* hist) {
  __shared__ uint32_t sc[NWAVE];
  const uint32_t trace = blockIdx.x;
  const uint32_t np = lay[trace].npasses;
  uint32_t* gh = hist + (uint64_t)trace * MAX_PASSES * RADIX;
  for (uint32_t q = 0; q < np; q++) {
    const uint32_t v = gh[q * RADIX + threadIdx.x];
    uint32_t tot;
    const uint32_t ex = block_excl_sum(v, sc, &tot);
    gh[q * RADIX + threadIdx.x] = ex;
  }
}

// ---------------------------------------------------------- k_sort_pass
//
// One stable LSD pass on the 8-bit digit at bits [2 + 8 pass, 10 + 8 pass).
// Keys are loaded wave-striped (key index = wave * 1024 + item * 64 + lane)
// so that lane order within an item is key order.  Each item's digit is
// matched across the wave with eight ballots; the lowest matching lane
// advances the wave's per-digit counter, which gives every key a stable
// rank within its wave.  Per-digit wave offsets, the tile's digit counts
// and the look-back over earlier tiles of the trace then give each key its
// destination; keys are staged in LDS in destination order and written out
// in runs per digit.

__global__ __launch_bounds__(NT) void k_sort_pass(const uint64_t* __restrict__ kin, uint64_t* __restrict__ kout,
                                                  const TraceDesc* __restrict__ desc, const TileRef* __restrict__ tiles,
                                                  const TraceLayout* __restrict__ lay, const uint32_t* __restrict__ hist,
                                                  uint64_t* status, Ctrl* ctrl, uint32_t pass, uint32_t tag) {
  __shared__ uint64_t s_keys[TILE];
  __shared__ uint32_t s_wh[NWAVE][RADIX];
  __shared__ uint32_t s_dstart[RADIX];
  __shared__ uint64_t s_gbase[RADIX];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_scan[NWAVE];

  if (pass >= __hip_atomic_load(&ctrl->max_passes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  if (threadIdx.x == 0) s_tile = atomicAdd(&ctrl->ticket[pass], 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const TileRef tr = tiles[tile];
  const TraceDesc T = desc[tr.trace];
  const TraceLayout L = lay[tr.trace];
  if (pass >= L.npasses) return;
  const uint32_t shift = 2 + RADIX_BITS * pass;
  const uint64_t start = (uint64_t)tr.local * TILE;
  const uint32_t n_in = (uint32_t)min<uint64_t>((uint64_t)TILE, T.n - start);
  const uint64_t* src = kin + T.off + start;

  for (uint32_t i = threadIdx.x; i < NWAVE * RADIX; i += NT) (&s_wh[0][0])[i] = 0;
  __syncthreads();

  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint64_t key[ITEMS];
  uint32_t rank[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const uint32_t j = wave * (ITEMS * 64) + i * 64 + lane;
    key[i] = (j < n_in) ? src[j] : ~0ull;  // padding sorts last (digit 255, after every real key)
  }
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    const uint32_t d = (uint32_t)(key[i] >> shift) & (RADIX - 1);
    uint64_t m = ~0ull;
#pragma unroll
    for (int b = 0; b < (int)RADIX_BITS; b++) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t before = (uint32_t)__popcll(m & lt_mask);
    const uint32_t old = s_wh[wave][d];
    if (before == 0) s_wh[wave][d] = old + (uint32_t)__popcll(m);
    rank[i] = old + before;
  }
  __syncthreads();

  // per digit: offsets of the waves, tile count, tile-local start
  const uint32_t d = threadIdx.x;
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
    uint64_t p = tile - 1;
    uint32_t spins = 0;
    while (true) {
      const uint64_t w = ld_agent(&status[p * RADIX + d]);
      if (status_tag(w) != tag || status_flag(w) == 0) {
        if (spin_exhausted(spins, ctrl)) break;
        continue;
      }
      excl += (uint32_t)w;
      if (status_flag(w) == FLAG_INCL) break;
      p--;
    }
    st_agent(&st[d], status_word(tag, FLAG_INCL, excl + pub));
  }
  const uint32_t* base = hist + (uint64_t)tr.trace * MAX_PASSES * RADIX + (uint64_t)pass * RADIX;
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
}

// --------------------------------------------------------------- k_scan
//
// Racing pairs per location over one tile of sorted keys.  Thread t holds
// keys 16 t .. 16 t + 15 of the tile.  Three workgroup passes:
//   A  segmented class counts per level (location, block, epoch, thread):
//      for every element, the counts of earlier elements of its open runs;
//   B  each element's pairs with earlier partners (segstate.h), summed per
//      location run;
//   C  the tile summary (State) for the look-back, whose inclusive prefix
//      gives the pair sums of the location run entering the tile.
// A location is reported by the tile holding its last element.  Counts
// inside a tile fit 16 bits and pair sums 32 bits; sums across tiles are
// 64-bit.

constexpr uint32_t LDS_PAD(uint32_t j) { return j + (j >> 4); }

struct Walk {
  uint64_t run[4];   // packed class counts of the open runs (16 bits each), flag = head seen
};

__device__ __forceinline__ uint32_t cnt16(uint64_t packed, uint32_t q) { return (uint32_t)(packed >> (16 * q)) & 0xFFFFu; }

__device__ __forceinline__ void state_words_store(uint64_t* slot, const State& s, uint32_t tag, uint32_t flag,
                                                  uint32_t lane) {
  uint32_t w = 0;
#pragma unroll
  for (int i = 0; i < SW; i++) {
    uint32_t v;
    if (i == 0) v = s.m;
    else if (i < 13) v = s.lead[(i - 1) / 3][(i - 1) % 3];
    else if (i < 25) v = s.trail[(i - 13) / 3][(i - 13) % 3];
    else if (i < 35) v = (uint32_t)(s.leadsum[(i - 25) / 2] >> (32 * ((i - 25) % 2)));
    else v = (uint32_t)(s.trailsum[(i - 35) / 2] >> (32 * ((i - 35) % 2)));
    if ((int)lane == i) w = v;
  }
  if (lane < (uint32_t)SW) st_agent(&slot[lane], status_word(tag, flag, w));
}

__device__ __forceinline__ State state_from_lanes(uint32_t w) {
  State s;
  s.m = __builtin_amdgcn_readlane(w, 0);
#pragma unroll
  for (int l = 0; l < 4; l++)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      s.lead[l][q] = __builtin_amdgcn_readlane(w, 1 + l * 3 + q);
      s.trail[l][q] = __builtin_amdgcn_readlane(w, 13 + l * 3 + q);
    }
#pragma unroll
  for (int k = 0; k < 5; k++) {
    s.leadsum[k] = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(w, 25 + 2 * k) |
                   ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(w, 26 + 2 * k) << 32);
    s.trailsum[k] = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(w, 35 + 2 * k) |
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(w, 36 + 2 * k) << 32);
  }
  return s;
}

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

__global__ __launch_bounds__(NT) void k_scan(const uint64_t* __restrict__ keys0, const uint64_t* __restrict__ keys1,
                                             const TraceDesc* __restrict__ desc, const TileRef* __restrict__ tiles,
                                             const TraceLayout* __restrict__ lay, uint64_t* seg_status,
                                             uint64_t* cnt_status, Ctrl* ctrl, Summary* summ, RaceOut* out,
                                             uint64_t out_cap, uint32_t n_tiles, uint32_t tag) {
  __shared__ uint64_t s_keys[LDS_PAD(TILE) + 1];
  __shared__ uint64_t s_scanA[NWAVE][4];
  __shared__ uint64_t s_scanB[NWAVE][3];
  __shared__ uint32_t s_scan32[NWAVE];
  __shared__ uint8_t s_firstlv[NT];
  __shared__ uint32_t s_lead[17];   // lead counts [l][c] (12), lead pair sums (5)
  __shared__ uint32_t s_min;
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_prev, s_next;
  __shared__ uint32_t s_taillast;
  __shared__ uint64_t s_open[5];
  __shared__ uint64_t s_outbase;

  if (__hip_atomic_load(&ctrl->error_flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(&ctrl->ticket[8], 1u);
  if (tid < 17) s_lead[tid] = 0;
  if (tid == 0) s_min = NO_HEAD;
  __syncthreads();
  const uint32_t tile = s_tile;
  const TileRef tr = tiles[tile];
  const TraceDesc T = desc[tr.trace];
  const TraceLayout L = lay[tr.trace];
  const uint64_t* keys = (L.npasses & 1u) ? keys1 : keys0;
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

  // ---- pass C: tile summary and look-back (wave 0)
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
    agg.trailsum[K_WW] = (uint32_t)totB[0];
    agg.trailsum[K_RW] = (uint32_t)(totB[0] >> 32) & 0x7FFFFFFFu;
    agg.trailsum[K_AW] = (uint32_t)totB[1];
    agg.trailsum[K_AR] = (uint32_t)(totB[1] >> 32) & 0x7FFFFFFFu;
    agg.trailsum[K_XB] = (uint32_t)totB[2];
    if (agg.m != 0)
      for (int k = 0; k < 5; k++) agg.trailsum[k] = 0;

    uint64_t* my = seg_status + (uint64_t)tile * 2 * SW;
    State E = identity();
    if (tr.local == 0) {
      state_words_store(my + SW, agg, tag, FLAG_INCL, lane);
    } else {
      state_words_store(my, agg, tag, FLAG_AGG, lane);
      uint64_t p = tile - 1;
      uint32_t spins = 0;
      while (true) {
        const uint64_t* ps = seg_status + p * 2 * SW;
        uint64_t wi = lane < (uint32_t)SW ? ld_agent(&ps[SW + lane]) : status_word(tag, 0, 0);
        if (__ballot(status_tag(wi) != tag) == 0) {
          E = combine(state_from_lanes((uint32_t)wi), E);
          break;
        }
        uint64_t wa = lane < (uint32_t)SW ? ld_agent(&ps[lane]) : status_word(tag, 0, 0);
        if (__ballot(status_tag(wa) != tag) == 0) {
          E = combine(state_from_lanes((uint32_t)wa), E);
          p--;
          continue;
        }
        if (spin_exhausted(spins, ctrl)) break;
      }
      state_words_store(my + SW, combine(E, agg), tag, FLAG_INCL, lane);
    }
    uint64_t open[5];
    open_sums(E, agg, open);
    if (lane < 5) s_open[lane] = open[lane];
  }
  __syncthreads();

  // ---- emission: a location is reported by the element that ends it
  uint32_t n_emit = 0;
  uint64_t pairs = 0;
  auto walk_emit = [&](bool write, uint64_t outpos) {
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
      const uint32_t j = ITEMS * tid + i;
      bool last;
      if (j + 1 == n_in) last = s_taillast != 0;
      else if (i + 1 < ITEMS) last = (meta[i + 1] & 7u) == 0;
      else last = s_firstlv[tid + 1] == 0;
      if (!last) continue;
      uint64_t S[5];
      if (seen0) {
        S[K_WW] = (uint32_t)s0; S[K_RW] = (uint32_t)(s0 >> 32);
        S[K_AW] = (uint32_t)s1; S[K_AR] = (uint32_t)(s1 >> 32);
        S[K_XB] = (uint32_t)s2;
      } else {
#pragma unroll
        for (int k = 0; k < 5; k++) S[k] = s_open[k];
      }
      if (S[K_WW] + S[K_RW] + S[K_AW] + S[K_AR] == 0) continue;
      if (write) {
        if (outpos < out_cap) {
          RaceOut e;
          uint32_t sp, blk;
          uint64_t unit;
          key_location(L, key[i], sp, blk, unit);
          e.trace = tr.trace;
          e.space = (uint8_t)sp;
          e.kinds = (uint8_t)((S[K_WW] ? 1 : 0) | (S[K_RW] ? 2 : 0) | (S[K_AW] ? 4 : 0) | (S[K_AR] ? 8 : 0) |
                              (S[K_XB] ? 16 : 0));
          e.reserved16 = 0;
          e.block = blk;
          e.reserved32 = 0;
          e.unit = unit;
          e.ww = S[K_WW]; e.rw = S[K_RW]; e.aw = S[K_AW]; e.ar = S[K_AR]; e.xb = S[K_XB];
          out[outpos] = e;
        }
        pairs += S[K_WW] + S[K_RW] + S[K_AW] + S[K_AR];
        outpos++;
      } else {
        n_emit++;
      }
    }
  };
  walk_emit(false, 0);
  uint32_t tile_emit;
  const uint32_t my_off = block_excl_sum(n_emit, s_scan32, &tile_emit);

  // ---- ordered output offset: look-back over the emission counts of all
  //      earlier tiles of the call
  if (tid == 0) {
    uint64_t excl = 0;
    if (tile == 0) {
      st_agent(&cnt_status[tile], status_word(tag, FLAG_INCL, tile_emit));
    } else {
      st_agent(&cnt_status[tile], status_word(tag, FLAG_AGG, tile_emit));
      uint64_t p = tile - 1;
      uint32_t spins = 0;
      while (true) {
        const uint64_t w = ld_agent(&cnt_status[p]);
        if (status_tag(w) != tag || status_flag(w) == 0) {
          if (spin_exhausted(spins, ctrl)) break;
          continue;
        }
        excl += (uint32_t)w;
        if (status_flag(w) == FLAG_INCL) break;
        p--;
      }
      st_agent(&cnt_status[tile], status_word(tag, FLAG_INCL, (uint32_t)(excl + tile_emit)));
    }
    s_outbase = excl;
    if (tile + 1 == n_tiles) ctrl->total_entries = excl + tile_emit;
  }
  __syncthreads();
  if (n_emit) walk_emit(true, s_outbase + my_off);

  // ---- per-trace summary
  pairs = __shfl_xor(pairs, 1, 64) + pairs;
  pairs = __shfl_xor(pairs, 2, 64) + pairs;
  pairs = __shfl_xor(pairs, 4, 64) + pairs;
  pairs = __shfl_xor(pairs, 8, 64) + pairs;
  pairs = __shfl_xor(pairs, 16, 64) + pairs;
  pairs = __shfl_xor(pairs, 32, 64) + pairs;
  if (lane == 0 && pairs) atomicAdd((unsigned long long*)&summ[tr.trace].n_pairs, (unsigned long long)pairs);
  if (tid == 0 && tile_emit) atomicAdd((unsigned long long*)&summ[tr.trace].n_race_locs, (unsigned long long)tile_emit);
}

__global__ void k_scan_reset(Ctrl* ctrl, Summary* summ, uint32_t n_traces) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctrl->ticket[8] = 0;
    ctrl->total_entries = 0;
  }
  if (i < n_traces) {
    summ[i].n_race_locs = 0;
    summ[i].n_pairs = 0;
  }
}

// -------------------------------------------------------- launch wrappers

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_init(const Buffers& b, hipStream_t s) {
  const uint32_t grid = max(1u, min(4096u, cdiv((uint64_t)b.n_traces * MAX_PASSES * RADIX, NT)));
  const uint32_t g2 = max(grid, cdiv(b.n_traces, NT));
  hipLaunchKernelGGL(k_init, dim3(g2), dim3(NT), 0, s, b.desc, b.n_traces, b.stats, b.summary, b.hist, b.ctrl);
  return hipGetLastError();
}
hipError_t launch_stats(const Buffers& b, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_stats, dim3(b.n_tiles), dim3(NT), 0, s, (const ulonglong2*)b.records, b.desc, b.tiles, b.stats);
  return hipGetLastError();
}
hipError_t launch_layout(const Buffers& b, hipStream_t s) {
  if (!b.n_traces) return hipSuccess;
  hipLaunchKernelGGL(k_layout, dim3(cdiv(b.n_traces, NT)), dim3(NT), 0, s, b.desc, b.n_traces, b.stats, b.layout,
                     b.ctrl);
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
  hipLaunchKernelGGL(k_digits, dim3(b.n_traces), dim3(NT), 0, s, b.layout, b.hist);
  return hipGetLastError();
}
hipError_t launch_sort_pass(const Buffers& b, uint32_t pass, uint32_t tag, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_sort_pass, dim3(b.n_tiles), dim3(NT), 0, s, b.keys[pass & 1], b.keys[(pass + 1) & 1], b.desc,
                     b.tiles, b.layout, b.hist, b.sort_status, b.ctrl, pass, tag);
  return hipGetLastError();
}
hipError_t launch_scan(const Buffers& b, uint32_t tag, hipStream_t s) {
  if (!b.n_tiles) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(b.n_tiles), dim3(NT), 0, s, b.keys[0], b.keys[1], b.desc, b.tiles, b.layout,
                     b.seg_status, b.cnt_status, b.ctrl, b.summary, b.out, b.out_cap, b.n_tiles, tag);
  return hipGetLastError();
}
hipError_t launch_scan_reset(const Buffers& b, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_reset, dim3(max(1u, cdiv(b.n_traces, NT))), dim3(NT), 0, s, b.ctrl, b.summary,
                     b.n_traces);
  return hipGetLastError();
}

}  // namespace sc
