// keys.h -- per-trace sort-key layout for the race check.
//
// Every record of a trace is packed into one key whose order groups
// the records first by location (the paper's Memory Unit, Sec. 4.2.1: one
// unit of global memory, or one unit of one block's shared memory, Alg. 3),
// then by block, by epoch (visit order) and by thread, with the action in
// the two lowest bits:
//
//   global : [0 | unit - gmin : ug | block : bb | epoch : eb | local tid : tb | side : sb | action : 2]
//   shared : [1 | block : bb | unit - smin : us | epoch : eb | local tid : tb | side : sb | action : 2]
//
// The side field is empty (sb = 0) except in the warp-aware check, where it
// holds the record's divergence bit above its statement id (Theorem 1,
// clauses 2 and 3): below the thread, so a thread's records stay one run and
// the threads of one warp stay adjacent.
//
// The fields between the space bit and the epoch field span wl = max(ug + bb,
// bb + us) bits in both layouts.  Field widths come from per-trace minima
// and maxima, so a key is lossless and the record can be read back from it.
// A key of at most 64 bits is one word; a wider one (up to 128 bits: a unit
// span near 2^64 in one trace) is a 128-bit integer, two words.
// Within a location the key orders records by (block, epoch, thread), which
// makes every group used by the race count contiguous after sorting.
//
// Functions are usable from host and device code.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define SC_HD __host__ __device__ __forceinline__
#else
#define SC_HD static inline
#endif

namespace sc {

// Per-trace statistics, reduced over all records of a trace.
struct TraceStats {
  uint64_t gmin, gmax;  // unit range of global records (gmin > gmax: none)
  uint64_t smin, smax;  // unit range of shared records
  uint64_t bad_index;   // smallest trace-relative index of an invalid record (~0: none)
  uint32_t max_tid;
  uint32_t max_epoch;
  uint32_t max_stmt;    // largest statement id (warp-aware check; 0 otherwise)
  uint32_t pad;
};

// Key layout of one trace.
struct TraceLayout {
  uint64_t gmin, smin;
  uint32_t tb, eb, bb, ug, us, wl;
  uint32_t key_bits;   // total bits including the action bits
  uint32_t npasses;    // radix passes over bits [2, key_bits) (pass_shift gives each pass's digit)
  uint32_t shift_e;    // epoch field
  uint32_t shift_b;    // block field of global keys; unit field of shared keys
  uint32_t shift_ug;   // unit field of global keys
  uint32_t shift_bs;   // block field of shared keys
  uint32_t shift_space;
  uint32_t error;      // LAYOUT_ERR_* bits
  uint32_t wide;       // 1: the key needs more than 64 bits (two-word keys)
  uint32_t max_epoch;  // largest epoch of the trace (its barrier boundaries are 0 .. max_epoch - 1)
  uint32_t sb;         // side field bits (0, or the divergence bit and the statement id's bits)
  uint64_t grange;     // largest minus smallest global unit (0 without global records)
  uint64_t srange;     // the same over shared units
};

// LAYOUT_ERR_* are per-trace layout errors; ERR_INTERNAL_BOUNDS is raised by
// the scatter's own check (a digit's destination range outside its trace)
// and reported as a device error.
enum : uint32_t { LAYOUT_ERR_WIDE = 1, LAYOUT_ERR_RECORD = 2, ERR_INTERNAL_BOUNDS = 4 };

// Radix digits: pass 0 sorts the 8 bits [2, 10); every later pass of a call
// sorts `db` bits (the call's digit width, RADIX_BITS or RADIX_WIDE_BITS),
// so pass p >= 1 sorts bits [10 + db (p - 1), 10 + db p).
constexpr uint32_t RADIX_BITS = 8;
constexpr uint32_t RADIX = 1u << RADIX_BITS;
constexpr uint32_t RADIX_WIDE_BITS = 9;
constexpr uint32_t RADIX_MAX = 1u << RADIX_WIDE_BITS;
constexpr uint32_t MAX_PASSES = 16;  // ceil(126 / 8)

SC_HD uint32_t pass_shift(uint32_t pass, uint32_t db) { return pass == 0 ? 2u : 2u + RADIX_BITS + db * (pass - 1); }

// Passes that sort `sorted` (>= 1) key bits with digits of width db after
// the first.
SC_HD uint32_t radix_passes(uint32_t sorted, uint32_t db) {
  return sorted <= RADIX_BITS ? 1u : 1u + (sorted - RADIX_BITS + db - 1) / db;
}

// A key of a trace wider than 64 bits: two words, one 128-bit integer.
typedef unsigned __int128 u128;

SC_HD uint32_t bits32(uint32_t x) { return x ? 32u - (uint32_t)__builtin_clz(x) : 0u; }
SC_HD uint32_t bits64(uint64_t x) { return x ? 64u - (uint32_t)__builtin_clzll(x) : 0u; }
SC_HD uint64_t lowmask(uint32_t b) { return b >= 64 ? ~0ull : ((1ull << b) - 1); }

SC_HD void stats_init(TraceStats& s) {
  s.gmin = ~0ull; s.gmax = 0; s.smin = ~0ull; s.smax = 0;
  s.bad_index = ~0ull; s.max_tid = 0; s.max_epoch = 0; s.max_stmt = 0; s.pad = 0;
}

// warp: the key carries the side field (divergence bit and statement id).
SC_HD TraceLayout make_layout(const TraceStats& s, uint32_t tpb, bool warp = false, uint32_t db = RADIX_BITS) {
  TraceLayout L;
  const bool has_g = s.gmin <= s.gmax;
  const bool has_s = s.smin <= s.smax;
  L.gmin = has_g ? s.gmin : 0;
  L.smin = has_s ? s.smin : 0;
  L.tb = bits32(tpb - 1);
  L.eb = bits32(s.max_epoch);
  L.bb = bits32(s.max_tid / tpb);
  L.ug = has_g ? bits64(s.gmax - s.gmin) : 0;
  L.us = has_s ? bits64(s.smax - s.smin) : 0;
  const uint32_t wg = L.ug + L.bb, ws = L.bb + L.us;
  L.wl = wg > ws ? wg : ws;
  L.sb = warp ? 1 + bits32(s.max_stmt) : 0;
  L.key_bits = 3 + L.sb + L.tb + L.eb + L.wl;
  L.shift_e = 2 + L.sb + L.tb;
  L.shift_b = L.shift_e + L.eb;
  L.shift_ug = L.shift_b + L.bb;
  L.shift_bs = L.shift_b + L.us;
  L.shift_space = L.shift_e + L.eb + L.wl;
  L.error = 0;
  L.wide = L.key_bits > 64 ? 1u : 0u;
  L.max_epoch = s.max_epoch;
  L.grange = has_g ? s.gmax - s.gmin : 0;
  L.srange = has_s ? s.smax - s.smin : 0;
  if (L.key_bits > 128) L.error |= LAYOUT_ERR_WIDE;
  if (s.bad_index != ~0ull) L.error |= LAYOUT_ERR_RECORD;
  L.npasses = L.error ? 0 : radix_passes(L.key_bits - 2, db);
  return L;
}

// How make_key_t finds a thread's block: a shift (the block size is a power
// of two, tb = log2 tpb), a division, or whichever of the two fits, chosen
// per call.  Callers that know the block size's form pick the first two:
// the third computes both on a device.
enum : int { BLK_ANY = 0, BLK_POW2 = 1, BLK_DIV = 2 };

// Divergence bit of a side word (its statement id is the other 31 bits).
constexpr uint32_t SIDE_DIVERGED = 0x80000000u;

// Key of one record (fields must be valid and within the trace's ranges);
// K is uint64_t for keys of at most 64 bits, u128 otherwise.  side: the
// record's side word when the layout has a side field (ignored otherwise).
template <typename K, int BLK = BLK_ANY>
SC_HD K make_key_t(const TraceLayout& L, uint64_t unit, uint32_t tid, uint32_t epoch, uint32_t action, uint32_t space,
                   uint32_t tpb, uint32_t side = 0) {
  const bool pow2 = BLK == BLK_POW2 || (BLK == BLK_ANY && (tpb & (tpb - 1)) == 0);
  const uint32_t blk = pow2 ? tid >> L.tb : tid / tpb;
  const uint32_t loc = tid - blk * tpb;
  K low = ((K)epoch << L.shift_e) | ((K)loc << (2 + L.sb)) | (K)(action & 3u);
  if (L.sb)
    low |= ((K)((side & SIDE_DIVERGED) ? 1u : 0u) << (1 + L.sb)) | ((K)(side & ~SIDE_DIVERGED) << 2);
  if (space == 0) return ((K)(unit - L.gmin) << L.shift_ug) | ((K)blk << L.shift_b) | low;
  return ((K)1 << L.shift_space) | ((K)blk << L.shift_bs) | ((K)(unit - L.smin) << L.shift_b) | low;
}
SC_HD uint64_t make_key(const TraceLayout& L, uint64_t unit, uint32_t tid, uint32_t epoch, uint32_t action,
                        uint32_t space, uint32_t tpb) {
  return make_key_t<uint64_t>(L, unit, tid, epoch, action, space, tpb);
}

// Highest set bit of a nonzero key.
SC_HD uint32_t top_bit(uint64_t x) { return 63u - (uint32_t)__builtin_clzll(x); }
SC_HD uint32_t top_bit(u128 x) {
  const uint64_t hi = (uint64_t)(x >> 64);
  return hi ? 127u - (uint32_t)__builtin_clzll(hi) : 63u - (uint32_t)__builtin_clzll((uint64_t)x);
}

// Nesting level at which key x starts a new group relative to the previous
// key p of the same trace: 0 new location, 1 new block (global only),
// 2 new epoch, 3 new thread, 4 same (location, block, epoch, thread).
template <typename K>
SC_HD uint32_t head_level_t(const TraceLayout& L, K p, K x) {
  // written with selects only: it runs for every key of the tile scan; the
  // action and side fields below the thread do not start a group
  const K d = (x ^ p) & ~(K)lowmask(2 + L.sb);
  const uint32_t hb = d != 0 ? top_bit(d) : 0u;  // highest differing bit
  const bool shared = ((x >> L.shift_space) & 1u) != 0;
  const uint32_t inner = hb >= L.shift_e ? 2u : 3u;          // epoch or thread
  const uint32_t lv_s = hb >= L.shift_b ? 0u : inner;        // shared: block is part of the location
  const uint32_t lv_g = hb >= L.shift_ug ? 0u : (hb >= L.shift_b ? 1u : inner);
  return d == 0 ? 4u : (shared ? lv_s : lv_g);
}
SC_HD uint32_t head_level(const TraceLayout& L, uint64_t p, uint64_t x) { return head_level_t<uint64_t>(L, p, x); }

// The same levels as four tests, h[l] = "key x starts a group at level l or
// coarser" (head_level_t(L, p, x) <= l), each one comparison of the bits
// where the keys differ against the lowest bit of a field: the location's
// (the unit's for global keys, the block's for shared keys, whose block is
// part of the location), the block's, the epoch's, and any difference at
// all.  Keys of different spaces differ in the space bit, above all of them.
template <typename K>
struct HeadTests {
  bool h[4];
};
// The thresholds of one trace (the lowest bits of its fields), computed once.
// Every threshold is a power of two at or above the thread field's lowest
// bit 2^(2 + sb), so the bits below it (action, side field), which start no
// group, need no masking: for such a threshold T, d >= T exactly when the
// masked difference is, and a difference above those bits is d >= 2^(2 + sb).
template <typename K>
struct HeadThresholds {
  K thread;  // the thread field's lowest bit
  K space;   // the space bit: a key at or above it is a shared key
  K unit_g, block, epoch;
};
template <typename K>
SC_HD HeadThresholds<K> head_thresholds_t(const TraceLayout& L) {
  HeadThresholds<K> t;
  t.thread = (K)1 << (2 + L.sb);
  t.space = (K)1 << L.shift_space;
  t.unit_g = (K)1 << L.shift_ug;
  t.block = (K)1 << L.shift_b;
  t.epoch = (K)1 << L.shift_e;
  return t;
}
template <typename K>
SC_HD HeadTests<K> head_tests_t(const HeadThresholds<K>& t, K p, K x) {
  const K d = x ^ p;
  HeadTests<K> r;
  r.h[1] = d >= t.block;
  r.h[0] = d >= t.unit_g || (x >= t.space && r.h[1]);  // shared: the block is part of the location
  r.h[2] = d >= t.epoch;
  r.h[3] = d >= t.thread;
  return r;
}
template <typename K>
SC_HD HeadTests<K> head_tests_t(const TraceLayout& L, K p, K x) {
  return head_tests_t<K>(head_thresholds_t<K>(L), p, x);
}

// Epoch and block-local thread of a key.
template <typename K>
SC_HD uint32_t key_epoch_t(const TraceLayout& L, K k) {
  return (uint32_t)((uint64_t)(k >> L.shift_e) & lowmask(L.eb));
}
template <typename K>
SC_HD uint32_t key_ltid_t(const TraceLayout& L, K k) {
  return (uint32_t)((uint64_t)(k >> (2 + L.sb)) & lowmask(L.tb));
}

// Side field of a key (warp-aware check): divergence bit and statement id.
template <typename K>
SC_HD bool key_diverged_t(const TraceLayout& L, K k) {
  return L.sb && ((uint64_t)(k >> (1 + L.sb)) & 1u);
}
template <typename K>
SC_HD uint32_t key_stmt_t(const TraceLayout& L, K k) {
  return L.sb ? (uint32_t)((uint64_t)(k >> 2) & lowmask(L.sb - 1)) : 0u;
}

// Location of a key: space, owning block (shared) or 0xFFFFFFFF, unit.
template <typename K>
SC_HD void key_location_t(const TraceLayout& L, K k, uint32_t& space, uint32_t& block, uint64_t& unit) {
  space = (uint32_t)((k >> L.shift_space) & 1u);
  if (space == 0) {
    block = 0xFFFFFFFFu;
    unit = ((uint64_t)(k >> L.shift_ug) & lowmask(L.ug)) + L.gmin;
  } else {
    block = (uint32_t)((uint64_t)(k >> L.shift_bs) & lowmask(L.bb));
    unit = ((uint64_t)(k >> L.shift_b) & lowmask(L.us)) + L.smin;
  }
}
SC_HD void key_location(const TraceLayout& L, uint64_t k, uint32_t& space, uint32_t& block, uint64_t& unit) {
  key_location_t<uint64_t>(L, k, space, block, unit);
}

}  // namespace sc
