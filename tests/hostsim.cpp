// hostsim.cpp -- CPU model of the GPU path's tiled race count (test only).
//
// Compiles the product's key-layout and monoid headers for the host and runs
// the same tile decomposition as the GPU kernels: keys are built and sorted
// per trace and cut into tiles; each tile is summarised from its own
// elements (carry-free) and reports the locations that start and end inside
// it; a location that crosses tiles is finished by the tile where it starts,
// by combining the summaries of the tiles it spans.  Tiles are additionally
// split into "thread" chunks whose summaries are combined, to exercise
// associativity at a second level.  The tests compare the output
// with the oracle; nothing here is used by the product path.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../paper_1905_01833_amd/csrc/barrier.h"
#include "../paper_1905_01833_amd/csrc/segstate.h"
#include "../paper_1905_01833_amd/csrc/tilewalk.h"

struct rec {
  uint64_t unit;
  uint32_t tid;
  uint16_t epoch;
  uint8_t action;
  uint8_t space;
};
struct race {
  uint32_t trace;
  uint8_t space, kinds;
  uint16_t r16;
  uint32_t block, r32;
  uint64_t unit, ww, rw, aw, ar, xb;
};

using namespace sc;

template <typename K>
static void emit(std::vector<race>& out, uint32_t tr, const TraceLayout& L, K key, const uint64_t s[5]) {
  if (s[K_WW] + s[K_RW] + s[K_AW] + s[K_AR] == 0) return;
  race e;
  std::memset(&e, 0, sizeof e);
  e.trace = tr;
  uint32_t sp, blk;
  uint64_t unit;
  key_location_t<K>(L, key, sp, blk, unit);
  e.space = (uint8_t)sp;
  e.block = blk;
  e.unit = unit;
  e.ww = s[K_WW]; e.rw = s[K_RW]; e.aw = s[K_AW]; e.ar = s[K_AR]; e.xb = s[K_XB];
  e.kinds = (uint8_t)((e.ww ? 1 : 0) | (e.rw ? 2 : 0) | (e.aw ? 4 : 0) | (e.ar ? 8 : 0) | (e.xb ? 16 : 0));
  out.push_back(e);
}

// K = uint64_t: one-word keys (a trace wider than 64 bits is an error, as
// in the GPU path's one-word mode); K = u128: two-word keys for every trace.
template <typename K>
static int64_t check_impl(const rec* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                          uint32_t tile, uint32_t chunk, race* out, uint64_t cap, uint32_t* max_passes) {
  std::vector<race> res;
  uint32_t mp = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], n = off[tr + 1] - off[tr];
    if (n == 0) continue;
    TraceStats S;
    stats_init(S);
    for (uint64_t i = 0; i < n; i++) {
      const rec& r = recs[lo + i];
      if (r.action > 2 || r.space > 1) { S.bad_index = std::min<uint64_t>(S.bad_index, i); continue; }
      if (r.space == 0) { S.gmin = std::min(S.gmin, r.unit); S.gmax = std::max(S.gmax, r.unit); }
      else { S.smin = std::min(S.smin, r.unit); S.smax = std::max(S.smax, r.unit); }
      S.max_tid = std::max(S.max_tid, r.tid);
      S.max_epoch = std::max<uint32_t>(S.max_epoch, r.epoch);
    }
    const TraceLayout L = make_layout(S, tpb[tr]);
    if (L.error) return -(int64_t)L.error;
    if (L.wide && sizeof(K) == 8) return -(int64_t)LAYOUT_ERR_WIDE;
    mp = std::max(mp, L.npasses);
    std::vector<K> k(n);
    for (uint64_t i = 0; i < n; i++) {
      const rec& r = recs[lo + i];
      k[i] = make_key_t<K>(L, r.unit, r.tid, r.epoch, r.action, r.space, tpb[tr]);
    }
    std::sort(k.begin(), k.end());
    // tile summaries, carry-free (as the tile scan computes them)
    const uint64_t nt = (n + tile - 1) / tile;
    std::vector<State> agg(nt);
    std::vector<uint32_t> lv(n);
    for (uint64_t i = 0; i < n; i++) lv[i] = (i == 0) ? 0 : head_level_t<K>(L, k[i - 1], k[i]);
    for (uint64_t t = 0; t < nt; t++) {
      const uint64_t t0 = t * tile, t1 = std::min<uint64_t>(n, t0 + tile);
      State a = identity();
      for (uint64_t c0 = t0; c0 < t1; c0 += chunk) {  // chunks combined: associativity at a second level
        State cs = identity();
        for (uint64_t i = c0; i < std::min<uint64_t>(t1, c0 + chunk); i++) push(cs, lv[i], action_class(k[i]));
        a = combine(a, cs);
      }
      agg[t] = a;
    }
    for (uint64_t t = 0; t < nt; t++) {
      const uint64_t t0 = t * tile, t1 = std::min<uint64_t>(n, t0 + tile);
      // locations that start and end inside the tile
      State run = identity();
      bool seen_head = false;
      for (uint64_t i = t0; i < t1; i++) {
        push(run, lv[i], action_class(k[i]));
        if (lv[i] == 0) seen_head = true;
        if (!seen_head) continue;  // the location entering the tile is finished by its owner
        const bool last = (i + 1 == n) || lv[i + 1] == 0;
        if (last) emit(res, tr, L, k[i], run.trailsum);
      }
      // a location that starts in this tile and continues into later tiles
      const bool owns = agg[t].m == 0 && t1 < n && lv[t1] != 0;
      if (!owns) continue;
      State S = agg[t];
      uint64_t u = t + 1;
      while (u < nt && agg[u].m != 0) S = combine(S, agg[u++]);
      uint64_t fin[5];
      if (u < nt) {
        open_sums(S, agg[u], fin);
      } else {
        const uint64_t* ts = tail_sums(S);
        for (int q = 0; q < 5; q++) fin[q] = ts[q];
      }
      emit(res, tr, L, k[t1 - 1], fin);
    }
  }
  if (max_passes) *max_passes = mp;
  if (res.size() > cap) return (int64_t)res.size();
  std::memcpy(out, res.data(), res.size() * sizeof(race));
  return (int64_t)res.size();
}

extern "C" int64_t hs_check(const rec* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                            uint32_t tile, uint32_t chunk, race* out, uint64_t cap, uint32_t* max_passes) {
  return check_impl<uint64_t>(recs, off, n_traces, tpb, tile, chunk, out, cap, max_passes);
}

extern "C" int64_t hs_check_wide(const rec* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                                 uint32_t tile, uint32_t chunk, race* out, uint64_t cap, uint32_t* max_passes) {
  return check_impl<u128>(recs, off, n_traces, tpb, tile, chunk, out, cap, max_passes);
}

// Barrier instances as the barrier kernel counts them: keys built and
// sorted per trace, barrier_instance() at every position, counts summed
// per (trace, boundary).  Output rows as the oracle's: trace, boundary,
// instances, racing, in (trace, boundary) order, rows with an instance only.
struct barrier_row {
  uint32_t trace, boundary;
  uint64_t instances, racing;
};

template <typename K>
static int64_t barriers_impl(const rec* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                             barrier_row* out, uint64_t cap) {
  std::vector<barrier_row> res;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], n = off[tr + 1] - off[tr];
    if (n == 0) continue;
    TraceStats S;
    stats_init(S);
    for (uint64_t i = 0; i < n; i++) {
      const rec& r = recs[lo + i];
      if (r.space == 0) { S.gmin = std::min(S.gmin, r.unit); S.gmax = std::max(S.gmax, r.unit); }
      else { S.smin = std::min(S.smin, r.unit); S.smax = std::max(S.smax, r.unit); }
      S.max_tid = std::max(S.max_tid, r.tid);
      S.max_epoch = std::max<uint32_t>(S.max_epoch, r.epoch);
    }
    const TraceLayout L = make_layout(S, tpb[tr]);
    if (L.error) return -(int64_t)L.error;
    if (L.wide && sizeof(K) == 8) return -(int64_t)LAYOUT_ERR_WIDE;
    std::vector<K> k(n);
    for (uint64_t i = 0; i < n; i++) {
      const rec& r = recs[lo + i];
      k[i] = make_key_t<K>(L, r.unit, r.tid, r.epoch, r.action, r.space, tpb[tr]);
    }
    std::sort(k.begin(), k.end());
    std::vector<uint64_t> inst(L.max_epoch + 1, 0), rac(L.max_epoch + 1, 0);
    for (uint64_t p = 0; p < n; p++) {
      uint32_t b;
      bool racing;
      if (!barrier_instance<K>(L, k.data(), n, p, &b, &racing)) continue;
      if (b >= L.max_epoch) return -1000;  // a boundary the trace cannot have
      inst[b]++;
      rac[b] += racing ? 1 : 0;
    }
    for (uint32_t b = 0; b < L.max_epoch; b++)
      if (inst[b]) res.push_back(barrier_row{tr, b, inst[b], rac[b]});
  }
  if (res.size() > cap) return (int64_t)res.size();
  std::memcpy(out, res.data(), res.size() * sizeof(barrier_row));
  return (int64_t)res.size();
}

extern "C" int64_t hs_barriers(const rec* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                               barrier_row* out, uint64_t cap) {
  return barriers_impl<uint64_t>(recs, off, n_traces, tpb, out, cap);
}

extern "C" int64_t hs_barriers_wide(const rec* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                                    barrier_row* out, uint64_t cap) {
  return barriers_impl<u128>(recs, off, n_traces, tpb, out, cap);
}

// Associativity check on random element sequences: fold(push) equals the
// combine() of arbitrary splits.  Returns 0 when all trials agree.
extern "C" int hs_assoc(uint64_t seed, int trials) {
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
  auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
  for (int t = 0; t < trials; t++) {
    const int n = 1 + (int)(rnd() % 40);
    std::vector<uint32_t> lv(n), cl(n);
    for (int i = 0; i < n; i++) { lv[i] = (uint32_t)(rnd() % 5); cl[i] = (uint32_t)(rnd() % 3); }
    State whole = identity();
    for (int i = 0; i < n; i++) push(whole, lv[i], cl[i]);
    // three-way split combined as (A B) C and A (B C)
    const int s1 = (int)(rnd() % (n + 1)), s2 = s1 + (int)(rnd() % (n - s1 + 1));
    State A = identity(), B = identity(), C = identity();
    for (int i = 0; i < s1; i++) push(A, lv[i], cl[i]);
    for (int i = s1; i < s2; i++) push(B, lv[i], cl[i]);
    for (int i = s2; i < n; i++) push(C, lv[i], cl[i]);
    const State l = combine(combine(A, B), C), r = combine(A, combine(B, C));
    for (const State* s : {&l, &r}) {
      if (s->m != whole.m) return 1;
      for (int k = 0; k < 5; k++) {
        if (s->trailsum[k] != whole.trailsum[k] && whole.m == 0) return 2;
        if (s->leadsum[k] != whole.leadsum[k]) return 3;
      }
      for (int l2 = 0; l2 < 4; l2++)
        for (int q = 0; q < 3; q++)
          if (s->trail[l2][q] != whole.trail[l2][q] || s->lead[l2][q] != whole.lead[l2][q]) return 4;
    }
  }
  return 0;
}

// head_tests_t (the scan's four threshold tests) against head_level_t on
// random layouts and key pairs: neighbours that differ in one chosen field,
// and random pairs, for both key widths and with or without a side field.
// Returns the number of disagreements.
template <typename K>
static int head_tests_impl(uint64_t seed, int trials) {
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 7;
  auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
  int bad = 0;
  for (int t = 0; t < trials; t++) {
    TraceStats S;
    stats_init(S);
    const uint32_t tpb = 1 + (uint32_t)(rnd() % 600);
    const uint64_t gspan = rnd() >> (rnd() % 64), sspan = rnd() >> (rnd() % 64);
    S.gmin = rnd() % 1000; S.gmax = S.gmin + gspan;
    S.smin = rnd() % 1000; S.smax = S.smin + sspan;
    if (rnd() % 5 == 0) { S.gmin = ~0ull; S.gmax = 0; }  // no global records
    S.max_tid = (uint32_t)(rnd() % 100000);
    S.max_epoch = (uint32_t)(rnd() % 70000 % 65536);
    S.max_stmt = (uint32_t)(rnd() % 1000);
    const bool warp = rnd() % 2;
    const TraceLayout L = make_layout(S, tpb, warp);
    if (L.error || (sizeof(K) == 8 && L.wide)) continue;
    auto rec_key = [&](uint32_t space, uint64_t unit, uint32_t tid, uint32_t epoch, uint32_t action, uint32_t side) {
      return make_key_t<K>(L, unit, tid, epoch, action, space, tpb, side);
    };
    for (int q = 0; q < 20; q++) {
      const bool has_g = S.gmin <= S.gmax;
      const uint32_t space = has_g ? (uint32_t)(rnd() % 2) : 1u;
      const uint64_t lo = space ? S.smin : S.gmin, span = space ? sspan : gspan;
      const uint64_t unit = lo + (span ? rnd() % (span + 1) : 0);
      const uint32_t tid = (uint32_t)(rnd() % (S.max_tid + 1)), ep = (uint32_t)(rnd() % (S.max_epoch + 1));
      const uint32_t act = (uint32_t)(rnd() % 3), side = (uint32_t)(rnd() % (S.max_stmt + 1)) | (rnd() % 2 ? SIDE_DIVERGED : 0u);
      const K a = rec_key(space, unit, tid, ep, act, side);
      // a neighbour: the same record with one field changed
      uint32_t space2 = space, tid2 = tid, ep2 = ep, act2 = act, side2 = side;
      uint64_t unit2 = unit;
      switch (rnd() % 7) {
        case 0: unit2 = lo + (span ? rnd() % (span + 1) : 0); break;
        case 1: tid2 = (uint32_t)(rnd() % (S.max_tid + 1)); break;
        case 2: ep2 = (uint32_t)(rnd() % (S.max_epoch + 1)); break;
        case 3: act2 = (uint32_t)(rnd() % 3); break;
        case 4: side2 = (uint32_t)(rnd() % (S.max_stmt + 1)); break;
        case 5: tid2 = tid ^ 1u; if (tid2 > S.max_tid) tid2 = tid; break;
        default:
          if (has_g) { space2 = 1u - space; unit2 = space2 ? S.smin : S.gmin; }
      }
      const K b = rec_key(space2, unit2, tid2, ep2, act2, side2);
      const K p = a < b ? a : b, y = a < b ? b : a;
      const uint32_t lv = head_level_t<K>(L, p, y);
      const HeadTests<K> h = head_tests_t<K>(L, p, y);
      for (uint32_t l = 0; l < 4; l++)
        if (h.h[l] != (lv <= l)) bad++;
    }
  }
  return bad;
}

extern "C" int hs_head_tests(uint64_t seed, int trials) {
  return head_tests_impl<uint64_t>(seed, trials) + head_tests_impl<u128>(seed + 1, trials);
}

// Tile walk of a launch as the tile kernels run it: the grid for `per_cu`
// workgroups per CU over n_cu CUs, every workgroup's tiles counted in
// count[n].  One-tile kernels (grid / 8 >= the tiles per XCD) visit only the
// first tile of their walk.  Returns the grid; *max_per_wg receives the most
// tiles any workgroup visited.
extern "C" uint32_t hs_tile_walk(uint32_t n, uint32_t per_cu, uint32_t n_cu, uint32_t* count, uint32_t* max_per_wg) {
  const uint32_t grid = tile_grid(n, per_cu, n_cu);
  const bool loop = grid / N_XCD < (n + N_XCD - 1) / N_XCD;
  *max_per_wg = 0;
  for (uint32_t wg = 0; wg < grid; wg++) {
    const TileWalk w = tile_walk(n, grid, wg);
    uint32_t k = 0;
    for (uint32_t t = w.first; t < w.end; t = loop ? t + w.step : w.end) {
      count[t]++;
      k++;
    }
    *max_per_wg = std::max(*max_per_wg, k);
  }
  return grid;
}

// The radix digit plan (pass_shift, radix_passes): for every sorted width
// and digit width, the passes' digits tile the bits [2, 2 + sorted) exactly,
// and a stable LSD sort with that plan (counting sort per digit, the
// all-ones padding of a partial tile included) equals a full sort of the
// keys.  Returns the number of failures.
template <typename K>
static int plan_sort_impl(uint64_t seed, int trials, uint32_t db) {
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 7;
  auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
  int bad = 0;
  const uint32_t maxbits = sizeof(K) == 8 ? 64 : 128;
  for (int t = 0; t < trials; t++) {
    const uint32_t key_bits = 3 + (uint32_t)(rnd() % (maxbits - 2));
    const uint32_t n = 1 + (uint32_t)(rnd() % 300);
    std::vector<K> k(n), pad(n + 5);
    for (uint32_t i = 0; i < n; i++) {
      K v = ((K)rnd() << 64 % (8 * sizeof(K))) ^ (K)rnd();
      if (key_bits < 8 * sizeof(K)) v &= (((K)1) << key_bits) - 1;
      if (rnd() % 4 == 0 && i) v = k[rnd() % i];  // repeats
      k[i] = v;
    }
    // the sort proper ignores the two action bits: bits >= 2 compared, ties
    // in input order (what a stable sort of bits [2, key_bits) gives)
    std::vector<K> want = k;
    std::stable_sort(want.begin(), want.end(), [](K a, K b) { return (a >> 2) < (b >> 2); });
    std::vector<K> cur = k;
    for (uint32_t i = 0; i < 5; i++) cur.push_back(~(K)0);  // padding ranks last in every pass
    const uint32_t np = radix_passes(key_bits - 2, db);
    for (uint32_t p = 0; p < np; p++) {
      const uint32_t sh = pass_shift(p, db), w = p == 0 ? RADIX_BITS : db;
      std::vector<std::vector<K>> bucket(1u << w);
      for (const K& v : cur) bucket[(uint32_t)(v >> sh) & ((1u << w) - 1)].push_back(v);
      cur.clear();
      for (auto& bk : bucket) cur.insert(cur.end(), bk.begin(), bk.end());
    }
    cur.resize(n);
    if (cur != want) bad++;
  }
  return bad;
}

extern "C" int hs_digit_plan(uint64_t seed, int trials) {
  int bad = 0;
  for (uint32_t db : {RADIX_BITS, RADIX_WIDE_BITS})
    for (uint32_t sorted = 1; sorted <= 126; sorted++) {
      const uint32_t np = radix_passes(sorted, db);
      if (pass_shift(0, db) != 2) bad++;
      for (uint32_t p = 0; p + 1 < np + 1; p++) {
        const uint32_t w = p == 0 ? RADIX_BITS : db;
        if (pass_shift(p + 1, db) != pass_shift(p, db) + w) bad++;
      }
      // the last pass starts inside the sorted bits and the passes reach their end
      if (!(pass_shift(np - 1, db) < 2 + sorted && pass_shift(np, db) >= 2 + sorted)) bad++;
      if (db == RADIX_BITS && np != (sorted + 7) / 8) bad++;
      if (np > MAX_PASSES) bad++;
    }
  for (uint32_t db : {RADIX_BITS, RADIX_WIDE_BITS})
    bad += plan_sort_impl<uint64_t>(seed + db, trials, db) + plan_sort_impl<u128>(seed + 2 * db, trials, db);
  return bad;
}
