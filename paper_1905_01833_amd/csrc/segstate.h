// segstate.h -- exact racing-pair counts over sorted keys, as a monoid.
//
// After sorting, the records of one location form a contiguous run, nested
// into runs of (location, block), (location, block, epoch) and (location,
// block, epoch, thread).  Walking the run in order, an element x of class c
// (read, write, atomic) races with every earlier element y of the same
// location that conflicts with it (Theorem 1: at least one write; atomics
// conflict with plain accesses only) and is concurrent with it: y lies in an
// earlier block (barriers order one block only), or in x's block and epoch
// but in an earlier thread.  So x contributes
//
//   sum over conflicting classes c' of  N_xb[c'] + N_in[c']
//
// pairs, where N_xb counts earlier elements of the location outside x's
// block run and N_in earlier elements of x's epoch run outside x's thread
// run.  Every unordered racing pair is counted once, at its later element.
// The per-location total is the entry the check reports.
//
// To split this walk over tiles, a range of elements is summarised by a
// State; combine(A, B) gives the summary of A followed by B, and the result
// is independent of how the sequence is split (the operation is
// associative, with identity()).  The counts of the carried-in open runs
// enter B's contributions linearly, which is what the correction term of
// combine() adds.
#pragma once
#include <stdint.h>

#include "keys.h"

namespace sc {

constexpr uint32_t NLEV = 4;     // location, block, epoch, thread
constexpr uint32_t NO_HEAD = 5;  // "no run starts in this range"
enum { CLS_R = 0, CLS_W = 1, CLS_A = 2 };
enum { K_WW = 0, K_RW = 1, K_AW = 2, K_AR = 3, K_XB = 4, NSUM = 5 };

struct State {
  uint32_t m;           // smallest head level inside the range (NO_HEAD: none)
  uint32_t lead[4][3];  // per level: class counts before the range's first head at that level or coarser
  uint32_t trail[4][3]; // per level: class counts of the run open at the end of the range
  uint64_t leadsum[5];  // pair sums of elements before the first location head
  uint64_t trailsum[5]; // pair sums of the last location run that starts in the range (m == 0)
};

// Pairs formed by one element of class c with earlier partners counted in
// xb[] (other blocks of its location) and in[] (other threads of its block
// and epoch).  T is uint32_t inside a tile and uint64_t across tiles.
template <typename T>
SC_HD void element_pairs(uint32_t c, const T xb[3], const T in[3], T out[5]) {
  const T r = xb[CLS_R] + in[CLS_R], w = xb[CLS_W] + in[CLS_W], a = xb[CLS_A] + in[CLS_A];
  out[K_WW] = out[K_RW] = out[K_AW] = out[K_AR] = out[K_XB] = 0;
  if (c == CLS_R) {
    out[K_RW] = w;
    out[K_AR] = a;
    out[K_XB] = xb[CLS_W] + xb[CLS_A];
  } else if (c == CLS_W) {
    out[K_WW] = w;
    out[K_RW] = r;
    out[K_AW] = a;
    out[K_XB] = xb[CLS_R] + xb[CLS_W] + xb[CLS_A];
  } else {
    out[K_AW] = w;
    out[K_AR] = r;
    out[K_XB] = xb[CLS_R] + xb[CLS_W];
  }
}

// Racing pairs between a group with class counts `later` and a group with
// class counts `earlier` (every cross pair conflicting by kind).
SC_HD void cross_pairs(const uint32_t later[3], const uint32_t earlier[3], uint64_t p[4]) {
  const uint64_t lr = later[CLS_R], lw = later[CLS_W], la = later[CLS_A];
  const uint64_t er = earlier[CLS_R], ew = earlier[CLS_W], ea = earlier[CLS_A];
  p[K_WW] = lw * ew;
  p[K_RW] = lr * ew + lw * er;
  p[K_AW] = la * ew + lw * ea;
  p[K_AR] = la * er + lr * ea;
}

SC_HD State identity() {
  State s;
  s.m = NO_HEAD;
  for (uint32_t l = 0; l < NLEV; l++)
    for (uint32_t c = 0; c < 3; c++) s.lead[l][c] = s.trail[l][c] = 0;
  for (uint32_t k = 0; k < NSUM; k++) s.leadsum[k] = s.trailsum[k] = 0;
  return s;
}

// Pair sums of the location run open at the end of a range.
SC_HD const uint64_t* tail_sums(const State& s) { return s.m == 0 ? s.trailsum : s.leadsum; }

// Pair sums of the location run that is open at the end of `a` and
// continues through the part of `b` before b's first location head.
SC_HD void open_sums(const State& a, const State& b, uint64_t out[5]) {
  const uint64_t* ta = tail_sums(a);
  for (uint32_t k = 0; k < NSUM; k++) out[k] = ta[k] + b.leadsum[k];
  // Elements of b before its first head at level <= l sit in runs that
  // started in `a`: add the pairs they form with a's open run counts,
  // signed + - + - over levels (location, block, epoch, thread); the first
  // two levels are the cross-block part.
  for (uint32_t l = 0; l < NLEV; l++) {
    uint64_t p[4];
    cross_pairs(b.lead[l], a.trail[l], p);
    const bool neg = (l & 1u) != 0;
    uint64_t tot = 0;
    for (uint32_t k = 0; k < 4; k++) {
      out[k] = neg ? out[k] - p[k] : out[k] + p[k];
      tot += p[k];
    }
    if (l < 2) out[K_XB] = neg ? out[K_XB] - tot : out[K_XB] + tot;
  }
}

SC_HD State combine(const State& a, const State& b) {
  State c;
  uint64_t open[5];
  open_sums(a, b, open);
  c.m = a.m < b.m ? a.m : b.m;
  for (uint32_t k = 0; k < NSUM; k++) {
    c.leadsum[k] = (a.m == 0) ? a.leadsum[k] : open[k];
    c.trailsum[k] = (b.m == 0) ? b.trailsum[k] : open[k];
  }
  for (uint32_t l = 0; l < NLEV; l++)
    for (uint32_t q = 0; q < 3; q++) {
      c.trail[l][q] = (b.m <= l) ? b.trail[l][q] : a.trail[l][q] + b.trail[l][q];
      c.lead[l][q] = (a.m <= l) ? a.lead[l][q] : a.lead[l][q] + b.lead[l][q];
    }
  return c;
}

// Append one element (head level lv relative to its predecessor, class c).
// When lv == 0 and the range already holds a location head, the run that
// ends here is complete: its sums are s.trailsum before the call.
SC_HD void push(State& s, uint32_t lv, uint32_t c) {
  for (uint32_t l = lv; l < NLEV; l++)
    for (uint32_t q = 0; q < 3; q++) s.trail[l][q] = 0;
  if (lv == 0)
    for (uint32_t k = 0; k < NSUM; k++) s.trailsum[k] = 0;
  if (lv < s.m) s.m = lv;
  uint64_t xb[3], in[3], v[5];
  for (uint32_t q = 0; q < 3; q++) {
    xb[q] = (uint64_t)s.trail[0][q] - s.trail[1][q];
    in[q] = (uint64_t)s.trail[2][q] - s.trail[3][q];
  }
  element_pairs<uint64_t>(c, xb, in, v);
  for (uint32_t k = 0; k < NSUM; k++) {
    if (s.m > 0) s.leadsum[k] += v[k];
    else s.trailsum[k] += v[k];
  }
  for (uint32_t l = 0; l < NLEV; l++) {
    s.trail[l][c]++;
    if (s.m > l) s.lead[l][c]++;
  }
}

SC_HD uint32_t action_class(uint64_t key) { return (uint32_t)(key & 3ull); }
SC_HD uint32_t action_class(u128 key) { return (uint32_t)((uint64_t)key & 3ull); }

}  // namespace sc
