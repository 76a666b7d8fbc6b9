// barrier.h -- barrier instances of the redundant-barrier check over sorted
// keys (paper Sec. 4.2.3, the second loop of Alg. 5).
//
// After sorting, the records of one location and block form runs of equal
// epoch in epoch order, so the records that a block's barrier at boundary b
// separates on that location are two neighbouring runs: epoch b, then
// epoch b + 1.  The first element of an epoch run whose preceding run is
// the previous epoch of the same location and block marks one instance of
// that barrier (a visit-order change of the location it causes).  Both
// runs are summarised per action class -- no thread, one thread (which), or
// several -- and the instance is racing when some pair across the two runs
// would race without the barrier: different threads, at least one write,
// not both atomic.
//
// Functions are usable from host and device code.
#pragma once
#include <stdint.h>

#include "keys.h"
#include "segstate.h"

namespace sc {

// Threads of one action class in a run: none, one (which), or several.
struct ThreadSet {
  uint32_t state;  // 0 none, 1 one thread, 2 several
  uint32_t tid;
};

SC_HD void ts_add(ThreadSet& s, uint32_t t) {
  if (s.state == 0) {
    s.state = 1;
    s.tid = t;
  } else if (s.state == 1 && s.tid != t) {
    s.state = 2;
  }
}

SC_HD ThreadSet ts_union(ThreadSet a, const ThreadSet& b) {
  if (b.state == 2) a.state = 2;
  else if (b.state == 1) ts_add(a, b.tid);
  return a;
}

// Whether a thread of `a` and a different thread of `b` exist.
SC_HD bool ts_pair(const ThreadSet& a, const ThreadSet& b) {
  if (a.state == 0 || b.state == 0) return false;
  return !(a.state == 1 && b.state == 1 && a.tid == b.tid);
}

template <typename K>
SC_HD void run_threads(const TraceLayout& L, K k, ThreadSet (&set)[3]) {
  const uint32_t c = action_class(k);
  if (c < 3) ts_add(set[c], key_ltid_t<K>(L, k));
}

// Whether the element at position p of a trace's n sorted keys is the head
// of a barrier instance; then *boundary is the barrier's boundary (the
// epoch before it) and *racing whether the instance races.  The runs are
// read from `keys` (any memory the caller can read; device code reads them
// from the key buffer).
template <typename K>
SC_HD bool barrier_instance(const TraceLayout& L, const K* keys, uint64_t n, uint64_t p, uint32_t* boundary,
                            bool* racing) {
  if (p == 0 || p >= n) return false;
  const K x = keys[p], w = keys[p - 1];
  if (head_level_t<K>(L, w, x) != 2) return false;  // a new epoch of the same location and block
  const uint32_t e1 = key_epoch_t<K>(L, x), e0 = key_epoch_t<K>(L, w);
  if (e1 != e0 + 1) return false;
  ThreadSet before[3] = {{0, 0}, {0, 0}, {0, 0}}, after[3] = {{0, 0}, {0, 0}, {0, 0}};
  uint64_t q = p - 1;
  run_threads<K>(L, w, before);
  while (q > 0) {  // back over the epoch-e0 run
    const K y = keys[q - 1];
    if (head_level_t<K>(L, y, keys[q]) < 3) break;
    run_threads<K>(L, y, before);
    q--;
  }
  q = p;
  run_threads<K>(L, x, after);
  while (q + 1 < n) {  // forward over the epoch-e1 run
    const K y = keys[q + 1];
    if (head_level_t<K>(L, keys[q], y) < 3) break;
    run_threads<K>(L, y, after);
    q++;
  }
  const ThreadSet any1 = ts_union(ts_union(after[CLS_R], after[CLS_W]), after[CLS_A]);
  *racing = ts_pair(before[CLS_W], any1) || ts_pair(ts_union(before[CLS_R], before[CLS_A]), after[CLS_W]) ||
            ts_pair(before[CLS_A], after[CLS_R]) || ts_pair(before[CLS_R], after[CLS_A]);
  *boundary = e0;
  return true;
}

}  // namespace sc
