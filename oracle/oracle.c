/*
 * oracle.c -- CPU oracle for the Memory-Model data-race check.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load this file's
 * library.  It shares no code, header, table or helper with the GPU path.
 *
 * What is computed (paper Sec. 4.2.3, Theorem 1; Alg. 5, data-race part):
 * two accesses (Unit Tuples) of one trace race when
 *   - they touch the same memory unit (same location: global memory is one
 *     array for all blocks, shared memory is private to a block, Alg. 3),
 *   - they come from different threads (Theorem 1, second condition),
 *   - they are concurrent: the same visit order, i.e. the same barrier
 *     interval (Theorem 1, first condition), or different blocks, since a
 *     barrier only orders the threads of one block (Sec. 2),
 *   - at least one writes (Theorem 1, third condition), where an atomic
 *     races with a plain read or write but not with another atomic.
 * The warp clauses (1)-(3) of Theorem 1 are not applied: records carry no
 * statement or divergence information, so every pair of distinct threads is
 * treated as potentially concurrent.
 *
 * For every location with at least one racing pair, one entry gives the
 * number of racing unordered record pairs by kind (write/write, read/write,
 * atomic/write, atomic/read) and how many of them span two blocks.
 *
 * Tier A (orc_brute_force) applies the pairwise definition literally to all
 * O(n^2) pairs.  Tier B (orc_closed_form) groups records by location, block,
 * epoch and thread with the C library's qsort and counts pairs from group
 * sizes by inclusion-exclusion:
 *   pairs_k(L) = K_k(L) - sum_b K_k(L_b) + sum_{b,e} K_k(L_be) - sum_{b,e,t} K_k(L_bet)
 * with K_WW = w(w-1)/2, K_RW = r w, K_AW = a w, K_AR = a r for a group with
 * r reads, w writes and a atomics.  A pair with the same thread is counted
 * +1-1+1-1 = 0 times, one in the same block and epoch from different threads
 * +1-1+1 = 1 time, one in the same block and different epochs +1-1 = 0
 * times, and one in different blocks +1 time.  The cross-block count is
 * sum_k [K_k(L) - sum_b K_k(L_b)].  Tier B is checked against Tier A by the
 * tests; it is not assumed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t unit;
  uint32_t tid;
  uint16_t epoch;
  uint8_t action; /* 0 read, 1 write, 2 atomic */
  uint8_t space;  /* 0 global, 1 shared */
} orc_record;

typedef struct {
  uint32_t trace;
  uint8_t space;
  uint8_t kinds; /* bit0 WW, bit1 RW, bit2 AW, bit3 AR, bit4 cross-block */
  uint16_t reserved16;
  uint32_t block; /* owning block for shared, 0xFFFFFFFF for global */
  uint32_t reserved32;
  uint64_t unit;
  uint64_t pairs_ww, pairs_rw, pairs_aw, pairs_ar, pairs_xblock;
} orc_race;

typedef struct {
  uint64_t n_records, n_race_locs, n_pairs;
} orc_summary;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERECORD = -2, ORC_ENOMEM = -3 };
enum { KIND_WW = 0, KIND_RW = 1, KIND_AW = 2, KIND_AR = 3 };

/* Kind of an unordered action pair, or -1 when the pair does not conflict
 * (read/read, atomic/atomic). */
static int kind_of(int a, int b) {
  if (a > b) { int t = a; a = b; b = t; }
  if (a == 0 && b == 0) return -1; /* R R */
  if (a == 0 && b == 1) return KIND_RW;
  if (a == 0 && b == 2) return KIND_AR;
  if (a == 1 && b == 1) return KIND_WW;
  if (a == 1 && b == 2) return KIND_AW;
  return -1; /* A A */
}

/* ---------- growable entry list ---------- */
typedef struct {
  orc_race* v;
  uint64_t n, cap;
} race_list;

static int push(race_list* L, const orc_race* e) {
  if (L->n == L->cap) {
    uint64_t nc = L->cap ? 2 * L->cap : 256;
    orc_race* nv = (orc_race*)realloc(L->v, nc * sizeof(orc_race));
    if (!nv) return ORC_ENOMEM;
    L->v = nv;
    L->cap = nc;
  }
  L->v[L->n++] = *e;
  return ORC_OK;
}

static int validate(const orc_record* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                    uint64_t* bad_index) {
  if (n_traces && (!off || !tpb)) return ORC_EINVAL;
  if (n_traces && off[0] != 0) return ORC_EINVAL;
  for (uint32_t t = 0; t < n_traces; t++) {
    if (off[t + 1] < off[t]) return ORC_EINVAL;
    if (tpb[t] == 0) return ORC_EINVAL;
  }
  uint64_t n = n_traces ? off[n_traces] : 0;
  if (n && !recs) return ORC_EINVAL;
  for (uint64_t i = 0; i < n; i++) {
    if (recs[i].action > 2 || recs[i].space > 1) {
      if (bad_index) *bad_index = i;
      return ORC_ERECORD;
    }
  }
  return ORC_OK;
}

static void finish_entry(orc_race* e) {
  e->kinds = (uint8_t)((e->pairs_ww ? 1 : 0) | (e->pairs_rw ? 2 : 0) | (e->pairs_aw ? 4 : 0) |
                       (e->pairs_ar ? 8 : 0) | (e->pairs_xblock ? 16 : 0));
}

/* ---------- location ordering shared by both tiers' outputs ---------- */
static int cmp_entry(const void* pa, const void* pb) {
  const orc_race* a = (const orc_race*)pa;
  const orc_race* b = (const orc_race*)pb;
  if (a->trace != b->trace) return a->trace < b->trace ? -1 : 1;
  if (a->space != b->space) return a->space < b->space ? -1 : 1;
  if (a->block != b->block) return a->block < b->block ? -1 : 1;
  if (a->unit != b->unit) return a->unit < b->unit ? -1 : 1;
  return 0;
}

static void summarise(const race_list* L, const uint64_t* off, uint32_t n_traces, orc_summary* S) {
  if (!S) return;
  for (uint32_t t = 0; t < n_traces; t++) {
    S[t].n_records = off[t + 1] - off[t];
    S[t].n_race_locs = 0;
    S[t].n_pairs = 0;
  }
  for (uint64_t i = 0; i < L->n; i++) {
    orc_summary* s = &S[L->v[i].trace];
    s->n_race_locs++;
    s->n_pairs += L->v[i].pairs_ww + L->v[i].pairs_rw + L->v[i].pairs_aw + L->v[i].pairs_ar;
  }
}

/* ======================= Tier A: brute force ======================= */

/* One racing pair becomes one "hit" on its location; hits are then sorted by
 * location and summed. */
int64_t orc_brute_force(const orc_record* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                        orc_race** out, orc_summary* summary, uint64_t* bad_index) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  race_list hits = {0, 0, 0};
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], hi = off[tr + 1];
    const uint32_t T = tpb[tr];
    for (uint64_t i = lo; i < hi; i++) {
      const orc_record* x = &recs[i];
      const uint32_t bx = x->tid / T;
      for (uint64_t j = i + 1; j < hi; j++) {
        const orc_record* y = &recs[j];
        const uint32_t by = y->tid / T;
        /* same memory unit: same space and unit; shared memory is per block */
        if (x->space != y->space || x->unit != y->unit) continue;
        if (x->space == 1 && bx != by) continue;
        /* different threads */
        if (x->tid == y->tid) continue;
        /* at least one write (atomics conflict with plain accesses only) */
        const int kind = kind_of(x->action, y->action);
        if (kind < 0) continue;
        /* concurrent: same barrier interval, or different blocks */
        if (!(bx != by || x->epoch == y->epoch)) continue;
        orc_race h;
        memset(&h, 0, sizeof h);
        h.trace = tr;
        h.space = x->space;
        h.block = x->space == 1 ? bx : 0xFFFFFFFFu;
        h.unit = x->unit;
        if (kind == KIND_WW) h.pairs_ww = 1;
        if (kind == KIND_RW) h.pairs_rw = 1;
        if (kind == KIND_AW) h.pairs_aw = 1;
        if (kind == KIND_AR) h.pairs_ar = 1;
        h.pairs_xblock = (bx != by) ? 1 : 0;
        if (push(&hits, &h)) { free(hits.v); return ORC_ENOMEM; }
      }
    }
  }
  if (hits.n) qsort(hits.v, hits.n, sizeof(orc_race), cmp_entry);
  race_list res = {0, 0, 0};
  for (uint64_t i = 0; i < hits.n;) {
    orc_race e = hits.v[i];
    uint64_t j = i + 1;
    while (j < hits.n && cmp_entry(&hits.v[j], &hits.v[i]) == 0) {
      e.pairs_ww += hits.v[j].pairs_ww;
      e.pairs_rw += hits.v[j].pairs_rw;
      e.pairs_aw += hits.v[j].pairs_aw;
      e.pairs_ar += hits.v[j].pairs_ar;
      e.pairs_xblock += hits.v[j].pairs_xblock;
      j++;
    }
    finish_entry(&e);
    if (push(&res, &e)) { free(hits.v); free(res.v); return ORC_ENOMEM; }
    i = j;
  }
  free(hits.v);
  summarise(&res, off, n_traces, summary);
  *out = res.v;
  return (int64_t)res.n;
}

/* ===================== Tier B: group counts ===================== */

typedef struct {
  uint64_t unit;
  uint32_t lblock; /* block if shared, 0xFFFFFFFF if global: part of the location */
  uint32_t block;
  uint32_t tid;
  uint16_t epoch;
  uint8_t space;
  uint8_t action;
} item;

static int cmp_item(const void* pa, const void* pb) {
  const item* a = (const item*)pa;
  const item* b = (const item*)pb;
  if (a->space != b->space) return a->space < b->space ? -1 : 1;
  if (a->lblock != b->lblock) return a->lblock < b->lblock ? -1 : 1;
  if (a->unit != b->unit) return a->unit < b->unit ? -1 : 1;
  if (a->block != b->block) return a->block < b->block ? -1 : 1;
  if (a->epoch != b->epoch) return a->epoch < b->epoch ? -1 : 1;
  if (a->tid != b->tid) return a->tid < b->tid ? -1 : 1;
  return 0;
}

typedef struct {
  uint64_t r, w, a;
} counts;

/* K_k of one group, k = WW, RW, AW, AR */
static void K(const counts* c, uint64_t k[4]) {
  k[KIND_WW] = c->w ? c->w * (c->w - 1) / 2 : 0;
  k[KIND_RW] = c->r * c->w;
  k[KIND_AW] = c->a * c->w;
  k[KIND_AR] = c->a * c->r;
}

static void add(counts* c, uint8_t action) {
  if (action == 0) c->r++;
  else if (action == 1) c->w++;
  else c->a++;
}

static int same_loc(const item* x, const item* y) {
  return x->space == y->space && x->lblock == y->lblock && x->unit == y->unit;
}

/* Tier B's counting over one sorted run of items of trace `tr`: every
 * location [i, iL) is split into its block, epoch and thread groups, and
 * its pairs are the inclusion-exclusion of the groups' K values. */
static int count_sorted(const item* it, uint64_t n, uint32_t tr, race_list* res) {
  uint64_t i = 0;
  while (i < n) {
    /* one location [i, iL) */
    uint64_t iL = i;
    counts cL = {0, 0, 0};
    while (iL < n && same_loc(&it[iL], &it[i])) add(&cL, it[iL++].action);
    uint64_t KL[4], SB[4] = {0, 0, 0, 0}, SE[4] = {0, 0, 0, 0}, ST[4] = {0, 0, 0, 0}, tmp[4];
    K(&cL, KL);
    for (uint64_t ib = i; ib < iL;) { /* block groups */
      uint64_t jb = ib;
      counts cB = {0, 0, 0};
      while (jb < iL && it[jb].block == it[ib].block) add(&cB, it[jb++].action);
      K(&cB, tmp);
      for (int k = 0; k < 4; k++) SB[k] += tmp[k];
      for (uint64_t ie = ib; ie < jb;) { /* epoch groups */
        uint64_t je = ie;
        counts cE = {0, 0, 0};
        while (je < jb && it[je].epoch == it[ie].epoch) add(&cE, it[je++].action);
        K(&cE, tmp);
        for (int k = 0; k < 4; k++) SE[k] += tmp[k];
        for (uint64_t itd = ie; itd < je;) { /* thread groups */
          uint64_t jt = itd;
          counts cT = {0, 0, 0};
          while (jt < je && it[jt].tid == it[itd].tid) add(&cT, it[jt++].action);
          K(&cT, tmp);
          for (int k = 0; k < 4; k++) ST[k] += tmp[k];
          itd = jt;
        }
        ie = je;
      }
      ib = jb;
    }
    uint64_t p[4], xb = 0;
    for (int k = 0; k < 4; k++) {
      p[k] = KL[k] - SB[k] + SE[k] - ST[k];
      xb += KL[k] - SB[k];
    }
    if (p[0] + p[1] + p[2] + p[3] > 0) {
      orc_race e;
      memset(&e, 0, sizeof e);
      e.trace = tr;
      e.space = it[i].space;
      e.block = it[i].lblock;
      e.unit = it[i].unit;
      e.pairs_ww = p[KIND_WW];
      e.pairs_rw = p[KIND_RW];
      e.pairs_aw = p[KIND_AW];
      e.pairs_ar = p[KIND_AR];
      e.pairs_xblock = xb;
      finish_entry(&e);
      if (push(res, &e)) return ORC_ENOMEM;
    }
    i = iL;
  }
  return ORC_OK;
}

static void to_item(const orc_record* r, uint32_t T, item* x) {
  x->unit = r->unit;
  x->block = r->tid / T;
  x->lblock = r->space == 1 ? x->block : 0xFFFFFFFFu;
  x->tid = r->tid;
  x->epoch = r->epoch;
  x->space = r->space;
  x->action = r->action;
}

int64_t orc_closed_form(const orc_record* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                        orc_race** out, orc_summary* summary, uint64_t* bad_index) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  race_list res = {0, 0, 0};
  uint64_t maxn = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++)
    if (off[tr + 1] - off[tr] > maxn) maxn = off[tr + 1] - off[tr];
  item* it = maxn ? (item*)malloc(maxn * sizeof(item)) : NULL;
  if (maxn && !it) return ORC_ENOMEM;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], n = off[tr + 1] - off[tr];
    const uint32_t T = tpb[tr];
    for (uint64_t i = 0; i < n; i++) to_item(&recs[lo + i], T, &it[i]);
    if (n) qsort(it, n, sizeof(item), cmp_item);
    if (count_sorted(it, n, tr, &res)) { free(it); free(res.v); return ORC_ENOMEM; }
  }
  free(it);
  summarise(&res, off, n_traces, summary);
  *out = res.v;
  return (int64_t)res.n;
}

/* ============ Tier B on many cores: the same counting, split up ============
 *
 * The work of orc_closed_form is divided among OpenMP threads without any
 * change to what is computed:
 *   - traces of at most `bucket_min` records are independent units, handed
 *     to the threads largest first;
 *   - a larger trace is split by a hash of the location into buckets; all
 *     records of one location fall into one bucket, so each bucket is
 *     sorted and counted by count_sorted exactly as a whole trace is, and
 *     the trace's entries are the union of its buckets' entries, put back
 *     in location order.
 * n_threads = 0 uses every core OpenMP sees. */
#ifdef _OPENMP
#include <omp.h>
#endif

static uint64_t loc_hash(const item* x) {
  uint64_t h = x->unit ^ ((uint64_t)x->lblock << 32) ^ ((uint64_t)x->space << 63);
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

typedef struct {
  uint32_t trace;
  uint64_t n;
} trace_ref;

static int cmp_trace_ref(const void* pa, const void* pb) {
  const trace_ref* a = (const trace_ref*)pa;
  const trace_ref* b = (const trace_ref*)pb;
  if (a->n != b->n) return a->n > b->n ? -1 : 1;
  return a->trace < b->trace ? -1 : (a->trace > b->trace);
}

/* One large trace, bucket by bucket on all threads; its entries go to *res. */
static int big_trace(const orc_record* recs, uint64_t lo, uint64_t n, uint32_t T, uint32_t tr, int nth,
                     race_list* res) {
  const uint32_t nb = (uint32_t)(8 * nth);
  item* it = (item*)malloc(n * sizeof(item));
  uint64_t* cnt = (uint64_t*)calloc((size_t)nth * nb, sizeof(uint64_t));
  uint64_t* start = (uint64_t*)calloc((size_t)nb + 1, sizeof(uint64_t));
  race_list* parts = (race_list*)calloc(nb, sizeof(race_list));
  int rc = ORC_OK;
  if (!it || !cnt || !start || !parts) { rc = ORC_ENOMEM; goto done; }
  /* bucket of every record, counted per thread over fixed chunks */
#pragma omp parallel num_threads(nth)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    const uint64_t c0 = n * (uint64_t)t / (uint64_t)nth, c1 = n * (uint64_t)(t + 1) / (uint64_t)nth;
    item x;
    for (uint64_t i = c0; i < c1; i++) {
      to_item(&recs[lo + i], T, &x);
      cnt[(size_t)t * nb + loc_hash(&x) % nb]++;
    }
  }
  /* bucket b's records go to [start[b], start[b+1]), thread by thread */
  {
    uint64_t run = 0;
    for (uint32_t b = 0; b < nb; b++) {
      start[b] = run;
      for (int t = 0; t < nth; t++) {
        const uint64_t c = cnt[(size_t)t * nb + b];
        cnt[(size_t)t * nb + b] = run;
        run += c;
      }
    }
    start[nb] = run;
  }
#pragma omp parallel num_threads(nth)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    const uint64_t c0 = n * (uint64_t)t / (uint64_t)nth, c1 = n * (uint64_t)(t + 1) / (uint64_t)nth;
    item x;
    for (uint64_t i = c0; i < c1; i++) {
      to_item(&recs[lo + i], T, &x);
      it[cnt[(size_t)t * nb + loc_hash(&x) % nb]++] = x;
    }
  }
  /* each bucket: sort and count as a whole trace */
  {
    int err = 0;
#pragma omp parallel for num_threads(nth) schedule(dynamic, 1) reduction(| : err)
    for (int64_t b = 0; b < (int64_t)nb; b++) {
      const uint64_t m = start[b + 1] - start[b];
      if (m) qsort(it + start[b], m, sizeof(item), cmp_item);
      if (count_sorted(it + start[b], m, tr, &parts[b])) err |= 1;
    }
    if (err) { rc = ORC_ENOMEM; goto done; }
  }
  {
    const uint64_t first = res->n;
    for (uint32_t b = 0; b < nb && rc == ORC_OK; b++)
      for (uint64_t k = 0; k < parts[b].n; k++)
        if (push(res, &parts[b].v[k])) { rc = ORC_ENOMEM; break; }
    if (rc == ORC_OK && res->n > first) qsort(res->v + first, res->n - first, sizeof(orc_race), cmp_entry);
  }
done:
  if (parts)
    for (uint32_t b = 0; b < nb; b++) free(parts[b].v);
  free(parts);
  free(start);
  free(cnt);
  free(it);
  return rc;
}

int64_t orc_closed_form_par(const orc_record* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                            orc_race** out, orc_summary* summary, uint64_t* bad_index, int n_threads,
                            uint64_t bucket_min) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  int nth = n_threads;
#ifdef _OPENMP
  if (nth <= 0) nth = omp_get_max_threads();
#endif
  if (nth <= 0) nth = 1;
  race_list* per = (race_list*)calloc(n_traces ? n_traces : 1, sizeof(race_list));
  trace_ref* order = (trace_ref*)malloc((n_traces ? n_traces : 1) * sizeof(trace_ref));
  if (!per || !order) { free(per); free(order); return ORC_ENOMEM; }
  uint32_t n_small = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t n = off[tr + 1] - off[tr];
    if (n <= bucket_min) order[n_small++] = (trace_ref){tr, n};
  }
  qsort(order, n_small, sizeof(trace_ref), cmp_trace_ref);
  int err = 0;
  /* small traces: one unit each, largest first */
#pragma omp parallel num_threads(nth) reduction(| : err)
  {
    item* it = NULL;
    uint64_t cap = 0;
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < (int64_t)n_small; k++) {
      const uint32_t tr = order[k].trace;
      const uint64_t lo = off[tr], n = order[k].n;
      if (n > cap) {
        free(it);
        it = (item*)malloc(n * sizeof(item));
        cap = it ? n : 0;
        if (!it) { err |= 1; continue; }
      }
      for (uint64_t i = 0; i < n; i++) to_item(&recs[lo + i], tpb[tr], &it[i]);
      if (n) qsort(it, n, sizeof(item), cmp_item);
      if (count_sorted(it, n, tr, &per[tr])) err |= 1;
    }
    free(it);
  }
  /* large traces: one at a time, bucket by bucket on all threads */
  for (uint32_t tr = 0; tr < n_traces && !err; tr++) {
    const uint64_t n = off[tr + 1] - off[tr];
    if (n > bucket_min && big_trace(recs, off[tr], n, tpb[tr], tr, nth, &per[tr])) err |= 1;
  }
  race_list res = {0, 0, 0};
  for (uint32_t tr = 0; tr < n_traces && !err; tr++)
    for (uint64_t k = 0; k < per[tr].n; k++)
      if (push(&res, &per[tr].v[k])) { err |= 1; break; }
  for (uint32_t tr = 0; tr < n_traces; tr++) free(per[tr].v);
  free(per);
  free(order);
  if (err) { free(res.v); return ORC_ENOMEM; }
  summarise(&res, off, n_traces, summary);
  *out = res.v;
  return (int64_t)res.n;
}

/* =============== Redundant barriers (Alg. 5, second loop) ===============
 *
 * Sec. 4.2.3: a barrier is redundant when removing it lets no data race be
 * detected; Alg. 5 checks, per memory unit, whether the tuples of adjacent
 * visit orders can be merged without a race, counts the mergeable changes
 * per barrier, and calls the barrier redundant when that count equals the
 * number of visit-order changes the barrier causes.
 *
 * Here, per trace: the barrier at boundary b of block B ends B's epoch b
 * (the threads of B pass it between their epoch-b and epoch-(b+1)
 * accesses).  An instance of it is a location L (a global unit, or a unit of
 * B's shared memory) on which block B has records in both epochs b and b+1
 * -- a visit-order change of L's unit that the barrier causes.  The
 * instance is racing when merging the two epochs would race: some record x
 * of epoch b and some record y of epoch b+1, both of block B on L, come
 * from different threads and conflict (at least one writes; not both
 * atomic).  Records of other blocks are concurrent with both epochs either
 * way, so the barrier does not separate them from anything.  For every
 * (trace, boundary) with at least one instance, one entry gives the number
 * of instances and of racing instances; the barrier is redundant when no
 * instance is racing.
 */
typedef struct {
  uint32_t trace;
  uint32_t boundary;
  uint64_t instances;
  uint64_t racing;
} orc_barrier;

typedef struct {
  orc_barrier* v;
  uint64_t n, cap;
} barrier_list;

static int push_barrier(barrier_list* L, const orc_barrier* e) {
  if (L->n == L->cap) {
    uint64_t nc = L->cap ? 2 * L->cap : 64;
    orc_barrier* nv = (orc_barrier*)realloc(L->v, nc * sizeof(orc_barrier));
    if (!nv) return ORC_ENOMEM;
    L->v = nv;
    L->cap = nc;
  }
  L->v[L->n++] = *e;
  return ORC_OK;
}

/* whether two actions conflict: at least one write, not both atomic */
static int conflicts(int a, int b) { return kind_of(a, b) >= 0; }

/* One instance found by the brute force: (trace, boundary, location, block)
 * and whether the pair that found it races. */
typedef struct {
  uint32_t trace, boundary, space, lblock, block, racing;
  uint64_t unit;
} inst_hit;

static int cmp_inst_hit(const void* pa, const void* pb) {
  const inst_hit* a = (const inst_hit*)pa;
  const inst_hit* b = (const inst_hit*)pb;
  if (a->trace != b->trace) return a->trace < b->trace ? -1 : 1;
  if (a->boundary != b->boundary) return a->boundary < b->boundary ? -1 : 1;
  if (a->space != b->space) return a->space < b->space ? -1 : 1;
  if (a->lblock != b->lblock) return a->lblock < b->lblock ? -1 : 1;
  if (a->unit != b->unit) return a->unit < b->unit ? -1 : 1;
  if (a->block != b->block) return a->block < b->block ? -1 : 1;
  return 0;
}

/* Instances of one sorted hit list, summed per (trace, boundary). */
static int collect_instances(inst_hit* hits, uint64_t nh, barrier_list* res) {
  if (nh) qsort(hits, nh, sizeof(inst_hit), cmp_inst_hit);
  for (uint64_t i = 0; i < nh;) {
    orc_barrier e = {hits[i].trace, hits[i].boundary, 0, 0};
    uint64_t j = i;
    while (j < nh && hits[j].trace == e.trace && hits[j].boundary == e.boundary) {
      /* one instance: all hits with the same location and block */
      uint64_t k = j;
      uint32_t racing = 0;
      while (k < nh && cmp_inst_hit(&hits[k], &hits[j]) == 0) racing |= hits[k++].racing;
      e.instances++;
      e.racing += racing;
      j = k;
    }
    if (push_barrier(res, &e)) return ORC_ENOMEM;
    i = j;
  }
  return ORC_OK;
}

/* Tier A: every pair of records of a trace, tested against the definition. */
int64_t orc_barriers_brute_force(const orc_record* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                                 orc_barrier** out, uint64_t* bad_index) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  inst_hit* hits = NULL;
  uint64_t nh = 0, cap = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint32_t T = tpb[tr];
    for (uint64_t i = off[tr]; i < off[tr + 1]; i++)
      for (uint64_t j = off[tr]; j < off[tr + 1]; j++) {
        const orc_record* x = &recs[i];
        const orc_record* y = &recs[j];
        const uint32_t bx = x->tid / T, by = y->tid / T;
        /* x in epoch b, y in epoch b + 1, both of one block, one location */
        if (bx != by || x->space != y->space || x->unit != y->unit) continue;
        if ((uint32_t)y->epoch != (uint32_t)x->epoch + 1) continue;
        if (nh == cap) {
          cap = cap ? 2 * cap : 256;
          inst_hit* nv = (inst_hit*)realloc(hits, cap * sizeof(inst_hit));
          if (!nv) { free(hits); return ORC_ENOMEM; }
          hits = nv;
        }
        inst_hit h;
        h.trace = tr;
        h.boundary = x->epoch;
        h.space = x->space;
        h.lblock = x->space == 1 ? bx : 0xFFFFFFFFu;
        h.block = bx;
        h.unit = x->unit;
        h.racing = (x->tid != y->tid && conflicts(x->action, y->action)) ? 1u : 0u;
        hits[nh++] = h;
      }
  }
  barrier_list res = {0, 0, 0};
  rc = collect_instances(hits, nh, &res);
  free(hits);
  if (rc) { free(res.v); return rc; }
  *out = res.v;
  return (int64_t)res.n;
}

/* Tier B: records grouped by location, block and epoch (sorted items); for
 * every two adjacent epoch groups of one block and location, an instance,
 * racing when some pair across the two groups races. */
int64_t orc_barriers(const orc_record* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                     orc_barrier** out, uint64_t* bad_index) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  uint64_t maxn = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++)
    if (off[tr + 1] - off[tr] > maxn) maxn = off[tr + 1] - off[tr];
  item* it = maxn ? (item*)malloc(maxn * sizeof(item)) : NULL;
  if (maxn && !it) return ORC_ENOMEM;
  inst_hit* hits = NULL;
  uint64_t nh = 0, cap = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], n = off[tr + 1] - off[tr];
    for (uint64_t i = 0; i < n; i++) to_item(&recs[lo + i], tpb[tr], &it[i]);
    if (n) qsort(it, n, sizeof(item), cmp_item);
    /* epoch groups [g0, g1) and [g1, g2) of one location and block */
    for (uint64_t g0 = 0; g0 < n;) {
      uint64_t g1 = g0;
      while (g1 < n && same_loc(&it[g1], &it[g0]) && it[g1].block == it[g0].block && it[g1].epoch == it[g0].epoch)
        g1++;
      if (g1 < n && same_loc(&it[g1], &it[g0]) && it[g1].block == it[g0].block &&
          (uint32_t)it[g1].epoch == (uint32_t)it[g0].epoch + 1) {
        uint64_t g2 = g1;
        while (g2 < n && same_loc(&it[g2], &it[g1]) && it[g2].block == it[g1].block && it[g2].epoch == it[g1].epoch)
          g2++;
        uint32_t racing = 0;
        for (uint64_t a = g0; a < g1 && !racing; a++)
          for (uint64_t b = g1; b < g2 && !racing; b++)
            if (it[a].tid != it[b].tid && conflicts(it[a].action, it[b].action)) racing = 1;
        if (nh == cap) {
          cap = cap ? 2 * cap : 256;
          inst_hit* nv = (inst_hit*)realloc(hits, cap * sizeof(inst_hit));
          if (!nv) { free(hits); free(it); return ORC_ENOMEM; }
          hits = nv;
        }
        inst_hit h;
        h.trace = tr;
        h.boundary = it[g0].epoch;
        h.space = it[g0].space;
        h.lblock = it[g0].lblock;
        h.block = it[g0].block;
        h.unit = it[g0].unit;
        h.racing = racing;
        hits[nh++] = h;
      }
      g0 = g1;
    }
  }
  free(it);
  barrier_list res = {0, 0, 0};
  rc = collect_instances(hits, nh, &res);
  free(hits);
  if (rc) { free(res.v); return rc; }
  *out = res.v;
  return (int64_t)res.n;
}

/* ===================== Barrier divergence (Alg. 4) =====================
 *
 * Alg. 4 reports a barrier divergence when a thread reaches the end of the
 * kernel while other threads of its block halt at a barrier (Sec. 4.2.2):
 * the halted thread waits at a barrier the finished one never reaches.  So,
 * given for every thread the number of barriers it arrived at before it
 * finished, a block diverges when those numbers are not all equal: a thread
 * with fewer arrivals finished while a thread with more waited at a barrier
 * it did not reach.  Per trace, threads are numbered block by block
 * (thread t is in block t / threads_per_block), and every block of the
 * trace is complete.  One entry per divergent block: the fewest and most
 * arrivals, and how many of its threads arrived at fewer than the most
 * (the threads that left early).
 */
typedef struct {
  uint32_t trace;
  uint32_t block;
  uint32_t min_barriers;
  uint32_t max_barriers;
  uint64_t early_threads;
} orc_divergence;

int64_t orc_divergence_check(const uint32_t* counts, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                             orc_divergence** out) {
  if (n_traces && (!off || !tpb)) return ORC_EINVAL;
  if (n_traces && off[0] != 0) return ORC_EINVAL;
  for (uint32_t t = 0; t < n_traces; t++) {
    if (off[t + 1] < off[t] || tpb[t] == 0) return ORC_EINVAL;
    if ((off[t + 1] - off[t]) % tpb[t] != 0) return ORC_EINVAL; /* whole blocks only */
  }
  if (n_traces && off[n_traces] && !counts) return ORC_EINVAL;
  orc_divergence* v = NULL;
  uint64_t n = 0, cap = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t n_blocks = (off[tr + 1] - off[tr]) / tpb[tr];
    for (uint64_t b = 0; b < n_blocks; b++) {
      const uint32_t* c = counts + off[tr] + b * tpb[tr];
      uint32_t lo = c[0], hi = c[0];
      for (uint32_t k = 1; k < tpb[tr]; k++) {
        if (c[k] < lo) lo = c[k];
        if (c[k] > hi) hi = c[k];
      }
      if (lo == hi) continue;
      uint64_t early = 0;
      for (uint32_t k = 0; k < tpb[tr]; k++) early += c[k] < hi ? 1 : 0;
      if (n == cap) {
        cap = cap ? 2 * cap : 64;
        orc_divergence* nv = (orc_divergence*)realloc(v, cap * sizeof(orc_divergence));
        if (!nv) { free(v); return ORC_ENOMEM; }
        v = nv;
      }
      orc_divergence d = {tr, (uint32_t)b, lo, hi, early};
      v[n++] = d;
    }
  }
  *out = v;
  return (int64_t)n;
}

/* ===================== EP fitness (Eq. 1, Sec. 4.1.1) =====================
 *
 * For one candidate input (one trace): g(i) is 1 when memory address i is
 * accessed at all and f(i) the number of threads that access it; the
 * primary fitness F = sum g / sum f is 1 when no two threads share an
 * address and smaller the more they do.  The secondary fitness is the
 * access range R = end - start.  Addresses are the locations of the race
 * check (a global unit, or a unit of one block's shared memory); threads
 * are grid-wide ids.  Per trace: the number of records, sum g (locations),
 * sum f (distinct (location, thread) pairs), the unit range of global and
 * of shared accesses (max - min, 0 without such accesses) and F (1 for a
 * trace without records).
 */
typedef struct {
  uint64_t n_records;
  uint64_t n_locations;
  uint64_t n_location_threads;
  uint64_t global_range;
  uint64_t shared_range;
  double fitness;
} orc_fitness;

typedef struct {
  uint64_t unit;
  uint32_t lblock;
  uint32_t tid;
  uint32_t space;
} loc_thread;

static int cmp_loc_thread(const void* pa, const void* pb) {
  const loc_thread* a = (const loc_thread*)pa;
  const loc_thread* b = (const loc_thread*)pb;
  if (a->space != b->space) return a->space < b->space ? -1 : 1;
  if (a->lblock != b->lblock) return a->lblock < b->lblock ? -1 : 1;
  if (a->unit != b->unit) return a->unit < b->unit ? -1 : 1;
  if (a->tid != b->tid) return a->tid < b->tid ? -1 : 1;
  return 0;
}

int orc_fitness_eval(const orc_record* recs, const uint64_t* off, uint32_t n_traces, const uint32_t* tpb,
                     orc_fitness* out, uint64_t* bad_index) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  uint64_t maxn = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++)
    if (off[tr + 1] - off[tr] > maxn) maxn = off[tr + 1] - off[tr];
  loc_thread* v = maxn ? (loc_thread*)malloc(maxn * sizeof(loc_thread)) : NULL;
  if (maxn && !v) return ORC_ENOMEM;
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], n = off[tr + 1] - off[tr];
    uint64_t gmin = UINT64_MAX, gmax = 0, smin = UINT64_MAX, smax = 0;
    for (uint64_t i = 0; i < n; i++) {
      const orc_record* r = &recs[lo + i];
      v[i].unit = r->unit;
      v[i].tid = r->tid;
      v[i].space = r->space;
      v[i].lblock = r->space == 1 ? r->tid / tpb[tr] : 0xFFFFFFFFu;
      if (r->space == 0) {
        if (r->unit < gmin) gmin = r->unit;
        if (r->unit > gmax) gmax = r->unit;
      } else {
        if (r->unit < smin) smin = r->unit;
        if (r->unit > smax) smax = r->unit;
      }
    }
    if (n) qsort(v, n, sizeof(loc_thread), cmp_loc_thread);
    uint64_t g = 0, f = 0;
    for (uint64_t i = 0; i < n; i++) {
      const int new_loc = i == 0 || v[i].space != v[i - 1].space || v[i].lblock != v[i - 1].lblock ||
                          v[i].unit != v[i - 1].unit;
      if (new_loc) g++;
      if (new_loc || v[i].tid != v[i - 1].tid) f++;
    }
    out[tr].n_records = n;
    out[tr].n_locations = g;
    out[tr].n_location_threads = f;
    out[tr].global_range = gmin <= gmax ? gmax - gmin : 0;
    out[tr].shared_range = smin <= smax ? smax - smin : 0;
    out[tr].fitness = f ? (double)g / (double)f : 1.0;
  }
  free(v);
  return ORC_OK;
}

/* ============ warp-aware race check (Theorem 1, clauses 1-3) ============
 *
 * Theorem 1, and the race loop of Alg. 5, refine the check for two threads
 * of one warp (32 consecutive threads of a block execute in lockstep,
 * Sec. 2): such a pair of accesses races only when the threads had
 * undergone branch divergence (clause 3), or when both write by the same
 * statement (clause 2); threads of different warps race as before
 * (clause 1).  Every record comes with a side word: bits 0-30 name the
 * statement (the static memory-access instruction) that made the access,
 * bit 31 is set when the access ran while its warp was diverged.  A
 * same-warp pair counts as having undergone divergence when either of its
 * records carries the bit.  The warp of a thread is its block and its
 * block-local id divided by 32 (CUDA's linear order within a block).
 * Records of different blocks are in different warps, so the cross-block
 * count equals the plain check's.
 *
 * Tier A (orc_brute_force_warp) adds the warp test to the pairwise
 * definition.  Tier B (orc_closed_form_warp) takes the plain group counts
 * and subtracts, per warp group g (the records of one location, block,
 * epoch and warp), the pairs the lockstep rule removes: among the records
 * of g without the divergence bit, the conflicting pairs of different
 * threads, K_k(g0) - sum_t K_k(g0_t), except the write/write pairs of one
 * statement, C2(w_{g0,s}) - sum_t C2(w_{g0,s,t}) summed over statements s,
 * which stay races.  C2(m) = m(m-1)/2. */
#define WARP_SIZE 32u
#define SD_DIVERGED 0x80000000u

static int same_warp(uint32_t t1, uint32_t t2, uint32_t T) {
  return t1 / T == t2 / T && (t1 % T) / WARP_SIZE == (t2 % T) / WARP_SIZE;
}

int64_t orc_brute_force_warp(const orc_record* recs, const uint32_t* sd, const uint64_t* off, uint32_t n_traces,
                             const uint32_t* tpb, orc_race** out, orc_summary* summary, uint64_t* bad_index) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  if (n_traces && off[n_traces] && !sd) return ORC_EINVAL;
  race_list hits = {0, 0, 0};
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], hi = off[tr + 1];
    const uint32_t T = tpb[tr];
    for (uint64_t i = lo; i < hi; i++) {
      const orc_record* x = &recs[i];
      const uint32_t bx = x->tid / T;
      for (uint64_t j = i + 1; j < hi; j++) {
        const orc_record* y = &recs[j];
        const uint32_t by = y->tid / T;
        if (x->space != y->space || x->unit != y->unit) continue;
        if (x->space == 1 && bx != by) continue;
        if (x->tid == y->tid) continue;
        const int kind = kind_of(x->action, y->action);
        if (kind < 0) continue;
        if (!(bx != by || x->epoch == y->epoch)) continue;
        /* one warp: lockstep orders the pair unless it diverged or both
         * write by the same statement */
        if (same_warp(x->tid, y->tid, T)) {
          const int diverged = ((sd[i] | sd[j]) & SD_DIVERGED) != 0;
          const int same_stmt_writes = x->action == 1 && y->action == 1 &&
                                       (sd[i] & ~SD_DIVERGED) == (sd[j] & ~SD_DIVERGED);
          if (!diverged && !same_stmt_writes) continue;
        }
        orc_race h;
        memset(&h, 0, sizeof h);
        h.trace = tr;
        h.space = x->space;
        h.block = x->space == 1 ? bx : 0xFFFFFFFFu;
        h.unit = x->unit;
        if (kind == KIND_WW) h.pairs_ww = 1;
        if (kind == KIND_RW) h.pairs_rw = 1;
        if (kind == KIND_AW) h.pairs_aw = 1;
        if (kind == KIND_AR) h.pairs_ar = 1;
        h.pairs_xblock = (bx != by) ? 1 : 0;
        if (push(&hits, &h)) { free(hits.v); return ORC_ENOMEM; }
      }
    }
  }
  if (hits.n) qsort(hits.v, hits.n, sizeof(orc_race), cmp_entry);
  race_list res = {0, 0, 0};
  for (uint64_t i = 0; i < hits.n;) {
    orc_race e = hits.v[i];
    uint64_t j = i + 1;
    while (j < hits.n && cmp_entry(&hits.v[j], &hits.v[i]) == 0) {
      e.pairs_ww += hits.v[j].pairs_ww;
      e.pairs_rw += hits.v[j].pairs_rw;
      e.pairs_aw += hits.v[j].pairs_aw;
      e.pairs_ar += hits.v[j].pairs_ar;
      e.pairs_xblock += hits.v[j].pairs_xblock;
      j++;
    }
    finish_entry(&e);
    if (push(&res, &e)) { free(hits.v); free(res.v); return ORC_ENOMEM; }
    i = j;
  }
  free(hits.v);
  summarise(&res, off, n_traces, summary);
  *out = res.v;
  return (int64_t)res.n;
}

typedef struct {
  item it;
  uint32_t sd;
} witem;

static int cmp_witem(const void* pa, const void* pb) { return cmp_item(&((const witem*)pa)->it, &((const witem*)pb)->it); }

/* (statement, thread) of a write, for the same-statement counts */
typedef struct {
  uint32_t stmt, tid;
} stmt_tid;

static int cmp_stmt_tid(const void* pa, const void* pb) {
  const stmt_tid* a = (const stmt_tid*)pa;
  const stmt_tid* b = (const stmt_tid*)pb;
  if (a->stmt != b->stmt) return a->stmt < b->stmt ? -1 : 1;
  if (a->tid != b->tid) return a->tid < b->tid ? -1 : 1;
  return 0;
}

static uint64_t c2(uint64_t m) { return m ? m * (m - 1) / 2 : 0; }

/* Pairs the lockstep rule removes from one warp group [i, j) (sorted by
 * thread), by kind; st is scratch for j - i entries. */
static void warp_group_removed(const witem* w, uint64_t i, uint64_t j, stmt_tid* st, uint64_t rem[4]) {
  counts g0 = {0, 0, 0};
  uint64_t sumT[4] = {0, 0, 0, 0}, tmp[4];
  uint64_t nw = 0;
  for (uint64_t a = i; a < j;) { /* thread groups */
    uint64_t b = a;
    counts t0 = {0, 0, 0};
    while (b < j && w[b].it.tid == w[a].it.tid) {
      if (!(w[b].sd & SD_DIVERGED)) {
        add(&t0, w[b].it.action);
        add(&g0, w[b].it.action);
        if (w[b].it.action == 1) {
          st[nw].stmt = w[b].sd & ~SD_DIVERGED;
          st[nw].tid = w[b].it.tid;
          nw++;
        }
      }
      b++;
    }
    K(&t0, tmp);
    for (int k = 0; k < 4; k++) sumT[k] += tmp[k];
    a = b;
  }
  K(&g0, tmp);
  for (int k = 0; k < 4; k++) rem[k] = tmp[k] - sumT[k];
  /* write/write pairs of one statement from different threads stay races */
  if (nw > 1) qsort(st, nw, sizeof(stmt_tid), cmp_stmt_tid);
  uint64_t keep = 0;
  for (uint64_t a = 0; a < nw;) {
    uint64_t b = a;
    while (b < nw && st[b].stmt == st[a].stmt) b++;
    keep += c2(b - a);
    for (uint64_t c = a; c < b;) {
      uint64_t d = c;
      while (d < b && st[d].tid == st[c].tid) d++;
      keep -= c2(d - c);
      c = d;
    }
    a = b;
  }
  rem[KIND_WW] -= keep;
}

static int count_sorted_warp(const witem* w, uint64_t n, uint32_t tr, uint32_t T, stmt_tid* st, race_list* res) {
  uint64_t i = 0;
  while (i < n) {
    uint64_t iL = i;
    counts cL = {0, 0, 0};
    while (iL < n && same_loc(&w[iL].it, &w[i].it)) add(&cL, w[iL++].it.action);
    uint64_t KL[4], SB[4] = {0, 0, 0, 0}, SE[4] = {0, 0, 0, 0}, ST[4] = {0, 0, 0, 0}, RM[4] = {0, 0, 0, 0};
    uint64_t tmp[4];
    K(&cL, KL);
    for (uint64_t ib = i; ib < iL;) { /* block groups */
      uint64_t jb = ib;
      counts cB = {0, 0, 0};
      while (jb < iL && w[jb].it.block == w[ib].it.block) add(&cB, w[jb++].it.action);
      K(&cB, tmp);
      for (int k = 0; k < 4; k++) SB[k] += tmp[k];
      for (uint64_t ie = ib; ie < jb;) { /* epoch groups */
        uint64_t je = ie;
        counts cE = {0, 0, 0};
        while (je < jb && w[je].it.epoch == w[ie].it.epoch) add(&cE, w[je++].it.action);
        K(&cE, tmp);
        for (int k = 0; k < 4; k++) SE[k] += tmp[k];
        for (uint64_t itd = ie; itd < je;) { /* thread groups */
          uint64_t jt = itd;
          counts cT = {0, 0, 0};
          while (jt < je && w[jt].it.tid == w[itd].it.tid) add(&cT, w[jt++].it.action);
          K(&cT, tmp);
          for (int k = 0; k < 4; k++) ST[k] += tmp[k];
          itd = jt;
        }
        for (uint64_t iw = ie; iw < je;) { /* warp groups (threads sorted, so contiguous) */
          uint64_t jw = iw;
          while (jw < je && same_warp(w[jw].it.tid, w[iw].it.tid, T)) jw++;
          warp_group_removed(w, iw, jw, st, tmp);
          for (int k = 0; k < 4; k++) RM[k] += tmp[k];
          iw = jw;
        }
        ie = je;
      }
      ib = jb;
    }
    uint64_t p[4], xb = 0;
    for (int k = 0; k < 4; k++) {
      p[k] = KL[k] - SB[k] + SE[k] - ST[k] - RM[k];
      xb += KL[k] - SB[k];
    }
    if (p[0] + p[1] + p[2] + p[3] > 0) {
      orc_race e;
      memset(&e, 0, sizeof e);
      e.trace = tr;
      e.space = w[i].it.space;
      e.block = w[i].it.lblock;
      e.unit = w[i].it.unit;
      e.pairs_ww = p[KIND_WW];
      e.pairs_rw = p[KIND_RW];
      e.pairs_aw = p[KIND_AW];
      e.pairs_ar = p[KIND_AR];
      e.pairs_xblock = xb;
      finish_entry(&e);
      if (push(res, &e)) return ORC_ENOMEM;
    }
    i = iL;
  }
  return ORC_OK;
}

int64_t orc_closed_form_warp(const orc_record* recs, const uint32_t* sd, const uint64_t* off, uint32_t n_traces,
                             const uint32_t* tpb, orc_race** out, orc_summary* summary, uint64_t* bad_index) {
  int rc = validate(recs, off, n_traces, tpb, bad_index);
  if (rc) return rc;
  if (n_traces && off[n_traces] && !sd) return ORC_EINVAL;
  race_list res = {0, 0, 0};
  uint64_t maxn = 0;
  for (uint32_t tr = 0; tr < n_traces; tr++)
    if (off[tr + 1] - off[tr] > maxn) maxn = off[tr + 1] - off[tr];
  witem* w = maxn ? (witem*)malloc(maxn * sizeof(witem)) : NULL;
  stmt_tid* st = maxn ? (stmt_tid*)malloc(maxn * sizeof(stmt_tid)) : NULL;
  if (maxn && (!w || !st)) { free(w); free(st); return ORC_ENOMEM; }
  for (uint32_t tr = 0; tr < n_traces; tr++) {
    const uint64_t lo = off[tr], n = off[tr + 1] - off[tr];
    const uint32_t T = tpb[tr];
    for (uint64_t i = 0; i < n; i++) {
      to_item(&recs[lo + i], T, &w[i].it);
      w[i].sd = sd[lo + i];
    }
    if (n) qsort(w, n, sizeof(witem), cmp_witem);
    if (count_sorted_warp(w, n, tr, T, st, &res)) { free(w); free(st); free(res.v); return ORC_ENOMEM; }
  }
  free(w);
  free(st);
  summarise(&res, off, n_traces, summary);
  *out = res.v;
  return (int64_t)res.n;
}

void orc_free(void* p) { free(p); }
