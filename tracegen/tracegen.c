/*
 * tracegen.c -- seeded synthetic Memory-Model traces.
 *
 * This module only produces input records; it holds none of the race-check
 * arithmetic.  Both the oracle and the GPU path consume its output.
 *
 * A record is one Unit Tuple of the paper's Memory Model (Sec. 4.2.1): the
 * accessed memory unit, the thread, the visit order (here: the number of
 * barriers the thread has passed, its "epoch") and the action, plus the
 * memory space (global or per-block shared, Sec. 4.2.2 / Alg. 3).
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed by the seed
 * and indexed by (access index, global thread id, purpose, trace), so every
 * record is reproducible independently of threading.  Zipf ranks use the
 * rejection-inversion method of Hoermann and Derflinger (ACM TOMACS 1996).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t unit;
  uint32_t tid;
  uint16_t epoch;
  uint8_t action; /* 0 read, 1 write, 2 atomic */
  uint8_t space;  /* 0 global, 1 shared */
} tg_record;

typedef struct {
  uint8_t space;
  uint8_t action_x; /* action of the targeted record */
  uint8_t action_y; /* action written into the rewritten record */
  uint8_t cross_block;
  uint32_t block; /* owning block if shared, 0xFFFFFFFF if global */
  uint64_t unit;
  uint64_t x_index; /* targeted record */
  uint64_t y_index; /* rewritten record */
} tg_injection;

typedef struct {
  uint32_t n_blocks;
  uint32_t tpb;        /* threads per block */
  uint32_t k;          /* accesses per thread */
  uint32_t per_epoch;  /* accesses between two barriers */
  double p_read;
  double p_write;      /* p_atomic = 1 - p_read - p_write */
  double p_shared;     /* probability that a read/write targets shared memory */
  uint32_t shared_words;      /* per-block shared window, in 4-byte words */
  uint32_t global_read_log2;  /* global read region = 2^this words */
  uint32_t atomic_bins_log2;  /* atomic bin region = 2^this words */
  double zipf_s;
  uint64_t n_records; /* emission-order prefix that exists (<= n_blocks*tpb*k) */
  double inject_rate;
  uint64_t seed;
  uint32_t trace_id;  /* mixed into every Philox counter */
} tg_params;

/* ---------------- Philox4x32-10 ---------------- */
static inline void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
  uint32_t n1 = (uint32_t)p1;
  uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
  uint32_t n3 = (uint32_t)p0;
  c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void tg_philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; r++) {
    philox_round(c, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

uint64_t tg_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct {
  uint32_t k0, k1, trace;
} rng_t;

static inline void draw(const rng_t* g, uint32_t a, uint32_t b, uint32_t purpose, uint32_t out[4]) {
  out[0] = a; out[1] = b; out[2] = purpose; out[3] = g->trace;
  tg_philox4x32_10(out, g->k0, g->k1);
}

/* 53-bit uniform double in [0,1) from two 32-bit words. */
static inline double u01(uint32_t x, uint32_t y) {
  return ((double)(x >> 5) * 67108864.0 + (double)(y >> 6)) * (1.0 / 9007199254740992.0);
}

/* ---------------- Zipf by rejection-inversion ---------------- */
typedef struct {
  double s, hx1, hN, sconst;
  uint64_t N;
} zipf_t;

static double zH(const zipf_t* z, double x) { /* integral of t^-s from 1 to x */
  return (pow(x, 1.0 - z->s) - 1.0) / (1.0 - z->s);
}
static double zHinv(const zipf_t* z, double y) {
  return pow(1.0 + y * (1.0 - z->s), 1.0 / (1.0 - z->s));
}
static double zh(const zipf_t* z, double x) { return pow(x, -z->s); }

static void zipf_init(zipf_t* z, uint64_t N, double s) {
  z->s = s;
  z->N = N;
  z->hx1 = zH(z, 1.5) - 1.0;
  z->hN = zH(z, (double)N + 0.5);
  z->sconst = 2.0 - zHinv(z, zH(z, 2.5) - zh(z, 2.0));
}

/* Returns a rank in [1, N]; draws are indexed by (a, b, purpose base). */
static uint64_t zipf_sample(const zipf_t* z, const rng_t* g, uint32_t a, uint32_t b, uint32_t pbase) {
  for (uint32_t attempt = 0;; attempt++) {
    uint32_t r[4];
    draw(g, a, b, pbase + attempt, r);
    for (int half = 0; half < 2; half++) {
      double U = u01(r[2 * half], r[2 * half + 1]);
      double u = z->hN + U * (z->hx1 - z->hN);
      double x = zHinv(z, u);
      double kf = floor(x + 0.5);
      if (kf < 1.0) kf = 1.0;
      if (kf > (double)z->N) kf = (double)z->N;
      if (kf - x <= z->sconst || u >= zH(z, kf + 0.5) - zh(z, kf)) return (uint64_t)kf;
    }
  }
}

/* Draw a Zipf rank (exposed for tests of the sampler). */
uint64_t tg_zipf_rank(uint64_t N, double s, uint64_t seed, uint32_t a, uint32_t b) {
  zipf_t z;
  zipf_init(&z, N, s);
  rng_t g = {(uint32_t)seed, (uint32_t)(seed >> 32), 0};
  return zipf_sample(&z, &g, a, b, 0);
}

/* ---------------- helpers ---------------- */
static inline uint64_t rank_to_unit(uint64_t r0, uint32_t log2n) {
  /* odd multiplier: a bijection on [0, 2^log2n) that scatters hot ranks */
  uint64_t m = (log2n >= 64) ? ~0ull : ((1ull << log2n) - 1);
  return (r0 * 0x9E3779B1ull) & m;
}

enum { P_ACTION = 0, P_SHARED_WRITE = 1, P_ZIPF = 16, P_SHREAD = 4096, P_ATOMIC = 8192 };

/* Fill one block's records (emission order: for each access index j, threads
 * 0..tpb-1).  Shared accesses are race-free by construction: within one
 * (block, epoch) a shared word is written only by its owner thread
 * own(u, e) = (u + 37 e) mod tpb, and reads avoid words written by another
 * thread in that (block, epoch).  Global reads hit a Zipf-distributed read
 * region that is never written; global writes go to a thread-private fresh
 * word; atomics go to a Zipf-distributed bin region that is never plainly
 * accessed. */
static void gen_block(const tg_params* P, const rng_t* g, const zipf_t* zr, const zipf_t* za,
                      uint32_t b, tg_record* out, int32_t* writer) {
  const uint64_t per_block = (uint64_t)P->tpb * P->k;
  const uint64_t base = (uint64_t)b * per_block;
  const uint64_t read_region = 1ull << P->global_read_log2;
  const uint64_t out_region = read_region;
  const uint64_t nthreads = (uint64_t)P->n_blocks * P->tpb;
  const uint64_t atomic_region = out_region + nthreads * P->k;
  const uint32_t W = P->shared_words;
  const uint32_t pe = P->per_epoch ? P->per_epoch : P->k;
  if (base >= P->n_records) return;

  for (uint32_t j0 = 0; j0 < P->k; j0 += pe) {
    const uint32_t e = j0 / pe;
    const uint32_t j1 = (j0 + pe < P->k) ? j0 + pe : P->k;
    for (uint32_t w = 0; w < W; w++) writer[w] = -1;
    /* phase 1: actions, writes and atomics */
    for (uint32_t j = j0; j < j1; j++) {
      for (uint32_t t = 0; t < P->tpb; t++) {
        const uint64_t idx = base + (uint64_t)j * P->tpb + t;
        if (idx >= P->n_records) continue;
        const uint32_t gtid = b * P->tpb + t;
        tg_record* r = &out[idx];
        uint32_t d[4];
        draw(g, j, gtid, P_ACTION, d);
        const double ua = u01(d[0], d[1]);
        const double us = (double)(d[2] >> 8) * (1.0 / 16777216.0);
        r->tid = gtid;
        r->epoch = (uint16_t)e;
        if (ua < P->p_read) {
          r->action = 0;
          r->space = (us < P->p_shared) ? 1 : 0;
          r->unit = 0; /* filled in phase 2 */
        } else if (ua < P->p_read + P->p_write) {
          r->action = 1;
          r->space = (us < P->p_shared) ? 1 : 0;
          if (r->space == 1) {
            const uint32_t own = (uint32_t)(((int64_t)t - 37 * (int64_t)e) % (int64_t)P->tpb + P->tpb) % P->tpb;
            const uint32_t nw = (own < W) ? (W - own + P->tpb - 1) / P->tpb : 0;
            if (nw == 0) {
              r->space = 0;
            } else {
              const uint32_t u = own + P->tpb * (d[3] % nw);
              r->unit = u;
              writer[u] = (int32_t)t;
            }
          }
          if (r->space == 0) r->unit = out_region + (uint64_t)gtid * P->k + j;
        } else {
          r->action = 2;
          r->space = 0;
          const uint64_t rank = zipf_sample(za, g, j, gtid, P_ATOMIC);
          r->unit = atomic_region + rank_to_unit(rank - 1, P->atomic_bins_log2);
        }
      }
    }
    /* phase 2: reads */
    for (uint32_t j = j0; j < j1; j++) {
      for (uint32_t t = 0; t < P->tpb; t++) {
        const uint64_t idx = base + (uint64_t)j * P->tpb + t;
        if (idx >= P->n_records) continue;
        tg_record* r = &out[idx];
        if (r->action != 0) continue;
        const uint32_t gtid = b * P->tpb + t;
        if (r->space == 0) {
          const uint64_t rank = zipf_sample(zr, g, j, gtid, P_ZIPF);
          r->unit = rank_to_unit(rank - 1, P->global_read_log2);
        } else {
          uint32_t d[4];
          draw(g, j, gtid, P_SHREAD, d);
          uint32_t u = d[0] % W;
          /* linear probe from a random start: the first word not written by
           * another thread in this (block, epoch) */
          for (uint32_t s = 0; s < W; s++) {
            const int32_t wr = writer[u];
            if (wr < 0 || wr == (int32_t)t) break;
            u = (u + 1 == W) ? 0 : u + 1;
          }
          r->unit = u;
        }
      }
    }
  }
}

/* ---------------- injection ---------------- */
typedef struct {
  uint64_t* slot;
  uint64_t cap;
} iset_t;

static int iset_has(const iset_t* s, uint64_t v) {
  uint64_t h = tg_splitmix64(v) & (s->cap - 1);
  while (s->slot[h] != ~0ull) {
    if (s->slot[h] == v) return 1;
    h = (h + 1) & (s->cap - 1);
  }
  return 0;
}
static void iset_add(iset_t* s, uint64_t v) {
  uint64_t h = tg_splitmix64(v) & (s->cap - 1);
  while (s->slot[h] != ~0ull) {
    if (s->slot[h] == v) return;
    h = (h + 1) & (s->cap - 1);
  }
  s->slot[h] = v;
}

/* Rewrite m = round(rate * n) records so that each creates a race with a
 * targeted record x.  Returns the number of injections made. */
static int64_t inject(const tg_params* P, const rng_t* g, tg_record* out, tg_injection* log, uint64_t log_cap) {
  const uint64_t n = P->n_records;
  const uint64_t m = (uint64_t)llround(P->inject_rate * (double)n);
  if (m == 0 || n < 2) return 0;
  const uint64_t per_block = (uint64_t)P->tpb * P->k;
  const uint32_t pe = P->per_epoch ? P->per_epoch : P->k;
  iset_t touched;
  touched.cap = 64;
  while (touched.cap < 8 * m + 64) touched.cap <<= 1;
  touched.slot = (uint64_t*)malloc(touched.cap * sizeof(uint64_t));
  if (!touched.slot) return -1;
  memset(touched.slot, 0xFF, touched.cap * sizeof(uint64_t));
  int64_t done = 0;
  uint32_t attempt = 0;
  for (uint64_t i = 0; i < m && attempt < 64u * (uint32_t)m + 1024u; attempt++) {
    uint32_t d[4], e4[4];
    draw(g, (uint32_t)attempt, 0xFFFFFFFFu, 0x100, d);
    draw(g, (uint32_t)attempt, 0xFFFFFFFEu, 0x101, e4);
    const uint64_t x = (((uint64_t)d[0] << 32) | d[1]) % n;
    if (iset_has(&touched, x)) continue;
    const tg_record rx = out[x];
    const uint32_t bx = (uint32_t)(x / per_block);
    const uint64_t rem = x % per_block;
    const uint32_t jx = (uint32_t)(rem / P->tpb);
    const uint32_t tx = (uint32_t)(rem % P->tpb);
    const uint32_t ex = jx / pe;
    int cross = 0;
    if (rx.space == 0 && P->n_blocks >= 2) cross = (d[2] & 1) ? 1 : 0;
    if (P->tpb < 2) {
      if (rx.space == 1 || P->n_blocks < 2) continue;
      cross = 1;
    }
    uint64_t y;
    if (!cross) {
      const uint32_t j0 = ex * pe;
      const uint32_t j1 = (j0 + pe < P->k) ? j0 + pe : P->k;
      const uint32_t jy = j0 + e4[0] % (j1 - j0);
      const uint32_t ty = (tx + 1 + e4[1] % (P->tpb - 1)) % P->tpb;
      y = (uint64_t)bx * per_block + (uint64_t)jy * P->tpb + ty;
    } else {
      const uint32_t by = (bx + 1 + e4[0] % (P->n_blocks - 1)) % P->n_blocks;
      const uint32_t jy = e4[1] % P->k;
      const uint32_t ty = e4[2] % P->tpb;
      y = (uint64_t)by * per_block + (uint64_t)jy * P->tpb + ty;
    }
    if (y >= n || y == x || iset_has(&touched, y)) continue;
    tg_record* ry = &out[y];
    ry->unit = rx.unit;
    ry->space = rx.space;
    ry->action = (rx.action == 2) ? 0 : 1; /* read against an atomic, else write */
    iset_add(&touched, x);
    iset_add(&touched, y);
    if (log && (uint64_t)done < log_cap) {
      tg_injection* L = &log[done];
      L->space = rx.space;
      L->action_x = rx.action;
      L->action_y = ry->action;
      L->cross_block = (uint8_t)cross;
      L->block = rx.space == 1 ? rx.tid / P->tpb : 0xFFFFFFFFu;
      L->unit = rx.unit;
      L->x_index = x;
      L->y_index = y;
    }
    done++;
    i++;
  }
  free(touched.slot);
  return done;
}

/* Generate one trace.  `out` holds n_records records; `log` (nullable)
 * receives up to log_cap injections.  Returns the number of injections, or a
 * negative value on bad parameters. */
static int params_ok(const tg_params* P) {
  if (!P || P->tpb == 0 || P->k == 0 || P->n_blocks == 0) return 0;
  if ((uint64_t)P->n_blocks * P->tpb * P->k < P->n_records) return 0;
  if (P->shared_words == 0 || P->global_read_log2 > 40 || P->atomic_bins_log2 > 32) return 0;
  if ((uint64_t)P->n_blocks * P->tpb > 0xFFFFFFFFull) return 0;
  if ((P->k + (P->per_epoch ? P->per_epoch : P->k) - 1) / (P->per_epoch ? P->per_epoch : P->k) > 65536u) return 0;
  return 1;
}

int64_t tg_generate(const tg_params* P, tg_record* out, tg_injection* log, uint64_t log_cap, int n_threads) {
  if (!out || !params_ok(P)) return -1;
  rng_t g = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32), P->trace_id};
  zipf_t zr, za;
  zipf_init(&zr, 1ull << P->global_read_log2, P->zipf_s);
  zipf_init(&za, 1ull << P->atomic_bins_log2, P->zipf_s);
  const int64_t nb = P->n_blocks;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
  {
    int32_t* writer = (int32_t*)malloc(sizeof(int32_t) * P->shared_words);
#pragma omp for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; b++) gen_block(P, &g, &zr, &za, (uint32_t)b, out, writer);
    free(writer);
  }
  return inject(P, &g, out, log, log_cap);
}

typedef struct {
  uint64_t n, i;
} size_by_index;

static int larger_first(const void* a, const void* b) {
  const size_by_index *x = (const size_by_index*)a, *y = (const size_by_index*)b;
  if (x->n != y->n) return x->n > y->n ? -1 : 1;
  return x->i < y->i ? -1 : (x->i > y->i);
}

/* Many traces at once: trace i (parameters P[i]) is written to
 * out + offsets[i] and its injections to log + log_off[i] (capacity
 * log_off[i+1] - log_off[i]); n_inj[i] receives the injection count.  The
 * records are the same as n_traces calls of tg_generate; the work is spread
 * over traces rather than over the blocks of one trace.  Returns 0, or -1
 * (nothing written) when some trace's parameters are invalid. */
int64_t tg_generate_batch(const tg_params* P, uint64_t n_traces, tg_record* out, const uint64_t* offsets,
                          tg_injection* log, const uint64_t* log_off, int64_t* n_inj, int n_threads) {
  if (!P || !out || !offsets || !log || !log_off || !n_inj) return -1;
  for (uint64_t i = 0; i < n_traces; i++)
    if (!params_ok(&P[i]) || offsets[i + 1] - offsets[i] != P[i].n_records) return -1;
  /* largest traces first, for balance */
  size_by_index* order = (size_by_index*)malloc(sizeof(size_by_index) * (n_traces ? n_traces : 1));
  if (!order) return -1;
  for (uint64_t i = 0; i < n_traces; i++) { order[i].n = P[i].n_records; order[i].i = i; }
  qsort(order, n_traces, sizeof(size_by_index), larger_first);
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
  {
    uint32_t cap = 0;
    int32_t* writer = NULL;
#pragma omp for schedule(dynamic, 1)
    for (int64_t j = 0; j < (int64_t)n_traces; j++) {
      const uint64_t i = order[j].i;
      const tg_params* p = &P[i];
      if (p->shared_words > cap) {
        free(writer);
        cap = p->shared_words;
        writer = (int32_t*)malloc(sizeof(int32_t) * cap);
      }
      rng_t g = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32), p->trace_id};
      zipf_t zr, za;
      zipf_init(&zr, 1ull << p->global_read_log2, p->zipf_s);
      zipf_init(&za, 1ull << p->atomic_bins_log2, p->zipf_s);
      tg_record* o = out + offsets[i];
      for (uint32_t b = 0; b < p->n_blocks; b++) gen_block(p, &g, &zr, &za, b, o, writer);
      n_inj[i] = inject(p, &g, o, log + log_off[i], log_off[i + 1] - log_off[i]);
    }
    free(writer);
  }
  free(order);
  return 0;
}

/* ---------------- hand-built trace: shared-memory tree reduction ----------
 * One block of 256 threads reduces in[0..255] (global units 0..255) through
 * s[0..255] (shared units 0..255) into out[0] (global unit 256), with the
 * usual sequential-addressing loop: stride 128, 64, ..., 1, a barrier after
 * the initial store (B0) and after every level (B1..B8).  `removed` names a
 * barrier to leave out (0..8), or -1 for none.  Records are emitted in the
 * round-robin statement order of the paper's simulation (Alg. 3 / Alg. 4).
 * Returns the record count (1279). */
int64_t tg_tree_reduction(int removed, tg_record* out) {
  const uint32_t T = 256;
  int64_t n = 0;
  uint16_t epoch = 0;
#define EMIT(U, TID, ACT, SP) \
  do { out[n].unit = (U); out[n].tid = (TID); out[n].epoch = epoch; out[n].action = (ACT); out[n].space = (SP); n++; } while (0)
  for (uint32_t t = 0; t < T; t++) EMIT(t, t, 0, 0);       /* read in[t] */
  for (uint32_t t = 0; t < T; t++) EMIT(t, t, 1, 1);       /* s[t] = in[t] */
  if (removed != 0) epoch++;                               /* B0 */
  for (int lvl = 1; lvl <= 8; lvl++) {
    const uint32_t sig = T >> lvl;
    for (uint32_t t = 0; t < sig; t++) EMIT(t, t, 0, 1);       /* read s[t] */
    for (uint32_t t = 0; t < sig; t++) EMIT(t + sig, t, 0, 1); /* read s[t+stride] */
    for (uint32_t t = 0; t < sig; t++) EMIT(t, t, 1, 1);       /* write s[t] */
    if (removed != lvl) epoch++;                               /* B_lvl */
  }
  EMIT(0, 0, 0, 1);   /* thread 0 reads s[0] */
  EMIT(256, 0, 1, 0); /* and writes out[0] */
#undef EMIT
  return n;
}
