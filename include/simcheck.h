/*
 * simcheck.h -- C ABI of the MI355X data-race check over Memory-Model traces.
 *
 * The operation (paper Sec. 4.2.3, Theorem 1, and the data-race loop of
 * Alg. 5): a trace is a multiset of accesses, each one Unit Tuple of the
 * paper's Memory Model (Sec. 4.2.1) -- memory unit, thread, visit order,
 * action -- plus its memory space.  Two records of one trace race when
 *   - they touch the same location: the same unit of global memory (one
 *     array for all blocks), or the same unit of one block's shared memory
 *     (shared memory is private to a block, Alg. 3);
 *   - their thread ids differ;
 *   - they are concurrent: the same epoch (visit order, i.e. the number of
 *     barriers the thread has passed; Sec. 4.2.2, Alg. 4) within one block,
 *     or different blocks (a barrier synchronises one block only, Sec. 2);
 *   - at least one writes, and they are not both atomic (an atomic races
 *     with a plain read or write).
 * The warp clauses (1)-(3) of Theorem 1 are not applied by this check
 * (records carry no statement or divergence data): every pair of distinct
 * threads counts as potentially concurrent.  sim_check_traces_warp applies
 * them to records that come with a side word of statement and divergence.
 *
 * For every racing location the library returns one entry with the exact
 * number of racing unordered record pairs by kind and the cross-block
 * subset; entries are ordered by (trace, space, block, unit), global before
 * shared.  The result depends only on the multiset of records of each trace.
 *
 * Conventions
 *   - Little-endian, C99, no C++ or HIP types across the ABI.
 *   - Return value 0 on success, a negative SIM_E* code on error.  On error
 *     *out is set to NULL, nothing partial is returned and the context stays
 *     usable; sim_last_error() describes the failure.
 *   - A context is used by one host thread at a time; several contexts may
 *     coexist.  All work runs on the GPU given to sim_create(); there is no
 *     CPU fallback -- creation fails when no usable gfx950 device exists.
 */
#ifndef SIMCHECK_H
#define SIMCHECK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ types */

/* One access record (16 bytes, 8-byte aligned).
 *   unit   : memory unit index within its space (4-byte word address)
 *   tid    : grid-wide linear thread id; block = tid / threads_per_block
 *   epoch  : barriers the thread had passed at the access (visit order)
 *   action : SIM_READ, SIM_WRITE or SIM_ATOMIC
 *   space  : SIM_GLOBAL or SIM_SHARED                                      */
typedef struct sim_record {
  uint64_t unit;
  uint32_t tid;
  uint16_t epoch;
  uint8_t action;
  uint8_t space;
} sim_record;

enum { SIM_READ = 0, SIM_WRITE = 1, SIM_ATOMIC = 2 };
enum { SIM_GLOBAL = 0, SIM_SHARED = 1 };

/* kinds bits of a sim_race */
enum {
  SIM_KIND_WW = 1,     /* write / write   */
  SIM_KIND_RW = 2,     /* read / write    */
  SIM_KIND_AW = 4,     /* atomic / write  */
  SIM_KIND_AR = 8,     /* atomic / read   */
  SIM_KIND_XBLOCK = 16 /* some racing pair spans two blocks */
};

/* One racing location (64 bytes). */
typedef struct sim_race {
  uint32_t trace;      /* index of the trace in the call */
  uint8_t space;       /* SIM_GLOBAL or SIM_SHARED */
  uint8_t kinds;       /* SIM_KIND_* bits: pairs_k > 0, pairs_xblock > 0 */
  uint16_t reserved16; /* 0 */
  uint32_t block;      /* owning block if SIM_SHARED, 0xFFFFFFFF if SIM_GLOBAL */
  uint32_t reserved32; /* 0 */
  uint64_t unit;
  uint64_t pairs_ww, pairs_rw, pairs_aw, pairs_ar; /* racing unordered record pairs by kind */
  uint64_t pairs_xblock; /* subset of the above whose two records are in different blocks */
} sim_race;

typedef struct sim_trace_summary {
  uint64_t n_records;   /* records of the trace */
  uint64_t n_race_locs; /* entries of the trace */
  uint64_t n_pairs;     /* sum of pairs_ww + pairs_rw + pairs_aw + pairs_ar */
} sim_trace_summary;

/* Result of one call; allocated by the library, freed by sim_result_free(). */
typedef struct sim_result {
  sim_race* races;            /* n_races entries, host memory */
  uint64_t n_races;
  sim_trace_summary* traces;  /* n_traces summaries, host memory */
  uint32_t n_traces;
} sim_result;

typedef struct sim_config {
  uint64_t reserve_records; /* allocate at creation every device buffer of a call of this many records
                               (0: grow on demand); later calls up to that size allocate nothing */
  uint32_t flags;           /* SIM_CFG_* */
  uint32_t reserve_traces;  /* ... in this many traces (0: 1) */
} sim_config;

enum {
  SIM_CFG_PROFILE = 1, /* record per-stage HIP events (see sim_stage_times); disables graphs */
  SIM_CFG_GRAPHS = 2   /* capture each call's launch sequence as a HIP graph and replay it while
                          calls keep the same shape (records pointer, offsets, threads per block,
                          stream); needs a non-NULL stream */
};

typedef struct sim_ctx sim_ctx;

/* error codes */
enum {
  SIM_OK = 0,
  SIM_EINVAL = -1,  /* null pointer, offsets not CSR, threads_per_block = 0, too many records */
  SIM_ERECORD = -2, /* action > 2 or space > 1; sim_last_error() names the first bad index */
  SIM_ENOMEM = -3,  /* device or host allocation failed */
  SIM_EDEVICE = -4, /* HIP runtime error (text in sim_last_error()) */
  SIM_EAGAIN = -5,  /* serving: result not ready yet, or the pending queue is full */
  SIM_ERANGE = -6,  /* a trace's sort key would need more than 128 bits (cannot happen with 32-bit thread
                       ids and 16-bit epochs: keys take at most 116 bits; kept for the ABI) */
  SIM_ENOSPC = -7   /* sim_check_traces_device_noalloc: the caller's output buffer, or the scratch, holds
                       fewer entries than the call has; *n_races gives the number of entries */
};

/* --------------------------------------------------------------- context */

/* Create a context on HIP device `hip_device` (must be gfx950).
 * cfg may be NULL.  Returns SIM_EDEVICE when the device is missing or not
 * gfx950.                                                                  */
int sim_create(sim_ctx** out, int hip_device, const sim_config* cfg);

/* Release a context and its device buffers.  NULL is ignored. */
void sim_destroy(sim_ctx* ctx);

/* Text of the last error on this context ("" if none).  Valid until the
 * next call on the context.                                                */
const char* sim_last_error(const sim_ctx* ctx);

/* ----------------------------------------------------------------- checks */

/* Check n_traces traces whose records sit in host memory.
 *   records           : offsets[n_traces] records, host memory, caller-owned
 *   offsets           : n_traces + 1 CSR offsets, host memory; offsets[0] = 0,
 *                       non-decreasing; trace i is records[offsets[i] ..
 *                       offsets[i+1])
 *   threads_per_block : n_traces values >= 1, host memory
 *   out               : receives the result (caller frees it)
 * n_traces = 0 and empty traces are valid.  Inputs are read only and must
 * stay valid until the call returns.  The records are copied to the device
 * on the context's stream.
 * Keys: a record's sort key packs its location, block, epoch and thread in
 * as few bits as the trace's ranges allow.  When some trace of a call needs
 * more than 64 bits (a unit span near 2^64), the call runs with 128-bit
 * keys: 16 bytes of key storage per record instead of 8, and a second
 * device round when the context's previous call did not need them.       */
int sim_check_traces(sim_ctx* ctx, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
                     const uint32_t* threads_per_block, sim_result** out);

/* Same check for records already in device memory of the context's GPU
 * (e.g. a torch tensor's storage).  offsets and threads_per_block are host
 * arrays as above (they size the launch grids).  stream is a hipStream_t
 * (NULL: the default stream); the library orders all of its work on it and
 * returns after the stream has finished the call's work.  The stream is not
 * owned by the library.                                                    */
int sim_check_traces_device(sim_ctx* ctx, const sim_record* d_records, const uint64_t* offsets,
                            uint32_t n_traces, const uint32_t* threads_per_block, void* stream,
                            sim_result** out);

/* The check of sim_check_traces_device without any allocation, for callers
 * that cannot allocate (code that runs under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Every device buffer of
 * the call comes from one fixed scratch array of 128 MiB per GPU that the
 * library holds until the process ends, and the call's tables from pinned
 * host memory sim_create() allocated; the result goes to the caller's
 * buffers.  No device, pinned or host memory is allocated by this call
 * (creating the context, earlier, does allocate).
 *   d_records, offsets, n_traces, threads_per_block, stream : as for
 *                       sim_check_traces_device
 *   races      : host memory, room for races_cap entries; receives the
 *                entries in the order of sim_check_traces
 *   n_races    : receives the number of entries (also on SIM_ENOSPC)
 *   traces     : host memory, n_traces summaries
 * Limits: at most 4096 traces and 6144 tiles (a trace of n records takes
 * ceil(n / 4096) tiles), and the call's device buffers must fit the scratch:
 * 16 bytes per record (32 with two-word keys, see sim_check_traces), about
 * 4.3 KiB per tile and 128 bytes per trace, the rest holding the entry list
 * (2^22 records in one trace leave room for about a million entries).  A call
 * beyond these limits fails with SIM_EINVAL; one with more entries than
 * races_cap or than the scratch holds with SIM_ENOSPC.  Calls on one GPU
 * share its scratch: calls that overlap in time on one GPU (from several
 * threads or contexts) race with each other and must be serialised by the
 * caller.  The scratch keeps the last call's contents; every call
 * initialises what it reads.                                               */
int sim_check_traces_device_noalloc(sim_ctx* ctx, const sim_record* d_records, const uint64_t* offsets,
                                    uint32_t n_traces, const uint32_t* threads_per_block, void* stream,
                                    sim_race* races, uint64_t races_cap, uint64_t* n_races,
                                    sim_trace_summary* traces);

/* Free a result.  NULL is ignored. */
void sim_result_free(sim_result* r);

/* ---------------------------------------------------- warp-aware check */

/* Side word of a record for the warp-aware check: the statement (static
 * memory-access instruction) that made the access in bits 0-30, and
 * SIM_SIDE_DIVERGED when the access ran while its warp was diverged (some
 * of the warp's threads on another control path).                         */
#define SIM_SIDE_DIVERGED 0x80000000u

/* The race check with the warp clauses of Theorem 1 (paper Sec. 4.2.3, and
 * the race loop of Alg. 5): the 32 threads of a warp (threads of one block
 * whose block-local ids agree after division by 32; Sec. 2) run in
 * lockstep, so two accesses by different threads of one warp race only
 * when the threads had diverged before them (either record carries
 * SIM_SIDE_DIVERGED; clause 3) or both are writes by the same statement
 * (clause 2).  Threads of different warps race as in sim_check_traces
 * (clause 1); cross-block pairs are never in one warp.  The result has the
 * form and order of sim_check_traces's, with the pair counts of this rule:
 * a location whose racing pairs are all ordered by lockstep has no entry.
 *   d_records, offsets, n_traces, threads_per_block, stream, out : as for
 *                       sim_check_traces_device
 *   d_side            : offsets[n_traces] side words, device memory of the
 *                       context's GPU, caller-owned, one per record in the
 *                       records' order
 * Errors and ownership as for sim_check_traces_device.  The statement ids
 * widen the sort key by 1 + log2 of the largest id bits.                  */
int sim_check_traces_warp_device(sim_ctx* ctx, const sim_record* d_records, const uint32_t* d_side,
                                 const uint64_t* offsets, uint32_t n_traces, const uint32_t* threads_per_block,
                                 void* stream, sim_result** out);

/* The same for records and side words in host memory (copied to the
 * device first). */
int sim_check_traces_warp(sim_ctx* ctx, const sim_record* records, const uint32_t* side, const uint64_t* offsets,
                          uint32_t n_traces, const uint32_t* threads_per_block, sim_result** out);

/* ------------------------------------------------------ redundant barriers */

/* One barrier boundary of one trace (24 bytes): the barrier a block passes
 * between its epoch `boundary` and epoch `boundary + 1` (paper Sec. 4.2.3
 * and the second loop of Alg. 5).  An instance is a location (a global
 * unit, or a unit of the block's shared memory) on which one block has
 * records in both of those epochs: a visit-order change the barrier causes.
 * The instance is racing when some pair of the block's records across the
 * barrier would race once the barrier were removed (different threads, at
 * least one write, not both atomic; the warp clauses are not applied).
 * Records of different blocks are never separated by a barrier.  The
 * barrier is redundant when none of its instances is racing: no race is
 * detected by removing it.  A barrier that several boundaries share (one
 * barrier statement in a loop) is redundant when all of them are; blocks
 * are taken to pass the same barrier statements in the same order.       */
typedef struct sim_barrier {
  uint32_t trace;     /* index of the trace in the call */
  uint32_t boundary;  /* epochs boundary and boundary + 1 */
  uint64_t instances; /* locations a block touches on both sides */
  uint64_t racing;    /* instances that would race without the barrier */
} sim_barrier;

typedef struct sim_barrier_result {
  sim_barrier* barriers; /* n_barriers entries, host memory: every (trace, boundary) with an instance,
                            ordered by trace, then boundary */
  uint64_t n_barriers;
} sim_barrier_result;

/* The race check of sim_check_traces_device and, over the same sorted keys,
 * the redundant-barrier check: *races as sim_check_traces_device gives it,
 * *barriers every (trace, boundary) that has an instance.  barriers may be
 * NULL (then only races).  Arguments, ownership and errors as for
 * sim_check_traces_device; on error both outputs are NULL.                */
int sim_check_sync_device(sim_ctx* ctx, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                          const uint32_t* threads_per_block, void* stream, sim_result** races,
                          sim_barrier_result** barriers);

/* The same for records in host memory (copied to the device first). */
int sim_check_sync(sim_ctx* ctx, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
                   const uint32_t* threads_per_block, sim_result** races, sim_barrier_result** barriers);

/* Free a barrier result.  NULL is ignored. */
void sim_barrier_result_free(sim_barrier_result* r);

/* ------------------------------------------------------------- EP fitness */

/* Fitness of one candidate input of the Evolutionary Programming search
 * (paper Sec. 4.1.1, Eq. 1), from its trace (48 bytes).  For every address
 * i the trace touches, g(i) = 1 and f(i) is the number of threads that
 * touch it; the primary fitness is F = sum g / sum f (1 when no address is
 * shared between threads, smaller the more threads share addresses), the
 * secondary score the access range R = end - start.  Addresses are the
 * locations of the race check (a global unit, or a unit of one block's
 * shared memory); threads are grid-wide ids; the range is taken per memory
 * space.                                                                   */
typedef struct sim_fitness {
  uint64_t n_records;
  uint64_t n_locations;        /* sum g: locations touched */
  uint64_t n_location_threads; /* sum f: distinct (location, thread) pairs */
  uint64_t global_range;       /* largest minus smallest global unit (0 without global records) */
  uint64_t shared_range;       /* the same over shared units */
  double fitness;              /* F = n_locations / n_location_threads (1.0 for an empty trace) */
} sim_fitness;

/* EP fitness of every trace of a call (one candidate per trace, e.g. a
 * population of them in one call).  Arguments as for
 * sim_check_traces_device; out: n_traces rows, host memory, caller-owned
 * (row i for trace i).  The records are sorted by (location, thread) on the
 * device -- the race check's sort with epoch and action left out of the
 * key -- and the rows are counted from the runs.  Errors as for
 * sim_check_traces_device; on error out is left unspecified.              */
int sim_eval_fitness_device(sim_ctx* ctx, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                            const uint32_t* threads_per_block, void* stream, sim_fitness* out);

/* The same for records in host memory (copied to the device first). */
int sim_eval_fitness(sim_ctx* ctx, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
                     const uint32_t* threads_per_block, sim_fitness* out);

/* ----------------------------------------------------- barrier divergence */

/* One block whose threads arrived at different numbers of barriers before
 * they finished (24 bytes).  Paper Sec. 4.2.2 and Alg. 4: a thread that
 * reaches the end of the kernel while another thread of its block is
 * halted at a barrier is a barrier divergence -- the halted thread waits at
 * a barrier the finished one never reaches.  Given every thread's number of
 * barrier arrivals at its end, a block diverges exactly when those numbers
 * are not all equal.                                                       */
typedef struct sim_divergence {
  uint32_t trace;         /* index of the trace in the call */
  uint32_t block;         /* block within the trace */
  uint32_t min_barriers;  /* fewest arrivals of a thread of the block */
  uint32_t max_barriers;  /* most arrivals */
  uint64_t early_threads; /* threads of the block with fewer than max_barriers arrivals */
} sim_divergence;

typedef struct sim_divergence_result {
  sim_divergence* blocks; /* n_blocks entries, host memory, ordered by trace, then block */
  uint64_t n_blocks;
} sim_divergence_result;

/* Barrier-divergence check of n_traces traces (Alg. 4).
 *   d_arrivals        : offsets[n_traces] counts, device memory of the
 *                       context's GPU, caller-owned: count i is the number
 *                       of barriers thread i of the call arrived at before
 *                       it finished.  Trace t's threads are d_arrivals[
 *                       offsets[t] .. offsets[t+1]), block by block: thread
 *                       k of the trace is in block k / threads_per_block[t]
 *   offsets           : n_traces + 1 CSR offsets over threads, host memory;
 *                       every trace holds whole blocks (SIM_EINVAL otherwise)
 *   threads_per_block : n_traces values >= 1, host memory
 *   stream            : hipStream_t (NULL: the default stream); the call
 *                       returns after the stream has finished its work
 *   out               : receives one entry per divergent block (caller frees
 *                       it with sim_divergence_result_free)
 * A call holds at most 2^32 - 1 threads.  Errors and ownership as for
 * sim_check_traces_device.                                                 */
int sim_check_divergence_device(sim_ctx* ctx, const uint32_t* d_arrivals, const uint64_t* offsets,
                                uint32_t n_traces, const uint32_t* threads_per_block, void* stream,
                                sim_divergence_result** out);

/* The same for arrival counts in host memory (copied to the device first). */
int sim_check_divergence(sim_ctx* ctx, const uint32_t* arrivals, const uint64_t* offsets, uint32_t n_traces,
                         const uint32_t* threads_per_block, sim_divergence_result** out);

/* Free a divergence result.  NULL is ignored. */
void sim_divergence_result_free(sim_divergence_result* r);

/* -------------------------------------------------------------- profiling */

/* Per-stage device time of the last call on a context created with
 * SIM_CFG_PROFILE, measured with HIP events on the stream the kernels ran
 * on.  Stages are listed by sim_stage_name(); launches counts the kernel
 * launches that did work in each stage.  Returns the number of stages
 * written (at most cap).                                                   */
typedef struct sim_stage_time {
  double ms;
  uint32_t launches;
  uint32_t reserved;
} sim_stage_time;

int sim_stage_times(const sim_ctx* ctx, sim_stage_time* out, int cap);
const char* sim_stage_name(int stage);

/* ----------------------------------------------------------------- tuning */

/* Launch shape of the tile kernels (tiles are 4096 records of one trace).
 * Shapes change speed only: every shape gives the same result.  A context
 * keeps one shape per size class; class k covers calls of 2^(k-1) ..
 * 2^k - 1 records in total (k = 0 .. 32, see sim_size_class).  A call uses
 * its class's shape, else that of the nearest class that has one, else the
 * default (all fields 0).                                                  */
typedef struct sim_tuning {
  uint32_t stream_wgs_per_cu; /* statistics, key and histogram kernels: workgroups per CU, each looping
                                 over tiles (0: one workgroup per tile); at most 64 */
  uint32_t sort_wgs_per_cu;   /* radix scatter kernel, same meaning */
  uint32_t scan_wgs_per_cu;   /* tile-scan kernel, same meaning */
  int32_t group_shift_bias;   /* added to log2 of the tiles per histogram group (by default about the
                                 square root of a trace's tiles); the result is clamped to 0 .. 12 */
  uint32_t scatter_threads;   /* threads of a radix scatter workgroup: 256 (16 keys each) or 512 (8 keys
                                 each; one-word keys only, two-word calls use 256); 0: by call size,
                                 512 up to 16384 tiles, else 256 */
  uint32_t digit_bits;        /* radix digit width of the passes after the first: 8 or 9; 0: by the
                                 key width of the context's previous call of the same kind (9 where
                                 it saves a pass; no-allocation calls always use 8) */
  double ms;                  /* sim_autotune: fastest time of one call in the chosen shape; else 0 */
} sim_tuning;

#define SIM_SIZE_CLASSES 33

/* Size class of a call of `total_records` records: its bit length (capped at 32). */
uint32_t sim_size_class(uint64_t total_records);

/* Set the shape of one size class (t = NULL: back to the default).
 * SIM_EINVAL for a class >= SIM_SIZE_CLASSES or fields out of range.      */
int sim_set_tuning(sim_ctx* ctx, uint32_t size_class, const sim_tuning* t);

/* Shape of one size class; returns 1 if the class has one (set or tuned),
 * 0 if it uses the default (then *t is all zero), SIM_EINVAL on bad
 * arguments.                                                               */
int sim_get_tuning(const sim_ctx* ctx, uint32_t size_class, sim_tuning* t);

/* Autotuner: time complete calls on the given input (arguments as for
 * sim_check_traces_device) under candidate shapes -- coordinate descent over
 * the workgroups per CU of the scatter (0, 1, 2, 4, 8), of the tile scan,
 * of the streaming kernels, then the histogram-group bias (-2 .. +2), then
 * the scatter's other thread count (256 or 512).  Each candidate runs
 * `reps` calls (0: 3; at least 5 when a call takes under 10 ms) taking turns
 * with as many calls of the current shape, so that a drift of the GPU's
 * speed during tuning reaches both; it replaces the current shape only when
 * its fastest call is at least 0.5 % faster than the current shape's.  The
 * chosen shape is stored for the input's size class and written to *best.
 * Results of the trial calls are discarded; on error the class keeps its
 * old shape.                                                               */
int sim_autotune(sim_ctx* ctx, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                 const uint32_t* threads_per_block, void* stream, uint32_t reps, sim_tuning* best);

/* ---------------------------------------------------------------- serving */

/* A server checks requests (each one call's worth of traces: records,
 * offsets, threads per block, as for sim_check_traces) that arrive over
 * time, with continuous batching: `slots` worker threads each own a context
 * (its own stream and device buffers); a free worker takes the pending
 * requests in arrival order, as many as fit its batch limits and the HBM
 * budget, checks them as ONE call (one trace list, so small requests share
 * every launch), and hands each request its own part of the result.
 * Requests that arrive while batches run wait for the next free worker;
 * batches of different workers overlap on the GPU.  A request's result is
 * the result sim_check_traces gives for it alone (trace numbers relative
 * to the request), including its error code: when a batch fails, its
 * requests are checked one by one so that one bad request fails alone.
 *
 * Admission by device-memory footprint.  A request's footprint is what its
 * check may hold on the device: its records when they come from host
 * memory (16 bytes each), two key buffers of 16 bytes per record (two-word
 * keys are possible until the device has seen the request), about 8.3 KiB
 * per 4096-record tile (tables for 9-bit radix digits) and 136 bytes per
 * trace of tables, and the output's first allocation (up to 64 Ki entries
 * of 64 bytes), each with 1/8 growth headroom.  Every worker is charged the device bytes it may hold: an idle
 * worker what it holds, a worker checking a batch the larger of that and
 * the batch's footprint, and its buffers never grow past its charge (a
 * worker whose buffers would grow past it releases them and allocates the
 * batch's sizes afresh).  A batch is admitted only while the charges of all
 * workers stay within the budget; when the first pending request fits no
 * worker, idle workers release their buffers.  A request whose output
 * outgrows the usual estimate (more than 64 Ki racing locations, or a tile
 * staging overflow) fails within its charge and is queued again, alone,
 * charged its worst case (an entry for every second record, in the output
 * and in staging).  A request whose footprint, or worst case when it comes
 * to that, exceeds the budget fails with SIM_ENOMEM.
 *
 * All server calls are thread-safe.                                        */
typedef struct sim_server sim_server;

typedef struct sim_server_config {
  uint64_t hbm_budget_bytes;   /* footprint of the batches on the GPU at most (0: 8 GiB) */
  uint64_t max_batch_records;  /* records per batch at most (0: 2^26; a larger request runs alone) */
  uint32_t slots;              /* worker threads = batches on the GPU at once (0: 2; at most 16) */
  uint32_t max_batch_requests; /* requests per batch at most (0: 1024) */
  uint32_t max_pending;        /* submitted requests not yet taken by a worker at most (0: 65536) */
  uint32_t reserved;
  uint64_t reserve_records;    /* each worker allocates its device buffers (records included) for a batch of
                                  this many records (in up to max_batch_requests traces) at creation, so
                                  that batches up to that size allocate nothing (0: grow on demand).  Its
                                  footprint must fit budget / slots (else SIM_EINVAL). */
} sim_server_config;

typedef struct sim_server_stats {
  uint64_t submitted, completed, failed; /* requests */
  uint64_t batches;                      /* batches run */
  uint64_t records;                      /* records of completed requests */
  double p50_ms, p99_ms, max_ms, mean_ms; /* latency of completed requests, submission to result ready */
  double records_per_s;                  /* records of completed requests / (last completion - first submission) */
  double mean_batch_requests;            /* completed requests per batch */
  uint64_t peak_inflight_bytes;          /* largest sum of the workers' charges (at most the budget) */
  uint64_t device_bytes;                 /* device buffers the workers hold now */
  uint64_t requeued;                     /* requests queued again, charged their worst case */
} sim_server_stats;

/* Create a server on HIP device `hip_device` (gfx950).  cfg may be NULL.  */
int sim_server_create(sim_server** out, int hip_device, const sim_server_config* cfg);

/* Finish every submitted request, stop the workers, free all results not
 * yet collected and the server.  NULL is ignored.                          */
void sim_server_destroy(sim_server* srv);

/* Submit one request (arguments as for sim_check_traces; host memory).
 * offsets and threads_per_block are copied; the records are read by a
 * worker later and must stay valid and unchanged until the request's
 * result has been collected (sim_poll / sim_wait returned something other
 * than SIM_EAGAIN).  *ticket identifies the request.  Errors: SIM_EINVAL
 * (bad tables), SIM_ENOMEM (footprint above the budget), SIM_EAGAIN
 * (max_pending requests wait already).                                     */
int sim_submit(sim_server* srv, const sim_record* records, const uint64_t* offsets, uint32_t n_traces,
               const uint32_t* threads_per_block, uint64_t* ticket);

/* Submit one request whose records already live in device memory of the
 * server's GPU (e.g. a torch tensor's storage): the workers read them where
 * they are, with no copy, so a batch of such requests moves no record over
 * PCIe.  d_records: offsets[n_traces] records, device memory, caller-owned;
 * it must stay valid and unchanged until the request's result has been
 * collected.  offsets and threads_per_block are host arrays, copied as for
 * sim_submit; errors as for sim_submit.  The footprint does not count the
 * records.                                                                 */
int sim_submit_device(sim_server* srv, const sim_record* d_records, const uint64_t* offsets, uint32_t n_traces,
                      const uint32_t* threads_per_block, uint64_t* ticket);

/* Collect a request's result: SIM_EAGAIN while it is pending; otherwise the
 * request's own return code, with *out set on success (caller frees it with
 * sim_result_free).  The ticket is consumed unless SIM_EAGAIN is returned;
 * an unknown ticket gives SIM_EINVAL.                                      */
int sim_poll(sim_server* srv, uint64_t ticket, sim_result** out);

/* As sim_poll, but blocks until the result is ready or timeout_ms passes
 * (negative: no limit; SIM_EAGAIN on timeout).                             */
int sim_wait(sim_server* srv, uint64_t ticket, int64_t timeout_ms, sim_result** out);

/* Counters and latency percentiles since creation or the last reset.      */
int sim_server_get_stats(sim_server* srv, sim_server_stats* out, int reset);

/* Text of the error of the last sim_submit / sim_poll / sim_wait that
 * failed on the calling thread ("" if none).                              */
const char* sim_server_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIMCHECK_H */
