"""CPU oracle for the Memory-Model data-race check.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH: only the tests, the smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code with
the GPU path and never imports it.

Two native tiers live in ``oracle.c`` (built into ``liboracle.so``):
  * ``brute_force`` -- Tier A, the pairwise race definition of Theorem 1
    (Sec. 4.2.3) applied to every pair, O(n^2);
  * ``closed_form`` -- Tier B, group counts by location / block / epoch /
    thread and inclusion-exclusion over them;
  * ``closed_form_par`` -- Tier B's same counting spread over OpenMP
    threads (by trace, and by location-hash bucket within a large trace).
``tier_a_py`` is a third, pure-Python rendering of the pairwise definition
for tiny inputs, written separately so that the C tiers can be checked
against it.  ``brute_force_warp``, ``closed_form_warp`` and
``tier_a_warp_py`` are the same three renderings of the warp-aware check
(Theorem 1 with its warp clauses), over records plus one side word each
(statement id, divergence bit).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RACE_DTYPE = np.dtype(
    [
        ("trace", "<u4"),
        ("space", "u1"),
        ("kinds", "u1"),
        ("reserved16", "<u2"),
        ("block", "<u4"),
        ("reserved32", "<u4"),
        ("unit", "<u8"),
        ("pairs_ww", "<u8"),
        ("pairs_rw", "<u8"),
        ("pairs_aw", "<u8"),
        ("pairs_ar", "<u8"),
        ("pairs_xblock", "<u8"),
    ]
)
assert RACE_DTYPE.itemsize == 64

SUMMARY_DTYPE = np.dtype([("n_records", "<u8"), ("n_race_locs", "<u8"), ("n_pairs", "<u8")])

KIND_BITS = {"ww": 1, "rw": 2, "aw": 4, "ar": 8, "xblock": 16}

BARRIER_DTYPE = np.dtype([("trace", "<u4"), ("boundary", "<u4"), ("instances", "<u8"), ("racing", "<u8")])
FITNESS_DTYPE = np.dtype([("n_records", "<u8"), ("n_locations", "<u8"), ("n_location_threads", "<u8"),
                          ("global_range", "<u8"), ("shared_range", "<u8"), ("fitness", "<f8")])
DIVERGENCE_DTYPE = np.dtype([("trace", "<u4"), ("block", "<u4"), ("min_barriers", "<u4"), ("max_barriers", "<u4"),
                             ("early_threads", "<u8")])


class OracleError(Exception):
    def __init__(self, code, bad_index=None):
        super().__init__(f"oracle rejected input (code {code}, bad index {bad_index})")
        self.code = code
        self.bad_index = bad_index


def build() -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        for name in ("orc_brute_force", "orc_closed_form"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int64
            f.argtypes = [
                ctypes.c_void_p,
                ctypes.c_void_p,
                ctypes.c_uint32,
                ctypes.c_void_p,
                ctypes.POINTER(ctypes.c_void_p),
                ctypes.c_void_p,
                ctypes.POINTER(ctypes.c_uint64),
            ]
        f = lib.orc_closed_form_par
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                      ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                      ctypes.c_int, ctypes.c_uint64]
        for name in ("orc_barriers_brute_force", "orc_barriers"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                          ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint64)]
        for name in ("orc_brute_force_warp", "orc_closed_form_warp"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                          ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
        f = lib.orc_fitness_eval
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.POINTER(ctypes.c_uint64)]
        f = lib.orc_divergence_check
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                      ctypes.POINTER(ctypes.c_void_p)]
        lib.orc_free.restype = None
        lib.orc_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _as_batch(records, offsets=None, tpb=None):
    records = np.ascontiguousarray(records)
    if offsets is None:
        offsets = np.array([0, len(records)], dtype=np.uint64)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    n_traces = len(offsets) - 1
    if tpb is None:
        raise ValueError("threads-per-block is required")
    tpb = np.asarray(tpb, dtype=np.uint32)
    if tpb.ndim == 0:
        tpb = np.full(n_traces, int(tpb), dtype=np.uint32)
    tpb = np.ascontiguousarray(tpb)
    return records, offsets, n_traces, tpb


def _run(fname, records, offsets, tpb, *extra):
    records, offsets, n_traces, tpb = _as_batch(records, offsets, tpb)
    lib = _load()
    out = ctypes.c_void_p()
    summ = np.zeros(max(n_traces, 1), dtype=SUMMARY_DTYPE)
    bad = ctypes.c_uint64(0)
    n = getattr(lib, fname)(
        records.ctypes.data if len(records) else None,
        offsets.ctypes.data,
        n_traces,
        tpb.ctypes.data,
        ctypes.byref(out),
        summ.ctypes.data,
        ctypes.byref(bad),
        *extra,
    )
    if n < 0:
        raise OracleError(int(n), int(bad.value) if n == -2 else None)
    races = np.zeros(n, dtype=RACE_DTYPE)
    if n:
        ctypes.memmove(races.ctypes.data, out.value, n * RACE_DTYPE.itemsize)
    if out.value:
        lib.orc_free(out)
    return races, summ[:n_traces]


def brute_force(records, offsets=None, tpb=None):
    """Tier A: every pair tested against the race definition."""
    return _run("orc_brute_force", records, offsets, tpb)


def closed_form(records, offsets=None, tpb=None):
    """Tier B: inclusion-exclusion over location/block/epoch/thread groups."""
    return _run("orc_closed_form", records, offsets, tpb)


def closed_form_par(records, offsets=None, tpb=None, threads=0, bucket_min=1 << 22):
    """Tier B's counting spread over OpenMP threads (0: every core): traces of
    at most bucket_min records are independent units, a larger trace is split
    into location-hash buckets counted separately.  Same result as
    closed_form."""
    return _run("orc_closed_form_par", records, offsets, tpb, int(threads), int(bucket_min))


SD_DIVERGED = 1 << 31  # side-word bit: the access ran while its warp was diverged


def _run_warp(fname, records, side, offsets, tpb):
    records, offsets, n_traces, tpb = _as_batch(records, offsets, tpb)
    side = np.ascontiguousarray(np.asarray(side, dtype=np.uint32))
    if len(side) != len(records):
        raise ValueError("one side word per record")
    lib = _load()
    out = ctypes.c_void_p()
    summ = np.zeros(max(n_traces, 1), dtype=SUMMARY_DTYPE)
    bad = ctypes.c_uint64(0)
    n = getattr(lib, fname)(records.ctypes.data if len(records) else None, side.ctypes.data if len(side) else None,
                            offsets.ctypes.data, n_traces, tpb.ctypes.data, ctypes.byref(out), summ.ctypes.data,
                            ctypes.byref(bad))
    if n < 0:
        raise OracleError(int(n), int(bad.value) if n == -2 else None)
    races = np.zeros(n, dtype=RACE_DTYPE)
    if n:
        ctypes.memmove(races.ctypes.data, out.value, n * RACE_DTYPE.itemsize)
    if out.value:
        lib.orc_free(out)
    return races, summ[:n_traces]


def brute_force_warp(records, side, offsets=None, tpb=None):
    """Warp-aware Tier A (Theorem 1 with clauses 1-3): every pair tested;
    a same-warp pair races only when either record carries SD_DIVERGED or
    both write by the same statement (side & ~SD_DIVERGED)."""
    return _run_warp("orc_brute_force_warp", records, side, offsets, tpb)


def closed_form_warp(records, side, offsets=None, tpb=None):
    """Warp-aware Tier B: the plain group counts minus, per warp group, the
    pairs that lockstep execution orders."""
    return _run_warp("orc_closed_form_warp", records, side, offsets, tpb)


def omp_threads():
    """Threads the parallel tier uses by default (OpenMP's maximum)."""
    import ctypes.util

    gomp = ctypes.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
    gomp.omp_get_max_threads.restype = ctypes.c_int
    return int(gomp.omp_get_max_threads())


def _run_barriers(fname, records, offsets, tpb):
    records, offsets, n_traces, tpb = _as_batch(records, offsets, tpb)
    lib = _load()
    out = ctypes.c_void_p()
    bad = ctypes.c_uint64(0)
    n = getattr(lib, fname)(records.ctypes.data if len(records) else None, offsets.ctypes.data, n_traces,
                            tpb.ctypes.data, ctypes.byref(out), ctypes.byref(bad))
    if n < 0:
        raise OracleError(int(n), int(bad.value) if n == -2 else None)
    res = np.zeros(n, dtype=BARRIER_DTYPE)
    if n:
        ctypes.memmove(res.ctypes.data, out.value, n * BARRIER_DTYPE.itemsize)
    if out.value:
        lib.orc_free(out)
    return res


def barriers_brute_force(records, offsets=None, tpb=None):
    """Barrier instances (Alg. 5, second loop), Tier A: every pair of
    records tested.  One entry per (trace, boundary) with an instance:
    instances, racing instances (the barrier is redundant when 0)."""
    return _run_barriers("orc_barriers_brute_force", records, offsets, tpb)


def barriers(records, offsets=None, tpb=None):
    """Barrier instances, Tier B: adjacent epoch groups of every location
    and block, compared pair by pair."""
    return _run_barriers("orc_barriers", records, offsets, tpb)


def barriers_py(records, tpb):
    """Pure-Python rendering for one tiny trace: {boundary: (instances,
    racing)}.  An instance is a (location, block) with records of that block
    in epochs b and b+1; it races when a pair across the two epochs has
    different threads and at least one write, not both atomic."""
    recs = [tuple(int(v) for v in r) for r in records]  # unit, tid, epoch, action, space
    groups = {}
    for u, t, e, a, s in recs:
        b = t // tpb
        loc = (s, b if s == 1 else None, u)
        groups.setdefault((loc, b), {}).setdefault(e, []).append((t, a))
    out = {}
    for (_, _), by_epoch in groups.items():
        for e, xs in by_epoch.items():
            ys = by_epoch.get(e + 1)
            if ys is None:
                continue
            racing = any(tx != ty and not (ax == 0 and ay == 0) and not (ax == 2 and ay == 2)
                         for tx, ax in xs for ty, ay in ys)
            inst, rac = out.get(e, (0, 0))
            out[e] = (inst + 1, rac + (1 if racing else 0))
    return out


def barriers_to_dict(res, trace=0):
    """{boundary: (instances, racing)} of one trace from a BARRIER_DTYPE array."""
    return {int(r["boundary"]): (int(r["instances"]), int(r["racing"])) for r in res if int(r["trace"]) == trace}


def fitness(records, offsets=None, tpb=None):
    """EP fitness of every trace (Eq. 1): FITNESS_DTYPE rows with the
    locations (sum g), distinct (location, thread) pairs (sum f), the global
    and shared unit ranges (R) and F = sum g / sum f."""
    records, offsets, n_traces, tpb = _as_batch(records, offsets, tpb)
    lib = _load()
    out = np.zeros(max(n_traces, 1), dtype=FITNESS_DTYPE)
    bad = ctypes.c_uint64(0)
    rc = lib.orc_fitness_eval(records.ctypes.data if len(records) else None, offsets.ctypes.data, n_traces,
                              tpb.ctypes.data, out.ctypes.data, ctypes.byref(bad))
    if rc < 0:
        raise OracleError(int(rc), int(bad.value) if rc == -2 else None)
    return out[:n_traces]


def divergence(counts, offsets, tpb):
    """Barrier divergence (Alg. 4): counts[i] is the number of barriers
    thread i arrived at before finishing; trace t holds threads
    offsets[t] .. offsets[t+1], block by block (whole blocks).  One
    DIVERGENCE_DTYPE row per block whose threads' counts differ."""
    counts = np.ascontiguousarray(np.asarray(counts, dtype=np.uint32))
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    n_traces = len(offsets) - 1
    tpb = np.asarray(tpb, dtype=np.uint32)
    if tpb.ndim == 0:
        tpb = np.full(n_traces, int(tpb), dtype=np.uint32)
    tpb = np.ascontiguousarray(tpb)
    lib = _load()
    out = ctypes.c_void_p()
    n = lib.orc_divergence_check(counts.ctypes.data if len(counts) else None, offsets.ctypes.data, n_traces,
                                 tpb.ctypes.data, ctypes.byref(out))
    if n < 0:
        raise OracleError(int(n))
    res = np.zeros(n, dtype=DIVERGENCE_DTYPE)
    if n:
        ctypes.memmove(res.ctypes.data, out.value, n * DIVERGENCE_DTYPE.itemsize)
    if out.value:
        lib.orc_free(out)
    return res


# ---------------------------------------------------------------------------
# Pure-Python Tier A for tiny traces (independent rendering of Theorem 1).
# ---------------------------------------------------------------------------

def tier_a_py(records, tpb, trace=0):
    """Return {(space, block_or_None, unit): {'ww','rw','aw','ar','xblock'}}
    for one trace, by testing every unordered pair of record positions."""
    recs = [tuple(int(v) for v in r) for r in records]  # unit, tid, epoch, action, space
    out = {}
    names = {frozenset(["W"]): "ww", frozenset(["R", "W"]): "rw",
             frozenset(["A", "W"]): "aw", frozenset(["A", "R"]): "ar"}
    letter = {0: "R", 1: "W", 2: "A"}
    for i in range(len(recs)):
        for j in range(i + 1, len(recs)):
            u1, t1, e1, a1, s1 = recs[i]
            u2, t2, e2, a2, s2 = recs[j]
            b1, b2 = t1 // tpb, t2 // tpb
            if s1 != s2 or u1 != u2:
                continue
            if s1 == 1 and b1 != b2:  # shared memory belongs to one block
                continue
            if t1 == t2:
                continue
            acts = frozenset([letter[a1], letter[a2]])
            if acts in (frozenset(["R"]), frozenset(["A"])):
                continue
            if b1 == b2 and e1 != e2:  # a barrier of the block separates them
                continue
            key = (s1, b1 if s1 == 1 else None, u1)
            d = out.setdefault(key, {"ww": 0, "rw": 0, "aw": 0, "ar": 0, "xblock": 0})
            d[names[acts]] += 1
            if b1 != b2:
                d["xblock"] += 1
    return out


def tier_a_warp_py(records, side, tpb, trace=0):
    """Pure-Python warp-aware rendering for one tiny trace, in the form of
    tier_a_py.  Threads of one warp: same block, same block-local id // 32.
    Such a pair is ordered by lockstep execution, and so does not race,
    unless one of its accesses ran diverged or both are writes by one
    statement."""
    recs = [tuple(int(v) for v in r) for r in records]  # unit, tid, epoch, action, space
    side = [int(v) for v in side]
    out = {}
    names = {frozenset(["W"]): "ww", frozenset(["R", "W"]): "rw",
             frozenset(["A", "W"]): "aw", frozenset(["A", "R"]): "ar"}
    letter = {0: "R", 1: "W", 2: "A"}
    for i in range(len(recs)):
        for j in range(i + 1, len(recs)):
            u1, t1, e1, a1, s1 = recs[i]
            u2, t2, e2, a2, s2 = recs[j]
            b1, b2 = t1 // tpb, t2 // tpb
            if s1 != s2 or u1 != u2 or (s1 == 1 and b1 != b2) or t1 == t2:
                continue
            acts = frozenset([letter[a1], letter[a2]])
            if acts in (frozenset(["R"]), frozenset(["A"])):
                continue
            if b1 == b2 and e1 != e2:
                continue
            if b1 == b2 and (t1 % tpb) // 32 == (t2 % tpb) // 32:
                diverged = bool((side[i] | side[j]) & SD_DIVERGED)
                one_stmt_writes = a1 == 1 and a2 == 1 and (side[i] & ~SD_DIVERGED) == (side[j] & ~SD_DIVERGED)
                if not diverged and not one_stmt_writes:
                    continue
            key = (s1, b1 if s1 == 1 else None, u1)
            d = out.setdefault(key, {"ww": 0, "rw": 0, "aw": 0, "ar": 0, "xblock": 0})
            d[names[acts]] += 1
            if b1 != b2:
                d["xblock"] += 1
    return out


def races_to_dict(races, trace=0, kinds=False):
    """Convert a RACE_DTYPE array (one trace) to the tier_a_py form; with
    kinds=True each entry also carries its kinds bits."""
    out = {}
    for r in races:
        if int(r["trace"]) != trace:
            continue
        key = (int(r["space"]), int(r["block"]) if int(r["space"]) == 1 else None, int(r["unit"]))
        out[key] = {
            "ww": int(r["pairs_ww"]),
            "rw": int(r["pairs_rw"]),
            "aw": int(r["pairs_aw"]),
            "ar": int(r["pairs_ar"]),
            "xblock": int(r["pairs_xblock"]),
        }
        if kinds:
            out[key]["kinds"] = int(r["kinds"])
    return out
