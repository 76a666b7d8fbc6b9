"""Seeded synthetic Memory-Model traces (input generation only).

Records follow the paper's Unit Tuple <visit order, thread id, action> of the
Memory Model (Sec. 4.2.1), extended with the accessed unit and memory space
(global memory is one array for all blocks, shared memory is per block,
Alg. 3).  This module holds none of the race-check arithmetic; the oracle
and the GPU path both consume what it produces.

The native part lives in ``tracegen.c`` and is built into ``libtracegen.so``
next to it (``build()``).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tracegen.c")
_LIB = os.path.join(_HERE, "libtracegen.so")

RECORD_DTYPE = np.dtype(
    [("unit", "<u8"), ("tid", "<u4"), ("epoch", "<u2"), ("action", "u1"), ("space", "u1")]
)
assert RECORD_DTYPE.itemsize == 16

INJ_DTYPE = np.dtype(
    [
        ("space", "u1"),
        ("action_x", "u1"),
        ("action_y", "u1"),
        ("cross_block", "u1"),
        ("block", "<u4"),
        ("unit", "<u8"),
        ("x_index", "<u8"),
        ("y_index", "<u8"),
    ]
)
assert INJ_DTYPE.itemsize == 32

READ, WRITE, ATOMIC = 0, 1, 2
GLOBAL, SHARED = 0, 1


class _Params(ctypes.Structure):
    _fields_ = [
        ("n_blocks", ctypes.c_uint32),
        ("tpb", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("per_epoch", ctypes.c_uint32),
        ("p_read", ctypes.c_double),
        ("p_write", ctypes.c_double),
        ("p_shared", ctypes.c_double),
        ("shared_words", ctypes.c_uint32),
        ("global_read_log2", ctypes.c_uint32),
        ("atomic_bins_log2", ctypes.c_uint32),
        ("zipf_s", ctypes.c_double),
        ("n_records", ctypes.c_uint64),
        ("inject_rate", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("trace_id", ctypes.c_uint32),
    ]


def build() -> str:
    """Compile libtracegen.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.tg_generate.restype = ctypes.c_int64
        lib.tg_generate.argtypes = [
            ctypes.POINTER(_Params),
            ctypes.c_void_p,
            ctypes.c_void_p,
            ctypes.c_uint64,
            ctypes.c_int,
        ]
        lib.tg_generate_batch.restype = ctypes.c_int64
        lib.tg_generate_batch.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.tg_tree_reduction.restype = ctypes.c_int64
        lib.tg_tree_reduction.argtypes = [ctypes.c_int, ctypes.c_void_p]
        lib.tg_splitmix64.restype = ctypes.c_uint64
        lib.tg_splitmix64.argtypes = [ctypes.c_uint64]
        lib.tg_philox4x32_10.restype = None
        lib.tg_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32, ctypes.c_uint32]
        lib.tg_zipf_rank.restype = ctypes.c_uint64
        lib.tg_zipf_rank.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        _lib = lib
    return _lib


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter under a 2-word key (for tests)."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    lib.tg_philox4x32_10(c, int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF)
    return [int(x) for x in c]


def splitmix64(x: int) -> int:
    return int(_load().tg_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def zipf_rank(n: int, s: float, seed: int, a: int, b: int) -> int:
    return int(_load().tg_zipf_rank(n, s, seed, a, b))


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _n_injections(rate: float, n: int) -> int:
    """Injections the C generator makes for a trace of n records: rate * n
    rounded half away from zero (llround), not Python's half-to-even."""
    return int(math.floor(rate * n + 0.5)) if rate > 0 else 0


def generate(
    n_blocks: int,
    tpb: int,
    k: int,
    *,
    per_epoch: int = 16,
    p_read: float = 0.75,
    p_write: float = 0.25,
    p_shared: float = 0.5,
    shared_words: int = 12288,
    global_read_log2: int = 24,
    atomic_bins_log2: int = 16,
    zipf_s: float = 1.1,
    n_records: int | None = None,
    inject_rate: float = 0.0,
    seed: int = 1,
    trace_id: int = 0,
    out: np.ndarray | None = None,
    threads: int | None = None,
):
    """Generate one trace; returns (records, injections)."""
    full = n_blocks * tpb * k
    n = full if n_records is None else int(n_records)
    if n > full:
        raise ValueError("n_records exceeds n_blocks * tpb * k")
    p = _Params(
        n_blocks, tpb, k, per_epoch, p_read, p_write, p_shared, shared_words,
        global_read_log2, atomic_bins_log2, zipf_s, n, inject_rate,
        int(seed) & 0xFFFFFFFFFFFFFFFF, trace_id,
    )
    if out is None:
        recs = np.zeros(n, dtype=RECORD_DTYPE)
    else:
        recs = out
        assert recs.dtype == RECORD_DTYPE and recs.shape == (n,) and recs.flags.c_contiguous
    m = _n_injections(inject_rate, n)
    log = np.zeros(max(m, 1), dtype=INJ_DTYPE)
    got = _load().tg_generate(
        ctypes.byref(p), recs.ctypes.data, log.ctypes.data, m, threads or _threads()
    )
    if got < 0:
        raise ValueError("tg_generate rejected its parameters")
    return recs, log[: int(got)]


def tree_reduction(removed: int = -1) -> np.ndarray:
    """Shared-memory tree reduction, 1 block x 256 threads, optionally with
    one barrier (0..8) left out.  1279 records."""
    recs = np.zeros(1279, dtype=RECORD_DTYPE)
    n = _load().tg_tree_reduction(int(removed), recs.ctypes.data)
    assert n == 1279
    return recs


# --------------------------------------------------------------------------
# Workloads.  Shapes follow the configurations of the synthetic benchmark
# suite that stands in for the paper's (unavailable) subject-kernel traces.
# --------------------------------------------------------------------------

def c0() -> np.ndarray:
    """Tree reduction with the barrier before level 3 (B2) removed."""
    return tree_reduction(2)


def c1(n_blocks: int = 1024, inject_rate: float = 1e-4, seed: int = 0x5EED0001, **kw):
    """1024 blocks x 256 threads x 64 accesses = 2^24 records; 75% reads;
    shared window 48 KiB per block; global reads Zipf(1.1) over 64 MiB."""
    return generate(
        n_blocks, 256, 64, per_epoch=16, p_read=0.75, p_write=0.25, p_shared=0.5,
        shared_words=12288, global_read_log2=24, atomic_bins_log2=16, zipf_s=1.1,
        inject_rate=inject_rate, seed=seed, **kw,
    )


def c2(n_blocks: int = 8192, inject_rate: float = 1e-5, seed: int = 0x5EED0002, **kw):
    """8192 blocks x 512 threads x 64 accesses = 2^28 records; 5% atomics;
    global reads Zipf(1.1) over 1 GiB."""
    return generate(
        n_blocks, 512, 64, per_epoch=16, p_read=0.75, p_write=0.20, p_shared=0.5,
        shared_words=12288, global_read_log2=28, atomic_bins_log2=16, zipf_s=1.1,
        inject_rate=inject_rate, seed=seed, **kw,
    )


def c3_shapes(n_traces: int = 4096, seed: int = 0x5EED0003, log2_min: float = 8.0, log2_max: float = 20.0):
    """Per-trace (n_records, n_blocks, k, seed) of the batched workload:
    sizes log-uniform 2^8..2^20, block counts log-uniform 1..256, 256
    threads per block, k = ceil(n / (blocks * 256))."""
    shapes = []
    for i in range(n_traces):
        s = splitmix64(seed ^ i)
        u1 = (splitmix64(s) >> 11) / float(1 << 53)
        u2 = (splitmix64(s ^ 0xA5A5A5A5A5A5A5A5) >> 11) / float(1 << 53)
        n = int(round(2.0 ** (log2_min + (log2_max - log2_min) * u1)))
        nb = int(round(2.0 ** (8.0 * u2)))
        nb = max(1, min(256, nb))
        k = int(math.ceil(n / (nb * 256)))
        shapes.append((n, nb, k, s))
    return shapes


def batch(shapes, inject_rate: float = 1e-4, threads: int | None = None):
    """Generate a batch of traces; returns (records, offsets, tpb, injections)
    with injections a list of (trace index, injection log).  Trace i is the
    same as ``generate`` with shape i (c1 distributions, 256 threads per
    block); traces are generated in parallel."""
    sizes = np.array([s[0] for s in shapes], dtype=np.uint64)
    offsets = np.zeros(len(shapes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    recs = np.zeros(int(offsets[-1]), dtype=RECORD_DTYPE)
    tpb = np.full(len(shapes), 256, dtype=np.uint32)
    params = (_Params * max(1, len(shapes)))()
    caps = np.zeros(len(shapes) + 1, dtype=np.uint64)
    for i, (n, nb, k, s) in enumerate(shapes):
        params[i] = _Params(nb, 256, k, 16, 0.75, 0.25, 0.5, 12288, 24, 16, 1.1, n, inject_rate,
                            int(s) & 0xFFFFFFFFFFFFFFFF, i)
        caps[i + 1] = caps[i] + max(1, _n_injections(inject_rate, n))
    logs = np.zeros(max(1, int(caps[-1])), dtype=INJ_DTYPE)
    counts = np.zeros(max(1, len(shapes)), dtype=np.int64)
    rc = _load().tg_generate_batch(params, len(shapes), recs.ctypes.data, offsets.ctypes.data, logs.ctypes.data,
                                   caps.ctypes.data, counts.ctypes.data, threads or _threads())
    if rc < 0:
        raise ValueError("tg_generate_batch rejected its parameters")
    inj = [(i, logs[int(caps[i]) : int(caps[i]) + min(int(counts[i]), int(caps[i + 1] - caps[i]))])
           for i in range(len(shapes))]
    return recs, offsets, tpb, inj


def random_small(rng: np.random.Generator, n: int, *, units: int = 4, blocks: int = 3, tpb: int = 3,
                 epochs: int = 3, atomics: bool = True):
    """Tiny trace over small domains so that collisions are frequent."""
    r = np.zeros(n, dtype=RECORD_DTYPE)
    r["unit"] = rng.integers(0, units, n)
    r["tid"] = rng.integers(0, blocks * tpb, n)
    r["epoch"] = rng.integers(0, epochs, n)
    r["action"] = rng.integers(0, 3 if atomics else 2, n)
    r["space"] = rng.integers(0, 2, n)
    return r


def arrivals(n_blocks: int, tpb: int, barriers: int, seed: int, diverge_rate: float = 1e-2):
    """Per-thread barrier arrival counts of one synthetic launch, block by
    block (uint32, n_blocks * tpb of them): every thread arrives at
    `barriers` barriers, except in about diverge_rate of the blocks, where a
    random subset of threads returns early after fewer (a thread-dependent
    branch around a barrier, or an early return).  Returns (counts, list of
    the blocks made divergent)."""
    rng = np.random.default_rng(seed)
    counts = np.full(n_blocks * tpb, barriers, dtype=np.uint32)
    if barriers == 0 or n_blocks == 0 or tpb < 2:
        return counts, []
    picked = np.flatnonzero(rng.random(n_blocks) < diverge_rate)
    for b in picked:
        blk = counts[b * tpb:(b + 1) * tpb]
        m = int(rng.integers(1, tpb))  # threads that leave early (at least one stays)
        who = rng.choice(tpb, size=m, replace=False)
        blk[who] = rng.integers(0, barriers, m).astype(np.uint32)
    return counts, [int(b) for b in picked]


def arrivals_batch(shapes, barriers: int = 4, diverge_rate: float = 1e-2, seed: int = 0x5EED0005):
    """Arrival counts of a batch of launches, one per (n_blocks, tpb) shape:
    (counts, CSR offsets over threads, threads per block)."""
    parts, tpbs = [], []
    for i, (nb, tp) in enumerate(shapes):
        c, _ = arrivals(nb, tp, barriers, splitmix64(seed ^ i), diverge_rate)
        parts.append(c)
        tpbs.append(tp)
    off = np.zeros(len(shapes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(c) for c in parts])
    counts = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint32)
    return counts, off, np.array(tpbs, dtype=np.uint32)
