"""Python binding of the MI355X data-race check (libsimcheck.so).

Argument marshalling only: every step of the check runs in the HIP kernels
behind the C ABI of include/simcheck.h.  The binding keeps the C names
(sim_create, sim_check_traces, sim_check_traces_device, ...) and adds a small
Context wrapper.  Loading fails loudly when the library is not built; there
is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import json
import os
import sys
import weakref

import numpy as np

from ._build import LIB, build_library

RECORD_DTYPE = np.dtype(
    [("unit", "<u8"), ("tid", "<u4"), ("epoch", "<u2"), ("action", "u1"), ("space", "u1")]
)
RACE_DTYPE = np.dtype(
    [
        ("trace", "<u4"), ("space", "u1"), ("kinds", "u1"), ("reserved16", "<u2"), ("block", "<u4"),
        ("reserved32", "<u4"), ("unit", "<u8"), ("pairs_ww", "<u8"), ("pairs_rw", "<u8"),
        ("pairs_aw", "<u8"), ("pairs_ar", "<u8"), ("pairs_xblock", "<u8"),
    ]
)
SUMMARY_DTYPE = np.dtype([("n_records", "<u8"), ("n_race_locs", "<u8"), ("n_pairs", "<u8")])
BARRIER_DTYPE = np.dtype([("trace", "<u4"), ("boundary", "<u4"), ("instances", "<u8"), ("racing", "<u8")])
FITNESS_DTYPE = np.dtype([("n_records", "<u8"), ("n_locations", "<u8"), ("n_location_threads", "<u8"),
                          ("global_range", "<u8"), ("shared_range", "<u8"), ("fitness", "<f8")])
DIVERGENCE_DTYPE = np.dtype([("trace", "<u4"), ("block", "<u4"), ("min_barriers", "<u4"), ("max_barriers", "<u4"),
                             ("early_threads", "<u8")])

SIM_OK, SIM_EINVAL, SIM_ERECORD, SIM_ENOMEM, SIM_EDEVICE, SIM_ERANGE, SIM_ENOSPC = 0, -1, -2, -3, -4, -6, -7
SIM_CFG_PROFILE = 1
SIM_CFG_GRAPHS = 2
STAGES = ["init", "stats", "layout", "keygen", "upsweep", "sort_pass", "scan_tiles", "scan_cross", "scan_out"]

# Symbols declared in include/simcheck.h.
EXPORTS = [
    "sim_create", "sim_destroy", "sim_last_error", "sim_check_traces", "sim_check_traces_device",
    "sim_check_traces_device_noalloc", "sim_result_free", "sim_check_traces_warp_device", "sim_check_traces_warp",
    "sim_check_sync_device", "sim_check_sync", "sim_barrier_result_free", "sim_eval_fitness_device",
    "sim_eval_fitness", "sim_check_divergence_device", "sim_check_divergence", "sim_divergence_result_free",
    "sim_stage_times", "sim_stage_name", "sim_size_class", "sim_set_tuning", "sim_get_tuning", "sim_autotune",
    "sim_server_create", "sim_server_destroy", "sim_submit", "sim_submit_device", "sim_poll", "sim_wait",
    "sim_server_get_stats", "sim_server_last_error",
]
SIM_EAGAIN = -5
SIM_SIZE_CLASSES = 33
TUNING_FIELDS = ("stream_wgs_per_cu", "sort_wgs_per_cu", "scan_wgs_per_cu", "group_shift_bias", "scatter_threads",
                 "digit_bits")


class SimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"simcheck error {code}: {msg}")
        self.code = code


class _Result(ctypes.Structure):
    _fields_ = [
        ("races", ctypes.c_void_p),
        ("n_races", ctypes.c_uint64),
        ("traces", ctypes.c_void_p),
        ("n_traces", ctypes.c_uint32),
    ]


class _BarrierResult(ctypes.Structure):
    _fields_ = [("barriers", ctypes.c_void_p), ("n_barriers", ctypes.c_uint64)]


class _DivergenceResult(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_void_p), ("n_blocks", ctypes.c_uint64)]


class _Config(ctypes.Structure):
    _fields_ = [("reserve_records", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("reserve_traces", ctypes.c_uint32)]


class _StageTime(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _Tuning(ctypes.Structure):
    _fields_ = [
        ("stream_wgs_per_cu", ctypes.c_uint32),
        ("sort_wgs_per_cu", ctypes.c_uint32),
        ("scan_wgs_per_cu", ctypes.c_uint32),
        ("group_shift_bias", ctypes.c_int32),
        ("scatter_threads", ctypes.c_uint32),
        ("digit_bits", ctypes.c_uint32),
        ("ms", ctypes.c_double),
    ]


def _tuning_dict(t: _Tuning) -> dict:
    d = {f: int(getattr(t, f)) for f in TUNING_FIELDS}
    d["ms"] = float(t.ms)
    return d


class _ServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("max_batch_records", ctypes.c_uint64),
        ("slots", ctypes.c_uint32),
        ("max_batch_requests", ctypes.c_uint32),
        ("max_pending", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("reserve_records", ctypes.c_uint64),
    ]


class _ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
        ("batches", ctypes.c_uint64), ("records", ctypes.c_uint64),
        ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double), ("records_per_s", ctypes.c_double), ("mean_batch_requests", ctypes.c_double),
        ("peak_inflight_bytes", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64), ("requeued", ctypes.c_uint64),
    ]


_lib = None


def lib_path() -> str:
    return LIB


def load() -> ctypes.CDLL:
    """Load libsimcheck.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise ImportError(f"{LIB} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    lib.sim_create.restype = ctypes.c_int
    lib.sim_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    lib.sim_destroy.restype = None
    lib.sim_destroy.argtypes = [P]
    lib.sim_last_error.restype = ctypes.c_char_p
    lib.sim_last_error.argtypes = [P]
    lib.sim_check_traces.restype = ctypes.c_int
    lib.sim_check_traces.argtypes = [P, P, P, ctypes.c_uint32, P, ctypes.POINTER(ctypes.POINTER(_Result))]
    lib.sim_check_traces_device.restype = ctypes.c_int
    lib.sim_check_traces_device.argtypes = [P, P, P, ctypes.c_uint32, P, P, ctypes.POINTER(ctypes.POINTER(_Result))]
    lib.sim_check_traces_device_noalloc.restype = ctypes.c_int
    lib.sim_check_traces_device_noalloc.argtypes = [P, P, P, ctypes.c_uint32, P, P, P, ctypes.c_uint64,
                                                    ctypes.POINTER(ctypes.c_uint64), P]
    lib.sim_check_sync_device.restype = ctypes.c_int
    lib.sim_check_sync_device.argtypes = [P, P, P, ctypes.c_uint32, P, P, ctypes.POINTER(ctypes.POINTER(_Result)),
                                          ctypes.POINTER(ctypes.POINTER(_BarrierResult))]
    lib.sim_check_sync.restype = ctypes.c_int
    lib.sim_check_sync.argtypes = [P, P, P, ctypes.c_uint32, P, ctypes.POINTER(ctypes.POINTER(_Result)),
                                   ctypes.POINTER(ctypes.POINTER(_BarrierResult))]
    lib.sim_barrier_result_free.restype = None
    lib.sim_barrier_result_free.argtypes = [ctypes.POINTER(_BarrierResult)]
    lib.sim_check_traces_warp_device.restype = ctypes.c_int
    lib.sim_check_traces_warp_device.argtypes = [P, P, P, P, ctypes.c_uint32, P, P,
                                                 ctypes.POINTER(ctypes.POINTER(_Result))]
    lib.sim_check_traces_warp.restype = ctypes.c_int
    lib.sim_check_traces_warp.argtypes = [P, P, P, P, ctypes.c_uint32, P, ctypes.POINTER(ctypes.POINTER(_Result))]
    lib.sim_eval_fitness_device.restype = ctypes.c_int
    lib.sim_eval_fitness_device.argtypes = [P, P, P, ctypes.c_uint32, P, P, P]
    lib.sim_eval_fitness.restype = ctypes.c_int
    lib.sim_eval_fitness.argtypes = [P, P, P, ctypes.c_uint32, P, P]
    lib.sim_check_divergence_device.restype = ctypes.c_int
    lib.sim_check_divergence_device.argtypes = [P, P, P, ctypes.c_uint32, P, P,
                                                ctypes.POINTER(ctypes.POINTER(_DivergenceResult))]
    lib.sim_check_divergence.restype = ctypes.c_int
    lib.sim_check_divergence.argtypes = [P, P, P, ctypes.c_uint32, P,
                                         ctypes.POINTER(ctypes.POINTER(_DivergenceResult))]
    lib.sim_divergence_result_free.restype = None
    lib.sim_divergence_result_free.argtypes = [ctypes.POINTER(_DivergenceResult)]
    lib.sim_result_free.restype = None
    lib.sim_result_free.argtypes = [ctypes.POINTER(_Result)]
    lib.sim_stage_times.restype = ctypes.c_int
    lib.sim_stage_times.argtypes = [P, ctypes.POINTER(_StageTime), ctypes.c_int]
    lib.sim_stage_name.restype = ctypes.c_char_p
    lib.sim_stage_name.argtypes = [ctypes.c_int]
    lib.sim_size_class.restype = ctypes.c_uint32
    lib.sim_size_class.argtypes = [ctypes.c_uint64]
    lib.sim_set_tuning.restype = ctypes.c_int
    lib.sim_set_tuning.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(_Tuning)]
    lib.sim_get_tuning.restype = ctypes.c_int
    lib.sim_get_tuning.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(_Tuning)]
    lib.sim_autotune.restype = ctypes.c_int
    lib.sim_autotune.argtypes = [P, P, P, ctypes.c_uint32, P, P, ctypes.c_uint32, ctypes.POINTER(_Tuning)]
    lib.sim_server_create.restype = ctypes.c_int
    lib.sim_server_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(_ServerConfig)]
    lib.sim_server_destroy.restype = None
    lib.sim_server_destroy.argtypes = [P]
    lib.sim_submit.restype = ctypes.c_int
    lib.sim_submit.argtypes = [P, P, P, ctypes.c_uint32, P, ctypes.POINTER(ctypes.c_uint64)]
    lib.sim_submit_device.restype = ctypes.c_int
    lib.sim_submit_device.argtypes = [P, P, P, ctypes.c_uint32, P, ctypes.POINTER(ctypes.c_uint64)]
    lib.sim_poll.restype = ctypes.c_int
    lib.sim_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.POINTER(_Result))]
    lib.sim_wait.restype = ctypes.c_int
    lib.sim_wait.argtypes = [P, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ctypes.POINTER(_Result))]
    lib.sim_server_get_stats.restype = ctypes.c_int
    lib.sim_server_get_stats.argtypes = [P, ctypes.POINTER(_ServerStats), ctypes.c_int]
    lib.sim_server_last_error.restype = ctypes.c_char_p
    lib.sim_server_last_error.argtypes = []
    _lib = lib
    return lib


# ------------------------------------------------------------ C-named API

def sim_create(hip_device: int = 0, profile: bool = False, reserve_records: int = 0,
               graphs: bool = False, reserve_traces: int = 0) -> ctypes.c_void_p:
    lib = load()
    ctx = ctypes.c_void_p()
    flags = (SIM_CFG_PROFILE if profile else 0) | (SIM_CFG_GRAPHS if graphs else 0)
    cfg = _Config(reserve_records, flags, reserve_traces)
    rc = lib.sim_create(ctypes.byref(ctx), hip_device, ctypes.byref(cfg))
    if rc != SIM_OK:
        raise SimError(rc, f"sim_create failed on device {hip_device} (needs a gfx950 GPU)")
    return ctx


def sim_destroy(ctx) -> None:
    load().sim_destroy(ctx)


def sim_last_error(ctx) -> str:
    return (load().sim_last_error(ctx) or b"").decode()


def _tables(offsets, tpb, n_records):
    if offsets is None:
        offsets = np.array([0, n_records], dtype=np.uint64)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    n_traces = len(offsets) - 1
    tpb = np.asarray(tpb, dtype=np.uint32)
    if tpb.ndim == 0:
        tpb = np.full(n_traces, int(tpb), dtype=np.uint32)
    tpb = np.ascontiguousarray(tpb)
    if len(tpb) != n_traces:
        raise ValueError("threads_per_block needs one value per trace")
    return offsets, n_traces, tpb


class _ResultMemory:
    """A library result (sim_result): freed with sim_result_free once the
    last array that views its entries or summaries is gone."""

    def __init__(self, res_p):
        self._p = res_p
        self._free = load().sim_result_free  # bound now: usable during shutdown

    def __del__(self):
        p, self._p = self._p, None
        if p is not None:
            self._free(p)


def _view(ptr, n, dtype, owner):
    """Array of n `dtype` items at host address ptr, owned by `owner`."""
    if n == 0:
        return np.zeros(0, dtype=dtype)
    buf = (ctypes.c_char * (n * dtype.itemsize)).from_address(ptr)
    buf._owner = owner  # the buffer, and so every array on it, keeps the result alive
    return np.frombuffer(buf, dtype=dtype)


def _take_result(res_p):
    """The entries and summaries of a result as arrays on the library's own
    memory (no copy)."""
    r = res_p.contents
    owner = _ResultMemory(res_p)
    return _view(r.races, r.n_races, RACE_DTYPE, owner), _view(r.traces, r.n_traces, SUMMARY_DTYPE, owner)


def sim_check_traces(ctx, records: np.ndarray, offsets=None, threads_per_block=1):
    """Check traces whose records are in host memory (numpy RECORD_DTYPE)."""
    lib = load()
    records = np.ascontiguousarray(records)
    if records.dtype.itemsize != 16:
        raise TypeError("records must be 16-byte sim_record entries")
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, len(records))
    out = ctypes.POINTER(_Result)()
    rc = lib.sim_check_traces(ctx, records.ctypes.data if len(records) else None, offsets.ctypes.data, n_traces,
                              tpb.ctypes.data, ctypes.byref(out))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return _take_result(out)


def sim_check_traces_device(ctx, d_records_ptr: int, n_records: int, offsets=None, threads_per_block=1, stream=None):
    """Check traces whose records are in device memory at d_records_ptr
    (e.g. tensor.data_ptr()); stream is a hipStream_t handle (int) or None."""
    lib = load()
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, n_records)
    if int(offsets[-1]) != n_records:
        raise ValueError("offsets[-1] must equal the number of device records")
    out = ctypes.POINTER(_Result)()
    rc = lib.sim_check_traces_device(ctx, ctypes.c_void_p(d_records_ptr) if n_records else None, offsets.ctypes.data,
                                     n_traces, tpb.ctypes.data, ctypes.c_void_p(stream or 0), ctypes.byref(out))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return _take_result(out)


SIM_SIDE_DIVERGED = 1 << 31  # side-word bit: the access ran while its warp was diverged


def sim_check_traces_warp(ctx, records: np.ndarray, side: np.ndarray, offsets=None, threads_per_block=1):
    """Warp-aware check of host records; side: one uint32 per record
    (statement id, SIM_SIDE_DIVERGED)."""
    lib = load()
    records = np.ascontiguousarray(records)
    side = np.ascontiguousarray(np.asarray(side, dtype=np.uint32))
    if records.dtype.itemsize != 16:
        raise TypeError("records must be 16-byte sim_record entries")
    if len(side) != len(records):
        raise ValueError("one side word per record")
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, len(records))
    out = ctypes.POINTER(_Result)()
    rc = lib.sim_check_traces_warp(ctx, records.ctypes.data if len(records) else None,
                                   side.ctypes.data if len(side) else None, offsets.ctypes.data, n_traces,
                                   tpb.ctypes.data, ctypes.byref(out))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return _take_result(out)


def sim_check_traces_warp_device(ctx, d_records_ptr: int, d_side_ptr: int, n_records: int, offsets=None,
                                 threads_per_block=1, stream=None):
    """Warp-aware check of device records, with one device side word per
    record at d_side_ptr."""
    lib = load()
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, n_records)
    if int(offsets[-1]) != n_records:
        raise ValueError("offsets[-1] must equal the number of device records")
    out = ctypes.POINTER(_Result)()
    rc = lib.sim_check_traces_warp_device(ctx, ctypes.c_void_p(d_records_ptr) if n_records else None,
                                          ctypes.c_void_p(d_side_ptr) if n_records else None, offsets.ctypes.data,
                                          n_traces, tpb.ctypes.data, ctypes.c_void_p(stream or 0), ctypes.byref(out))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return _take_result(out)


def sim_check_traces_device_noalloc(ctx, d_records_ptr: int, n_records: int, offsets=None, threads_per_block=1,
                                    stream=None, races_cap: int = 1 << 16, races_out=None, traces_out=None):
    """The no-allocation check (records in device memory, every device
    buffer from the library's fixed scratch).  races_out / traces_out are
    the caller's host arrays (RACE_DTYPE with room for races_cap entries,
    SUMMARY_DTYPE with one per trace); made here when not given.  Returns
    (races, summaries) as views of them."""
    lib = load()
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, n_records)
    if int(offsets[-1]) != n_records:
        raise ValueError("offsets[-1] must equal the number of device records")
    if races_out is None:
        races_out = np.zeros(races_cap, dtype=RACE_DTYPE)
    if traces_out is None:
        traces_out = np.zeros(max(n_traces, 1), dtype=SUMMARY_DTYPE)
    if races_out.dtype != RACE_DTYPE or traces_out.dtype != SUMMARY_DTYPE or len(traces_out) < n_traces:
        raise ValueError("races_out / traces_out have the wrong type or size")
    n = ctypes.c_uint64(0)
    rc = lib.sim_check_traces_device_noalloc(
        ctx, ctypes.c_void_p(d_records_ptr) if n_records else None, offsets.ctypes.data, n_traces, tpb.ctypes.data,
        ctypes.c_void_p(stream or 0), races_out.ctypes.data if len(races_out) else None, len(races_out),
        ctypes.byref(n), traces_out.ctypes.data)
    if rc != SIM_OK:
        err = SimError(rc, sim_last_error(ctx))
        err.n_races = int(n.value)
        raise err
    return races_out[: n.value], traces_out[:n_traces]


def _take_barriers(res_p):
    r = res_p.contents
    out = np.zeros(r.n_barriers, dtype=BARRIER_DTYPE)
    if r.n_barriers:
        ctypes.memmove(out.ctypes.data, r.barriers, r.n_barriers * BARRIER_DTYPE.itemsize)
    load().sim_barrier_result_free(res_p)
    return out


def sim_check_sync_device(ctx, d_records_ptr: int, n_records: int, offsets=None, threads_per_block=1, stream=None):
    """Race check and redundant-barrier check of device records: returns
    (races, summaries, barriers), barriers a BARRIER_DTYPE array with one
    row per (trace, boundary) that has an instance."""
    lib = load()
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, n_records)
    if int(offsets[-1]) != n_records:
        raise ValueError("offsets[-1] must equal the number of device records")
    out = ctypes.POINTER(_Result)()
    bar = ctypes.POINTER(_BarrierResult)()
    rc = lib.sim_check_sync_device(ctx, ctypes.c_void_p(d_records_ptr) if n_records else None, offsets.ctypes.data,
                                   n_traces, tpb.ctypes.data, ctypes.c_void_p(stream or 0), ctypes.byref(out),
                                   ctypes.byref(bar))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    races, summ = _take_result(out)
    return races, summ, _take_barriers(bar)


def sim_check_sync(ctx, records: np.ndarray, offsets=None, threads_per_block=1):
    """sim_check_sync_device for records in host memory."""
    lib = load()
    records = np.ascontiguousarray(records)
    if records.dtype.itemsize != 16:
        raise TypeError("records must be 16-byte sim_record entries")
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, len(records))
    out = ctypes.POINTER(_Result)()
    bar = ctypes.POINTER(_BarrierResult)()
    rc = lib.sim_check_sync(ctx, records.ctypes.data if len(records) else None, offsets.ctypes.data, n_traces,
                            tpb.ctypes.data, ctypes.byref(out), ctypes.byref(bar))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    races, summ = _take_result(out)
    return races, summ, _take_barriers(bar)


def sim_eval_fitness(ctx, records: np.ndarray, offsets=None, threads_per_block=1):
    """EP fitness (Eq. 1) of every trace of host records: a FITNESS_DTYPE
    row per trace."""
    lib = load()
    records = np.ascontiguousarray(records)
    if records.dtype.itemsize != 16:
        raise TypeError("records must be 16-byte sim_record entries")
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, len(records))
    out = np.zeros(max(n_traces, 1), dtype=FITNESS_DTYPE)
    rc = lib.sim_eval_fitness(ctx, records.ctypes.data if len(records) else None, offsets.ctypes.data, n_traces,
                              tpb.ctypes.data, out.ctypes.data)
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return out[:n_traces]


def sim_eval_fitness_device(ctx, d_records_ptr: int, n_records: int, offsets=None, threads_per_block=1,
                            stream=None):
    """sim_eval_fitness for records in device memory at d_records_ptr."""
    lib = load()
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, n_records)
    if int(offsets[-1]) != n_records:
        raise ValueError("offsets[-1] must equal the number of device records")
    out = np.zeros(max(n_traces, 1), dtype=FITNESS_DTYPE)
    rc = lib.sim_eval_fitness_device(ctx, ctypes.c_void_p(d_records_ptr) if n_records else None, offsets.ctypes.data,
                                     n_traces, tpb.ctypes.data, ctypes.c_void_p(stream or 0), out.ctypes.data)
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return out[:n_traces]


def _thread_tables(offsets, tpb):
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    n_traces = len(offsets) - 1
    tpb = np.asarray(tpb, dtype=np.uint32)
    if tpb.ndim == 0:
        tpb = np.full(n_traces, int(tpb), dtype=np.uint32)
    tpb = np.ascontiguousarray(tpb)
    if len(tpb) != n_traces:
        raise ValueError("threads_per_block needs one value per trace")
    return offsets, n_traces, tpb


def _take_divergence(res_p):
    r = res_p.contents
    out = np.zeros(r.n_blocks, dtype=DIVERGENCE_DTYPE)
    if r.n_blocks:
        ctypes.memmove(out.ctypes.data, r.blocks, r.n_blocks * DIVERGENCE_DTYPE.itemsize)
    load().sim_divergence_result_free(res_p)
    return out


def sim_check_divergence(ctx, arrivals: np.ndarray, offsets, threads_per_block):
    """Barrier-divergence check (Alg. 4) of per-thread barrier arrival counts
    in host memory (uint32, block by block; offsets: CSR over threads).
    Returns a DIVERGENCE_DTYPE array, one row per divergent block."""
    lib = load()
    arrivals = np.ascontiguousarray(np.asarray(arrivals, dtype=np.uint32))
    offsets, n_traces, tpb = _thread_tables(offsets, threads_per_block)
    out = ctypes.POINTER(_DivergenceResult)()
    rc = lib.sim_check_divergence(ctx, arrivals.ctypes.data if len(arrivals) else None, offsets.ctypes.data,
                                  n_traces, tpb.ctypes.data, ctypes.byref(out))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return _take_divergence(out)


def sim_check_divergence_device(ctx, d_arrivals_ptr: int, n_threads: int, offsets, threads_per_block, stream=None):
    """sim_check_divergence for counts in device memory at d_arrivals_ptr."""
    lib = load()
    offsets, n_traces, tpb = _thread_tables(offsets, threads_per_block)
    if int(offsets[-1]) != n_threads:
        raise ValueError("offsets[-1] must equal the number of device counts")
    out = ctypes.POINTER(_DivergenceResult)()
    rc = lib.sim_check_divergence_device(ctx, ctypes.c_void_p(d_arrivals_ptr) if n_threads else None,
                                         offsets.ctypes.data, n_traces, tpb.ctypes.data,
                                         ctypes.c_void_p(stream or 0), ctypes.byref(out))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return _take_divergence(out)


def sim_stage_times(ctx):
    lib = load()
    arr = (_StageTime * 16)()
    n = lib.sim_stage_times(ctx, arr, 16)
    return {lib.sim_stage_name(i).decode(): (arr[i].ms, arr[i].launches) for i in range(n)}


def sim_size_class(total_records: int) -> int:
    return int(load().sim_size_class(int(total_records)))


def sim_set_tuning(ctx, size_class: int, tuning: dict | None) -> None:
    """Set the launch shape of one size class (None: back to the default)."""
    t = None
    if tuning is not None:
        t = _Tuning(*(int(tuning.get(f, 0)) for f in TUNING_FIELDS), float(tuning.get("ms", 0.0)))
    rc = load().sim_set_tuning(ctx, size_class, ctypes.byref(t) if t is not None else None)
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))


def sim_get_tuning(ctx, size_class: int):
    """(is_set, shape) of one size class."""
    t = _Tuning()
    rc = load().sim_get_tuning(ctx, size_class, ctypes.byref(t))
    if rc < 0:
        raise SimError(rc, "bad size class")
    return rc == 1, _tuning_dict(t)


def sim_autotune(ctx, d_records_ptr: int, n_records: int, offsets=None, threads_per_block=1, stream=None,
                 reps: int = 3) -> dict:
    """Time candidate launch shapes on the given device records; the best is
    kept for the input's size class and returned."""
    offsets, n_traces, tpb = _tables(offsets, threads_per_block, n_records)
    if int(offsets[-1]) != n_records:
        raise ValueError("offsets[-1] must equal the number of device records")
    t = _Tuning()
    rc = load().sim_autotune(ctx, ctypes.c_void_p(d_records_ptr) if n_records else None, offsets.ctypes.data,
                             n_traces, tpb.ctypes.data, ctypes.c_void_p(stream or 0), reps, ctypes.byref(t))
    if rc != SIM_OK:
        raise SimError(rc, sim_last_error(ctx))
    return _tuning_dict(t)


# ----------------------------------------------------------- convenience

# Contexts and servers still open at interpreter exit are closed by an
# atexit hook, while the HIP runtime is fully alive: atexit hooks run at the
# start of interpreter finalisation, before module teardown and before the
# C-level exit handlers that finalise the HIP runtime (and a profiler's
# tool library).  A destructor that runs later, during finalisation, does
# not call into HIP at all (the handle is left to process exit).
_open_handles = weakref.WeakSet()
_atexit_registered = False


def _close_open_handles():
    for h in list(_open_handles):
        try:
            h.close()
        except Exception:
            pass


def _track(obj):
    global _atexit_registered
    if not _atexit_registered:
        atexit.register(_close_open_handles)
        _atexit_registered = True
    _open_handles.add(obj)


class Context:
    """One library context on one GPU."""

    def __init__(self, device: int = 0, profile: bool = False, reserve_records: int = 0, graphs: bool = False,
                 reserve_traces: int = 0):
        self._ctx = sim_create(device, profile=profile, reserve_records=reserve_records, graphs=graphs,
                               reserve_traces=reserve_traces)
        _track(self)

    def close(self):
        if self._ctx:
            sim_destroy(self._ctx)
            self._ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be cleared when
        # a destructor runs during interpreter shutdown)
        if not getattr(self, "_ctx", None) or _finalizing():  # (also after a failed __init__)
            return
        try:
            self.close()
        except Exception:
            pass

    def check_traces(self, records, offsets=None, threads_per_block=1):
        return sim_check_traces(self._ctx, records, offsets, threads_per_block)

    def check_traces_device(self, tensor, offsets=None, threads_per_block=1, stream=None):
        """tensor: a device tensor whose storage holds sim_record entries
        (16 bytes each, e.g. uint8 [n, 16] or int64 [n, 2])."""
        ptr, n, stream = self._device_args(tensor, stream)
        return sim_check_traces_device(self._ctx, ptr, n, offsets, threads_per_block, stream)

    def check_traces_warp(self, records, side, offsets=None, threads_per_block=1):
        """Warp-aware check of host records (side: uint32 per record)."""
        return sim_check_traces_warp(self._ctx, records, side, offsets, threads_per_block)

    def check_traces_warp_device(self, tensor, side_tensor, offsets=None, threads_per_block=1, stream=None):
        """Warp-aware check of a device tensor of records, with a device
        tensor of one uint32 side word per record."""
        ptr, n, stream = self._device_args(tensor, stream)
        if side_tensor.numel() * side_tensor.element_size() != 4 * n:
            raise ValueError("one 4-byte side word per record")
        return sim_check_traces_warp_device(self._ctx, ptr, side_tensor.data_ptr(), n, offsets, threads_per_block,
                                            stream)

    def check_sync(self, records, offsets=None, threads_per_block=1):
        """Races and barrier instances of host records."""
        return sim_check_sync(self._ctx, records, offsets, threads_per_block)

    def check_sync_device(self, tensor, offsets=None, threads_per_block=1, stream=None):
        """Races and barrier instances of a device tensor of records."""
        ptr, n, stream = self._device_args(tensor, stream)
        return sim_check_sync_device(self._ctx, ptr, n, offsets, threads_per_block, stream)

    def eval_fitness(self, records, offsets=None, threads_per_block=1):
        """EP fitness rows of host records."""
        return sim_eval_fitness(self._ctx, records, offsets, threads_per_block)

    def eval_fitness_device(self, tensor, offsets=None, threads_per_block=1, stream=None):
        """EP fitness rows of a device tensor of records."""
        ptr, n, stream = self._device_args(tensor, stream)
        return sim_eval_fitness_device(self._ctx, ptr, n, offsets, threads_per_block, stream)

    def check_divergence(self, arrivals, offsets, threads_per_block):
        """Barrier divergence of host arrival counts (numpy uint32)."""
        return sim_check_divergence(self._ctx, arrivals, offsets, threads_per_block)

    def check_divergence_device(self, tensor, offsets, threads_per_block, stream=None):
        """Barrier divergence of a contiguous device tensor of 32-bit arrival
        counts (int32 or uint32)."""
        if tensor.element_size() != 4 or not tensor.is_contiguous():
            raise ValueError("arrival counts must be a contiguous tensor of 32-bit integers")
        if stream is None:
            import torch

            stream = torch.cuda.current_stream(tensor.device).cuda_stream
        return sim_check_divergence_device(self._ctx, tensor.data_ptr(), tensor.numel(), offsets, threads_per_block,
                                           stream)

    def check_traces_device_noalloc(self, tensor, offsets=None, threads_per_block=1, stream=None,
                                    races_cap: int = 1 << 16, races_out=None, traces_out=None):
        """sim_check_traces_device_noalloc on a device tensor (as in
        check_traces_device); the result lands in host arrays."""
        ptr, n, stream = self._device_args(tensor, stream)
        return sim_check_traces_device_noalloc(self._ctx, ptr, n, offsets, threads_per_block, stream, races_cap,
                                               races_out, traces_out)

    @staticmethod
    def _device_args(tensor, stream):
        nbytes = tensor.numel() * tensor.element_size()
        if nbytes % 16:
            raise ValueError("tensor size is not a multiple of 16 bytes")
        if not tensor.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if stream is None:
            import torch

            stream = torch.cuda.current_stream(tensor.device).cuda_stream
        return tensor.data_ptr(), nbytes // 16, stream

    def stage_times(self):
        return sim_stage_times(self._ctx)

    def autotune(self, tensor, offsets=None, threads_per_block=1, stream=None, reps: int = 3) -> dict:
        """Autotune the launch shape for calls the size of this input (device
        tensor as in check_traces_device); returns the shape, with its size
        class under "size_class"."""
        ptr, n, stream = self._device_args(tensor, stream)
        d = sim_autotune(self._ctx, ptr, n, offsets, threads_per_block, stream, reps)
        d["size_class"] = sim_size_class(n)
        return d

    def set_tuning(self, size_class: int, tuning: dict | None) -> None:
        sim_set_tuning(self._ctx, size_class, tuning)

    def tuning(self, size_class: int):
        return sim_get_tuning(self._ctx, size_class)

    def save_tuning(self, path: str) -> None:
        """Write every set size class's shape to a JSON file (the tuning
        cache), merged with what the file already holds."""
        data = load_tuning_file(path)
        for k in range(SIM_SIZE_CLASSES):
            is_set, t = self.tuning(k)
            if is_set:
                data[str(k)] = t
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"format": "simcheck-tuning-1", "classes": data}, f, indent=1, sort_keys=True)
        os.replace(tmp, path)

    def load_tuning(self, path: str) -> int:
        """Set the shapes stored in a tuning cache file; returns how many."""
        data = load_tuning_file(path)
        for k, t in data.items():
            self.set_tuning(int(k), t)
        return len(data)

    def last_error(self) -> str:
        return sim_last_error(self._ctx)


def load_tuning_file(path: str) -> dict:
    """Size class -> shape from a tuning cache file ({} if it is absent)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    if d.get("format") != "simcheck-tuning-1":
        raise ValueError(f"{path}: not a tuning cache file")
    out = {}
    for k, t in d.get("classes", {}).items():
        if not (0 <= int(k) < SIM_SIZE_CLASSES):
            raise ValueError(f"{path}: size class {k} out of range")
        out[str(int(k))] = {f: int(t.get(f, 0)) for f in TUNING_FIELDS} | {"ms": float(t.get("ms", 0.0))}
    return out


# ---------------------------------------------------------------- serving

class Server:
    """Request loop with continuous batching (sim_server_* of the C ABI).

    submit() keeps a reference to the request's arrays until its result is
    collected, as the C ABI requires."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, slots: int = 0, max_batch_records: int = 0,
                 max_batch_requests: int = 0, max_pending: int = 0, reserve_records: int = 0):
        lib = load()
        cfg = _ServerConfig(hbm_budget_bytes, max_batch_records, slots, max_batch_requests, max_pending, 0,
                            reserve_records)
        self._srv = ctypes.c_void_p()
        rc = lib.sim_server_create(ctypes.byref(self._srv), device, ctypes.byref(cfg))
        if rc != SIM_OK:
            raise SimError(rc, lib.sim_server_last_error().decode())
        self._keep = {}
        _track(self)

    def close(self):
        if self._srv:
            load().sim_server_destroy(self._srv)
            self._srv = None
            self._keep.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be cleared when
        # a destructor runs during interpreter shutdown)
        if not getattr(self, "_srv", None) or _finalizing():  # (also after a failed __init__)
            return
        try:
            self.close()
        except Exception:
            pass

    def submit(self, records: np.ndarray, offsets=None, threads_per_block=1) -> int:
        lib = load()
        records = np.ascontiguousarray(records)
        if records.dtype.itemsize != 16:
            raise TypeError("records must be 16-byte sim_record entries")
        offsets, n_traces, tpb = _tables(offsets, threads_per_block, len(records))
        t = ctypes.c_uint64(0)
        rc = lib.sim_submit(self._srv, records.ctypes.data if len(records) else None, offsets.ctypes.data, n_traces,
                            tpb.ctypes.data, ctypes.byref(t))
        if rc != SIM_OK:
            raise SimError(rc, lib.sim_server_last_error().decode())
        self._keep[t.value] = records
        return t.value

    def submit_device(self, tensor, offsets=None, threads_per_block=1) -> int:
        """Submit a request whose records are a device tensor on the server's
        GPU (16-byte sim_record entries, contiguous); the workers read them
        in place.  The tensor is kept alive until the result is collected."""
        lib = load()
        nbytes = tensor.numel() * tensor.element_size()
        if nbytes % 16 or not tensor.is_contiguous():
            raise ValueError("tensor must be contiguous 16-byte sim_record entries")
        n = nbytes // 16
        offsets, n_traces, tpb = _tables(offsets, threads_per_block, n)
        if int(offsets[-1]) != n:
            raise ValueError("offsets[-1] must equal the number of device records")
        t = ctypes.c_uint64(0)
        rc = lib.sim_submit_device(self._srv, ctypes.c_void_p(tensor.data_ptr()) if n else None, offsets.ctypes.data,
                                   n_traces, tpb.ctypes.data, ctypes.byref(t))
        if rc != SIM_OK:
            raise SimError(rc, lib.sim_server_last_error().decode())
        self._keep[t.value] = tensor
        return t.value

    def _collect(self, rc, ticket, out):
        lib = load()
        if rc == SIM_EAGAIN:
            return None
        self._keep.pop(ticket, None)
        if rc != SIM_OK:
            raise SimError(rc, lib.sim_server_last_error().decode())
        return _take_result(out)

    def poll(self, ticket: int):
        """(races, summaries) when ready, None while pending; raises the
        request's error."""
        out = ctypes.POINTER(_Result)()
        return self._collect(load().sim_poll(self._srv, ticket, ctypes.byref(out)), ticket, out)

    def wait(self, ticket: int, timeout_ms: int = -1):
        out = ctypes.POINTER(_Result)()
        return self._collect(load().sim_wait(self._srv, ticket, timeout_ms, ctypes.byref(out)), ticket, out)

    def stats(self, reset: bool = False) -> dict:
        st = _ServerStats()
        rc = load().sim_server_get_stats(self._srv, ctypes.byref(st), 1 if reset else 0)
        if rc != SIM_OK:
            raise SimError(rc, "stats")
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}
