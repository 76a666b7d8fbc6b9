"""CPU tests of the product's host-side logic and library boundary (no GPU).

* The host model (tests/hostsim.cpp) compiles the product's key-layout and
  pair-count monoid headers for the CPU and runs the GPU path's tile
  decomposition; it must reproduce the oracle exactly.
* libsimcheck.so must load and export every function declared in
  include/simcheck.h; without a GPU, sim_create must fail cleanly.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import tracegen
from tracegen import RECORD_DTYPE

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOSTSIM = os.path.join(ROOT, "tests", "libhostsim.so")


def _hostsim():
    if not os.path.exists(HOSTSIM):
        import subprocess
        subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                        os.path.join(ROOT, "tests", "hostsim.cpp"), "-o", HOSTSIM], check=True)
    lib = ctypes.CDLL(HOSTSIM)
    lib.hs_check.restype = ctypes.c_int64
    lib.hs_check.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                                     ctypes.c_uint64, ctypes.c_void_p]
    lib.hs_check_wide.restype = ctypes.c_int64
    lib.hs_check_wide.argtypes = lib.hs_check.argtypes
    lib.hs_tile_walk.restype = ctypes.c_uint32
    lib.hs_tile_walk.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_uint32)]
    lib.hs_assoc.restype = ctypes.c_int
    lib.hs_assoc.argtypes = [ctypes.c_uint64, ctypes.c_int]
    lib.hs_head_tests.restype = ctypes.c_int
    lib.hs_head_tests.argtypes = [ctypes.c_uint64, ctypes.c_int]
    for name in ("hs_barriers", "hs_barriers_wide"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_uint64]
    return lib


def hs_barriers(recs, off, tpb, wide=False):
    lib = _hostsim()
    off = np.ascontiguousarray(np.asarray(off, dtype=np.uint64))
    tpb = np.ascontiguousarray(np.asarray(tpb, dtype=np.uint32))
    if tpb.ndim == 0 or len(tpb) != len(off) - 1:
        tpb = np.full(len(off) - 1, int(np.asarray(tpb).flat[0]), dtype=np.uint32)
    out = np.zeros(max(1, len(recs)), dtype=oracle.BARRIER_DTYPE)
    fn = lib.hs_barriers_wide if wide else lib.hs_barriers
    n = fn(recs.ctypes.data if len(recs) else None, off.ctypes.data, len(off) - 1, tpb.ctypes.data,
           out.ctypes.data, len(out))
    assert n >= 0, n
    return out[:n]


def hs_check(recs, off, tpb, tile, chunk, wide=False, expect_error=False):
    lib = _hostsim()
    off = np.ascontiguousarray(np.asarray(off, dtype=np.uint64))
    tpb = np.ascontiguousarray(np.asarray(tpb, dtype=np.uint32))
    out = np.zeros(len(recs) + 1, dtype=oracle.RACE_DTYPE)
    mp = ctypes.c_uint32(0)
    fn = lib.hs_check_wide if wide else lib.hs_check
    n = fn(recs.ctypes.data, off.ctypes.data, len(off) - 1, tpb.ctypes.data, tile, chunk,
           out.ctypes.data, len(out), ctypes.byref(mp))
    if expect_error:
        return n
    assert n >= 0, n
    return out[:n], int(mp.value)


def wide_trace(rng, n, tpb=64):
    """Units drawn from a few values spread over 2^62, thread ids up to 2^20,
    epochs up to 999: the lossless key needs more than 64 bits."""
    r = np.zeros(n, dtype=RECORD_DTYPE)
    pool = rng.integers(0, 1 << 62, 12, dtype=np.uint64)
    pool[0], pool[1] = 0, (1 << 62) - 1
    r["unit"] = pool[rng.integers(0, len(pool), n)]
    r["tid"] = rng.integers(0, 1 << 20, n)
    few = rng.random(n) < 0.5  # half the records in three blocks: same-block races
    r["tid"][few] = rng.integers(0, 3 * tpb, int(few.sum()))
    r["epoch"] = rng.integers(0, 3, n)
    r["epoch"][0] = 999
    r["action"] = rng.integers(0, 3, n)
    r["space"] = (rng.random(n) < 0.3).astype(np.uint8)
    return r


def test_monoid_associative():
    assert _hostsim().hs_assoc(12345, 50000) == 0


def test_head_tests_match_head_levels():
    """The scan's four threshold tests (keys.h head_tests_t) give the same
    head levels as head_level_t, on random layouts (with and without the
    warp side field, one- and two-word keys) and neighbouring keys that
    differ in one field."""
    assert _hostsim().hs_head_tests(2024, 20000) == 0


def test_radix_digit_plan():
    """The radix passes (keys.h pass_shift / radix_passes) with 8-bit digits,
    and with 9-bit digits after the first pass: their digits tile the sorted
    key bits exactly, 8-bit plans take ceil(bits / 8) passes, and a stable
    LSD sort under either plan (all-ones padding included) equals a full
    sort of random one- and two-word keys."""
    assert _hostsim().hs_digit_plan(77, 400) == 0


def test_nine_bit_digits_save_a_pass_where_expected():
    """9-bit digits after the 8-bit first pass save a pass exactly where
    1 + ceil((b - 8) / 9) < ceil(b / 8): for the sorted widths of the
    batched workload's largest traces (41..44 bits) but not for 45..48."""
    import math

    def p8(b):
        return math.ceil(b / 8)

    def p9(b):
        return 1 if b <= 8 else 1 + math.ceil((b - 8) / 9)

    assert [b for b in range(40, 49) if p9(b) < p8(b)] == [41, 42, 43, 44]
    assert p8(42) == 6 and p9(42) == 5


@pytest.mark.parametrize("seed", range(120))
def test_host_model_matches_oracle_small(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 300))
    tpb = int(rng.integers(1, 6))
    r = tracegen.random_small(rng, n, units=int(rng.integers(1, 8)), blocks=int(rng.integers(1, 4)), tpb=tpb,
                              epochs=int(rng.integers(1, 4)))
    want, _ = oracle.closed_form(r, tpb=tpb)
    for tile, chunk in [(1, 1), (2, 1), (5, 2), (17, 4), (4096, 16)]:
        got, _ = hs_check(r, [0, n], [tpb], tile, chunk)
        assert got.tobytes() == want.tobytes(), (tile, chunk)


def test_host_model_generated_and_mega_location():
    r, _ = tracegen.c1(n_blocks=8, inject_rate=2e-3)
    want, _ = oracle.closed_form(r, tpb=256)
    got, mp = hs_check(r, [0, len(r)], [256], 4096, 16)
    assert got.tobytes() == want.tobytes() and len(want) > 0
    assert mp >= 1
    # one global unit hit by every record: a location spanning many tiles
    rng = np.random.default_rng(9)
    m = tracegen.random_small(rng, 30000, units=1, blocks=6, tpb=64, epochs=3)
    m["space"] = 0
    want, _ = oracle.closed_form(m, tpb=64)
    for tile in (4096, 1000, 64):
        got, _ = hs_check(m, [0, len(m)], [64], tile, 16)
        assert got.tobytes() == want.tobytes()


@pytest.mark.parametrize("n", [1, 7, 8, 9, 63, 64, 65, 1000, 4097, 131075])
@pytest.mark.parametrize("per_cu", [0, 1, 2, 4, 8, 64])
def test_tile_walk_covers_every_tile_once(n, per_cu):
    """Every launch shape visits each tile of the queue exactly once; the
    one-workgroup-per-tile shape gives no workgroup a second tile; a
    persistent grid stays within its per-CU budget (rounded to 8)."""
    lib = _hostsim()
    for n_cu in (256, 3, 80):
        count = np.zeros(n, dtype=np.uint32)
        mx = ctypes.c_uint32(0)
        grid = lib.hs_tile_walk(n, per_cu, n_cu, count.ctypes.data, ctypes.byref(mx))
        assert (count == 1).all(), (n, per_cu, n_cu)
        assert grid % 8 == 0 and grid >= 8
        if per_cu == 0:
            assert mx.value == 1 and grid < n + 8
        else:
            assert grid <= max(8, -(-min(n, per_cu * n_cu) // 8) * 8)


def test_header_exports_match_library():
    import paper_1905_01833_amd as pkg

    hdr = open(os.path.join(ROOT, "include", "simcheck.h")).read()
    declared = set(re.findall(r"^(?:int|void|uint32_t|const char\*)\s+(sim_\w+)\(", hdr, re.M))
    assert declared == set(pkg.EXPORTS)
    lib = pkg.load()
    for name in declared:
        assert hasattr(lib, name), name


def test_create_fails_cleanly_without_gpu():
    import paper_1905_01833_amd as pkg

    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(pkg.SimError) as ei:
        pkg.Context(0)
    assert ei.value.code == pkg.SIM_EDEVICE


def test_server_create_fails_cleanly_without_gpu():
    import paper_1905_01833_amd as pkg

    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(pkg.SimError) as ei:
        pkg.Server(0, slots=2)
    assert ei.value.code == pkg.SIM_EDEVICE
    with pytest.raises(pkg.SimError) as ei:
        pkg.Server(0, slots=17)
    assert ei.value.code == pkg.SIM_EINVAL


@pytest.mark.parametrize("seed", range(12))
def test_host_model_two_word_keys(seed):
    """Keys wider than 64 bits: the one-word model refuses the trace (as the
    GPU path's one-word mode does), the two-word model matches the oracle;
    on narrow traces the two models agree."""
    rng = np.random.default_rng(seed)
    w = wide_trace(rng, 2500)
    want, _ = oracle.closed_form(w, tpb=64)
    assert len(want) > 0
    assert hs_check(w, [0, len(w)], [64], 4096, 16, expect_error=True) < 0
    for tile, chunk in [(4096, 16), (97, 5)]:
        got, mp = hs_check(w, [0, len(w)], [64], tile, chunk, wide=True)
        assert got.tobytes() == want.tobytes(), (tile, chunk)
        assert 8 < mp <= 16
    r = tracegen.random_small(rng, 400, units=5, blocks=3, tpb=3, epochs=3)
    a, _ = hs_check(r, [0, len(r)], [3], 50, 4)
    b, _ = hs_check(r, [0, len(r)], [3], 50, 4, wide=True)
    assert a.tobytes() == b.tobytes()


def test_abi_structs_match_binding(tmp_path):
    """The Python binding's ctypes mirrors have the sizes and field offsets
    of the structs that include/simcheck.h declares (checked with a probe
    compiled against the header by gcc)."""
    import subprocess

    import paper_1905_01833_amd as pkg

    pairs = {
        "sim_result": pkg._Result, "sim_config": pkg._Config, "sim_stage_time": pkg._StageTime,
        "sim_tuning": pkg._Tuning, "sim_server_config": pkg._ServerConfig, "sim_server_stats": pkg._ServerStats,
        "sim_barrier_result": pkg._BarrierResult, "sim_divergence_result": pkg._DivergenceResult,
    }
    dtypes = {
        "sim_record": pkg.RECORD_DTYPE, "sim_race": pkg.RACE_DTYPE, "sim_trace_summary": pkg.SUMMARY_DTYPE,
        "sim_barrier": pkg.BARRIER_DTYPE, "sim_fitness": pkg.FITNESS_DTYPE, "sim_divergence": pkg.DIVERGENCE_DTYPE,
    }
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "simcheck.h"', "int main(void) {"]
    for c_name, py in pairs.items():
        lines.append(f'  printf("{c_name} size %zu\\n", sizeof({c_name}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{c_name} {f} %zu\\n", offsetof({c_name}, {f}));')
    for c_name, dt in dtypes.items():
        lines.append(f'  printf("{c_name} size %zu\\n", sizeof({c_name}));')
        for f in dt.names:
            lines.append(f'  printf("{c_name} {f} %zu\\n", offsetof({c_name}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for c_name, py in pairs.items():
        assert got[(c_name, "size")] == ctypes.sizeof(py), c_name
        for f, _ in py._fields_:
            assert got[(c_name, f)] == getattr(py, f).offset, (c_name, f)
    for c_name, dt in dtypes.items():
        assert got[(c_name, "size")] == dt.itemsize, c_name
        for f in dt.names:
            assert got[(c_name, f)] == dt.fields[f][1], (c_name, f)


# ------------------------------------------- barrier instances (host model)

def test_host_barrier_model_tree_family():
    """The barrier kernel's per-element rule (barrier.h), run on the CPU
    over sorted keys, against the oracle on the tree-reduction family."""
    for removed in range(-1, 9):
        r = tracegen.tree_reduction(removed)
        off = np.array([0, len(r)], dtype=np.uint64)
        got = hs_barriers(r, off, 256)
        want = oracle.barriers(r, tpb=256)
        assert got.tobytes() == want.tobytes(), removed


@pytest.mark.parametrize("seed", range(40))
def test_host_barrier_model_random(seed):
    rng = np.random.default_rng(2000 + seed)
    tpb = int(rng.integers(1, 6))
    k = int(rng.integers(1, 4))
    traces = [tracegen.random_small(rng, int(rng.integers(0, 200)), units=int(rng.integers(1, 6)),
                                    blocks=int(rng.integers(1, 4)), tpb=tpb, epochs=int(rng.integers(1, 6)))
              for _ in range(k)]
    recs = np.concatenate(traces)
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    want = oracle.barriers(recs, off, tpb)
    assert hs_barriers(recs, off, tpb).tobytes() == want.tobytes()
    assert hs_barriers(recs, off, tpb, wide=True).tobytes() == want.tobytes()


def test_host_barrier_model_generated():
    shapes = tracegen.c3_shapes(24, log2_max=15)
    recs, off, tpb, _ = tracegen.batch(shapes, inject_rate=1e-3)
    want = oracle.barriers(recs, off, tpb)
    assert len(want) > 0 and int(want["racing"].sum()) > 0
    assert hs_barriers(recs, off, tpb).tobytes() == want.tobytes()


@pytest.mark.parametrize("seed", range(4))
def test_host_barrier_model_two_word_keys(seed):
    rng = np.random.default_rng(3000 + seed)
    r = wide_trace(rng, 3000)
    off = np.array([0, len(r)], dtype=np.uint64)
    want = oracle.barriers(r, off, 64)
    assert hs_barriers(r, off, 64, wide=True).tobytes() == want.tobytes()
