"""Pins for the oracle's EP fitness (Eq. 1 and the secondary score of
Sec. 4.1.1), on the CPU: hand-derived values on the tree reduction and the
paper's examples, closed cases, invariants, a pure-Python rendering;
planted mistakes must each fail a pin."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import tracegen
from golden_io import trace_fixture
from tracegen import RECORD_DTYPE

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
FIELDS = ("n_records", "n_locations", "n_location_threads", "global_range", "shared_range")


def row(f):
    return tuple(int(f[k]) for k in FIELDS) + (float(f["fitness"]),)


def test_tree_reduction():
    """Tree reduction: global in[0..255] read once each by its own thread
    and out[0] (unit 256) written by thread 0: 257 locations with one thread
    each.  Shared s[u], u >= 1: stored by thread u and read by thread
    u - s_k at the one level k where u is in [s_k, 2 s_k) (s[1] by thread 0
    at level 8): two threads; s[0] only by thread 0.  Sum g = 257 + 256 =
    513, sum f = 257 + 1 + 255 * 2 = 768, F = 513 / 768; global units span
    0..256, shared 0..255."""
    f = oracle.fitness(tracegen.tree_reduction(-1), tpb=256)[0]
    assert row(f) == (1279, 513, 768, 256, 255, 513 / 768)
    # barriers do not change which threads touch which addresses
    for k in range(9):
        assert row(oracle.fitness(tracegen.tree_reduction(k), tpb=256)[0])[1:] == row(f)[1:]


def test_paper_examples():
    # Sec. 3.4 kaldi pattern: threads 0..5 write out[0], out[1], out[2],
    # out[1], out[2], out[3]: 4 addresses, 6 (address, thread) pairs
    recs, tpb, _ = trace_fixture("kaldi_copy.txt")
    assert row(oracle.fitness(recs, tpb=tpb)[0]) == (6, 4, 6, 3, 0, 4 / 6)
    # Sec. 4.2.1 Memory Unit: threads 1, 2, 3 (3 twice) on one shared unit
    recs, tpb, _ = trace_fixture("fig6_unit.txt")
    assert row(oracle.fitness(recs, tpb=tpb)[0]) == (4, 1, 3, 0, 0, 1 / 3)


def test_closed_cases():
    # every thread its own addresses: F = 1 (no two threads share one)
    r = np.zeros(64, dtype=RECORD_DTYPE)
    r["tid"] = np.arange(64) // 4
    r["unit"] = np.arange(64) + 1000
    assert row(oracle.fitness(r, tpb=8)[0]) == (64, 64, 64, 63, 0, 1.0)
    # all T threads on one address: F = 1 / T
    r["unit"] = 7
    assert row(oracle.fitness(r, tpb=8)[0]) == (64, 1, 16, 0, 0, 1 / 16)
    # the same unit in shared memory of two blocks: two locations
    r["space"] = 1
    assert row(oracle.fitness(r, tpb=8)[0]) == (64, 2, 16, 0, 0, 2 / 16)
    # no records: F = 1, nothing accessed
    assert row(oracle.fitness(r[:0], tpb=8)[0]) == (0, 0, 0, 0, 0, 1.0)


def fitness_py(recs, tpb):
    locs, pairs = set(), set()
    g = [int(x["unit"]) for x in recs if int(x["space"]) == 0]
    s = [int(x["unit"]) for x in recs if int(x["space"]) == 1]
    for x in recs:
        u, t, sp = int(x["unit"]), int(x["tid"]), int(x["space"])
        loc = (sp, t // tpb if sp == 1 else None, u)
        locs.add(loc)
        pairs.add((loc, t))
    return (len(recs), len(locs), len(pairs), max(g) - min(g) if g else 0, max(s) - min(s) if s else 0,
            len(locs) / len(pairs) if pairs else 1.0)


@pytest.mark.parametrize("seed", range(30))
def test_matches_python_rendering_and_invariants(seed):
    rng = np.random.default_rng(700 + seed)
    tpb = int(rng.integers(1, 6))
    r = tracegen.random_small(rng, int(rng.integers(0, 120)), units=int(rng.integers(1, 9)),
                              blocks=int(rng.integers(1, 4)), tpb=tpb, epochs=3)
    want = fitness_py(r, tpb)
    assert row(oracle.fitness(r, tpb=tpb)[0]) == want
    # order, epochs, actions and repeated records do not matter
    p = r[rng.permutation(len(r))].copy()
    p["epoch"] = rng.integers(0, 9, len(p))
    p["action"] = rng.integers(0, 3, len(p))
    assert row(oracle.fitness(np.concatenate([p, p[: len(p) // 2]]), tpb=tpb)[0])[1:] == want[1:]


def test_batch_is_per_trace():
    traces = [tracegen.tree_reduction(-1), tracegen.c0()[:0], tracegen.c0()]
    recs = np.concatenate(traces)
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    got = oracle.fitness(recs, off, 256)
    for i, t in enumerate(traces):
        assert got[i].tobytes() == oracle.fitness(t, tpb=256)[0].tobytes()


MUTANTS = {
    "records_not_threads": ("if (new_loc || v[i].tid != v[i - 1].tid) f++;", "f++;"),
    "shared_not_per_block": ("v[i].lblock = r->space == 1 ? r->tid / tpb[tr] : 0xFFFFFFFFu;", "v[i].lblock = 0;"),
    "ratio_inverted": ("out[tr].fitness = f ? (double)g / (double)f : 1.0;",
                       "out[tr].fitness = g ? (double)f / (double)g : 1.0;"),
    "range_of_all_spaces": ("out[tr].shared_range = smin <= smax ? smax - smin : 0;",
                            "out[tr].shared_range = gmin <= gmax ? gmax - gmin : 0;"),
}


def _pins_pass():
    try:
        test_tree_reduction()
        test_paper_examples()
        test_closed_cases()
        for seed in range(10):
            test_matches_python_rendering_and_invariants(seed)
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_fitness_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c), "-o", str(so)], check=True)
    saved = oracle._load()
    mutant = ctypes.CDLL(so)
    f = mutant.orc_fitness_eval
    f.restype = saved.orc_fitness_eval.restype
    f.argtypes = saved.orc_fitness_eval.argtypes
    oracle._lib = mutant
    try:
        assert not _pins_pass(), f"mutant {name} survived every pin"
    finally:
        oracle._lib = saved
