"""Pins for the oracle's redundant-barrier check (Alg. 5, second loop;
Sec. 4.2.3), on the CPU.

Checked against things other than itself: hand-derived results on the
tree-reduction family and on hand-built fixtures, the relation to the race
check (removing a barrier adds exactly the races its racing instances
predict), and agreement of three separately written renderings (C brute
force over all pairs, C grouped by location / block / epoch, pure Python).
Planted mistakes in copies of the oracle must each fail a pin.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import tracegen
from golden_io import barrier_fixture, trace_fixture

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


def as_dict(res):
    return oracle.barriers_to_dict(res)


def both(recs, tpb):
    a = oracle.barriers_brute_force(recs, tpb=tpb)
    b = oracle.barriers(recs, tpb=tpb)
    return a, b


# ------------------------------------------------------ hand-derived cases

def test_tree_reduction_all_barriers():
    """Tree reduction with every barrier (B0 after the initial stores, B_k
    after level k).  Boundary 0: every shared unit is touched on both sides
    (256 instances); units 128..255 are written by thread u and read by
    thread u - 128 at level 1 (128 racing).  Boundary k = 1..7: level k
    touches units [0, 2 s_k), level k + 1 units [0, s_k) with s_k = 256 >> k
    (s_k instances); units [s_k / 2, s_k) are written by thread u at level k
    and read by thread u - s_k / 2 at level k + 1 (128 >> k racing); below
    s_k / 2 the same thread reads and writes.  Boundary 8: only s[0] is on
    both sides, touched by thread 0 alone -- B8 is the redundant barrier."""
    r = tracegen.tree_reduction(-1)
    want = {k: (256 >> k, 128 >> k) for k in range(8)}
    want[8] = (1, 0)
    a, b = both(r, 256)
    assert as_dict(a) == want
    assert as_dict(b) == want
    assert oracle.barriers_py(r, 256) == want
    redundant = [int(e["boundary"]) for e in b if int(e["racing"]) == 0]
    assert redundant == [8]


@pytest.mark.parametrize("removed", range(8))
def test_tree_reduction_racing_instances_are_the_races_of_removal(removed):
    """Removing B_k from the tree reduction creates exactly 128 >> k racing
    locations (the race check's pin); with B_k present, boundary k has
    exactly that many racing instances, on the same units."""
    full = tracegen.tree_reduction(-1)
    races, _ = oracle.closed_form(tracegen.tree_reduction(removed), tpb=256)
    assert len(races) == 128 >> removed
    b = oracle.barriers(full, tpb=256)
    assert as_dict(b)[removed][1] == len(races)


def test_hand_fixture():
    recs, tpb, want = barrier_fixture("barriers_hand.txt")
    a, b = both(recs, tpb)
    assert as_dict(a) == want
    assert as_dict(b) == want
    assert oracle.barriers_py(recs, tpb) == want


def test_memory_unit_example():
    """Sec. 4.2.1's Memory Unit (reads of threads 1, 2, 3 at visit order 0,
    thread 3 again at 1): one instance of boundary 0, not racing; with
    thread 2 writing instead, the write races with thread 3's later read."""
    recs, tpb, _ = trace_fixture("fig6_unit.txt")
    assert as_dict(oracle.barriers(recs, tpb=tpb)) == {0: (1, 0)}
    recs, tpb, _ = trace_fixture("fig6_unit_write.txt")
    assert as_dict(oracle.barriers(recs, tpb=tpb)) == {0: (1, 1)}
    assert oracle.barriers_py(recs, tpb) == {0: (1, 1)}


def test_single_epoch_and_empty():
    r = tracegen.random_small(np.random.default_rng(3), 50, units=3, blocks=2, tpb=4, epochs=1)
    assert len(oracle.barriers(r, tpb=4)) == 0
    assert len(oracle.barriers(r[:0], tpb=4)) == 0


def test_batches_number_their_traces():
    traces = [tracegen.tree_reduction(-1), tracegen.c0(), tracegen.tree_reduction(-1)[:10]]
    recs = np.concatenate(traces)
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    res = oracle.barriers(recs, off, 256)
    for i, t in enumerate(traces):
        mine = res[res["trace"] == i].copy()
        alone = oracle.barriers(t, tpb=256)
        alone["trace"] = i
        assert mine.tobytes() == alone.tobytes()


# --------------------------------------------------- three renderings agree

@pytest.mark.parametrize("seed", range(60))
def test_three_renderings_agree(seed):
    rng = np.random.default_rng(900 + seed)
    tpb = int(rng.integers(1, 5))
    r = tracegen.random_small(rng, int(rng.integers(0, 80)), units=int(rng.integers(1, 5)),
                              blocks=int(rng.integers(1, 4)), tpb=tpb, epochs=int(rng.integers(1, 5)))
    a, b = both(r, tpb)
    assert a.tobytes() == b.tobytes()
    assert as_dict(b) == oracle.barriers_py(r, tpb)


# --------------------------- relation to the race check: removing a barrier

def remove_boundary(recs, b):
    """The trace with the barrier at boundary b taken out (every block):
    epochs above b move down by one."""
    r = recs.copy()
    up = r["epoch"] > b
    r["epoch"][up] -= 1
    return r


@pytest.mark.parametrize("seed", range(30))
def test_removing_a_barrier_adds_the_predicted_races(seed):
    """One block: the locations whose racing-pair count grows when the
    barrier at boundary b is removed are exactly as many as the racing
    instances of b (each location has at most one instance of b)."""
    rng = np.random.default_rng(1300 + seed)
    tpb = 8
    r = tracegen.random_small(rng, int(rng.integers(10, 120)), units=int(rng.integers(2, 8)), blocks=1, tpb=tpb,
                              epochs=int(rng.integers(2, 5)))
    base, _ = oracle.closed_form(r, tpb=tpb)
    base_pairs = {k: sum(v[f] for f in ("ww", "rw", "aw", "ar")) for k, v in oracle.races_to_dict(base).items()}
    got = as_dict(oracle.barriers(r, tpb=tpb))
    for b in range(int(r["epoch"].max()) if len(r) else 0):
        merged, _ = oracle.closed_form(remove_boundary(r, b), tpb=tpb)
        grew = 0
        for k, v in oracle.races_to_dict(merged).items():
            if sum(v[f] for f in ("ww", "rw", "aw", "ar")) > base_pairs.get(k, 0):
                grew += 1
        assert got.get(b, (0, 0))[1] == grew, (seed, b)


# ---------------------------------------------------------------- mutants

MUTANTS = {
    "brute_any_later_epoch": ("if ((uint32_t)y->epoch != (uint32_t)x->epoch + 1) continue;",
                              "if ((uint32_t)y->epoch <= (uint32_t)x->epoch) continue;"),
    "brute_cross_block": ("if (bx != by || x->space != y->space || x->unit != y->unit) continue;",
                          "if (x->space != y->space || x->unit != y->unit) continue;"),
    "brute_same_thread_races": ("h.racing = (x->tid != y->tid && conflicts(x->action, y->action)) ? 1u : 0u;",
                                "h.racing = conflicts(x->action, y->action) ? 1u : 0u;"),
    "brute_reads_race": ("h.racing = (x->tid != y->tid && conflicts(x->action, y->action)) ? 1u : 0u;",
                         "h.racing = (x->tid != y->tid) ? 1u : 0u;"),
    "grouped_any_next_epoch": ("(uint32_t)it[g1].epoch == (uint32_t)it[g0].epoch + 1) {",
                               "(uint32_t)it[g1].epoch > (uint32_t)it[g0].epoch) {"),
    "grouped_ignores_block": ("if (g1 < n && same_loc(&it[g1], &it[g0]) && it[g1].block == it[g0].block &&",
                              "if (g1 < n && same_loc(&it[g1], &it[g0]) &&"),
    "grouped_same_thread_races": ("if (it[a].tid != it[b].tid && conflicts(it[a].action, it[b].action)) racing = 1;",
                                  "if (conflicts(it[a].action, it[b].action)) racing = 1;"),
    "count_racing_as_instances": ("      e.racing += racing;", "      e.racing += 1;"),
    "instances_from_racing": ("      e.instances++;", "      e.instances += racing;"),
    "boundary_of_later_epoch": ("        h.boundary = x->epoch;", "        h.boundary = y->epoch;"),
}


def _pins_pass():
    r = tracegen.tree_reduction(-1)
    want = {k: (256 >> k, 128 >> k) for k in range(8)}
    want[8] = (1, 0)
    for fn in (oracle.barriers_brute_force, oracle.barriers):
        if as_dict(fn(r, tpb=256)) != want:
            return False
    recs, tpb, want = barrier_fixture("barriers_hand.txt")
    for fn in (oracle.barriers_brute_force, oracle.barriers):
        if as_dict(fn(recs, tpb=tpb)) != want:
            return False
    for seed in range(20):
        rng = np.random.default_rng(900 + seed)
        tpb = int(rng.integers(1, 5))
        r = tracegen.random_small(rng, int(rng.integers(0, 80)), units=int(rng.integers(1, 5)),
                                  blocks=int(rng.integers(1, 4)), tpb=tpb, epochs=int(rng.integers(1, 5)))
        want = oracle.barriers_py(r, tpb)
        for fn in (oracle.barriers_brute_force, oracle.barriers):
            if as_dict(fn(r, tpb=tpb)) != want:
                return False
    return True


def test_real_oracle_passes_barrier_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_barrier_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found once"
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c), "-o", str(so)], check=True)
    saved = oracle._load()
    mutant = ctypes.CDLL(so)
    for fname in ("orc_barriers_brute_force", "orc_barriers", "orc_brute_force", "orc_closed_form",
                  "orc_closed_form_par"):
        f = getattr(mutant, fname)
        f.restype = getattr(saved, fname).restype
        f.argtypes = getattr(saved, fname).argtypes
    mutant.orc_free.restype = None
    mutant.orc_free.argtypes = [ctypes.c_void_p]
    oracle._lib = mutant
    try:
        assert not _pins_pass(), f"mutant {name} survived every pin"
    finally:
        oracle._lib = saved
