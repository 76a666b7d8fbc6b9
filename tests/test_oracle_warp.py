"""Pins for the oracle's warp-aware race check (Theorem 1 with its warp
clauses (1)-(3); the race loop of Alg. 5), on the CPU.

Each record has a side word: the statement that made the access (bits 0-30)
and a divergence bit (bit 31, oracle.SD_DIVERGED).  A warp is 32 threads of
one block, by block-local id.  Checked against things other than the
oracle itself: counts derived by hand for short CUDA patterns (a
warp-synchronous reduction, lanes writing one word, a divergent branch,
partial warps), the plain check it refines (every divergence bit set gives
the plain result; the refinement only removes same-warp pairs), and
agreement of three separately written renderings (C brute force, C group
counts, pure Python).  Planted mistakes in copies of the oracle must each
fail a pin.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import tracegen

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
DIV = oracle.SD_DIVERGED


class Trace:
    """Records and side words of one hand-built trace."""

    def __init__(self):
        self.rows, self.side = [], []

    def add(self, unit, tid, epoch, action, space, stmt, diverged=False):
        self.rows.append((unit, tid, epoch, action, space))
        self.side.append(stmt | (DIV if diverged else 0))

    def arrays(self):
        r = np.zeros(len(self.rows), dtype=tracegen.RECORD_DTYPE)
        for i, (u, t, e, a, s) in enumerate(self.rows):
            r[i] = (u, t, e, a, s)
        return r, np.array(self.side, dtype=np.uint32)


def both(recs, side, tpb):
    a = oracle.races_to_dict(oracle.brute_force_warp(recs, side, tpb=tpb)[0], kinds=True)
    b = oracle.races_to_dict(oracle.closed_form_warp(recs, side, tpb=tpb)[0], kinds=True)
    assert a == b
    return a


def warp_sync_reduction(active=32, diverged=False):
    """The unrolled last-warp reduction over shared s[0..63], one block of
    64 threads.  Epoch 0: thread t stores s[t] (statement 0).  A barrier.
    Epoch 1: if (t < active) for d = 32, 16, 8, 4, 2, 1:
    s[t] = s[t] + s[t + d] -- a load of s[t], a load of s[t + d] and a store
    of s[t], three statements per step.  Threads 32..63 form the second
    warp and skip the branch."""
    tr = Trace()
    for t in range(64):
        tr.add(t, t, 0, 1, 1, 0)
    for k, d in enumerate((32, 16, 8, 4, 2, 1)):
        for t in range(active):
            tr.add(t, t, 1, 0, 1, 1 + 3 * k, diverged)
            tr.add(t + d, t, 1, 0, 1, 2 + 3 * k, diverged)
            tr.add(t, t, 1, 1, 1, 3 + 3 * k, diverged)
    return tr.arrays()


def test_warp_synchronous_reduction():
    """Plain check: s[u], u < 32, is written by thread u at all six steps
    and read by thread u - d at step d for each d in {1, 2, 4, 8, 16} with
    d <= u; those reads pair with the six writes: 6 * #{d <= u} read/write
    pairs (u = 1: 6, 2-3: 12, 4-7: 18, 8-15: 24, 16-31: 30), 774 in all over
    31 words.  Warp-aware: all of these pairs are in one warp, without
    divergence, and made by different statements, so lockstep orders them:
    nothing races."""
    recs, side = warp_sync_reduction()
    plain = oracle.races_to_dict(oracle.brute_force(recs, tpb=64)[0])
    want = {}
    for u in range(1, 32):
        nd = sum(1 for d in (1, 2, 4, 8, 16) if d <= u)
        want[(1, 0, u)] = {"ww": 0, "rw": 6 * nd, "aw": 0, "ar": 0, "xblock": 0}
    assert plain == want
    assert sum(v["rw"] for v in want.values()) == 774
    assert both(recs, side, 64) == {}
    # every access diverged: the same pairs as the plain check
    recs, side = warp_sync_reduction(diverged=True)
    assert {k: {f: v[f] for f in ("ww", "rw", "aw", "ar", "xblock")} for k, v in both(recs, side, 64).items()} == want


def test_half_warp_branch_is_divergent():
    """if (t < 16) ...: half of warp 0 runs the reduction, so its accesses
    carry the divergence bit; the pairs are those of the plain check on the
    same accesses."""
    recs, side = warp_sync_reduction(active=16, diverged=True)
    plain = oracle.races_to_dict(oracle.closed_form(recs, tpb=64)[0])
    got = both(recs, side, 64)
    assert got and {k: {f: v[f] for f in ("ww", "rw", "aw", "ar", "xblock")} for k, v in got.items()} == plain


def test_one_word_written_by_every_lane():
    """Every lane of one warp stores s[0] by statement A, then by statement
    B, in one barrier interval.  Plain: 64 writes by 32 threads, pairs of
    different threads C(64,2) - 32 = 1984.  Warp-aware: lockstep orders
    A-B pairs; same-statement pairs stay races (clause 2): 2 * C(32,2) =
    992, write/write."""
    tr = Trace()
    for stmt in (10, 11):
        for t in range(32):
            tr.add(0, t, 0, 1, 1, stmt)
    recs, side = tr.arrays()
    assert oracle.races_to_dict(oracle.brute_force(recs, tpb=32)[0])[(1, 0, 0)]["ww"] == 1984
    assert both(recs, side, 32) == {(1, 0, 0): {"ww": 992, "rw": 0, "aw": 0, "ar": 0, "xblock": 0, "kinds": 1}}


def test_store_in_a_loop():
    """for (k = 0; k < 2; k++) s[0] = v; by every lane of one warp: one
    statement stores twice per thread.  Every pair of different threads is
    a same-statement store pair (clause 2), so the warp-aware count equals
    the plain one: C(64,2) - 32 = 1984 (a thread's own two stores never
    pair)."""
    tr = Trace()
    for k in range(2):
        for t in range(32):
            tr.add(0, t, 0, 1, 1, 12)
    recs, side = tr.arrays()
    assert both(recs, side, 32) == {(1, 0, 0): {"ww": 1984, "rw": 0, "aw": 0, "ar": 0, "xblock": 0, "kinds": 1}}


def test_two_warps_write_one_word():
    """The same two stores by 64 threads (two warps).  Plain: C(128,2) - 64
    = 8064.  Warp-aware: 992 inside each warp, and every pair across the
    two warps races (clause 1): 64 * 64 = 4096; 6080 in all."""
    tr = Trace()
    for stmt in (10, 11):
        for t in range(64):
            tr.add(0, t, 0, 1, 1, stmt)
    recs, side = tr.arrays()
    assert oracle.races_to_dict(oracle.brute_force(recs, tpb=64)[0])[(1, 0, 0)]["ww"] == 8064
    assert both(recs, side, 64)[(1, 0, 0)]["ww"] == 992 + 992 + 4096


def test_divergent_branch():
    """if (lane < 16) s[0] = x (statement A) else y = s[0] (statement B),
    one warp: the two sides ran diverged, so every pair of different
    threads races (clause 3): the 16 stores pairwise, C(16,2) = 120 (they
    also share a statement), and 16 x 16 = 256 store/load pairs.  Without
    the divergence bits only the same-statement stores would remain."""
    tr = Trace()
    for t in range(32):
        if t < 16:
            tr.add(0, t, 0, 1, 1, 20, diverged=True)
        else:
            tr.add(0, t, 0, 0, 1, 21, diverged=True)
    recs, side = tr.arrays()
    assert both(recs, side, 32) == {(1, 0, 0): {"ww": 120, "rw": 256, "aw": 0, "ar": 0, "xblock": 0, "kinds": 3}}
    assert both(recs, side & ~np.uint32(DIV), 32) == {
        (1, 0, 0): {"ww": 120, "rw": 0, "aw": 0, "ar": 0, "xblock": 0, "kinds": 1}}


def test_partial_warps_and_blocks():
    """48 threads per block: warp 0 is block-local 0..31, warp 1 is 32..47.
    Stores to global word 0, each by its own statement, no divergence, by
    threads 0 and 31 (block 0, warp 0), 32 (block 0, warp 1) and 48 (block
    1, local 0).  0-31: one warp, different statements: ordered.  0-32,
    31-32: different warps: 2 races.  48 with each of the other three:
    different blocks: 3 races, all cross-block.  5 write/write pairs, 3 of
    them cross-block."""
    tr = Trace()
    for k, t in enumerate((0, 31, 32, 48)):
        tr.add(0, t, 0, 1, 0, 30 + k)
    recs, side = tr.arrays()
    assert both(recs, side, 48) == {(0, None, 0): {"ww": 5, "rw": 0, "aw": 0, "ar": 0, "xblock": 3, "kinds": 17}}


def test_atomics_and_reads_in_one_warp():
    """One warp, no divergence: an atomic by lane 0 and a load by lane 1
    (different statements) are ordered; atomics of every lane by one
    statement never race each other (atomics only race plain accesses)."""
    tr = Trace()
    for t in range(32):
        tr.add(5, t, 0, 2, 0, 40)
    tr.add(5, 1, 0, 0, 0, 41)
    recs, side = tr.arrays()
    assert both(recs, side, 32) == {}
    side2 = side.copy()
    side2[-1] |= DIV  # the load ran diverged: it races with the 31 atomics of other lanes
    assert both(recs, side2, 32) == {(0, None, 5): {"ww": 0, "rw": 0, "aw": 0, "ar": 31, "xblock": 0, "kinds": 8}}


def random_warp_trace(rng, n):
    tpb = int(rng.choice([32, 40, 48, 64]))
    blocks = int(rng.integers(1, 3))
    r = np.zeros(n, dtype=tracegen.RECORD_DTYPE)
    r["unit"] = rng.integers(0, 3, n)
    r["tid"] = rng.integers(0, blocks * tpb, n)
    r["epoch"] = rng.integers(0, 2, n)
    r["action"] = rng.integers(0, 3, n)
    r["space"] = rng.integers(0, 2, n)
    side = (rng.integers(0, 3, n).astype(np.uint32) | np.where(rng.random(n) < 0.2, DIV, 0).astype(np.uint32))
    return r, side, tpb


@pytest.mark.parametrize("seed", range(40))
def test_three_renderings_agree(seed):
    rng = np.random.default_rng(seed)
    r, side, tpb = random_warp_trace(rng, int(rng.integers(0, 70)))
    want = oracle.tier_a_warp_py(r, side, tpb)
    assert oracle.races_to_dict(oracle.brute_force_warp(r, side, tpb=tpb)[0]) == want
    assert oracle.races_to_dict(oracle.closed_form_warp(r, side, tpb=tpb)[0]) == want


@pytest.mark.parametrize("seed", range(6))
def test_refines_the_plain_check(seed):
    """On generated traces (few blocks, so same-warp pairs are common): the
    warp-aware counts never exceed the plain ones, the cross-block counts
    are equal, and with every divergence bit set the result is the plain
    result."""
    recs, _ = tracegen.c1(n_blocks=2, inject_rate=3e-2, seed=1000 + seed)
    rng = np.random.default_rng(seed)
    side = rng.integers(0, 4, len(recs)).astype(np.uint32) | np.where(rng.random(len(recs)) < 0.1, DIV, 0).astype(
        np.uint32)
    plain = oracle.races_to_dict(oracle.closed_form(recs, tpb=256)[0])
    warp = oracle.races_to_dict(oracle.closed_form_warp(recs, side, tpb=256)[0])
    assert set(warp) <= set(plain) and plain
    for k, v in warp.items():
        for f in ("ww", "rw", "aw", "ar"):
            assert v[f] <= plain[k][f]
        assert v["xblock"] == plain[k]["xblock"]
    all_div = oracle.closed_form_warp(recs, side | np.uint32(DIV), tpb=256)
    assert all_div[0].tobytes() == oracle.closed_form(recs, tpb=256)[0].tobytes()
    assert len(oracle.closed_form_warp(recs, side, tpb=256)[0]) < len(plain) or any(
        warp[k] != plain[k] for k in warp)


def test_batches_number_their_traces():
    recs, side = warp_sync_reduction(diverged=True)
    r2, s2 = warp_sync_reduction()
    allr = np.concatenate([recs, r2, recs])
    alls = np.concatenate([side, s2, side])
    off = np.array([0, len(recs), len(recs) + len(r2), len(allr)], dtype=np.uint64)
    res, summ = oracle.closed_form_warp(allr, alls, off, tpb=[64, 64, 64])
    single, _ = oracle.closed_form_warp(recs, side, tpb=64)
    assert sorted(set(res["trace"].tolist())) == [0, 2]
    assert len(res) == 2 * len(single)
    assert [int(s["n_race_locs"]) for s in summ] == [31, 0, 31]


# ---------------------------------------------------------------- mutants

def _pins_pass():
    try:
        test_warp_synchronous_reduction()
        test_one_word_written_by_every_lane()
        test_store_in_a_loop()
        test_two_warps_write_one_word()
        test_divergent_branch()
        test_partial_warps_and_blocks()
        test_atomics_and_reads_in_one_warp()
        for seed in range(12):
            test_three_renderings_agree(seed)
    except AssertionError:
        return False
    return True


MUTANTS = {
    "warp_of_64": ("#define WARP_SIZE 32u", "#define WARP_SIZE 64u"),
    "brute_divergence_ignored": ("const int diverged = ((sd[i] | sd[j]) & SD_DIVERGED) != 0;",
                                 "const int diverged = 0;"),
    "closed_divergence_ignored": ("if (!(w[b].sd & SD_DIVERGED)) {", "if (1) {"),
    "brute_same_stmt_any_action": ("const int same_stmt_writes = x->action == 1 && y->action == 1 &&",
                                   "const int same_stmt_writes = 1 &&"),
    "warp_ignores_block": ("return t1 / T == t2 / T && (t1 % T) / WARP_SIZE == (t2 % T) / WARP_SIZE;",
                           "return (t1 % T) / WARP_SIZE == (t2 % T) / WARP_SIZE;"),
    "closed_same_stmt_not_kept": ("rem[KIND_WW] -= keep;", ""),
    "closed_thread_term_dropped": ("rem[k] = tmp[k] - sumT[k];", "rem[k] = tmp[k];"),
    "closed_keep_counts_same_thread": ("keep -= c2(d - c);", ""),
}


def _build_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mut = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mut)
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c), "-o", str(so)], check=True)
    return str(so)


def test_real_oracle_passes_warp_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_warp_mutant_is_caught(name, tmp_path):
    so = _build_mutant(name, tmp_path)
    saved = oracle._load()
    mutant = ctypes.CDLL(so)
    for fname in ("orc_brute_force", "orc_closed_form", "orc_brute_force_warp", "orc_closed_form_warp"):
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
