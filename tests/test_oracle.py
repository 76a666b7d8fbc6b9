"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: the hand-written
truth table and trace fixtures under tests/golden/ (each citing the passage
it follows), hand-derived results on the tree-reduction family, invariants of
the race relation, exhaustive agreement between three separately written
renderings (C brute force, pure-Python brute force, C group-count closed
form), and the race-free-by-construction property of the generator.
"""
import numpy as np
import pytest

import oracle
import tracegen
from golden_io import counts_only, trace_fixture, truth_table
from tracegen import RECORD_DTYPE

FIXTURES = ["fig6_unit.txt", "fig6_unit_write.txt", "kaldi_copy.txt", "mixed_kinds.txt"]


def as_dict(races, trace=0):
    return oracle.races_to_dict(races, trace)


def with_kinds(races, trace=0):
    return oracle.races_to_dict(races, trace, kinds=True)


# ---------------------------------------------------------------- fixtures

@pytest.mark.parametrize("row", truth_table(), ids=lambda r: r[0] if isinstance(r, str) else None)
def test_truth_table(row):
    line, recs, exp = row
    for fn in (oracle.brute_force, oracle.closed_form):
        races, _ = fn(recs, tpb=2)
        assert with_kinds(races) == exp, (fn.__name__, line)
    assert oracle.tier_a_py(recs, 2) == counts_only(exp)


@pytest.mark.parametrize("name", FIXTURES)
def test_trace_fixtures(name):
    recs, tpb, exp = trace_fixture(name)
    for fn in (oracle.brute_force, oracle.closed_form):
        races, summ = fn(recs, tpb=tpb)
        assert with_kinds(races) == exp
        assert int(summ[0]["n_records"]) == len(recs)
        assert int(summ[0]["n_race_locs"]) == len(exp)
        assert int(summ[0]["n_pairs"]) == sum(d["ww"] + d["rw"] + d["aw"] + d["ar"] for d in exp.values())
    assert oracle.tier_a_py(recs, tpb) == counts_only(exp)


def test_kaldi_names_the_papers_thread_pair():
    # Sec. 3.4: threads (0 1 0) and (1 0 0) race (write & write).  With
    # block (3, 2) their linear ids are 0 + 3*1 = 3 and 1 + 3*0 = 1.
    recs, tpb, _ = trace_fixture("kaldi_copy.txt")
    writers = sorted(int(r["tid"]) for r in recs if int(r["unit"]) == 1)
    assert writers == [1, 3]
    races, _ = oracle.brute_force(recs, tpb=tpb)
    e = [r for r in races if int(r["unit"]) == 1][0]
    assert int(e["pairs_ww"]) == 1 and int(e["kinds"]) == 1


# --------------------------------------------------- tree reduction family

def test_tree_reduction_size():
    # 256 loads + 256 stores + 3 * (128 + 64 + ... + 1) + 2 final accesses
    assert len(tracegen.tree_reduction()) == 256 + 256 + 3 * 255 + 2 == 1279


@pytest.mark.parametrize("removed", list(range(-1, 9)))
def test_tree_reduction_family(removed):
    """Hand derivation: with barrier B_k (k < 8) missing, level k's (or the
    initial store's, k = 0) write of s[u] by thread u and level k+1's read of
    s[u] by thread u - stride_{k+1} share an epoch, for u in
    [128 >> k, 256 >> k): exactly 128 >> k shared entries with one read/write
    pair each.  Every other same-epoch pair on a shared word belongs to one
    thread.  Without B8 only thread 0 touches s[0] afterwards: no race.  With
    every barrier present there is no race (the barrier-fixes-race pattern of
    the paper's Sec. 2 examples)."""
    recs = tracegen.tree_reduction(removed)
    if 0 <= removed < 8:
        lo, hi = 128 >> removed, 256 >> removed
        exp = {(1, 0, u): {"ww": 0, "rw": 1, "aw": 0, "ar": 0, "xblock": 0} for u in range(lo, hi)}
    else:
        exp = {}
    a, _ = oracle.brute_force(recs, tpb=256)
    b, _ = oracle.closed_form(recs, tpb=256)
    assert as_dict(a) == exp
    assert as_dict(b) == exp
    assert (a == b).all()


def test_c0_is_tree_without_b2():
    races, summ = oracle.closed_form(tracegen.c0(), tpb=256)
    assert len(races) == 32
    assert list(races["unit"]) == list(range(32, 64))
    assert int(summ[0]["n_pairs"]) == 32


# ------------------------------------------------------- special cases

def test_one_thread_per_block_never_races():
    # Sec. 2 (redundant-barrier example): with one thread per block every
    # shared word is touched by a single thread.
    rng = np.random.default_rng(5)
    r = tracegen.random_small(rng, 300, units=3, blocks=1, tpb=1, epochs=3)
    for fn in (oracle.brute_force, oracle.closed_form):
        races, _ = fn(r, tpb=1)
        assert len(races) == 0


def test_all_reads_and_all_atomics_never_race():
    rng = np.random.default_rng(6)
    r = tracegen.random_small(rng, 500, units=2, blocks=2, tpb=4, epochs=2)
    r["action"] = 0
    assert len(oracle.closed_form(r, tpb=4)[0]) == 0
    r["action"] = 2
    assert len(oracle.closed_form(r, tpb=4)[0]) == 0


def test_empty_inputs():
    r = np.zeros(0, dtype=RECORD_DTYPE)
    races, summ = oracle.closed_form(r, offsets=[0], tpb=[])
    assert len(races) == 0 and len(summ) == 0
    races, summ = oracle.closed_form(r, offsets=[0, 0, 0], tpb=[3, 4])
    assert len(races) == 0 and list(summ["n_records"]) == [0, 0]


def test_invalid_records_are_rejected():
    r = tracegen.random_small(np.random.default_rng(1), 10)
    r["action"][7] = 3
    with pytest.raises(oracle.OracleError) as ei:
        oracle.closed_form(r, tpb=3)
    assert ei.value.code == -2 and ei.value.bad_index == 7
    r["action"][7] = 0
    r["space"][2] = 2
    with pytest.raises(oracle.OracleError) as ei:
        oracle.brute_force(r, tpb=3)
    assert ei.value.bad_index == 2
    with pytest.raises(oracle.OracleError):
        oracle.closed_form(r[:0], offsets=[0, 0], tpb=[0])


def test_pair_counts_large_group():
    """Closed form on a group too large to have been checked exhaustively:
    one global unit, 1 block of 64 threads, one epoch, every thread writes
    twice and reads three times.  Racing pairs by hand: writes 128, reads
    192; write/write pairs from different threads C(128,2) - 64 * C(2,2);
    read/write pairs 128 * 192 - 64 * (2 * 3)."""
    r = np.zeros(64 * 5, dtype=RECORD_DTYPE)
    i = 0
    for t in range(64):
        for a in (1, 1, 0, 0, 0):
            r[i] = (9, t, 0, a, 0)
            i += 1
    races, _ = oracle.closed_form(r, tpb=64)
    assert len(races) == 1
    assert int(races[0]["pairs_ww"]) == 128 * 127 // 2 - 64
    assert int(races[0]["pairs_rw"]) == 128 * 192 - 64 * 6
    assert int(races[0]["pairs_xblock"]) == 0
    br, _ = oracle.brute_force(r, tpb=64)
    assert (br == races).all()


# ---------------------------------------------- agreement of three tiers

@pytest.mark.parametrize("seed", range(60))
def test_three_tiers_agree_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 65))
    tpb = int(rng.integers(1, 5))
    r = tracegen.random_small(rng, n, units=int(rng.integers(1, 5)), blocks=int(rng.integers(1, 4)),
                              tpb=tpb, epochs=int(rng.integers(1, 4)))
    a, sa = oracle.brute_force(r, tpb=tpb)
    b, sb = oracle.closed_form(r, tpb=tpb)
    assert (a == b).all() and len(a) == len(b)
    assert (sa == sb).all()
    assert oracle.tier_a_py(r, tpb) == as_dict(a)


@pytest.mark.parametrize("seed", range(4))
def test_tiers_agree_medium(seed):
    rng = np.random.default_rng(100 + seed)
    r = tracegen.random_small(rng, 3000, units=40, blocks=4, tpb=8, epochs=4)
    a, _ = oracle.brute_force(r, tpb=8)
    b, _ = oracle.closed_form(r, tpb=8)
    assert len(a) > 0 and len(a) == len(b) and (a == b).all()


@pytest.mark.parametrize("seed", range(12))
def test_parallel_tier_b_equals_tier_b(seed):
    """The OpenMP driver of Tier B (by trace, and by location-hash bucket
    inside a trace) gives Tier B's result byte for byte: tiny random batches
    in bucket mode (bucket_min = 0) and trace mode, over 1 to 5 threads."""
    rng = np.random.default_rng(400 + seed)
    k = int(rng.integers(1, 6))
    traces = [tracegen.random_small(rng, int(rng.integers(0, 300)), units=int(rng.integers(1, 30)),
                                    blocks=int(rng.integers(1, 4)), tpb=4, epochs=3) for _ in range(k)]
    recs = np.concatenate(traces)
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    want, wsum = oracle.closed_form(recs, off, 4)
    for threads in (1, 2, 5):
        for bucket_min in (0, 100, 1 << 22):
            got, gsum = oracle.closed_form_par(recs, off, 4, threads=threads, bucket_min=bucket_min)
            assert got.tobytes() == want.tobytes(), (threads, bucket_min)
            assert gsum.tobytes() == wsum.tobytes()


def test_parallel_tier_b_on_generated_traces():
    """The same on a generated c1-shaped trace (64 blocks, 2^20 records,
    injected races) split into buckets, and on a batch of 40 traces."""
    r, _ = tracegen.c1(n_blocks=64, inject_rate=1e-3)
    want, wsum = oracle.closed_form(r, tpb=256)
    got, gsum = oracle.closed_form_par(r, tpb=256, threads=4, bucket_min=1 << 16)
    assert len(want) > 0 and got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes()
    shapes = tracegen.c3_shapes(40, log2_max=15)
    recs, off, tpb, _ = tracegen.batch(shapes, inject_rate=1e-3)
    want, wsum = oracle.closed_form(recs, off, tpb)
    got, gsum = oracle.closed_form_par(recs, off, tpb, threads=3, bucket_min=1 << 13)
    assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes()


def test_batched_equals_concatenation():
    rng = np.random.default_rng(11)
    traces = [tracegen.random_small(rng, int(rng.integers(0, 200)), units=6, blocks=3, tpb=3) for _ in range(7)]
    tpbs = [3, 3, 3, 3, 3, 3, 3]
    recs = np.concatenate(traces)
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    batch, summ = oracle.closed_form(recs, offsets=off, tpb=tpbs)
    parts = []
    for i, t in enumerate(traces):
        p, s = oracle.closed_form(t, tpb=3)
        p["trace"] = i
        parts.append(p)
        assert (summ[i] == s[0]).all()
    assert (np.concatenate(parts) == batch).all()


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("seed", range(8))
def test_permutation_invariance(seed):
    rng = np.random.default_rng(200 + seed)
    r = tracegen.random_small(rng, 2000, units=30, blocks=3, tpb=5, epochs=3)
    a, _ = oracle.closed_form(r, tpb=5)
    b, _ = oracle.closed_form(r[rng.permutation(len(r))], tpb=5)
    assert len(a) > 0 and (a == b).all()


def _straddling_racing_pairs(r, tpb, block, epoch, first_half):
    """Racing pairs of one block and epoch with one record on each side of a
    split (different threads, conflicting actions, same unit and space)."""
    idx = np.nonzero((r["tid"] // tpb == block) & (r["epoch"] == epoch))[0]
    cnt = 0
    for i in idx:
        for j in idx:
            if not (first_half[i] and not first_half[j]):
                continue
            x, y = r[i], r[j]
            if x["space"] != y["space"] or x["unit"] != y["unit"] or x["tid"] == y["tid"]:
                continue
            acts = {int(x["action"]), int(y["action"])}
            if acts == {0} or acts == {2}:
                continue
            cnt += 1
    return cnt


@pytest.mark.parametrize("seed", range(6))
def test_barrier_insertion_removes_exactly_the_straddling_pairs(seed):
    rng = np.random.default_rng(300 + seed)
    tpb = 4
    r = tracegen.random_small(rng, 400, units=5, blocks=2, tpb=tpb, epochs=3)
    block, epoch = 1, 1
    first = rng.random(len(r)) < 0.5
    before, _ = oracle.closed_form(r, tpb=tpb)
    s = r.copy()
    in_blk = s["tid"] // tpb == block
    # the barrier splits `epoch` of `block`: later epochs of the block move up
    s["epoch"][in_blk & (s["epoch"] > epoch)] += 1
    s["epoch"][in_blk & (s["epoch"] == epoch) & ~first] += 1
    after, _ = oracle.closed_form(s, tpb=tpb)
    tot = lambda x: int(sum(int(e["pairs_ww"] + e["pairs_rw"] + e["pairs_aw"] + e["pairs_ar"]) for e in x))
    removed = _straddling_racing_pairs(r, tpb, block, epoch, first)
    assert tot(before) - tot(after) == removed
    # never increases any per-location count
    d0, d1 = as_dict(before), as_dict(after)
    for k, v in d1.items():
        for kind in ("ww", "rw", "aw", "ar", "xblock"):
            assert v[kind] <= d0[k][kind]


@pytest.mark.parametrize("seed", range(6))
def test_barrier_removal_never_decreases(seed):
    rng = np.random.default_rng(400 + seed)
    r = tracegen.random_small(rng, 600, units=8, blocks=3, tpb=3, epochs=4)
    before = as_dict(oracle.closed_form(r, tpb=3)[0])
    s = r.copy()
    blk = s["tid"] // 3 == 2
    s["epoch"][blk & (s["epoch"] >= 2)] -= 1  # merge epochs 1 and 2 of block 2
    after = as_dict(oracle.closed_form(s, tpb=3)[0])
    for k, v in before.items():
        for kind in v:
            assert after[k][kind] >= v[kind]


@pytest.mark.parametrize("seed", range(4))
def test_relabelling(seed):
    rng = np.random.default_rng(500 + seed)
    tpb = 4
    r = tracegen.random_small(rng, 1500, units=20, blocks=3, tpb=tpb, epochs=3)
    base = as_dict(oracle.closed_form(r, tpb=tpb)[0])
    # bijective relabelling of units within each space
    perm = {0: rng.permutation(20) + 1000, 1: rng.permutation(20) + 77}
    s = r.copy()
    for sp in (0, 1):
        m = s["space"] == sp
        s["unit"][m] = perm[sp][r["unit"][m]]
    mapped = as_dict(oracle.closed_form(s, tpb=tpb)[0])
    assert mapped == {(k[0], k[1], int(perm[k[0]][k[2]])): v for k, v in base.items()}
    # relabelling thread ids inside each block (block kept)
    s = r.copy()
    local = rng.permutation(tpb)
    s["tid"] = (r["tid"] // tpb) * tpb + local[r["tid"] % tpb]
    assert as_dict(oracle.closed_form(s, tpb=tpb)[0]) == base


# ---------------------------------------------------------- generator

def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 published with Random123.
    assert tracegen.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert tracegen.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert tracegen.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                                  [0xA4093822, 0x299F31D0]) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_zipf_head_frequencies():
    n, s = 1 << 24, 1.1
    H = float(np.sum(np.arange(1, n + 1, dtype=np.float64) ** -s))
    draws = np.array([tracegen.zipf_rank(n, s, 77, i, 3) for i in range(20000)])
    assert draws.min() >= 1 and draws.max() <= n
    for k in (1, 2, 3):
        p = k ** -s / H
        f = float(np.mean(draws == k))
        assert abs(f - p) < 5 * np.sqrt(p * (1 - p) / len(draws)) + 1e-3, (k, f, p)


def test_generator_deterministic_and_thread_independent():
    a, la = tracegen.c1(n_blocks=8, inject_rate=1e-3, threads=1)
    b, lb = tracegen.c1(n_blocks=8, inject_rate=1e-3, threads=4)
    assert (a == b).all() and (la == lb).all()


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
def test_generator_race_free_without_injection(cfg):
    if cfg == "c1":
        r, _ = tracegen.c1(n_blocks=64, inject_rate=0.0)
        off, tpb = None, 256
    elif cfg == "c2":
        r, _ = tracegen.c2(n_blocks=16, inject_rate=0.0)
        off, tpb = None, 512
        assert np.mean(r["action"] == 2) > 0.03
    else:
        shapes = tracegen.c3_shapes(24, log2_max=15)
        r, off, tpb, _ = tracegen.batch(shapes, inject_rate=0.0)
    races, _ = oracle.closed_form(r, offsets=off, tpb=tpb)
    assert len(races) == 0


def test_injected_locations_are_found_and_spot_checked():
    r, inj = tracegen.c1(n_blocks=32, inject_rate=2e-4, seed=0x1234)
    races, _ = oracle.closed_form(r, tpb=256)
    got = as_dict(races)
    assert len(inj) == round(2e-4 * len(r))
    for e in inj:
        key = (int(e["space"]), int(e["block"]) if int(e["space"]) == 1 else None, int(e["unit"]))
        assert key in got
    # spot brute force: every racing location plus random others, on the
    # extracted records of that location
    rng = np.random.default_rng(3)
    blocks = r["tid"] // 256
    keys = list(got.keys())
    others = rng.choice(len(r), 64, replace=False)
    for i in others:
        keys.append((int(r["space"][i]), int(blocks[i]) if r["space"][i] == 1 else None, int(r["unit"][i])))
    for key in keys:
        sp, blk, unit = key
        m = (r["space"] == sp) & (r["unit"] == unit)
        if sp == 1:
            m &= blocks == blk
        sub = r[m]
        if len(sub) > 4096:
            continue
        bf, _ = oracle.brute_force(sub, tpb=256)
        assert as_dict(bf).get(key) == got.get(key)


def test_batch_injection_logs_stay_with_their_trace():
    """rate * n = 28.5 and 2.5: the generator rounds half away from zero;
    each trace's log holds exactly its own injections, and the oracle
    reports every logged location in that trace."""
    shapes = [(285000, 194, 6, 8434942963311516179), (25000, 3, 33, 77), (4096, 1, 16, 5)]
    recs, off, tpb, inj = tracegen.batch(shapes, inject_rate=1e-4)
    counts = [len(log) for _, log in inj]
    assert counts == [29, 3, 0]
    for i, log in inj:
        lo, hi = int(off[i]), int(off[i + 1])
        want, _ = oracle.closed_form(recs[lo:hi], tpb=256)
        for e in log:
            assert int(e["x_index"]) < hi - lo and int(e["y_index"]) < hi - lo
            hit = (want["unit"] == e["unit"]) & (want["space"] == e["space"])
            if int(e["space"]) == 1:
                hit &= want["block"] == e["block"]
            assert hit.any(), (i, e)
