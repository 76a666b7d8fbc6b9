"""GPU parity of the warp-aware race check (Theorem 1's warp clauses;
sim_check_traces_warp_device / sim_check_traces_warp, through the C ABI)
with the oracle, byte for byte.

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic; expected values come from oracle/ only."""
import numpy as np
import pytest

import oracle
import tracegen
from test_oracle_warp import Trace, warp_sync_reduction

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DIV = oracle.SD_DIVERGED


def say(msg):
    print(f"[gpu-warp] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1905_01833_amd as pkg

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    c.close()


def run_device(ctx, recs, side, offsets, tpb):
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    dside = torch.from_numpy(side.astype(np.uint32).view(np.int32)).to("cuda:0")
    got = ctx.check_traces_warp_device(dev, dside, offsets, tpb)
    torch.cuda.synchronize()
    return got


def check(ctx, recs, side, offsets, tpb, name):
    say(name)
    got, summ = run_device(ctx, recs, side, offsets, tpb)
    want, wsum = oracle.closed_form_warp(recs, side, offsets, tpb)
    assert got.tobytes() == want.tobytes(), name
    assert summ.tobytes() == wsum.tobytes(), name
    return got


def hand_patterns():
    out = {}
    out["reduction"] = warp_sync_reduction() + (64,)
    out["reduction_diverged"] = warp_sync_reduction(diverged=True) + (64,)
    out["half_warp"] = warp_sync_reduction(active=16, diverged=True) + (64,)
    tr = Trace()
    for stmt in (10, 11):
        for t in range(32):
            tr.add(0, t, 0, 1, 1, stmt)
    out["lanes_store_one_word"] = tr.arrays() + (32,)
    tr = Trace()
    for k in range(2):
        for t in range(32):
            tr.add(0, t, 0, 1, 1, 12)
    out["store_in_loop"] = tr.arrays() + (32,)
    tr = Trace()
    for t in range(32):
        tr.add(0, t, 0, 1 if t < 16 else 0, 1, 20 if t < 16 else 21, diverged=True)
    out["divergent_branch"] = tr.arrays() + (32,)
    tr = Trace()
    for k, t in enumerate((0, 31, 32, 48)):
        tr.add(0, t, 0, 1, 0, 30 + k)
    out["partial_warps"] = tr.arrays() + (48,)
    tr = Trace()
    for t in range(32):
        tr.add(5, t, 0, 2, 0, 40)
    tr.add(5, 1, 0, 0, 0, 41, diverged=True)
    out["atomics"] = tr.arrays() + (32,)
    return out


@pytest.mark.parametrize("name", sorted(hand_patterns()))
def test_hand_patterns(ctx, name):
    recs, side, tpb = hand_patterns()[name]
    check(ctx, recs, side, None, tpb, name)


def test_hand_patterns_batched(ctx):
    pats = hand_patterns()
    names = sorted(pats)
    recs = np.concatenate([pats[n][0] for n in names])
    side = np.concatenate([pats[n][1] for n in names])
    off = np.cumsum([0] + [len(pats[n][0]) for n in names]).astype(np.uint64)
    tpb = np.array([pats[n][2] for n in names], dtype=np.uint32)
    got = check(ctx, recs, side, off, tpb, "hand patterns in one call")
    # only the warp-synchronous reduction has no race left (the atomics
    # pattern's load ran diverged here)
    assert set(got["trace"].tolist()) == {i for i, n in enumerate(names) if n != "reduction"}


def random_batch(seed, n_traces):
    rng = np.random.default_rng(seed)
    recs, sides, sizes, tpbs = [], [], [], []
    for _ in range(n_traces):
        n = int(rng.integers(0, 80))
        tpb = int(rng.choice([1, 3, 32, 40, 48, 64, 100]))
        blocks = int(rng.integers(1, 3))
        r = np.zeros(n, dtype=tracegen.RECORD_DTYPE)
        r["unit"] = rng.integers(0, 3, n)
        r["tid"] = rng.integers(0, blocks * tpb, n)
        r["epoch"] = rng.integers(0, 2, n)
        r["action"] = rng.integers(0, 3, n)
        r["space"] = rng.integers(0, 2, n)
        s = rng.integers(0, int(rng.choice([1, 3, 1000])), n).astype(np.uint32)
        s |= np.where(rng.random(n) < 0.2, DIV, 0).astype(np.uint32)
        recs.append(r)
        sides.append(s)
        sizes.append(n)
        tpbs.append(tpb)
    off = np.cumsum([0] + sizes).astype(np.uint64)
    return np.concatenate(recs), np.concatenate(sides), off, np.array(tpbs, dtype=np.uint32)


@pytest.mark.parametrize("seed", range(4))
def test_random_tiny_batch(ctx, seed):
    recs, side, off, tpb = random_batch(seed, 300)
    got = check(ctx, recs, side, off, tpb, f"random batch {seed}")
    # the brute force on a few traces as well
    for t in range(0, 300, 37):
        lo, hi = int(off[t]), int(off[t + 1])
        br, _ = oracle.brute_force_warp(recs[lo:hi], side[lo:hi], tpb=int(tpb[t]))
        mine = got[got["trace"] == t].copy()
        mine["trace"] = 0
        assert mine.tobytes() == br.tobytes()


def side_words(recs, seed, n_stmts=6, div_rate=0.1):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n_stmts, len(recs)).astype(np.uint32)
    return s | np.where(rng.random(len(recs)) < div_rate, DIV, 0).astype(np.uint32)


@pytest.mark.parametrize("n_blocks", [1, 3, 8])
def test_generated_traces_across_tiles(ctx, n_blocks):
    """Generated traces (several tiles and a ragged end) with many injected
    races: same-warp pairs among them are common."""
    recs, _ = tracegen.c1(n_blocks=n_blocks, inject_rate=2e-2, seed=77 + n_blocks)
    recs = recs[: len(recs) - 1234]
    side = side_words(recs, n_blocks)
    got = check(ctx, recs, side, None, 256, f"generated {n_blocks} blocks, {len(recs)} records")
    plain, _ = oracle.closed_form(recs, tpb=256)
    assert 0 < len(got) <= len(plain)


def test_all_diverged_equals_plain(ctx):
    recs, _ = tracegen.c1(n_blocks=4, inject_rate=1e-2, seed=5)
    side = side_words(recs, 5) | np.uint32(DIV)
    say("all diverged")
    got, _ = run_device(ctx, recs, side, None, 256)
    plain, _ = ctx.check_traces_device(torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0"), None, 256)
    torch.cuda.synchronize()
    assert got.tobytes() == plain.tobytes()


def test_two_word_keys(ctx):
    """A trace whose units span 2^60 words needs a two-word key; with the
    side field it stays one call."""
    recs, side, _ = warp_sync_reduction() + (64,)
    wide = recs.copy()
    wide["space"] = 0
    wide["unit"] = wide["unit"] * np.uint64(1 << 50) + np.uint64(7)
    both_r = np.concatenate([recs, wide])
    both_s = np.concatenate([side, side | np.uint32(DIV)])
    off = np.array([0, len(recs), len(both_r)], dtype=np.uint64)
    check(ctx, both_r, both_s, off, np.array([64, 64], dtype=np.uint32), "two-word keys")


def test_host_entry_point_equals_device(ctx):
    recs, side, off, tpb = random_batch(11, 100)
    say("host entry point")
    got_h = ctx.check_traces_warp(recs, side, off, tpb)
    got_d = run_device(ctx, recs, side, off, tpb)
    assert got_h[0].tobytes() == got_d[0].tobytes() and got_h[1].tobytes() == got_d[1].tobytes()


def test_plain_check_unchanged_after_warp_calls(ctx):
    """A context runs plain and warp-aware calls in turn (their keys differ
    in width); each result stays the oracle's."""
    recs, _ = tracegen.c1(n_blocks=2, inject_rate=1e-2, seed=9)
    side = side_words(recs, 9)
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    want_p, _ = oracle.closed_form(recs, tpb=256)
    want_w, _ = oracle.closed_form_warp(recs, side, tpb=256)
    say("plain / warp alternating")
    for _ in range(2):
        p, _ = ctx.check_traces_device(dev, None, 256)
        w, _ = run_device(ctx, recs, side, None, 256)
        assert p.tobytes() == want_p.tobytes() and w.tobytes() == want_w.tobytes()


def test_empty_and_errors(ctx):
    import paper_1905_01833_amd as pkg

    say("empty and errors")
    empty = np.zeros(0, dtype=tracegen.RECORD_DTYPE)
    races, summ = ctx.check_traces_warp(empty, np.zeros(0, dtype=np.uint32), np.array([0, 0], dtype=np.uint64), 32)
    assert len(races) == 0 and int(summ[0]["n_records"]) == 0
    recs, side, _ = hand_patterns()["divergent_branch"]
    with pytest.raises(ValueError):
        ctx.check_traces_warp(recs, side[:-1], None, 32)
    bad = recs.copy()
    bad[3]["action"] = 7
    with pytest.raises(pkg.SimError) as ei:
        ctx.check_traces_warp(bad, side, None, 32)
    assert ei.value.code == pkg.SIM_ERECORD
    lib = pkg.load()
    import ctypes

    out = ctypes.POINTER(pkg._Result)()
    off = np.array([0, len(recs)], dtype=np.uint64)
    tpb = np.array([32], dtype=np.uint32)
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    rc = lib.sim_check_traces_warp_device(ctx._ctx, ctypes.c_void_p(dev.data_ptr()), None, off.ctypes.data, 1,
                                          tpb.ctypes.data, None, ctypes.byref(out))
    assert rc == pkg.SIM_EINVAL
    # the context still works
    check(ctx, recs, side, None, 32, "after errors")


def test_c1_full_size(ctx):
    """The 2^24-record trace with synthetic side words (8 statements, 5 %
    diverged), whole entry list against the oracle."""
    recs, _ = tracegen.c1()
    side = side_words(recs, 123, n_stmts=8, div_rate=0.05)
    check(ctx, recs, side, None, 256, "c1 full size, 2^24 records")
