"""GPU parity of the radix sort's digit widths: passes after the first with
8-bit or 9-bit digits (sim_tuning.digit_bits forces one; by default a call
takes 9 bits where the previous call's widest key sorts in fewer passes
with them).  Every check goes through the C ABI and compares with the
oracle byte for byte: the race entries and summaries, the redundant-barrier
rows, the fitness rows and the warp-aware entries.

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic; expected values come from oracle/ only."""
import numpy as np
import pytest

import oracle
import tracegen
from tracegen import RECORD_DTYPE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-digits] {msg}", flush=True)


@pytest.fixture(scope="module")
def pkg():
    import paper_1905_01833_amd as p

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return p


@pytest.fixture(scope="module")
def ctx(pkg):
    c = pkg.Context(0)
    yield c
    c.close()


def to_dev(recs):
    return torch.from_numpy(np.ascontiguousarray(recs).view(np.uint8).reshape(-1, 16)).to("cuda:0")


class forced:
    """Force the digit width of one context for calls of n records."""

    def __init__(self, pkg, ctx, n, bits):
        self.ctx, self.cls, self.bits = ctx, pkg.sim_size_class(n), bits

    def __enter__(self):
        self.ctx.set_tuning(self.cls, {"digit_bits": self.bits})

    def __exit__(self, *exc):
        self.ctx.set_tuning(self.cls, None)


def mixed_batch():
    """Short traces (sorted whole in LDS) beside a 32-block trace of several
    hundred tiles whose keys sort 41 bits (six 8-bit passes, five with
    9-bit digits after the first) and a ragged end."""
    shapes = tracegen.c3_shapes(48, log2_max=15, seed=11)
    small, off, tpb, _ = tracegen.batch(shapes, inject_rate=5e-4)
    big, _ = tracegen.c1(n_blocks=32, inject_rate=5e-4, seed=21)
    big = big[: len(big) - 777]
    recs = np.concatenate([small, big])
    off = np.concatenate([off, [off[-1] + len(big)]]).astype(np.uint64)
    tpb = np.concatenate([tpb, [256]]).astype(np.uint32)
    return recs, off, tpb


@pytest.mark.parametrize("bits", [8, 9])
def test_forced_width_batched(pkg, ctx, bits):
    recs, off, tpb = mixed_batch()
    want, wsum = oracle.closed_form(recs, off, tpb)
    dev = to_dev(recs)
    with forced(pkg, ctx, len(recs), bits):
        for rep in range(2):
            say(f"batched, {bits}-bit digits, call {rep}")
            got, gsum = ctx.check_traces_device(dev, off, tpb)
            torch.cuda.synchronize()
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), (bits, rep)
        say(f"batched, {bits}-bit digits, host entry point")
        got, gsum = ctx.check_traces(recs, off, tpb)
        assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes()


@pytest.mark.parametrize("bits", [8, 9])
def test_forced_width_unfused_first_pass(pkg, ctx, bits):
    """200 threads per block: the first pass is key generation's digit
    histogram plus an 8-bit scatter, then passes of the forced width."""
    recs, _ = tracegen.generate(24, 200, 64, inject_rate=1e-3, seed=31)
    recs = recs[: len(recs) - 1001]
    say(f"200 threads per block, {bits}-bit digits, {len(recs)} records")
    want, wsum = oracle.closed_form(recs, None, 200)
    with forced(pkg, ctx, len(recs), bits):
        got, gsum = ctx.check_traces_device(to_dev(recs), None, 200)
        torch.cuda.synchronize()
    assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes()


@pytest.mark.parametrize("bits", [8, 9])
def test_forced_width_two_word_keys(pkg, ctx, bits):
    """Global units spread over 2^61 words: 77-bit keys (75 bits sorted), two
    words, ten 8-bit passes or nine with 9-bit digits after the first."""
    recs, _ = tracegen.c1(n_blocks=8, inject_rate=1e-3, seed=41)
    g = recs["space"] == 0
    recs["unit"][g] = recs["unit"][g] * np.uint64(1 << 36) + np.uint64(3)
    say(f"two-word keys, {bits}-bit digits, {len(recs)} records")
    want, wsum = oracle.closed_form(recs, None, 256)
    with forced(pkg, ctx, len(recs), bits):
        for rep in range(2):  # the first call finds it needs two-word keys and runs again
            got, gsum = ctx.check_traces_device(to_dev(recs), None, 256)
            torch.cuda.synchronize()
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), rep


@pytest.mark.parametrize("bits", [8, 9])
def test_forced_width_adjacent_checks(pkg, ctx, bits):
    """The redundant-barrier rows, the fitness rows and the warp-aware
    entries, all over keys sorted with the forced width."""
    recs, off, tpb = mixed_batch()
    dev = to_dev(recs)
    with forced(pkg, ctx, len(recs), bits):
        say(f"barrier check, {bits}-bit digits")
        races, summ, bars = ctx.check_sync_device(dev, off, tpb)
        torch.cuda.synchronize()
        assert bars.tobytes() == oracle.barriers(recs, off, tpb).tobytes()
        wr, ws = oracle.closed_form(recs, off, tpb)
        assert races.tobytes() == wr.tobytes() and summ.tobytes() == ws.tobytes()
        say(f"fitness, {bits}-bit digits")
        fit = ctx.eval_fitness_device(dev, off, tpb)
        torch.cuda.synchronize()
        assert fit.tobytes() == oracle.fitness(recs, off, tpb).tobytes()
        rng = np.random.default_rng(bits)
        side = rng.integers(0, 8, len(recs)).astype(np.uint32)
        side |= np.where(rng.random(len(recs)) < 0.05, oracle.SD_DIVERGED, 0).astype(np.uint32)
        say(f"warp-aware check, {bits}-bit digits")
        dside = torch.from_numpy(side.view(np.int32)).to("cuda:0")
        got, gsum = ctx.check_traces_warp_device(dev, dside, off, tpb)
        torch.cuda.synchronize()
        want, wsum = oracle.closed_form_warp(recs, side, off, tpb)
        assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes()


def test_automatic_width_saves_a_pass(pkg):
    """By default a context's first call sorts with 8-bit digits; the next
    call on keys of the same width (41 bits here) takes 9-bit digits and one
    global pass fewer.  Both results are the oracle's."""
    recs, _ = tracegen.c1(n_blocks=32, inject_rate=5e-4, seed=51)
    want, wsum = oracle.closed_form(recs, None, 256)
    dev = to_dev(recs)
    c = pkg.Context(0, profile=True)
    try:
        passes = []
        for rep in range(3):
            say(f"automatic width, call {rep}")
            got, gsum = c.check_traces_device(dev, None, 256)
            torch.cuda.synchronize()
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), rep
            passes.append(c.stage_times()["sort_pass"][1])
        # pass 0 is key generation's; then five 8-bit passes, or four 9-bit ones
        assert passes == [5, 4, 4], passes
    finally:
        c.close()


def test_graph_replays_with_nine_bit_digits(pkg):
    """Graph capture and replays of calls that sort with 9-bit digits, and
    a call of another key width in between (its own width and graph)."""
    recs, off, tpb = mixed_batch()
    want, wsum = oracle.closed_form(recs, off, tpb)
    other, _ = tracegen.c1(n_blocks=4, inject_rate=1e-3, seed=61)
    want_o, wsum_o = oracle.closed_form(other, None, 256)
    dev, dev_o = to_dev(recs), to_dev(other)
    c = pkg.Context(0, graphs=True)
    try:
        stream = torch.cuda.Stream()
        for rep in range(5):
            say(f"graph replay {rep}")
            with torch.cuda.stream(stream):
                got, gsum = c.check_traces_device(dev, off, tpb, stream=stream.cuda_stream)
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), rep
            if rep == 2:
                with torch.cuda.stream(stream):
                    got, gsum = c.check_traces_device(dev_o, None, 256, stream=stream.cuda_stream)
                assert got.tobytes() == want_o.tobytes() and gsum.tobytes() == wsum_o.tobytes()
    finally:
        c.close()


def test_tuning_rejects_other_widths(pkg, ctx):
    say("digit width out of range")
    for bad in (7, 10, 16):
        with pytest.raises(pkg.SimError) as ei:
            ctx.set_tuning(20, {"digit_bits": bad})
        assert ei.value.code == pkg.SIM_EINVAL
    ctx.set_tuning(20, {"digit_bits": 9})
    is_set, t = ctx.tuning(20)
    assert is_set and t["digit_bits"] == 9
    ctx.set_tuning(20, None)
    empty = np.zeros(0, dtype=RECORD_DTYPE)
    races, summ = ctx.check_traces(empty, np.array([0, 0], dtype=np.uint64), 256)
    assert len(races) == 0
