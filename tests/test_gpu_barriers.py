"""GPU parity of the redundant-barrier check (sim_check_sync_device /
sim_check_sync, through the C ABI) with the oracle, byte for byte, and of
the race list it returns beside it with the plain race check's.

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic; expected values come from oracle/ only."""
import numpy as np
import pytest

import oracle
import tracegen
from golden_io import barrier_fixture, trace_fixture
from tracegen import RECORD_DTYPE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_1905_01833_amd as pkg

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    c.close()


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def batch_of(traces):
    recs = np.concatenate(traces) if traces else np.zeros(0, dtype=RECORD_DTYPE)
    off = np.zeros(len(traces) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(t) for t in traces])
    return recs, off


def assert_sync_parity(ctx, recs, off, tpb, name, host=False):
    off = np.asarray(off, dtype=np.uint64)
    tpb = np.asarray(tpb, dtype=np.uint32)
    if tpb.ndim == 0:
        tpb = np.full(len(off) - 1, int(tpb), dtype=np.uint32)
    say(f"barriers {name}: {len(recs)} records, {len(off) - 1} traces")
    if host:
        races, summ, bars = ctx.check_sync(recs, off, tpb)
    else:
        dev = torch.from_numpy(np.ascontiguousarray(recs).view(np.uint8).reshape(-1, 16)).to("cuda:0")
        torch.cuda.synchronize()
        races, summ, bars = ctx.check_sync_device(dev, off, tpb)
        torch.cuda.synchronize()
    want = oracle.barriers(recs, off, tpb)
    assert len(bars) == len(want), (name, len(bars), len(want))
    assert bars.tobytes() == want.tobytes(), name
    wr, ws = oracle.closed_form(recs, off, tpb) if len(recs) <= (1 << 22) else oracle.closed_form_par(recs, off, tpb)
    assert races.tobytes() == wr.tobytes() and summ.tobytes() == ws.tobytes(), name
    return bars


def test_tree_family(ctx):
    traces = [tracegen.tree_reduction(k) for k in range(-1, 9)]
    recs, off = batch_of(traces)
    bars = assert_sync_parity(ctx, recs, off, 256, "tree family")
    full = bars[bars["trace"] == 0]
    assert [int(b["boundary"]) for b in full if int(b["racing"]) == 0] == [8]  # B8 is redundant


def test_hand_fixtures(ctx):
    for name in ("barriers_hand.txt",):
        recs, tpb, _ = barrier_fixture(name)
        assert_sync_parity(ctx, recs, np.array([0, len(recs)]), tpb, name)
    for name in ("fig6_unit.txt", "fig6_unit_write.txt", "kaldi_copy.txt", "mixed_kinds.txt"):
        recs, tpb, _ = trace_fixture(name)
        assert_sync_parity(ctx, recs, np.array([0, len(recs)]), tpb, name)


def test_random_tiny_batch(ctx):
    rng = np.random.default_rng(71)
    traces, tpbs = [], []
    for _ in range(300):
        tpb = int(rng.integers(1, 6))
        traces.append(tracegen.random_small(rng, int(rng.integers(0, 150)), units=int(rng.integers(1, 6)),
                                            blocks=int(rng.integers(1, 4)), tpb=tpb, epochs=int(rng.integers(1, 6))))
        tpbs.append(tpb)
    recs, off = batch_of(traces)
    assert_sync_parity(ctx, recs, off, tpbs, "300 tiny traces")
    assert_sync_parity(ctx, recs, off, tpbs, "300 tiny traces, host records", host=True)


def test_generated_batch_and_tiles(ctx):
    shapes = tracegen.c3_shapes(64, log2_max=17)
    recs, off, tpb, _ = tracegen.batch(shapes, inject_rate=1e-3)
    bars = assert_sync_parity(ctx, recs, off, tpb, "64 generated traces")
    assert int(bars["racing"].sum()) > 0
    # one location across many tiles and epochs: a long run on both sides
    n = 60000
    r = np.zeros(n, dtype=RECORD_DTYPE)
    r["unit"] = 5
    r["tid"] = np.arange(n) % 256
    r["epoch"] = np.arange(n) // 6000
    r["action"] = (np.arange(n) % 7 == 0).astype(np.uint8)
    assert_sync_parity(ctx, r, np.array([0, n]), 256, "one location, 10 epochs, 15 tiles")


def test_many_epochs(ctx):
    """Boundaries beyond the kernel's 256 LDS bins go straight to the
    counters in device memory."""
    rng = np.random.default_rng(5)
    n = 20000
    r = np.zeros(n, dtype=RECORD_DTYPE)
    r["unit"] = rng.integers(0, 40, n)
    r["tid"] = rng.integers(0, 64, n)
    r["epoch"] = rng.integers(0, 700, n)
    r["action"] = rng.integers(0, 3, n)
    r["space"] = rng.integers(0, 2, n)
    assert_sync_parity(ctx, r, np.array([0, n]), 32, "700 epochs")


def test_two_word_keys(ctx):
    rng = np.random.default_rng(8)
    r = np.zeros(5000, dtype=RECORD_DTYPE)
    pool = rng.integers(0, 1 << 62, 8, dtype=np.uint64)
    pool[0], pool[1] = 0, (1 << 62) - 1
    r["unit"] = pool[rng.integers(0, 8, len(r))]
    r["tid"] = rng.integers(0, 4 * 64, len(r))
    r["epoch"] = rng.integers(0, 4, len(r))
    r["action"] = rng.integers(0, 3, len(r))
    r["space"] = (rng.random(len(r)) < 0.3).astype(np.uint8)
    assert_sync_parity(ctx, r, np.array([0, len(r)]), 64, "two-word keys")


def test_c1_full_size(ctx):
    r, _ = tracegen.c1()
    assert_sync_parity(ctx, r, np.array([0, len(r)]), 256, "c1 full (2^24 records)")


def test_errors_and_empty(ctx):
    import paper_1905_01833_amd as pkg

    r = tracegen.c0().copy()
    r["space"][10] = 3
    dev = torch.from_numpy(r.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    say("barriers: invalid record")
    with pytest.raises(pkg.SimError) as ei:
        ctx.check_sync_device(dev, np.array([0, len(r)]), 256)
    assert ei.value.code == pkg.SIM_ERECORD
    say("barriers: empty call")
    races, summ, bars = ctx.check_sync(np.zeros(0, dtype=RECORD_DTYPE), np.array([0, 0]), 256)
    assert len(races) == 0 and len(bars) == 0 and len(summ) == 1
    assert_sync_parity(ctx, tracegen.c0(), np.array([0, 1279]), 256, "c0 after errors")
