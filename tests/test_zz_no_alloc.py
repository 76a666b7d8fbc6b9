"""The no-allocation entry point (sim_check_traces_device_noalloc) against
the ordinary one (sim_check_traces_device), both through the C ABI: the
same entries and summaries, bit for bit, on calls in a row whose inputs
shrink (the scratch keeps the previous call's contents), and the oracle
beside them.  Also its limits: a caller buffer that is too small, and a
call that does not fit the scratch."""
import numpy as np
import pytest

import oracle
import tracegen
from tracegen import RECORD_DTYPE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def pkg():
    import paper_1905_01833_amd as p

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return p


def on_device(recs):
    return torch.from_numpy(np.ascontiguousarray(recs).view(np.uint8).reshape(-1, 16)).to("cuda:0")


def both(ctx, recs, off, tpb, name, cap=1 << 20):
    say(f"no-alloc {name}: {len(recs)} records, {len(off) - 1} traces")
    dev = on_device(recs)
    torch.cuda.synchronize()
    want, wsum = ctx.check_traces_device(dev, off, tpb)
    got, gsum = ctx.check_traces_device_noalloc(dev, off, tpb, races_cap=cap)
    torch.cuda.synchronize()
    assert len(got) == len(want), (name, len(got), len(want))
    assert got.tobytes() == want.tobytes(), name
    assert gsum.tobytes() == wsum.tobytes(), name
    return got, gsum


def test_noalloc_equals_ordinary_entry_point(pkg):
    ctx = pkg.Context(0)
    try:
        # 1: one c1-shaped trace of 2^22 records (256 blocks x 256 threads)
        r1, _ = tracegen.c1(n_blocks=256, inject_rate=1e-4)
        off1 = np.array([0, len(r1)], dtype=np.uint64)
        got1, _ = both(ctx, r1, off1, np.array([256], dtype=np.uint32), "2^22-record trace")
        assert len(got1) > 0
        # 2: a smaller call of 48 traces of uneven size
        shapes = tracegen.c3_shapes(48, log2_max=16)
        r2, off2, tpb2, _ = tracegen.batch(shapes, inject_rate=5e-4)
        got2, gsum2 = both(ctx, r2, off2, tpb2, "48 traces")
        want2, wsum2 = oracle.closed_form(r2, off2, tpb2)
        assert got2.tobytes() == want2.tobytes() and gsum2.tobytes() == wsum2.tobytes()
        # 3: smaller still -- the tree reduction (one tile, sorted in LDS)
        r3 = tracegen.c0()
        got3, _ = both(ctx, r3, np.array([0, len(r3)], dtype=np.uint64), np.array([256], dtype=np.uint32), "c0")
        assert len(got3) == 32
    finally:
        ctx.close()


def test_noalloc_staging_overflow_and_repeats(pkg):
    # 150k locations with one write/write pair each: tiles hold more racing
    # locations than their key slices, so the call stages in the scratch
    n = 150000
    r = np.zeros(2 * n, dtype=RECORD_DTYPE)
    r["unit"] = np.repeat(np.arange(n, dtype=np.uint64) * 3, 2)
    r["tid"] = np.tile([0, 1], n)
    r["action"] = 1
    off = np.array([0, len(r)], dtype=np.uint64)
    ctx = pkg.Context(0)
    try:
        got, _ = both(ctx, r, off, np.array([2], dtype=np.uint32), "150k racing locations")
        assert len(got) == n
        small = r[: 2 * 1000]
        got, _ = both(ctx, small, np.array([0, len(small)], dtype=np.uint64), np.array([2], dtype=np.uint32),
                      "1000 racing locations after 150k")
        assert len(got) == 1000
    finally:
        ctx.close()


def test_noalloc_limits(pkg):
    ctx = pkg.Context(0)
    try:
        # the caller's buffer holds fewer entries than the call has
        r = tracegen.c0()
        dev = on_device(r)
        off = np.array([0, len(r)], dtype=np.uint64)
        say("no-alloc: output buffer of 10 entries for 32")
        with pytest.raises(pkg.SimError) as ei:
            ctx.check_traces_device_noalloc(dev, off, 256, races_cap=10)
        assert ei.value.code == pkg.SIM_ENOSPC and ei.value.n_races == 32
        # the context still works, and a large enough buffer gets the entries
        got, _ = ctx.check_traces_device_noalloc(dev, off, 256, races_cap=32)
        assert len(got) == 32
        # calls beyond the limits are refused on the host before anything
        # runs (the records are real device memory all the same: 2^24 zero
        # records, valid ones)
        big = 1 << 24
        zeros = torch.zeros(big * 16, dtype=torch.uint8, device="cuda:0")
        torch.cuda.synchronize()
        say("no-alloc: 2^24 records, beyond the scratch")
        with pytest.raises(pkg.SimError) as ei:
            ctx.check_traces_device_noalloc(zeros, np.array([0, big], dtype=np.uint64), 256)
        assert ei.value.code == pkg.SIM_EINVAL and "scratch" in str(ei.value)
        say("no-alloc: 4097 traces, beyond the trace limit")
        with pytest.raises(pkg.SimError) as ei:
            ctx.check_traces_device_noalloc(zeros[: 4097 * 16], np.arange(0, 4098, dtype=np.uint64), 256)
        assert ei.value.code == pkg.SIM_EINVAL and "traces" in str(ei.value)
        del zeros
        got, _ = ctx.check_traces_device_noalloc(dev, off, 256)
        assert len(got) == 32
    finally:
        ctx.close()
