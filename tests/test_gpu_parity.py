"""GPU parity: the HIP path (through the C ABI) against the oracle, bit-exact.

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic; expected values come from oracle/ only.
"""
import numpy as np
import pytest

import oracle
import tracegen
from golden_io import trace_fixture, truth_table
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


def run_device(ctx, recs, offsets, tpb):
    dev = torch.from_numpy(np.ascontiguousarray(recs).view(np.uint8).reshape(-1, 16)).to("cuda:0")
    races, summ = ctx.check_traces_device(dev, offsets, tpb)
    torch.cuda.synchronize()
    return races, summ


def assert_parity(ctx, recs, offsets=None, tpb=256, host=False, name=""):
    if offsets is None:
        offsets = np.array([0, len(recs)], dtype=np.uint64)
    offsets = np.asarray(offsets, dtype=np.uint64)
    tpb = np.asarray(tpb, dtype=np.uint32)
    if tpb.ndim == 0:
        tpb = np.full(len(offsets) - 1, int(tpb), dtype=np.uint32)
    say(f"{name}: {len(recs)} records, {len(offsets) - 1} traces")
    want, wsum = oracle.closed_form(recs, offsets, tpb)
    if host:
        got, gsum = ctx.check_traces(recs, offsets, tpb)
    else:
        got, gsum = run_device(ctx, recs, offsets, tpb)
    assert len(got) == len(want), (name, len(got), len(want))
    assert got.tobytes() == want.tobytes(), name
    assert gsum.tobytes() == wsum.tobytes(), name
    return got


def batch_of(traces):
    recs = np.concatenate(traces) if traces else np.zeros(0, dtype=RECORD_DTYPE)
    off = np.zeros(len(traces) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(t) for t in traces])
    return recs, off


# ------------------------------------------------------------- hand cases

def test_c0_tree_reduction(ctx):
    got = assert_parity(ctx, tracegen.c0(), tpb=256, name="c0")
    assert len(got) == 32 and list(got["unit"]) == list(range(32, 64))


def test_tree_family_batched(ctx):
    traces = [tracegen.tree_reduction(k) for k in range(-1, 9)]
    recs, off = batch_of(traces)
    got = assert_parity(ctx, recs, off, 256, name="tree family")
    per_trace = np.bincount(got["trace"], minlength=10)
    assert list(per_trace) == [0] + [128 >> k for k in range(8)] + [0]


def test_truth_table_batched(ctx):
    rows = truth_table()
    recs, off = batch_of([r for _, r, _ in rows])
    got = assert_parity(ctx, recs, off, 2, name="truth table")
    for i, (line, _, exp) in enumerate(rows):
        assert oracle.races_to_dict(got[got["trace"] == i], trace=i, kinds=True) == exp, line


@pytest.mark.parametrize("name", ["fig6_unit.txt", "fig6_unit_write.txt", "kaldi_copy.txt", "mixed_kinds.txt"])
def test_fixtures(ctx, name):
    recs, tpb, exp = trace_fixture(name)
    got = assert_parity(ctx, recs, tpb=tpb, name=name)
    assert oracle.races_to_dict(got, kinds=True) == exp


# ------------------------------------------------------------ random cases

def test_random_tiny_batch(ctx):
    rng = np.random.default_rng(1)
    traces, tpbs = [], []
    for _ in range(400):
        tpb = int(rng.integers(1, 5))
        traces.append(tracegen.random_small(rng, int(rng.integers(0, 65)), units=int(rng.integers(1, 5)),
                                            blocks=int(rng.integers(1, 4)), tpb=tpb, epochs=int(rng.integers(1, 4))))
        tpbs.append(tpb)
    recs, off = batch_of(traces)
    assert_parity(ctx, recs, off, tpbs, name="400 tiny traces")
    # the pairwise definition itself on a sample of them
    got, _ = ctx.check_traces(recs, off, tpbs)
    for i in range(0, 400, 37):
        bf, _ = oracle.brute_force(traces[i], tpb=tpbs[i])
        sub = got[got["trace"] == i].copy()
        sub["trace"] = 0
        assert sub.tobytes() == bf.tobytes()


@pytest.mark.parametrize("n", [4096 - 1, 4096, 4096 + 1, 3 * 4096 + 123, 10 * 4096 + 4095])
def test_tile_boundaries(ctx, n):
    rng = np.random.default_rng(n)
    r = tracegen.random_small(rng, n, units=50, blocks=5, tpb=7, epochs=4)
    assert_parity(ctx, r, tpb=7, name=f"ragged n={n}")


def test_host_entry_point(ctx):
    rng = np.random.default_rng(2)
    r = tracegen.random_small(rng, 20000, units=300, blocks=4, tpb=16, epochs=3)
    assert_parity(ctx, r, tpb=16, host=True, name="host records")


def test_mega_location(ctx):
    rng = np.random.default_rng(3)
    m = tracegen.random_small(rng, 60000, units=1, blocks=9, tpb=128, epochs=5)
    m["space"] = 0
    assert_parity(ctx, m, tpb=128, name="one global unit, 60k records")
    m["space"] = 1
    assert_parity(ctx, m, tpb=128, name="one shared unit per block, 60k records")


def test_uniform_groups(ctx):
    r = np.zeros(50000, dtype=RECORD_DTYPE)
    r["unit"] = 77
    r["tid"] = 5
    r["action"] = np.arange(50000) % 3
    got = assert_parity(ctx, r, tpb=32, name="one thread, one unit")
    assert len(got) == 0
    r["tid"][::2] = 6
    assert_parity(ctx, r, tpb=32, name="two threads, one unit")


def test_many_racing_locations_grow_output(ctx):
    # 150k locations with one write/write pair each: more than the initial
    # output buffer, exercising the rescan path
    n = 150000
    r = np.zeros(2 * n, dtype=RECORD_DTYPE)
    r["unit"] = np.repeat(np.arange(n, dtype=np.uint64) * 3, 2)
    r["tid"] = np.tile([0, 1], n)
    r["action"] = 1
    got = assert_parity(ctx, r, tpb=2, name="150k racing locations")
    assert len(got) == n


def test_location_lengths_across_threads(ctx):
    """Locations of 1 to 40 records in a repeating cycle, so that a thread's
    16 elements hold no, one or several complete locations and its first
    element belongs to a location that started in an earlier thread, a
    location that ends in it or one that runs on: every way the tile scan
    writes an entry (from the sums its pair pass kept, or by walking the
    thread's elements again) and locations that cross threads and tiles.
    Two threads per block, three barrier intervals, all three actions."""
    rng = np.random.default_rng(17)
    lens = np.tile(np.arange(1, 41), 600)
    n = int(lens.sum())
    r = np.zeros(n, dtype=RECORD_DTYPE)
    r["unit"] = np.repeat(np.arange(len(lens), dtype=np.uint64) * 5, lens)
    r["tid"] = rng.integers(0, 8, n)
    r["epoch"] = rng.integers(0, 3, n)
    r["action"] = rng.choice(np.array([0, 1, 2], dtype=np.uint8), n, p=[0.6, 0.3, 0.1])
    got = assert_parity(ctx, r, tpb=2, name="locations of 1..40 records")
    assert len(got) > 10000
    r["space"] = 1
    assert_parity(ctx, r, tpb=2, name="shared locations of 1..40 records")


def test_batched_mixed_sizes(ctx):
    shapes = tracegen.c3_shapes(48, log2_max=16)
    recs, off, tpb, inj = tracegen.batch(shapes, inject_rate=5e-4)
    got = assert_parity(ctx, recs, off, tpb, name="48 generated traces")
    for i, log in inj:
        for e in log:
            blk = int(e["block"])
            hit = (got["trace"] == i) & (got["space"] == e["space"]) & (got["unit"] == e["unit"])
            if int(e["space"]) == 1:
                hit &= got["block"] == blk
            assert hit.any()


def test_short_traces_sorted_in_lds():
    """Traces of up to four tiles (one-word keys) are sorted whole in one
    workgroup's LDS: alone (no global pass at all), mixed with longer traces
    (after the fused pass 0 when every block size is a power of two >= 256,
    from pass 0 otherwise), with key widths from 2 to 8 radix passes, sizes
    1..16384, and on a context whose remembered pass count comes from other
    calls."""
    import paper_1905_01833_amd as pkg

    rng = np.random.default_rng(77)

    def gen(n, unit_bits, tpb, blocks):
        r = np.zeros(n, dtype=RECORD_DTYPE)
        r["unit"] = rng.integers(0, 1 << unit_bits, n, dtype=np.uint64)
        r["unit"][: n // 2] = rng.integers(0, 8, n // 2)  # collisions
        r["tid"] = rng.integers(0, blocks * tpb, n)
        r["epoch"] = rng.integers(0, 4, n)
        r["action"] = rng.integers(0, 3, n)
        r["space"] = rng.integers(0, 2, n)
        return r

    sizes = [1, 2, 100, 1000, 4095, 4096, 4097, 8192, 12289, 16384]
    fresh = pkg.Context(0)
    try:
        for tpb, blocks in ((256, 8), (4, 3)):
            small = [gen(n, ub, tpb, blocks) for n in sizes for ub in (3, 20, 33)]
            recs, off = batch_of(small)
            assert_parity(fresh, recs, off, tpb, name=f"{len(small)} short traces, tpb {tpb}")
            big = gen(4 * 4096 + 17, 33, tpb, blocks)
            recs, off = batch_of(small[:5] + [big] + small[5:])
            assert_parity(fresh, recs, off, tpb, name=f"short traces around a 5-tile trace, tpb {tpb}")
            assert_parity(fresh, small[4], None, tpb, name=f"one one-tile trace after a mixed call, tpb {tpb}")
            assert_parity(fresh, small[-1], None, tpb, name=f"one 4-tile trace, tpb {tpb}")
            assert_parity(fresh, big, None, tpb, name=f"the 5-tile trace alone, tpb {tpb}")
    finally:
        fresh.close()


def test_empty_and_mixed_empty(ctx):
    r = np.zeros(0, dtype=RECORD_DTYPE)
    races, summ = ctx.check_traces(r, np.array([0], dtype=np.uint64), np.zeros(0, dtype=np.uint32))
    assert len(races) == 0 and len(summ) == 0
    traces = [np.zeros(0, dtype=RECORD_DTYPE), tracegen.c0(), np.zeros(0, dtype=RECORD_DTYPE), tracegen.c0()[:5]]
    recs, off = batch_of(traces)
    assert_parity(ctx, recs, off, [3, 256, 9, 256], name="empty traces mixed in")


# ------------------------------------------------------------ invariants

def test_permutation_invariance(ctx):
    r, _ = tracegen.c1(n_blocks=32, inject_rate=5e-4)
    a = assert_parity(ctx, r, tpb=256, name="c1 x32 blocks")
    perm = np.random.default_rng(4).permutation(len(r))
    b, _ = run_device(ctx, r[perm], None, 256)
    assert a.tobytes() == b.tobytes()


def test_results_identical_across_repeats_and_contexts(ctx):
    import paper_1905_01833_amd as pkg

    r, _ = tracegen.c1(n_blocks=16, inject_rate=1e-3, seed=77)
    first, _ = run_device(ctx, r, None, 256)
    for _ in range(3):
        again, _ = run_device(ctx, r, None, 256)
        assert again.tobytes() == first.tobytes()
    other = pkg.Context(0)
    try:
        got, _ = other.check_traces(r, None, 256)
        assert got.tobytes() == first.tobytes()
    finally:
        other.close()


def test_graph_replays_match_eager():
    """Graph mode: the first call of a shape is captured, later ones replay
    the graph.  Replays are interleaved with eager work of other shapes and
    host synchronisations, and every result is checked."""
    import paper_1905_01833_amd as pkg

    g = pkg.Context(0, graphs=True)
    try:
        r, _ = tracegen.c1(n_blocks=16, inject_rate=1e-3, seed=99)
        want, wsum = oracle.closed_form(r, tpb=256)
        dev = torch.from_numpy(r.view(np.uint8).reshape(-1, 16)).to("cuda:0")
        other = tracegen.c0()
        other_want, _ = oracle.closed_form(other, tpb=256)
        stream = torch.cuda.Stream()
        for rep in range(6):
            say(f"graph replay {rep}")
            with torch.cuda.stream(stream):
                got, gsum = g.check_traces_device(dev, None, 256, stream=stream.cuda_stream)
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), rep
            torch.cuda.synchronize()
            if rep % 2 == 1:  # a different shape in between forces a new capture
                o, _ = g.check_traces(other, None, 256)
                assert o.tobytes() == other_want.tobytes()
            x = torch.randn(1 << 20, device="cuda:0").sum().item()  # unrelated eager work
            assert x == x
    finally:
        g.close()


# ------------------------------------------------------------ error paths

def test_error_paths_leave_context_usable(ctx):
    import paper_1905_01833_amd as pkg

    r = tracegen.c0().copy()
    r["action"][500] = 7
    say("invalid action")
    with pytest.raises(pkg.SimError) as ei:
        ctx.check_traces(r, None, 256)
    assert ei.value.code == pkg.SIM_ERECORD and "500" in str(ei.value)
    r["action"][500] = 0
    r["space"][12] = 3
    with pytest.raises(pkg.SimError) as ei:
        run_device(ctx, r, None, 256)
    assert ei.value.code == pkg.SIM_ERECORD and "12" in str(ei.value)
    say("bad offsets / tpb")
    good = tracegen.c0()
    with pytest.raises(pkg.SimError) as ei:
        ctx.check_traces(good, np.array([0, 700, 600, 1279], dtype=np.uint64), [256, 256, 256])
    assert ei.value.code == pkg.SIM_EINVAL
    with pytest.raises(pkg.SimError) as ei:
        ctx.check_traces(good, None, 0)
    assert ei.value.code == pkg.SIM_EINVAL
    say("key wider than 64 bits: two-word keys, same context")
    w = np.zeros(4, dtype=RECORD_DTYPE)
    w["unit"] = [0, 1 << 62, 5, 5]
    w["tid"] = [0, 1 << 20, 3, 1 << 21]
    w["action"] = 1
    got = assert_parity(ctx, w, tpb=1024, name="86-bit keys")
    assert len(got) == 1 and int(got["unit"][0]) == 5
    assert_parity(ctx, good, tpb=256, name="after errors")


# ---------------------------------------------------------- full sizes

def test_c1_full_size(ctx):
    """The benchmark workload at full size: 1024 blocks x 256 threads,
    2^24 records, injection rate 1e-4; complete comparison."""
    r, inj = tracegen.c1()
    assert len(r) == 1 << 24
    got = assert_parity(ctx, r, tpb=256, name="c1 full")
    keys = set(zip(got["space"].tolist(), got["block"].tolist(), got["unit"].tolist()))
    for e in inj:
        blk = int(e["block"]) if int(e["space"]) == 1 else 0xFFFFFFFF
        assert (int(e["space"]), blk, int(e["unit"])) in keys


# ------------------------------------------------------ launch shapes (batched)

SHAPES = [
    {"stream_wgs_per_cu": 0, "sort_wgs_per_cu": 0, "scan_wgs_per_cu": 0, "group_shift_bias": 0},
    {"stream_wgs_per_cu": 1, "sort_wgs_per_cu": 1, "scan_wgs_per_cu": 1, "group_shift_bias": -1},
    {"stream_wgs_per_cu": 2, "sort_wgs_per_cu": 1, "scan_wgs_per_cu": 1, "group_shift_bias": 1,
     "scatter_threads": 512, "digit_bits": 9},
    {"stream_wgs_per_cu": 8, "sort_wgs_per_cu": 4, "scan_wgs_per_cu": 2, "group_shift_bias": -12,
     "digit_bits": 9},
    {"stream_wgs_per_cu": 0, "sort_wgs_per_cu": 2, "scan_wgs_per_cu": 0, "group_shift_bias": 12,
     "scatter_threads": 512},
    {"stream_wgs_per_cu": 0, "sort_wgs_per_cu": 0, "scan_wgs_per_cu": 0, "group_shift_bias": 0,
     "scatter_threads": 512},
    {"stream_wgs_per_cu": 0, "sort_wgs_per_cu": 1, "scan_wgs_per_cu": 0, "group_shift_bias": 0,
     "scatter_threads": 256},
    {"stream_wgs_per_cu": 0, "sort_wgs_per_cu": 0, "scan_wgs_per_cu": 0, "group_shift_bias": 12,
     "scatter_threads": 256, "digit_bits": 9},
    {"stream_wgs_per_cu": 1, "sort_wgs_per_cu": 2, "scan_wgs_per_cu": 1, "group_shift_bias": 0,
     "digit_bits": 8},
]


def test_every_launch_shape_bit_exact(ctx):
    """Persistent (looping) and one-tile-per-workgroup kernels, and histogram
    groups from one tile to whole traces, give identical results.  The
    input has more tiles than one workgroup per CU, so the small grids loop."""
    big, _ = tracegen.c1(n_blocks=96, inject_rate=3e-4, seed=123)
    shapes = tracegen.c3_shapes(40, log2_max=17, seed=5)
    small, off, tpb, _ = tracegen.batch(shapes, inject_rate=5e-4)
    recs = np.concatenate([small, big])
    off = np.concatenate([off, [off[-1] + len(big)]]).astype(np.uint64)
    tpb = np.concatenate([tpb, [256]]).astype(np.uint32)
    assert (len(recs) + 4095) // 4096 > 300
    want, wsum = oracle.closed_form(recs, off, tpb)
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    cls = tracegen_size_class(len(recs))
    try:
        for sh in SHAPES:
            say(f"shape {sh}")
            ctx.set_tuning(cls, sh)
            got, gsum = ctx.check_traces_device(dev, off, tpb)
            torch.cuda.synchronize()
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), sh
    finally:
        ctx.set_tuning(cls, None)


def tracegen_size_class(n):
    import paper_1905_01833_amd as pkg

    return pkg.sim_size_class(n)


def test_autotune_and_tuning_cache(ctx, tmp_path):
    import paper_1905_01833_amd as pkg

    shapes = tracegen.c3_shapes(64, log2_max=16, seed=6)
    recs, off, tpb, _ = tracegen.batch(shapes, inject_rate=5e-4)
    want, wsum = oracle.closed_form(recs, off, tpb)
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    say("autotune 64 traces")
    g = pkg.Context(0, graphs=True)
    try:
        best = g.autotune(dev, off, tpb, reps=1)
        assert best["ms"] > 0
        is_set, t = g.tuning(best["size_class"])
        assert is_set and all(t[f] == best[f] for f in pkg.TUNING_FIELDS)
        for rep in range(3):  # graph capture and replays with the tuned shape
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                got, gsum = g.check_traces_device(dev, off, tpb, stream=stream.cuda_stream)
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), rep
        path = str(tmp_path / "tuning.json")
        g.save_tuning(path)
    finally:
        g.close()
    h = pkg.Context(0)
    try:
        assert h.load_tuning(path) == 1
        is_set, t = h.tuning(best["size_class"])
        assert is_set and all(t[f] == best[f] for f in pkg.TUNING_FIELDS)
        got, _ = h.check_traces(recs, off, tpb)
        assert got.tobytes() == want.tobytes()
    finally:
        h.close()
    with pytest.raises(pkg.SimError):
        ctx.set_tuning(40, None)


# ------------------------------------------------------------- full sizes

def _location_ids(recs, tpb):
    """One integer per record naming its location: the unit for global
    memory, (1 << 62) | block << 24 | unit for shared memory."""
    unit = recs["unit"].astype(np.uint64)
    block = (recs["tid"] // np.uint32(tpb)).astype(np.uint64)
    shared = recs["space"] == 1
    return np.where(shared, (np.uint64(1) << np.uint64(62)) | (block << np.uint64(24)) | unit, unit)


def test_c2_full_size(ctx):
    """The large configuration (8192 blocks x 512 threads, 2^28 records, 5%
    atomics) at full size in one call: the whole entry list and summary
    equal the oracle's (its group-count tier on every host core), and every
    injected location is reported."""
    r, inj = tracegen.c2()
    assert len(r) == 1 << 28
    say("c2 full: 2^28 records")
    got, summ = run_device(ctx, r, None, 512)
    say("c2 full: oracle")
    want, wsum = oracle.closed_form_par(r, tpb=512)
    assert len(got) == len(want) > 0
    assert got.tobytes() == want.tobytes()
    assert summ.tobytes() == wsum.tobytes()
    keys = set(zip(got["space"].tolist(), got["block"].tolist(), got["unit"].tolist()))
    for e in inj:
        blk = int(e["block"]) if int(e["space"]) == 1 else 0xFFFFFFFF
        assert (int(e["space"]), blk, int(e["unit"])) in keys
    # Tier A (brute force) on the records of a few reported locations
    ids = _location_ids(r, 512)
    rng = np.random.default_rng(7)
    pick = got[rng.choice(len(got), size=min(24, len(got)), replace=False)]
    lids = np.where(pick["space"] == 1,
                    (np.uint64(1) << np.uint64(62)) | (pick["block"].astype(np.uint64) << np.uint64(24))
                    | pick["unit"].astype(np.uint64), pick["unit"].astype(np.uint64))
    sel = np.isin(ids, lids)
    sub_r, sub_ids = r[sel], ids[sel]
    checked = 0
    for e, lid in zip(pick, lids):
        sub = sub_r[sub_ids == lid]
        if len(sub) <= 4096:
            br, _ = oracle.brute_force(sub, tpb=512)
            assert len(br) == 1 and br.tobytes() == e.tobytes()
            checked += 1
    assert checked > 0


def test_c3_full_size(ctx):
    """The batched configuration (4096 traces, log-uniform 2^8..2^20
    records) in one call with the autotuned launch shape and a graph
    replay: the whole entry list and every summary equal the oracle's, and
    injected locations of every trace are reported."""
    import paper_1905_01833_amd as pkg

    shapes = tracegen.c3_shapes(4096)
    recs, off, tpb, inj = tracegen.batch(shapes, inject_rate=1e-4)
    say(f"c3 full: {len(recs)} records, 4096 traces")
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    g = pkg.Context(0, graphs=True)
    try:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            g.autotune(dev, off, tpb, stream=stream.cuda_stream, reps=1)
            got, summ = g.check_traces_device(dev, off, tpb, stream=stream.cuda_stream)
            again, _ = g.check_traces_device(dev, off, tpb, stream=stream.cuda_stream)  # graph replay
        torch.cuda.synchronize()
    finally:
        g.close()
    del dev
    assert again.tobytes() == got.tobytes()
    say("c3 full: oracle")
    want, wsum = oracle.closed_form_par(recs, off, tpb)
    assert len(got) == len(want) > 0
    assert got.tobytes() == want.tobytes()
    assert summ.tobytes() == wsum.tobytes()
    keys = set(zip(got["trace"].tolist(), got["space"].tolist(), got["block"].tolist(), got["unit"].tolist()))
    for i, log in inj:
        for e in log:
            blk = int(e["block"]) if int(e["space"]) == 1 else 0xFFFFFFFF
            assert (i, int(e["space"]), blk, int(e["unit"])) in keys


def test_widest_keys_and_mixed_pass_counts(ctx):
    """A trace whose key takes all 64 bits (8 radix passes: unit range 2^33,
    1024 blocks, 1024 epochs, 256 threads per block) batched with traces of
    2-pass keys, on a fresh context (no remembered pass count) and again on
    a warm one; also alone, where fewer passes were remembered."""
    import paper_1905_01833_amd as pkg

    rng = np.random.default_rng(64)
    n = 60000
    w = np.zeros(n, dtype=RECORD_DTYPE)
    w["unit"] = rng.integers(0, 1 << 33, n, dtype=np.uint64)
    w["unit"][: n // 2] = rng.integers(0, 64, n // 2)  # collisions in the low units
    w["unit"][n - 1] = (1 << 33) - 1  # the full unit range: 33 bits
    w["tid"] = rng.integers(0, 1024 * 256, n)
    w["tid"][:8] = [0, 1024 * 256 - 1, 5, 6, 7, 8, 9, 10]
    w["epoch"] = rng.integers(0, 1024, n)
    w["epoch"][0] = 1023
    w["action"] = rng.integers(0, 3, n)
    w["space"] = 0
    small = tracegen.random_small(rng, 3000, units=6, blocks=2, tpb=4, epochs=2)
    recs, off = batch_of([small, w, small[:100]])
    tpb = [4, 256, 4]
    fresh = pkg.Context(0)
    try:
        assert_parity(fresh, recs, off, tpb, name="64-bit keys batched, fresh context")
        assert_parity(fresh, recs, off, tpb, name="64-bit keys batched, warm context")
        assert_parity(fresh, small, None, 4, name="2-pass trace after 8")
        assert_parity(fresh, w, None, 256, name="64-bit keys alone after 2")
    finally:
        fresh.close()


def test_two_word_keys(ctx):
    """Traces whose lossless key needs more than 64 bits (units spread over
    2^62, thread ids up to 2^20, epochs up to 999) run with two-word keys:
    alone, batched with one-word traces, across tiles, and back to one-word
    calls on the same context; also under graph replay."""
    import paper_1905_01833_amd as pkg

    rng = np.random.default_rng(128)

    def wide(n, tpb=64):
        r = np.zeros(n, dtype=RECORD_DTYPE)
        pool = rng.integers(0, 1 << 62, 40, dtype=np.uint64)
        pool[0], pool[1] = 0, (1 << 62) - 1
        r["unit"] = pool[rng.integers(0, len(pool), n)]
        r["tid"] = rng.integers(0, 1 << 20, n)
        few = rng.random(n) < 0.5
        r["tid"][few] = rng.integers(0, 3 * tpb, int(few.sum()))
        r["epoch"] = rng.integers(0, 3, n)
        r["epoch"][0] = 999
        r["action"] = rng.integers(0, 3, n)
        r["space"] = (rng.random(n) < 0.3).astype(np.uint8)
        return r

    w1 = wide(30000)
    got = assert_parity(ctx, w1, tpb=64, name="two-word keys, 30000 records")
    assert len(got) > 0
    narrow = tracegen.random_small(rng, 9000, units=20, blocks=3, tpb=5, epochs=3)
    recs, off = batch_of([narrow, wide(5000, tpb=256), narrow[:77], wide(12345)])
    assert_parity(ctx, recs, off, [5, 256, 5, 64], name="two-word and one-word traces batched")
    assert_parity(ctx, narrow, tpb=5, name="one-word call after two-word calls")
    assert_parity(ctx, w1, tpb=64, name="two-word call after a one-word call")
    g = pkg.Context(0, graphs=True)
    try:
        want, wsum = oracle.closed_form(w1, tpb=64)
        dev = torch.from_numpy(w1.view(np.uint8).reshape(-1, 16)).to("cuda:0")
        stream = torch.cuda.Stream()
        for rep in range(4):
            say(f"two-word keys, graph replay {rep}")
            with torch.cuda.stream(stream):
                got, gsum = g.check_traces_device(dev, None, 64, stream=stream.cuda_stream)
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), rep
    finally:
        g.close()
