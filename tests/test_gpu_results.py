"""Result memory: entry lists of 1 MiB and more come from a small pool of
pinned host blocks that sim_result_free recycles (at most eight blocks;
beyond that, plain host memory).  Results held at the same time, freed in
any order and then reused must each stay the oracle's, byte for byte.

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic; expected values come from oracle/ only."""
import gc

import numpy as np
import pytest

import oracle
import tracegen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-results] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_1905_01833_amd as pkg

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    c.close()


def test_large_results_held_freed_and_reused(ctx):
    recs, _ = tracegen.c1(n_blocks=64, inject_rate=5e-2, seed=71)
    want, wsum = oracle.closed_form(recs, None, 256)
    assert len(want) * 64 >= 1 << 20, len(want)  # large enough for a pinned block
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    for rnd in range(2):
        held = []
        for k in range(10):  # more results alive than pinned blocks
            say(f"round {rnd}, call {k}: {len(want)} entries")
            got, gsum = ctx.check_traces_device(dev, None, 256)
            torch.cuda.synchronize()
            held.append((got, gsum))
        for got, gsum in held:
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes()
        # free in a mixed order; each remaining result is untouched
        for k in (3, 0, 7, 9, 1):
            held[k] = None
        gc.collect()
        for item in held:
            if item is not None:
                assert item[0].tobytes() == want.tobytes()
        held.clear()
        gc.collect()
    # a small result after the large ones (plain host memory)
    say("small result")
    small = recs[:5000]
    got, _ = ctx.check_traces_device(dev[:5000], None, 256)
    torch.cuda.synchronize()
    assert got.tobytes() == oracle.closed_form(small, None, 256)[0].tobytes()


def test_call_tables_follow_every_change_of_shape():
    """Calls whose trace tables differ in the split of the same records, or
    only in threads per block, alternate on one context (with and without
    graph replay): every call uses its own tables, never the previous
    call's, and equals the oracle."""
    import paper_1905_01833_amd as pkg

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    recs, _ = tracegen.c1(n_blocks=16, inject_rate=2e-3, seed=81)
    n = len(recs)
    shapes = [
        (np.array([0, n // 3, n], dtype=np.uint64), np.array([256, 256], dtype=np.uint32)),
        (np.array([0, n // 2, n], dtype=np.uint64), np.array([256, 256], dtype=np.uint32)),
        (np.array([0, n // 2, n], dtype=np.uint64), np.array([256, 512], dtype=np.uint32)),
    ]
    wants = [oracle.closed_form(recs, off, tpb) for off, tpb in shapes]
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    for graphs in (False, True):
        c = pkg.Context(0, graphs=graphs)
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                for rep in range(3):
                    for k, (off, tpb) in enumerate(shapes):
                        say(f"graphs={graphs}, round {rep}, shape {k}")
                        got, gsum = c.check_traces_device(dev, off, tpb, stream=stream.cuda_stream)
                        torch.cuda.synchronize()
                        want, wsum = wants[k]
                        assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), (graphs, rep, k)
        finally:
            c.close()
