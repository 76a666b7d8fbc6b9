"""GPU parity of the barrier-divergence check (Alg. 4; sim_check_divergence
and sim_check_divergence_device, through the C ABI) with the oracle, byte
for byte.

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic (tracegen); expected values come from oracle/ only."""
import numpy as np
import pytest

import oracle
import tracegen
from test_oracle_divergence import PATTERNS, grid_counts

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


def both(ctx, counts, off, tpb):
    """Host-memory and device-tensor entry points; both must agree."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    a = ctx.check_divergence(counts, off, tpb)
    d = torch.from_numpy(counts.view(np.int32)).to("cuda:0")
    b = ctx.check_divergence_device(d, off, tpb)
    torch.cuda.synchronize()
    assert a.tobytes() == b.tobytes()
    return a


def same_as_oracle(ctx, counts, off, tpb):
    got = both(ctx, counts, off, tpb)
    want = oracle.divergence(counts, off, tpb)
    assert len(got) == len(want)
    assert got.tobytes() == want.tobytes()
    return got


@pytest.mark.parametrize("name", sorted(PATTERNS))
def test_control_flow_patterns(ctx, name):
    say(f"divergence pattern {name}")
    n_blocks, tpb, arr, want = PATTERNS[name]
    c = grid_counts(n_blocks, tpb, arr)
    got = same_as_oracle(ctx, c, [0, len(c)], tpb)
    assert [tuple(int(x) for x in r) for r in got] == want


@pytest.mark.parametrize("tpb", [1, 2, 3, 31, 32, 33, 63, 64, 65, 100, 256, 257, 512, 1024, 4096, 5000])
def test_block_sizes(ctx, tpb):
    # every segment width of the kernel: several blocks per wave (tpb <= 64),
    # one wave striding over a block, chunks of one block
    say(f"divergence block size {tpb}")
    n_blocks = max(3, 20000 // tpb)
    c, picked = tracegen.arrivals(n_blocks, tpb, 5, 11 + tpb, diverge_rate=0.3)
    got = same_as_oracle(ctx, c, [0, len(c)], tpb)
    assert [int(r["block"]) for r in got] == (picked if tpb > 1 else [])


@pytest.mark.parametrize("seed", range(8))
def test_random_batches(ctx, seed):
    say(f"divergence random batch seed {seed}")
    rng = np.random.default_rng(900 + seed)
    shapes = [(int(rng.integers(0, 40)), int(rng.integers(1, 300))) for _ in range(int(rng.integers(1, 30)))]
    c, off, tpb = tracegen.arrivals_batch(shapes, barriers=int(rng.integers(1, 6)), diverge_rate=0.2, seed=seed)
    # also equal counts that are not the maximum: arbitrary values per thread
    mask = rng.random(len(c)) < 0.02
    c[mask] = rng.integers(0, 1 << 31, int(mask.sum())).astype(np.uint32)
    same_as_oracle(ctx, c, off, tpb)


def test_launch_shapes_at_size(ctx):
    # one launch of 1024 x 256 threads, one of 8192 x 512, and a batch of
    # 4096 launches with the batched workload's block counts
    say("divergence 1024 x 256")
    c, picked = tracegen.arrivals(1024, 256, 4, 0x5EED0001, diverge_rate=1e-2)
    got = same_as_oracle(ctx, c, [0, len(c)], 256)
    assert [int(r["block"]) for r in got] == picked
    say("divergence 8192 x 512")
    c, picked = tracegen.arrivals(8192, 512, 4, 0x5EED0002, diverge_rate=1e-3)
    got = same_as_oracle(ctx, c, [0, len(c)], 512)
    assert [int(r["block"]) for r in got] == picked
    say("divergence batch of 4096 launches")
    shapes = [(nb, 256) for (_, nb, _, _) in tracegen.c3_shapes()]
    c, off, tpb = tracegen.arrivals_batch(shapes, diverge_rate=1e-2)
    same_as_oracle(ctx, c, off, tpb)


def test_empty_and_errors(ctx):
    import paper_1905_01833_amd as pkg

    say("divergence empty calls and errors")
    assert len(ctx.check_divergence(np.zeros(0, np.uint32), [0], [])) == 0
    assert len(ctx.check_divergence(np.zeros(0, np.uint32), [0, 0, 0], [4, 7])) == 0
    with pytest.raises(pkg.SimError) as e:
        ctx.check_divergence(np.zeros(10, np.uint32), [0, 10], [4])  # not whole blocks
    assert e.value.code == pkg.SIM_EINVAL
    with pytest.raises(pkg.SimError) as e:
        ctx.check_divergence(np.zeros(8, np.uint32), [0, 8], [0])
    assert e.value.code == pkg.SIM_EINVAL
    with pytest.raises(pkg.SimError) as e:
        ctx.check_divergence(np.zeros(8, np.uint32), [0, 8, 4], [4, 4])
    assert e.value.code == pkg.SIM_EINVAL
    # the context stays usable, also for the race check
    c = grid_counts(2, 32, PATTERNS["early_return"][2])
    same_as_oracle(ctx, c, [0, len(c)], 32)
