"""GPU parity of the EP fitness count (Eq. 1; sim_eval_fitness and
sim_eval_fitness_device, through the C ABI) with the oracle, byte for byte
(the fitness value included: both sides divide the same two integers in
IEEE double).

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic (tracegen); expected values come from oracle/ only."""
import numpy as np
import pytest

import oracle
import tracegen
from golden_io import trace_fixture
from test_host import wide_trace
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


def to_dev(recs):
    return torch.from_numpy(np.ascontiguousarray(recs).view(np.uint8).reshape(-1, 16)).to("cuda:0")


def same_as_oracle(ctx, recs, off, tpb, host=True):
    want = oracle.fitness(recs, off, tpb)
    got = ctx.eval_fitness_device(to_dev(recs), off, tpb)
    torch.cuda.synchronize()
    assert got.tobytes() == want.tobytes()
    if host:
        assert ctx.eval_fitness(recs, off, tpb).tobytes() == want.tobytes()
    return got


@pytest.mark.parametrize("name", ["fig6_unit.txt", "fig6_unit_write.txt", "kaldi_copy.txt", "mixed_kinds.txt"])
def test_fixtures(ctx, name):
    say(f"fitness fixture {name}")
    recs, tpb, _ = trace_fixture(name)
    same_as_oracle(ctx, recs, [0, len(recs)], tpb)


def test_tree_family(ctx):
    say("fitness tree-reduction family")
    traces = [tracegen.tree_reduction(k) for k in range(-1, 9)]
    recs, off = batch_of(traces)
    got = same_as_oracle(ctx, recs, off, [256] * len(traces))
    # removing a barrier moves no access: every member has the same row
    assert len(set(r.tobytes() for r in got)) == 1


@pytest.mark.parametrize("seed", range(12))
def test_random_small_batches(ctx, seed):
    say(f"fitness random batch seed {seed}")
    rng = np.random.default_rng(1300 + seed)
    traces, tpbs = [], []
    for _ in range(int(rng.integers(1, 40))):
        n = int(rng.integers(0, 3000))
        tp = int(rng.integers(1, 9))
        traces.append(tracegen.random_small(rng, n, units=int(rng.integers(1, 50)), blocks=int(rng.integers(1, 5)),
                                            tpb=tp, epochs=int(rng.integers(1, 4))))
        tpbs.append(tp)
    recs, off = batch_of(traces)
    same_as_oracle(ctx, recs, off, tpbs)


@pytest.mark.parametrize("n", [4095, 4096, 4097, 16385, 45055])
def test_tile_boundaries(ctx, n):
    say(f"fitness tile boundaries n={n}")
    rng = np.random.default_rng(n)
    r = tracegen.random_small(rng, n, units=700, blocks=4, tpb=256, epochs=5)
    same_as_oracle(ctx, r, [0, n], 256)
    same_as_oracle(ctx, r, [0, n], 100, host=False)  # not a power of two: no fused first pass


@pytest.mark.parametrize("seed", range(4))
def test_two_word_keys(ctx, seed):
    say(f"fitness two-word keys seed {seed}")
    rng = np.random.default_rng(seed)
    w = wide_trace(rng, 3000)
    r = tracegen.random_small(rng, 5000, units=30, blocks=3, tpb=64, epochs=2)
    recs, off = batch_of([w, r])
    same_as_oracle(ctx, recs, off, [64, 64])


def test_population_of_candidates(ctx):
    # one generation of the EP search: 50 parents and 100 children, each a
    # candidate launch traced with the batched workload's distributions
    say("fitness population of 150 candidates")
    shapes = tracegen.c3_shapes(n_traces=150, seed=0x5EED0006, log2_max=18.0)
    recs, off, tpb, _ = tracegen.batch(shapes)
    same_as_oracle(ctx, recs, off, tpb)


def test_full_size_trace(ctx):
    say("fitness 1024 x 256 trace of 2^24 records")
    recs, _ = tracegen.c1()
    same_as_oracle(ctx, recs, [0, len(recs)], 256, host=False)


def test_modes_interleave(ctx):
    # the race check and the fitness count keep separate pass counts and
    # key widths; alternating them gives the same results
    say("fitness interleaved with the race check")
    rng = np.random.default_rng(77)
    a = tracegen.random_small(rng, 20000, units=3000, blocks=8, tpb=256, epochs=9)
    w = wide_trace(rng, 2000)
    for recs, tp in [(a, 256), (w, 64), (a, 256)]:
        same_as_oracle(ctx, recs, [0, len(recs)], tp, host=False)
        races, summ = ctx.check_traces_device(to_dev(recs), [0, len(recs)], tp)
        torch.cuda.synchronize()
        want, wsum = oracle.closed_form(recs, [0, len(recs)], tp)
        assert races.tobytes() == want.tobytes()


def test_empty_and_errors(ctx):
    import paper_1905_01833_amd as pkg

    say("fitness empty traces and errors")
    e = np.zeros(0, dtype=RECORD_DTYPE)
    assert len(ctx.eval_fitness(e, [0], [])) == 0
    got = ctx.eval_fitness(e, [0, 0, 0], [1, 1])
    assert got.tobytes() == oracle.fitness(e, [0, 0, 0], [1, 1]).tobytes()
    rng = np.random.default_rng(5)
    r = tracegen.random_small(rng, 100)
    recs, off = batch_of([e, r, e])
    same_as_oracle(ctx, recs, off, [3, 3, 3])
    bad = r.copy()
    bad["action"][17] = 3
    with pytest.raises(pkg.SimError) as ei:
        ctx.eval_fitness(bad, [0, len(bad)], 3)
    assert ei.value.code == pkg.SIM_ERECORD
    same_as_oracle(ctx, r, [0, len(r)], 3)  # the context stays usable
