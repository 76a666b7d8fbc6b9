"""GPU parity of the radix offsets' two row widths.  In-group digit offsets
are 16-bit when no histogram group of the call has more than 16 tiles (an
offset then sums at most 15 tiles of 4096 keys) and 32-bit otherwise.  A
trace of 256 tiles (groups of 16 tiles) whose keys mostly share one
location, block and interval shares the digits of those fields across most
keys, so the in-group offsets of those passes come close to their largest
values; the same records with wider groups
(group_shift_bias, or a longer trace in the call) take the 32-bit rows.
Every check goes through the C ABI and compares with the oracle byte for
byte.

Every case prints its name before it touches the GPU.  Inputs are seeded
and synthetic; expected values come from oracle/ only."""
import numpy as np
import pytest

import oracle
from tracegen import ATOMIC, READ, RECORD_DTYPE, WRITE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TILE = 4096


def say(msg):
    print(f"[gpu-offsets] {msg}", flush=True)


@pytest.fixture(scope="module")
def pkg():
    import paper_1905_01833_amd as p

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return p


def to_dev(recs):
    return torch.from_numpy(np.ascontiguousarray(recs).view(np.uint8).reshape(-1, 16)).to("cuda:0")


def hot_trace(n_tiles, seed):
    """n_tiles x 4096 records, most of them on one global location from the
    threads of block 0 in the first barrier interval (so the digits of the
    passes over those key fields agree on most keys), the rest spread over
    four locations, 64 blocks of 256 threads and three intervals; 80 %
    reads, 15 % writes, 5 % atomics."""
    n = n_tiles * TILE
    rng = np.random.default_rng(seed)
    r = np.zeros(n, dtype=RECORD_DTYPE)
    hot = rng.random(n) < 0.85
    r["unit"] = np.where(hot, 0, rng.integers(0, 4, n) * 64)
    r["tid"] = np.where(hot, rng.integers(0, 256, n), rng.integers(0, 256 * 64, n))
    r["epoch"] = np.where(hot, 0, rng.integers(0, 3, n))
    r["action"] = rng.choice(np.array([READ, WRITE, ATOMIC], dtype=np.uint8), n, p=[0.8, 0.15, 0.05])
    return r


@pytest.mark.parametrize("bias", [0, 1])
def test_hot_trace_group_widths(pkg, bias):
    """256 tiles: groups of 16 tiles (16-bit offsets) by default, of 32 with
    the bias (32-bit offsets); both equal the oracle."""
    recs = hot_trace(256, seed=7)
    want, wsum = oracle.closed_form(recs, None, 256)
    assert len(want) == 4
    dev = to_dev(recs)
    c = pkg.Context(0)
    try:
        c.set_tuning(pkg.sim_size_class(len(recs)), {"group_shift_bias": bias})
        for rep in range(2):
            say(f"one trace of 256 tiles, group shift bias {bias}, call {rep}")
            got, gsum = c.check_traces_device(dev, None, 256)
            torch.cuda.synchronize()
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), (bias, rep)
    finally:
        c.close()


def test_batch_widths_alternate(pkg):
    """The 256-tile trace alone (16-bit rows), then beside a 300-tile trace
    (its groups of 32 tiles make the call's rows 32-bit), on one context."""
    a = hot_trace(256, seed=8)
    b = hot_trace(300, seed=9)
    both = np.concatenate([a, b])
    off2 = np.array([0, len(a), len(both)], dtype=np.uint64)
    tpb2 = np.array([256, 256], dtype=np.uint32)
    cases = [
        ("alone", a, None, 256, oracle.closed_form(a, None, 256)),
        ("beside a 300-tile trace", both, off2, tpb2, oracle.closed_form(both, off2, tpb2)),
    ]
    devs = [to_dev(x[1]) for x in cases]
    c = pkg.Context(0)
    try:
        for rep in range(2):
            for (name, _, off, tpb, (want, wsum)), dev in zip(cases, devs):
                say(f"{name}, call {rep}")
                got, gsum = c.check_traces_device(dev, off, tpb)
                torch.cuda.synchronize()
                assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), (name, rep)
    finally:
        c.close()


def wide_hot_trace(n_tiles, seed):
    """As hot_trace, with two-word keys: units spread over 2^62 and thread
    ids up to 2^20 outside the hot part."""
    r = hot_trace(n_tiles, seed)
    rng = np.random.default_rng(seed + 1000)
    cold = r["unit"] != 0
    pool = rng.integers(0, 1 << 62, 16, dtype=np.uint64)
    r["unit"][cold] = pool[rng.integers(0, len(pool), int(cold.sum()))]
    r["tid"][cold] = rng.integers(0, 1 << 20, int(cold.sum()))
    r["unit"][-1] = (1 << 62) - 1
    return r


@pytest.mark.parametrize("n_tiles", [256, 300])
def test_two_word_keys_both_widths(pkg, n_tiles):
    """Two-word keys with 16-bit offset rows (256 tiles: groups of 16) and
    32-bit ones (300 tiles: groups of 32)."""
    recs = wide_hot_trace(n_tiles, seed=11)
    want, wsum = oracle.closed_form(recs, None, 256)
    dev = to_dev(recs)
    c = pkg.Context(0)
    try:
        for rep in range(2):
            say(f"two-word keys, {n_tiles} tiles, call {rep}")
            got, gsum = c.check_traces_device(dev, None, 256)
            torch.cuda.synchronize()
            assert got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes(), (n_tiles, rep)
    finally:
        c.close()
