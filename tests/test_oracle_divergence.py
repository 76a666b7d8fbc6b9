"""Pins for the oracle's barrier-divergence check (Alg. 4, Sec. 4.2.2), on
the CPU: the per-thread barrier arrival counts of small CUDA control-flow
patterns, derived by hand from what each thread executes; a pure-Python
rendering on random counts; planted mistakes must each fail a pin."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


def grid_counts(n_blocks, tpb, arrivals):
    """Barrier arrivals of every thread of a grid, block by block, from a
    function of (blockIdx.x, threadIdx.x) that says how many barriers the
    thread's path through the kernel calls."""
    return np.array([arrivals(b, t) for b in range(n_blocks) for t in range(tpb)], dtype=np.uint32)


def rows(res):
    return [tuple(int(r[f]) for f in ("trace", "block", "min_barriers", "max_barriers", "early_threads")) for r in res]


# Patterns and what every thread executes:
#   branch_barrier   if (threadIdx.x < 100) __syncthreads();
#                    threads 0..99 call it once, 100..255 never: every block
#                    diverges, 156 threads leave early.
#   block_uniform    if (blockIdx.x % 2) __syncthreads();
#                    all threads of a block take the same path: none.
#   loop_by_thread   for (i = 0; i < threadIdx.x % 4; i++) __syncthreads();
#                    (8 threads) counts 0 1 2 3 0 1 2 3: min 0, max 3, six
#                    threads below 3.
#   early_return     if (threadIdx.x == 5) return; __syncthreads(); __syncthreads();
#                    thread 5 arrives at none, the rest at two.
#   uniform_loop     for (i = 0; i < 3; i++) __syncthreads();  -- none.
PATTERNS = {
    "branch_barrier": (4, 256, lambda b, t: 1 if t < 100 else 0, [(0, b, 0, 1, 156) for b in range(4)]),
    "block_uniform": (6, 64, lambda b, t: 1 if b % 2 else 0, []),
    "loop_by_thread": (3, 8, lambda b, t: t % 4, [(0, b, 0, 3, 6) for b in range(3)]),
    "early_return": (2, 32, lambda b, t: 0 if t == 5 else 2, [(0, 0, 0, 2, 1), (0, 1, 0, 2, 1)]),
    "uniform_loop": (5, 128, lambda b, t: 3, []),
}


@pytest.mark.parametrize("name", sorted(PATTERNS))
def test_control_flow_patterns(name):
    n_blocks, tpb, arrivals, want = PATTERNS[name]
    c = grid_counts(n_blocks, tpb, arrivals)
    assert rows(oracle.divergence(c, [0, len(c)], tpb)) == want


def test_batch_numbers_traces_and_single_thread_blocks():
    a = grid_counts(4, 256, PATTERNS["branch_barrier"][2])
    b = grid_counts(6, 64, PATTERNS["block_uniform"][2])
    one = np.arange(10, dtype=np.uint32)  # one thread per block never diverges
    c = np.concatenate([a, b, one])
    off = [0, len(a), len(a) + len(b), len(c)]
    got = rows(oracle.divergence(c, off, [256, 64, 1]))
    assert got == [(0, k, 0, 1, 156) for k in range(4)]


def divergence_py(counts, off, tpb):
    out = []
    for t in range(len(off) - 1):
        c = [int(x) for x in counts[off[t]: off[t + 1]]]
        for b in range(len(c) // tpb[t]):
            blk = c[b * tpb[t]: (b + 1) * tpb[t]]
            lo, hi = min(blk), max(blk)
            if lo != hi:
                out.append((t, b, lo, hi, sum(1 for x in blk if x < hi)))
    return out


@pytest.mark.parametrize("seed", range(30))
def test_matches_python_rendering(seed):
    rng = np.random.default_rng(500 + seed)
    k = int(rng.integers(1, 5))
    tpbs = [int(rng.integers(1, 9)) for _ in range(k)]
    sizes = [tp * int(rng.integers(0, 6)) for tp in tpbs]
    counts = rng.integers(0, 3, sum(sizes)).astype(np.uint32)
    # some blocks uniform
    counts[rng.random(len(counts)) < 0.5] = 1
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    assert rows(oracle.divergence(counts, off, tpbs)) == divergence_py(counts, off, tpbs)


def test_partial_blocks_are_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.divergence(np.zeros(10, dtype=np.uint32), [0, 10], 4)


MUTANTS = {
    "min_from_zero": ("      uint32_t lo = c[0], hi = c[0];", "      uint32_t lo = 0, hi = c[0];"),
    "early_counts_equal": ("early += c[k] < hi ? 1 : 0;", "early += c[k] <= hi ? 1 : 0;"),
    "early_below_min": ("early += c[k] < hi ? 1 : 0;", "early += c[k] == lo ? 1 : 0;"),
    "block_stride_one_less": ("const uint32_t* c = counts + off[tr] + b * tpb[tr];",
                              "const uint32_t* c = counts + off[tr] + b * (tpb[tr] - 1);"),
}


def _pins_pass():
    for name, (n_blocks, tpb, arrivals, want) in PATTERNS.items():
        c = grid_counts(n_blocks, tpb, arrivals)
        if rows(oracle.divergence(c, [0, len(c)], tpb)) != want:
            return False
    for seed in range(10):
        rng = np.random.default_rng(500 + seed)
        tpbs = [int(rng.integers(1, 9)) for _ in range(3)]
        sizes = [tp * int(rng.integers(0, 6)) for tp in tpbs]
        counts = rng.integers(0, 3, sum(sizes)).astype(np.uint32)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
        if rows(oracle.divergence(counts, off, tpbs)) != divergence_py(counts, off, tpbs):
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_divergence_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c), "-o", str(so)], check=True)
    saved = oracle._load()
    mutant = ctypes.CDLL(so)
    f = mutant.orc_divergence_check
    f.restype = saved.orc_divergence_check.restype
    f.argtypes = saved.orc_divergence_check.argtypes
    mutant.orc_free.restype = None
    mutant.orc_free.argtypes = [ctypes.c_void_p]
    oracle._lib = mutant
    try:
        assert not _pins_pass(), f"mutant {name} survived every pin"
    finally:
        oracle._lib = saved
