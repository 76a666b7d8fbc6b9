"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch every one of them.

Each mutant is the oracle's C source with one textual change (a dropped
term, a flipped sign, a transposed operand, a lost condition), compiled into
a temporary library and swapped in for the real one while the pin checks
run.  A mutant that passes all pins would mean the pins cannot see that kind
of mistake.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import tracegen
from golden_io import trace_fixture, truth_table

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "drop_thread_term": ("p[k] = KL[k] - SB[k] + SE[k] - ST[k];", "p[k] = KL[k] - SB[k] + SE[k];"),
    "flip_epoch_sign": ("p[k] = KL[k] - SB[k] + SE[k] - ST[k];", "p[k] = KL[k] - SB[k] - SE[k] + ST[k];"),
    "xblock_no_block_term": ("xb += KL[k] - SB[k];", "xb += KL[k];"),
    "rw_transposed": ("k[KIND_RW] = c->r * c->w;", "k[KIND_RW] = c->r * c->r;"),
    "ww_ordered_pairs": ("k[KIND_WW] = c->w ? c->w * (c->w - 1) / 2 : 0;", "k[KIND_WW] = c->w * c->w / 2;"),
    "aw_ar_swapped": ("if (a == 1 && b == 2) return KIND_AW;", "if (a == 1 && b == 2) return KIND_AR;"),
    "atomics_race_each_other": ("return -1; /* A A */", "return KIND_AW; /* A A */"),
    "brute_no_cross_block": ("if (!(bx != by || x->epoch == y->epoch)) continue;",
                             "if (!(x->epoch == y->epoch)) continue;"),
    "brute_shared_not_per_block": ("if (x->space == 1 && bx != by) continue;", ""),
    "closed_shared_not_per_block": ("x->lblock = r->space == 1 ? x->block : 0xFFFFFFFFu;",
                                    "x->lblock = 0xFFFFFFFFu;"),
    "closed_epoch_groups_by_block": ("while (je < jb && it[je].epoch == it[ie].epoch)",
                                     "while (je < jb && it[je].block == it[ie].block)"),
    "brute_same_thread_allowed": ("if (x->tid == y->tid) continue;", ""),
    "kinds_aw_ar_swapped": ("(e->pairs_aw ? 4 : 0) |\n                       (e->pairs_ar ? 8 : 0)",
                            "(e->pairs_aw ? 8 : 0) |\n                       (e->pairs_ar ? 4 : 0)"),
    "kinds_xblock_dropped": (" | (e->pairs_xblock ? 16 : 0)", ""),
    "kinds_rw_from_ww": ("(e->pairs_rw ? 2 : 0)", "(e->pairs_ww ? 2 : 0)"),
    "kinds_ww_bit_dropped": ("(e->pairs_ww ? 1 : 0) | ", ""),
    "block_from_wrong_tpb": ("  x->block = r->tid / T;", "  x->block = r->tid / (T + 1);"),
}


def _build_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mut = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mut)
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c), "-o", str(so)], check=True)
    return str(so)


def _pins_pass():
    """The pin checks, run against whatever library oracle._lib holds."""
    for line, recs, exp in truth_table():
        for fn in (oracle.brute_force, oracle.closed_form):
            if oracle.races_to_dict(fn(recs, tpb=2)[0], kinds=True) != exp:
                return False
    for name in ("fig6_unit.txt", "fig6_unit_write.txt", "kaldi_copy.txt", "mixed_kinds.txt"):
        recs, tpb, exp = trace_fixture(name)
        for fn in (oracle.brute_force, oracle.closed_form):
            if oracle.races_to_dict(fn(recs, tpb=tpb)[0], kinds=True) != exp:
                return False
    for removed in range(-1, 9):
        recs = tracegen.tree_reduction(removed)
        n_exp = (128 >> removed) if 0 <= removed < 8 else 0
        for fn in (oracle.brute_force, oracle.closed_form):
            if len(fn(recs, tpb=256)[0]) != n_exp:
                return False
    for seed in range(30):
        rng = np.random.default_rng(seed)
        tpb = int(rng.integers(1, 5))
        r = tracegen.random_small(rng, int(rng.integers(0, 65)), units=int(rng.integers(1, 5)),
                                  blocks=int(rng.integers(1, 4)), tpb=tpb, epochs=int(rng.integers(1, 4)))
        want = oracle.tier_a_py(r, tpb)
        for fn in (oracle.brute_force, oracle.closed_form):
            if oracle.races_to_dict(fn(r, tpb=tpb)[0]) != want:
                return False
    return True


def test_real_oracle_passes_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    so = _build_mutant(name, tmp_path)
    saved = oracle._load()
    mutant = ctypes.CDLL(so)
    for fname in ("orc_brute_force", "orc_closed_form"):
        f = getattr(mutant, fname)
        f.restype = getattr(saved, fname).restype
        f.argtypes = getattr(saved, fname).argtypes
    mutant.orc_free.restype = None
    mutant.orc_free.argtypes = [ctypes.c_void_p]
    oracle._lib = mutant
    try:
        assert not _pins_pass(), f"mutant {name} survived every pin"
    finally:
        oracle._lib = saved
