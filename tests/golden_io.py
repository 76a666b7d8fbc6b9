"""Parsers for the hand-written fixtures under tests/golden/."""
import os

import numpy as np

from tracegen import RECORD_DTYPE

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
ACT = {"R": 0, "W": 1, "A": 2}
SPACE = {"G": 0, "S": 1}
# kinds bits of an entry, as the interface defines them
KIND_BIT = {"WW": 1, "RW": 2, "AW": 4, "AR": 8, "XBLOCK": 16}


def _kinds(text):
    """Bits of a hand-written kinds column ("-" or tag names)."""
    text = text.strip()
    if text == "-":
        return 0
    bits = 0
    for tag in text.split():
        bits |= KIND_BIT[tag]
    return bits


def _check_kinds(counts, bits, line):
    """The fixture's own consistency: a kind is listed iff its count > 0."""
    want = sum(b for k, b in KIND_BIT.items() if counts[k.lower()] > 0)
    assert want == bits, f"kinds column disagrees with the counts: {line}"


def counts_only(exp):
    """Expected dict without the kinds bits (for renderings that only count)."""
    return {k: {f: v for f, v in d.items() if f != "kinds"} for k, d in exp.items()}


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line


def truth_table():
    """Yield (records, expected dict with kinds bits) per row of truth_table.txt."""
    rows = []
    for line in _lines("truth_table.txt"):
        lhs, rhs, kinds = line.split("|")
        sp, a1, a2, t1, t2, e1, e2, u1, u2 = lhs.split()
        ww, rw, aw, ar, xb = (int(v) for v in rhs.split())
        bits = _kinds(kinds)
        r = np.zeros(2, dtype=RECORD_DTYPE)
        s1, s2 = (0, 1) if sp == "X" else (SPACE[sp], SPACE[sp])
        r[0] = (int(u1), int(t1), int(e1), ACT[a1], s1)
        r[1] = (int(u2), int(t2), int(e2), ACT[a2], s2)
        exp = {}
        if ww + rw + aw + ar:
            block = (int(t1) // 2) if s1 == 1 else None
            exp[(s1, block, int(u1))] = {"ww": ww, "rw": rw, "aw": aw, "ar": ar, "xblock": xb, "kinds": bits}
            _check_kinds(exp[(s1, block, int(u1))], bits, line)
        else:
            assert bits == 0, line
        rows.append((line, r, exp))
    return rows


def trace_fixture(name):
    """Return (records, tpb, expected dict with kinds bits) of a trace fixture."""
    tpb = None
    recs = []
    exp = {}
    for line in _lines(name):
        f = line.split()
        if f[0] == "tpb":
            tpb = int(f[1])
        elif f[0] == "rec":
            recs.append((int(f[1]), int(f[2]), int(f[3]), ACT[f[4]], SPACE[f[5]]))
        elif f[0] == "expect":
            lhs, rhs, kinds = line[len("expect"):].split("|")
            sp, blk, unit = lhs.split()
            ww, rw, aw, ar, xb = (int(v) for v in rhs.split())
            key = (SPACE[sp], None if blk == "-" else int(blk), int(unit))
            exp[key] = {"ww": ww, "rw": rw, "aw": aw, "ar": ar, "xblock": xb, "kinds": _kinds(kinds)}
            _check_kinds(exp[key], exp[key]["kinds"], line)
    r = np.zeros(len(recs), dtype=RECORD_DTYPE)
    for i, v in enumerate(recs):
        r[i] = v
    return r, tpb, exp


def barrier_fixture(name):
    """Return (records, tpb, {boundary: (instances, racing)}) of a barrier
    fixture (rec lines as in trace fixtures, expect_barrier lines)."""
    tpb = None
    recs = []
    exp = {}
    for line in _lines(name):
        f = line.split()
        if f[0] == "tpb":
            tpb = int(f[1])
        elif f[0] == "rec":
            recs.append((int(f[1]), int(f[2]), int(f[3]), ACT[f[4]], SPACE[f[5]]))
        elif f[0] == "expect_barrier":
            lhs, rhs = line[len("expect_barrier"):].split("|")
            inst, rac = (int(v) for v in rhs.split())
            exp[int(lhs)] = (inst, rac)
    r = np.zeros(len(recs), dtype=RECORD_DTYPE)
    for i, v in enumerate(recs):
        r[i] = v
    return r, tpb, exp
