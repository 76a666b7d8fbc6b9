"""Parsers for the hand-written fixtures under tests/golden/."""
import os

import numpy as np

from tracegen import RECORD_DTYPE

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
ACT = {"R": 0, "W": 1, "A": 2}
SPACE = {"G": 0, "S": 1}


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line


def truth_table():
    """Yield (records, expected dict) per row of truth_table.txt."""
    rows = []
    for line in _lines("truth_table.txt"):
        lhs, rhs = line.split("|")
        sp, a1, a2, t1, t2, e1, e2, u1, u2 = lhs.split()
        ww, rw, aw, ar, xb = (int(v) for v in rhs.split())
        r = np.zeros(2, dtype=RECORD_DTYPE)
        s1, s2 = (0, 1) if sp == "X" else (SPACE[sp], SPACE[sp])
        r[0] = (int(u1), int(t1), int(e1), ACT[a1], s1)
        r[1] = (int(u2), int(t2), int(e2), ACT[a2], s2)
        exp = {}
        if ww + rw + aw + ar:
            block = (int(t1) // 2) if s1 == 1 else None
            exp[(s1, block, int(u1))] = {"ww": ww, "rw": rw, "aw": aw, "ar": ar, "xblock": xb}
        rows.append((line, r, exp))
    return rows


def trace_fixture(name):
    """Return (records, tpb, expected dict) of a trace fixture."""
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
            lhs, rhs = line[len("expect"):].split("|")
            sp, blk, unit = lhs.split()
            ww, rw, aw, ar, xb = (int(v) for v in rhs.split())
            key = (SPACE[sp], None if blk == "-" else int(blk), int(unit))
            exp[key] = {"ww": ww, "rw": rw, "aw": aw, "ar": ar, "xblock": xb}
    r = np.zeros(len(recs), dtype=RECORD_DTYPE)
    for i, v in enumerate(recs):
        r[i] = v
    return r, tpb, exp
