"""The oracle's D2Q9 tables against the values the paper prints (tests/golden)."""
import ctypes as C
import math
import os

import numpy as np

from oracle.oracle import lib, ptr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d2q9_eq17_eq20.txt")


def read_golden():
    rows, cs2 = [], None
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "cs2":
                cs2 = int(line[1]) / int(line[2])
            else:
                rows.append([int(v) for v in line])
    return rows, cs2


def test_oracle_lattice_matches_printed_eq17_eq20():
    rows, cs2 = read_golden()
    ex = (C.c_int32 * 9)()
    ey = (C.c_int32 * 9)()
    w = np.zeros(9)
    lib().orc_lattice(ex, ey, ptr(w))
    assert len(rows) == 9
    for a, wn, wd, an, ad, l2 in rows:
        assert w[a] == wn / wd
        length = math.sqrt(l2)
        ang = math.pi * an / ad
        assert abs(ex[a] - length * math.cos(ang)) < 1e-12 and abs(ey[a] - length * math.sin(ang)) < 1e-12
    # second moment of the weights is c_s^2 I (the printed c_s = 1/sqrt(3))
    exs, eys = np.array(ex[:], float), np.array(ey[:], float)
    assert abs(np.sum(w * exs * exs) - cs2) < 1e-15 and abs(np.sum(w * eys * eys) - cs2) < 1e-15
    assert abs(np.sum(w * exs * eys)) < 1e-15
