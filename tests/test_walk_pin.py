"""Hand-computed pin of the oracle's level walk (Algorithm 1 as the rounds of Sec. 4.1, the
sketch filter of Sec. 4.2 with the threshold of Sec. 5.1, the stopping bound of Lemma 1).

A ten-point index is written out by hand: two tables (L = 2) of K = 4 bits, M = 2 sketches
(table j reads sketch j mod 2), the query q = e_0 in d = 4.  Point x has
x = (c_x, sqrt(1 - c_x^2), 0, 0), so its FP32 inner product with q is exactly c_x, and its
sketches differ from the query's in exactly h_x bits.  The query's codes (table 0: 1011,
table 1: 0100) and sketches are set by the signs of the hyperplanes' first coordinates.
Every expected value below follows by hand from those numbers; the arithmetic is in the
comments (theta/pi = acos(c)/pi, tau = (1 + eps) 64 theta/pi, p = 1 - theta/pi).

Sorted table 0 (code: point):  1:7  3:4  6:8  8:6  9:5  10:0  10:3  11:2  11:9  14:1
Sorted table 1 (code: point):  0:6  2:0  4:8  5:1  5:7  6:4  7:5  9:9  12:2  15:3
Query code 11 in table 0 starts the window at entry 7; query code 4 in table 1 at entry 2.
"""
import math
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

C = [0.25, 0.9375, 0.5, 0.75, -0.5, 0.875, 0.0, 0.625, 0.125, 0.375]  # c_x = <x, q>
H = [30, 5, 20, 22, 40, 9, 14, 24, 33, 26]                            # Hamming distance h_x
CODES = [[10, 14, 11, 10, 3, 9, 8, 1, 6, 11],                         # table 0 code of x
         [2, 5, 12, 15, 6, 7, 0, 5, 4, 9]]                            # table 1 code of x
QCODE = [0b1011, 0b0100]
K, L, M, D, N = 4, 2, 2, 4, 10
QSK = [0x5A5A_F00F_3C3C_0FF0, 0x0123_4567_89AB_CDEF]                  # query sketches


def _instance():
    X = np.zeros((N, D), dtype=np.float32)
    for x, c in enumerate(C):
        X[x, 0] = c
        X[x, 1] = math.sqrt(1.0 - c * c)
    # hyperplanes: rows j K + (s - 1) are h_{s,j} (s = 1 the most significant bit), then the
    # 64 M sketch rows; only the first coordinate meets q = e_0, and bit = 1 iff it is >= 0
    hp = np.zeros((L * K + 64 * M, D), dtype=np.float32)
    for j in range(L):
        for s in range(K):
            hp[j * K + s, 0] = 1.0 if (QCODE[j] >> (K - 1 - s)) & 1 else -1.0
    for m in range(M):
        for b in range(64):
            hp[L * K + 64 * m + b, 0] = 1.0 if (QSK[m] >> b) & 1 else -1.0
    # point sketches: the query's with the lowest h_x bits flipped
    sk = np.zeros((M, N), dtype=np.uint64)
    for m in range(M):
        for x in range(N):
            sk[m, x] = QSK[m] ^ ((1 << H[x]) - 1)
    tcode = np.zeros((L, N), dtype=np.uint32)
    tidx = np.zeros((L, N), dtype=np.uint32)
    for j in range(L):
        order = sorted(range(N), key=lambda x: (CODES[j][x], x))
        tcode[j] = [CODES[j][x] for x in order]
        tidx[j] = order
    tsk = np.stack([sk[j % M, tidx[j]] for j in range(L)])
    q = np.zeros((1, D), dtype=np.float32)
    q[0, 0] = 1.0
    return X, hp, tcode, tidx, tsk, q


def _ids(*xs):
    m = 0
    for x in xs:
        m |= 1 << x
    return m


# Walk with segments of B = 1 (windows grow exactly to the prefix ranges):
#  level 4: tau 64 (top-k empty).  New: table 0 entries 7, 8 (points 2, 9); table 1 entry 2
#           (point 8).  All pass.  Top-2: 2 (.5), 9 (.375).
#           Exact rule: p = .622357, 2 log1p(-p^4) = -0.325 > ln .1 = -2.303: go on.
#  level 3: tau from ip_k = .375: theta/pi = .377643, 64 x = 24.169 -> 24.  New: table 0
#           entries 5, 6 (points 0, 3); table 1 entries 3, 4 (points 1, 7).  h: 0 -> 30 fails,
#           3 -> 22, 1 -> 5, 7 -> 24 pass (24 <= 24).  Top-2: 1 (.9375), 3 (.75).
#           Exact: p = .769947, 2 log1p(-p^3) = -1.219: go on.  Filter-aware (q = P[Bin(64,
#           .230053) <= 24] = .99709, g_s = 1): 2 log(1 - q p^3) = -1.214: go on.
#           (A threshold from rank k-1 = .5 would be 21 and reject 3 and 7; one refreshed
#           after table 0, from top {3, 2}, would be 21 for table 1 and reject 7.)
#  level 2: tau from .75: 64 x .230053 = 14.723 -> 14.  New: table 0 entries 3, 4 (points
#           6, 5); table 1 entries 5, 6 (points 4, 5).  6 -> 14 passes, 5 -> 9 passes twice,
#           4 -> 40 fails.  Top-2: 1, 5 (.875).
#           Exact: p = .839139, 2 log1p(-p^2) = -2.436 <= -2.303: STOP (exact rule).
#           Filter-aware: q = P[Bin(64, .160861) <= 14] = .91913, 2 log(1 - q p^2) = -2.084:
#           go on.  Algorithm 1: L p^2 = 1.408 < ln 10 = 2.303: go on.
#  level 1: tau from .875: 64 x .160861 = 10.295 -> 10.  New: table 0 entry 9 (point 1);
#           table 1 entries 0, 1 (points 6, 0).  1 -> 5 passes; 6 -> 14, 0 -> 30 fail.
#           Filter-aware: q = .54311, 2 log(1 - q p) = -1.217: go on.  Algorithm 1:
#           L p = 1.678 < 2.303: go on.
#  level 0: linear scan, all ten points re-ranked: top-2 1, 5.
LEVELS_B1 = {
    #   tau, new ids, passing ids, c_scan, c_pass, c_rerank, top-k ids
    4: (64, _ids(2, 9, 8), _ids(2, 9, 8), 3, 3, 3, _ids(2, 9)),
    3: (24, _ids(0, 3, 1, 7), _ids(3, 1, 7), 7, 6, 6, _ids(1, 3)),
    2: (14, _ids(6, 5, 4), _ids(6, 5), 11, 9, 9, _ids(1, 5)),
    1: (10, _ids(1, 6, 0), _ids(1), 14, 10, 10, _ids(1, 5)),
}
# B = 2: table 0's windows fall on segment boundaries (the same new entries); table 1's
# window, starting at entry 2, takes [2, 4) at level 4 (points 8 and 1, though point 1's
# code 5 does not share the 4-bit prefix), [4, 6) at level 3, [6, 8) at level 2.
#  level 4: tau 64.  New: points 2, 9 (table 0), 8, 1 (table 1); all pass.  Top-2: 1, 2.
#           Exact: p = 2/3, 2 log1p(-(2/3)^4) = -0.440: go on (filter-aware the same, q = 1).
#  level 3: tau from .5: 64/3 = 21.333 -> 21.  New: 0, 3 (table 0), 7, 4 (table 1):
#           h = 30, 22, 24, 40 all fail.  Exact: 2 log1p(-(2/3)^3) = -0.703: go on;
#           filter-aware (q = P[Bin(64, 1/3) <= 21] = .52350): -0.337: go on.
#  level 2: tau 21.  New: 6, 5 (table 0), 5, 9 (table 1): 6 -> 14, 5 -> 9 (twice) pass,
#           9 -> 26 fails.  Top-2: 1, 5.  Exact: -2.436: STOP; filter-aware (q = .99973):
#           2 log(1 - q p^2) = -2.435 <= -2.303: STOP.
LEVELS_B2 = {
    4: (64, _ids(2, 9, 8, 1), _ids(2, 9, 8, 1), 4, 4, 4, _ids(1, 2)),
    3: (21, _ids(0, 3, 7, 4), 0, 8, 4, 4, _ids(1, 2)),
    2: (21, _ids(6, 5, 9), _ids(6, 5), 12, 7, 7, _ids(1, 5)),
}

# (B, rule, eps) -> (stop level, levels walked with their expected rows, c_rerank at the end)
CASES = {
    (1, oracle.RULE_EXACT, 0.0): (2, {i: LEVELS_B1[i] for i in (4, 3, 2)}, 9),
    (1, oracle.RULE_FILTER, 0.0): (0, LEVELS_B1, 20),
    (1, oracle.RULE_ALG1, 0.0): (0, LEVELS_B1, 20),
    (2, oracle.RULE_EXACT, 0.0): (2, LEVELS_B2, 7),
    (2, oracle.RULE_FILTER, 0.0): (2, LEVELS_B2, 7),
    # eps = 0.25: level 3's threshold is 1.25 x 24.169 = 30.211 -> 30, so point 0 (h = 30)
    # passes too; level 2's is 1.25 x 14.723 = 18.404 -> 18 (the same entries pass)
    (1, oracle.RULE_EXACT, 0.25): (2, {4: LEVELS_B1[4], 3: (30, _ids(0, 3, 1, 7), _ids(0, 3, 1, 7), 7, 7, 7,
                                                             _ids(1, 3)),
                                       2: (18, _ids(6, 5, 4), _ids(6, 5), 11, 10, 10, _ids(1, 5))}, 10),
}


def _walk(B, rule, eps, lib_search=None):
    X, hp, tcode, tidx, tsk, q = _instance()
    fn = lib_search or oracle.search_tables
    return fn(X, hp, tcode, tidx, tsk, K, M, q, 2, 0.9, eps=eps, B=B, rule=rule, trace=True)


def test_instance_is_what_the_docstring_says():
    X, hp, tcode, tidx, tsk, q = _instance()
    assert tcode[0].tolist() == [1, 3, 6, 8, 9, 10, 10, 11, 11, 14]
    assert tidx[0].tolist() == [7, 4, 8, 6, 5, 0, 3, 2, 9, 1]
    assert tcode[1].tolist() == [0, 2, 4, 5, 5, 6, 7, 9, 12, 15]
    assert tidx[1].tolist() == [6, 0, 8, 1, 7, 4, 5, 9, 2, 3]
    # the query hashes to the codes and sketches the walk assumes
    codes, sks = oracle.hash_codes(q, hp, L, K, M)
    assert codes[:, 0].tolist() == QCODE
    assert [int(v) for v in sks[:, 0]] == QSK
    for x in range(N):
        assert oracle.ip32(X[x], q[0]) == np.float32(C[x])
        for j in range(L):
            e = tidx[j].tolist().index(x)
            assert bin(int(tsk[j, e]) ^ QSK[j % M]).count("1") == H[x]


@pytest.mark.parametrize("case", sorted(CASES), ids=lambda c: f"B{c[0]}-rule{c[1]}-eps{c[2]}")
def test_level_walk_by_hand(case):
    B, rule, eps = case
    stop, levels, rerank = CASES[case]
    r = _walk(B, rule, eps)
    lv = r.levels
    for i in range(K, -1, -1):
        if i in levels:
            tau, new, pas, cs, cp, cr, top = levels[i]
            got = tuple(int(v) for v in lv[i, :7])
            assert got == (tau, new, pas, cs, cp, cr, top), f"level {i}: {got}"
            assert lv[i, 7] == (1 if i == stop else 0), f"level {i} stop flag"
        elif i == 0 and stop == 0:
            assert lv[0, 0] == -1 and lv[0, 7] == 1
        else:
            assert lv[i, 0] == -2, f"level {i} should not be reached"
    assert int(r.stop_level[0]) == stop
    assert r.ids[0].tolist() == [1, 5]
    assert r.ips[0].tolist() == [0.9375, 0.875]
    last = levels[min(levels)]
    assert int(r.c_scan[0]) == last[3] and int(r.c_pass[0]) == last[4]
    assert int(r.c_rerank[0]) == rerank


def test_window_trace_by_hand():
    """lo_i, hi_i and the windows after each level, per table (B = 1 and B = 2)."""
    r = _walk(1, oracle.RULE_FILTER, 0.0)
    lo_hi = {4: [(7, 9), (2, 3)], 3: [(5, 9), (2, 5)], 2: [(3, 9), (2, 7)], 1: [(3, 10), (0, 7)]}
    for i, rows in lo_hi.items():
        for j, (lo, hi) in enumerate(rows):
            assert tuple(r.trace[i, j]) == (lo, hi, lo, hi)
    r = _walk(2, oracle.RULE_FILTER, 0.0)
    win = {4: [(7, 9, 7, 9), (2, 3, 2, 4)], 3: [(5, 9, 5, 9), (2, 5, 2, 6)], 2: [(3, 9, 3, 9), (2, 7, 2, 8)]}
    for i, rows in win.items():
        for j, row in enumerate(rows):
            assert tuple(r.trace[i, j]) == row


# --------------------------------------------------------------- negative controls
# The pins above must fail for the two readings of the threshold that Sec. 4.2 / 5.1 do
# not take here: a threshold from another rank of the top-k, and a threshold refreshed
# inside a level after each table.  Each is planted in a copy of the oracle built in a
# temporary directory (the committed oracle is not touched).
_SRC = os.path.join(os.path.dirname(oracle.__file__), "puffinn_oracle.c")

_RANK = ("tau = oracle_tau(top->v[k - 1].ip, eps);", "tau = oracle_tau(top->v[k > 1 ? k - 2 : 0].ip, eps);")
_REFRESH = (
    "                    if (list_push(fresh, c)) return OR_ENOMEM;\n                }\n            }\n        }\n",
    "                    if (list_push(fresh, c)) return OR_ENOMEM;\n                }\n            }\n"
    "            if (accumulate(top, fresh, k)) return OR_ENOMEM;\n"
    "            fresh->len = 0;\n"
    "            if (filter_on && top->len == k) {\n"
    "                tau = oracle_tau(top->v[k - 1].ip, eps);\n"
    "                tau_int = tau >= 64.0 ? 64 : (tau < -1.0 ? -1 : (int32_t)floor(tau));\n"
    "            }\n"
    "        }\n",
)


def _mutant_search(tmp, name, plant):
    src = open(_SRC).read()
    assert src.count(plant[0]) == 1, "the planted line must occur once"
    path = os.path.join(tmp, name + ".c")
    open(path, "w").write(src.replace(plant[0], plant[1]))
    so = os.path.join(tmp, name + ".so")
    subprocess.run(["gcc", "-O1", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, path, "-lm"], check=True)
    import ctypes

    lib = ctypes.CDLL(so)
    lib.oracle_search.restype = ctypes.c_int
    lib.oracle_search.argtypes = oracle.lib().oracle_search.argtypes
    lib.oracle_hash.argtypes = oracle.lib().oracle_hash.argtypes

    def search(*a, **kw):
        saved = oracle._lib
        oracle._lib = lib
        try:
            return oracle.search_tables(*a, **kw)
        finally:
            oracle._lib = saved

    return search


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("plant", [_RANK, _REFRESH], ids=["tau-from-rank-k-1", "tau-refreshed-per-table"])
def test_pins_reject_other_threshold_readings(plant):
    with tempfile.TemporaryDirectory() as tmp:
        search = _mutant_search(tmp, "mutant", plant)
        r = _walk(1, oracle.RULE_EXACT, 0.0, lib_search=search)
        ok = r.levels[3, 2] == LEVELS_B1[3][2] and r.levels[3, 4] == LEVELS_B1[3][4]
        assert not ok, "the planted threshold reading went unnoticed"
