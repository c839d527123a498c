"""CPU oracle of the adaptive k-NN query path (PUFFINN, ESA 2019) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  It wraps ``liboracle.so`` (plain C, see ``puffinn_oracle.c``)
with numpy and shares no code with the GPU library in ``paper_1906_12211_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "puffinn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RULE_FILTER = 0
RULE_EXACT = 1
RULE_ALG1 = 2
RULE_POOL = 3
DEFAULT_POOL = 3072
DEFAULT_K = 24
DEFAULT_M = 32
DEFAULT_B = 12
DEFAULT_GROUPS = 16  # stopping tests per level (at most L): the method's default parameter
DEFAULT_TEST_ENTRIES = 256  # a group's test waits for this many entries since the previous one


def build(verbose: bool = False) -> str:
    """Compile liboracle.so in place (gcc, OpenMP, no FMA contraction)."""
    cmd = [
        "gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
        "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_D = ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_splitmix64.restype = _U64
        L.oracle_splitmix64.argtypes = [_U64, _U64]
        L.oracle_hyperplanes.restype = None
        L.oracle_hyperplanes.argtypes = [_U64, _I64, _I32, _P]
        L.oracle_normalize.restype = _I64
        L.oracle_normalize.argtypes = [_P, _I64, _I32]
        L.oracle_num_tables.restype = _I64
        L.oracle_num_tables.argtypes = [_I64, _I32, _I32, _I32, _I32, _I32, _U64]
        L.oracle_cp_dims.restype = _I32
        L.oracle_cp_dims.argtypes = [_I32, _P, _P]
        L.oracle_cp_value.restype = ctypes.c_uint32
        L.oracle_cp_value.argtypes = [_P, _I32, _U64, _U64]
        L.oracle_cp_hash.restype = None
        L.oracle_cp_hash.argtypes = [_P, _I64, _I32, _U64, _I32, _I32, _P]
        L.oracle_cp_table.restype = None
        L.oracle_cp_table.argtypes = [_U64, _I32, _I32, _P]
        L.oracle_cp_prob.restype = _D
        L.oracle_cp_prob.argtypes = [_P, _I32, ctypes.c_float, _I32]
        L.oracle_pool_select.restype = ctypes.c_int
        L.oracle_pool_select.argtypes = [_U64, _I32, _I32, _I32, _P]
        L.oracle_hash.restype = None
        L.oracle_hash.argtypes = [_P, _I64, _I32, _P, _I32, _I32, _I32, _P, _I32, _P, _P]
        L.oracle_build_tables.restype = ctypes.c_int
        L.oracle_build_tables.argtypes = [_P, _I64, _I32, _I32, _P, _P, _P]
        L.oracle_table_sketches.restype = None
        L.oracle_table_sketches.argtypes = [_P, _P, _I64, _I32, _I32, _P]
        L.oracle_ip32.restype = ctypes.c_float
        L.oracle_ip32.argtypes = [_P, _P, _I32]
        L.oracle_ip64.restype = _D
        L.oracle_ip64.argtypes = [_P, _P, _I32]
        L.oracle_collision_prob.restype = _D
        L.oracle_collision_prob.argtypes = [ctypes.c_float]
        L.oracle_tau.restype = _D
        L.oracle_tau.argtypes = [ctypes.c_float, _D]
        L.oracle_stop.restype = ctypes.c_int
        L.oracle_stop.argtypes = [ctypes.c_float, _I32, _I32, _I32, _D, _I32, _I32, _I32, _P, _I32,
                                  ctypes.POINTER(_D)]
        L.oracle_stop_partial.restype = ctypes.c_int
        L.oracle_stop_partial.argtypes = [ctypes.c_float, _I32, _I32, _I32, _I32, _I32, _D, _I32, _I32, _I32, _P,
                                          _I32, ctypes.POINTER(_D)]
        L.oracle_binom_cdf64.restype = _D
        L.oracle_binom_cdf64.argtypes = [_D, _I32]
        L.oracle_search.restype = ctypes.c_int
        L.oracle_search.argtypes = [
            _P, _I64, _I32, _P, _P, _P, _P, _I32, _I32, _I32, _P, _I32, _P, _U64,
            _P, _I64, _I32, _D, _D, _I32, _I32, _I32, _I32, _I32,
            _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
        ]
        L.oracle_bruteforce.restype = ctypes.c_int
        L.oracle_bruteforce.argtypes = [_P, _I64, _I32, _P, _I64, _I32, _P, _P]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [_I32]
        L.oracle_num_threads.argtypes = []
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------- primitives
def splitmix64(seed: int, s: int) -> int:
    return int(lib().oracle_splitmix64(seed, s))


def hyperplanes(seed: int, rows: int, d: int) -> np.ndarray:
    out = np.empty((rows, d), dtype=np.float32)
    lib().oracle_hyperplanes(seed, rows, d, _ptr(out))
    return out


def normalize(x: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(x, dtype=np.float32).copy()
    bad = lib().oracle_normalize(_ptr(y), y.shape[0], y.shape[1])
    if bad >= 0:
        raise ValueError(f"row {bad} has zero or non-finite norm")
    return y


def num_tables(n: int, d: int, budget: int, K: int = DEFAULT_K, M: int = DEFAULT_M, pool: int = 0,
               cp: bool = False) -> int:
    return int(lib().oracle_num_tables(n, d, K, M, pool, 1 if cp else 0, budget))


CP_MC_DRAWS = 1000   # Monte Carlo functions per tabulated similarity (Sec. 4.3)
CP_GRID = 41         # similarities -1, -0.95, ..., 1


def cp_dims(d: int):
    """(d', ell): the padded power-of-two dimension and the bits of one FHT-CP value."""
    dp, ell = ctypes.c_int32(), ctypes.c_int32()
    lib().oracle_cp_dims(d, ctypes.byref(dp), ctypes.byref(ell))
    return dp.value, ell.value


def cp_value(x: np.ndarray, seed: int, fn: int) -> int:
    x = np.ascontiguousarray(x, dtype=np.float32)
    return int(lib().oracle_cp_value(_ptr(x), x.shape[0], seed, fn))


def cp_hash(x: np.ndarray, seed: int, L: int, K: int) -> np.ndarray:
    """codes[L][n] of normalised rows x under FHT cross-polytope tables."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, d = x.shape
    codes = np.empty((L, n), dtype=np.uint32)
    lib().oracle_cp_hash(_ptr(x), n, d, seed, L, K, _ptr(codes))
    return codes


def cp_table(seed: int, d: int, draws: int = CP_MC_DRAWS) -> np.ndarray:
    """tab[g][b]: collision probability of b-bit prefixes at similarity -1 + 0.05 g."""
    _, ell = cp_dims(d)
    tab = np.empty((CP_GRID, ell + 1), dtype=np.float64)
    lib().oracle_cp_table(seed, d, draws, _ptr(tab))
    return tab


def cp_prob(tab: np.ndarray, ip: float, i: int) -> float:
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    return float(lib().oracle_cp_prob(_ptr(tab), tab.shape[1] - 1, ip, i))


def pool_select(seed: int, pool: int, L: int, K: int) -> np.ndarray:
    """sel[L][K]: pool index of h_{t+1,j} for every trie j (pooling, Sec. 3.2)."""
    sel = np.empty((L, K), dtype=np.int32)
    rc = lib().oracle_pool_select(seed, pool, L, K, _ptr(sel))
    if rc:
        raise ValueError(f"oracle_pool_select rc={rc}")
    return sel


def hash_codes(x: np.ndarray, hp: np.ndarray, L: int, K: int, M: int, sel: np.ndarray | None = None):
    """codes[L][n] (u32), sketches[M][n] (u64) of normalised rows x; with sel (pooling)
    hp holds the pool functions, then the sketch functions."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, d = x.shape
    pool = 0
    if sel is None:
        assert hp.shape == (L * K + 64 * M, d)
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        assert sel.shape == (L, K)
        pool = hp.shape[0] - 64 * M
    codes = np.empty((L, n), dtype=np.uint32)
    sk = np.empty((M, n), dtype=np.uint64)
    lib().oracle_hash(_ptr(x), n, d, _ptr(np.ascontiguousarray(hp)), L, K, M, _ptr(sel), pool, _ptr(codes),
                      _ptr(sk))
    return codes, sk


def build_tables(codes: np.ndarray, K: int):
    L, n = codes.shape
    P = min(13, K)
    tcode = np.empty((L, n), dtype=np.uint32)
    tidx = np.empty((L, n), dtype=np.uint32)
    off = np.empty((L, (1 << P) + 1), dtype=np.uint32)
    rc = lib().oracle_build_tables(_ptr(np.ascontiguousarray(codes)), n, L, K, _ptr(tcode), _ptr(tidx), _ptr(off))
    if rc:
        raise MemoryError("oracle_build_tables")
    return tcode, tidx, off


def table_sketches(tidx: np.ndarray, sketches: np.ndarray) -> np.ndarray:
    L, n = tidx.shape
    M = sketches.shape[0]
    tsk = np.empty((L, n), dtype=np.uint64)
    lib().oracle_table_sketches(_ptr(tidx), _ptr(np.ascontiguousarray(sketches)), n, L, M, _ptr(tsk))
    return tsk


def ip32(x: np.ndarray, q: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    return float(lib().oracle_ip32(_ptr(x), _ptr(q), x.shape[0]))


def ip64(x: np.ndarray, q: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    return float(lib().oracle_ip64(_ptr(x), _ptr(q), x.shape[0]))


def collision_prob(ip: float) -> float:
    return float(lib().oracle_collision_prob(ip))


def tau(ip_k: float, eps: float = 0.0) -> float:
    return float(lib().oracle_tau(ip_k, eps))


def stop(ip_k: float, i: int, L: int, delta: float, rule: int = RULE_EXACT, M: int = DEFAULT_M,
         tau_int: int = 64, pool: int = 0, cptab: np.ndarray | None = None):
    m = _D()
    tab = None if cptab is None else np.ascontiguousarray(cptab, dtype=np.float64)
    ell = 0 if tab is None else tab.shape[1] - 1
    r = lib().oracle_stop(ip_k, i, L, M, delta, rule, tau_int, pool, _ptr(tab), ell, ctypes.byref(m))
    return bool(r), float(m.value)


def stop_partial(ip_k: float, i: int, a: int, L: int, K: int, delta: float, rule: int = RULE_EXACT,
                 M: int = DEFAULT_M, tau_int: int = 64, pool: int = 0, cptab: np.ndarray | None = None):
    """The stopping test with the first a of L repetitions at level i and the rest at level
    i + 1 (none taken when i = K)."""
    m = _D()
    tab = None if cptab is None else np.ascontiguousarray(cptab, dtype=np.float64)
    ell = 0 if tab is None else tab.shape[1] - 1
    r = lib().oracle_stop_partial(ip_k, i, a, L, M, K, delta, rule, tau_int, pool, _ptr(tab), ell, ctypes.byref(m))
    return bool(r), float(m.value)


def binom_cdf64(t: float, T: int) -> float:
    return float(lib().oracle_binom_cdf64(t, T))


def bruteforce(points_n: np.ndarray, queries_n: np.ndarray, k: int):
    """Exact k-NN of normalised queries over normalised points: (ids, FP64 ips)."""
    p = np.ascontiguousarray(points_n, dtype=np.float32)
    q = np.ascontiguousarray(queries_n, dtype=np.float32)
    m = q.shape[0]
    ids = np.empty((m, k), dtype=np.int32)
    ips = np.empty((m, k), dtype=np.float64)
    rc = lib().oracle_bruteforce(_ptr(p), p.shape[0], p.shape[1], _ptr(q), m, k, _ptr(ids), _ptr(ips))
    if rc:
        raise ValueError(f"oracle_bruteforce rc={rc}")
    return ids, ips


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(t: int) -> None:
    """Threads of the following oracle calls (timing only)."""
    lib().oracle_set_threads(int(t))


# ----------------------------------------------------------------------------- index
@dataclass
class SearchResult:
    ids: np.ndarray
    ips: np.ndarray
    ips64: np.ndarray
    stop_level: np.ndarray
    c_scan: np.ndarray
    c_pass: np.ndarray
    c_rerank: np.ndarray
    boundary: np.ndarray
    trace: np.ndarray | None = None
    levels: np.ndarray | None = None  # (K+1) x 8, see level_trace()


class OracleIndex:
    """The index of Sec. 4.1-4.2 built step by step on the CPU."""

    def __init__(self, points: np.ndarray, budget: int, seed: int = 42, K: int = DEFAULT_K,
                 M: int = DEFAULT_M, L: int | None = None, pool: int = 0, cp: bool = False):
        """pool = m > 0: the tries sample their K functions from a pool of m (Sec. 3.2);
        cp: FHT cross-polytope codes with Monte Carlo collision tables (Sec. 4.3)."""
        pts = np.ascontiguousarray(points, dtype=np.float32)
        self.n, self.d = pts.shape
        self.K, self.M, self.pool, self.cp, self.seed = K, M, int(pool), bool(cp), seed
        if self.cp and self.pool:
            raise ValueError("pooling is for hyperplane functions here")
        self.L = num_tables(self.n, self.d, budget, K, M, self.pool, self.cp) if L is None else int(L)
        if self.L < 1:
            raise ValueError("memory budget holds no table")
        self.points = normalize(pts)
        self.cptab = None
        if self.cp:
            self.sel = None
            self.hp = hyperplanes(seed, 64 * M, self.d)
            self.cptab = cp_table(seed, self.d)
            self.codes = cp_hash(self.points, seed, self.L, K)
            _, self.sketches = hash_codes(self.points, self.hp, 0, K, M)
            self.tcode, self.tidx, self.off = build_tables(self.codes, K)
            self.tsk = table_sketches(self.tidx, self.sketches)
            return
        if self.pool:
            self.sel = pool_select(seed, self.pool, self.L, K)
            self.hp = hyperplanes(seed, self.pool + 64 * M, self.d)
        else:
            self.sel = None
            self.hp = hyperplanes(seed, self.L * K + 64 * M, self.d)
        codes, self.sketches = hash_codes(self.points, self.hp, self.L, K, M, self.sel)
        self.codes = codes
        self.tcode, self.tidx, self.off = build_tables(codes, K)
        self.tsk = table_sketches(self.tidx, self.sketches)

    def search(self, queries: np.ndarray, k: int, recall: float, eps: float = 0.0,
               B: int = DEFAULT_B, rule: int = RULE_FILTER, filter_on: bool = True,
               trace: bool = False, groups: int | None = None, test_entries: int | None = None) -> SearchResult:
        """groups: stopping tests per level (None: min(L, DEFAULT_GROUPS)); test_entries: a
        group's test is skipped while fewer entries were read since the previous test (None:
        DEFAULT_TEST_ENTRIES; 0: a test after every group)."""
        if groups is None:
            groups = min(self.L, DEFAULT_GROUPS)
        if test_entries is None:
            test_entries = DEFAULT_TEST_ENTRIES
        return search_tables(self.points, self.hp, self.tcode, self.tidx, self.tsk, self.K, self.M, queries, k,
                             recall, eps=eps, B=B, rule=rule, filter_on=filter_on, trace=trace, groups=groups,
                             test_entries=test_entries,
                             sel=getattr(self, "sel", None), pool=getattr(self, "pool", 0),
                             cptab=getattr(self, "cptab", None), seed=getattr(self, "seed", 0))


LEVEL_TRACE_W = 8  # columns of SearchResult.levels


def search_tables(points: np.ndarray, hp: np.ndarray, tcode: np.ndarray, tidx: np.ndarray, tsk: np.ndarray,
                  K: int, M: int, queries: np.ndarray, k: int, recall: float, eps: float = 0.0,
                  B: int = DEFAULT_B, rule: int = RULE_FILTER, filter_on: bool = True, trace: bool = False,
                  sel: np.ndarray | None = None, pool: int = 0, cptab: np.ndarray | None = None,
                  seed: int = 0, groups: int = 1, test_entries: int = 0) -> SearchResult:
    """The adaptive query over given tables: normalised points (n x d), the hyperplanes
    the queries are hashed with, and the L sorted tables (codes, positions, table-local
    sketches).  groups: the stopping test runs after each of that many consecutive groups
    of tables in a level (1: once per level); test_entries > 0 skips a group's test while
    fewer entries than that were read since the level's previous test.  With trace=True the walk of query 0 is
    recorded: ``trace`` per level and
    table (lo_i, hi_i, c_lo, c_hi), ``levels`` per level (threshold used, masks of the new,
    passing and top-k point ids, c_scan, c_pass, c_rerank, stopped)."""
    points = np.ascontiguousarray(points, dtype=np.float32)
    n, d = points.shape
    tcode = np.ascontiguousarray(tcode, dtype=np.uint32)
    tidx = np.ascontiguousarray(tidx, dtype=np.uint32)
    tsk = np.ascontiguousarray(tsk, dtype=np.uint64)
    L = tcode.shape[0]
    assert tcode.shape == tidx.shape == tsk.shape == (L, n)
    hp = np.ascontiguousarray(hp, dtype=np.float32)
    q = np.ascontiguousarray(queries, dtype=np.float32)
    assert q.ndim == 2 and q.shape[1] == d
    m = q.shape[0]
    ids = np.empty((m, k), dtype=np.int32)
    ips = np.empty((m, k), dtype=np.float32)
    ips64 = np.empty((m, k), dtype=np.float64)
    sl = np.empty(m, dtype=np.int32)
    cs = np.empty(m, dtype=np.int64)
    cp = np.empty(m, dtype=np.int64)
    cr = np.empty(m, dtype=np.int64)
    bd = np.empty(m, dtype=np.int32)
    tr = np.zeros((K + 1, L, 4), dtype=np.int64) if trace else None
    lt = np.zeros((K + 1, LEVEL_TRACE_W), dtype=np.int64) if trace else None
    sel = None if sel is None else np.ascontiguousarray(sel, dtype=np.int32)
    tab = None if cptab is None else np.ascontiguousarray(cptab, dtype=np.float64)
    rc = lib().oracle_search(
        _ptr(points), n, d, _ptr(hp), _ptr(tcode), _ptr(tidx), _ptr(tsk), L, K, M, _ptr(sel), pool,
        _ptr(tab), seed, _ptr(q), m, k, recall, eps, B, rule,
        1 if filter_on else 0, int(groups), int(test_entries), _ptr(ids), _ptr(ips), _ptr(ips64), _ptr(sl), _ptr(cs),
        _ptr(cp), _ptr(cr), _ptr(bd), _ptr(tr), _ptr(lt))
    if rc:
        raise ValueError(f"oracle_search rc={rc}")
    return SearchResult(ids, ips, ips64, sl, cs, cp, cr, bd, tr, lt)
