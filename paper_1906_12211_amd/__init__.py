"""Python binding of libpfhip.so, the gfx950 adaptive k-NN index (PUFFINN, ESA 2019).

Argument marshalling only: every step of build and search runs in the HIP library.
Functions carry the C-ABI names of ``include/pfhip.h``; ``Index`` wraps them for numpy
arrays (host memory) and torch tensors (device memory on the current HIP stream).
The library must be built first (``python -m paper_1906_12211_amd.build``); importing
works without it, but every call raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libpfhip.so")

PF_OK, PF_EINVAL, PF_EBUDGET, PF_ENOMEM, PF_EDEVICE, PF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PF_HOST, PF_DEVICE = 0, 1
PF_RULE_FILTER, PF_RULE_EXACT, PF_RULE_ALG1, PF_RULE_POOL = 0, 1, 2, 3
PF_HASH_BF16X3, PF_HASH_FP64 = 0, 1
(PF_EXPORT_POINTS, PF_EXPORT_HYPERPLANES, PF_EXPORT_CODES, PF_EXPORT_IDX,
 PF_EXPORT_SKETCHES, PF_EXPORT_OFFSETS, PF_EXPORT_POOL_SEL, PF_EXPORT_CP_TABLE, PF_EXPORT_ROWS8) = range(9)
PF_FAMILY_HP, PF_FAMILY_FHTCP = 0, 1
PF_MAX_TABLES, PF_MAX_K, PF_MAX_DIM = 512, 256, 4096

PF_BATCH_LEARNED, PF_BATCH_AUTOTUNE = 1, 2

PF_SCHED_IN, PF_SCHED_OUT, PF_SCHED_PARAMS = 98, 2, 29442

EXPORTED = ["pf_normalize", "pf_build_index", "pf_plan_index", "pf_search", "pf_search_ex", "pf_search_batch", "pf_search_noalloc", "pf_hash",
            "pf_export", "pf_index_info", "pf_last_timing", "pf_free_index", "pf_last_error", "pf_version",
            "pf_tile_count", "pf_tile_name", "pf_read_bandwidth", "pf_random_read_rate",
            "pf_sched_create", "pf_sched_free", "pf_sched_params", "pf_features", "pf_sched_predict",
            "pf_sched_grad", "pf_sched_train", "pf_sched_save", "pf_sched_load", "pf_index_set_scheduler"]


class PfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class pf_build_opts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("K", ctypes.c_int32), ("M", ctypes.c_int32),
                ("hash_mode", ctypes.c_int32), ("L_override", ctypes.c_int32), ("pool", ctypes.c_int32),
                ("family", ctypes.c_int32), ("pos_bytes", ctypes.c_int32),
                ("prefix_bits", ctypes.c_int32)]


class pf_search_opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("B", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("no_filter", ctypes.c_int32), ("timing", ctypes.c_int32), ("no_prefilter", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("groups", ctypes.c_int32), ("test_entries", ctypes.c_int32)]


class pf_query_stats(ctypes.Structure):
    _fields_ = [("stop_level", ctypes.c_int32), ("wave_us", ctypes.c_int32),
                ("c_scan", ctypes.c_int64), ("c_pass", ctypes.c_int64), ("c_rerank", ctypes.c_int64),
                ("c_exact", ctypes.c_int64), ("c_upper", ctypes.c_int64), ("c_q8", ctypes.c_int64)]


class pf_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("L", ctypes.c_int32),
                ("K", ctypes.c_int32), ("M", ctypes.c_int32), ("P", ctypes.c_int32),
                ("pool", ctypes.c_int32), ("family", ctypes.c_int32), ("bytes_budget_rule", ctypes.c_uint64),
                ("bytes_device", ctypes.c_uint64), ("build_ms", ctypes.c_double),
                ("pos_bytes", ctypes.c_int32)]


class pf_timing(ctypes.Structure):
    _fields_ = [("normalize_ms", ctypes.c_double), ("hash_ms", ctypes.c_double),
                ("ranges_ms", ctypes.c_double), ("search_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("tile", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("order_ms", ctypes.c_double), ("slots", ctypes.c_int64), ("groups", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I32, _I64, _U64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double


def lib():
    """Load libpfhip.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1906_12211_amd.build`")
        # torch ships its own HIP runtime under the same soname; load it first so that the
        # process holds one runtime, shared by torch's tensors/streams and this library
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        L.pf_last_error.restype = ctypes.c_char_p
        L.pf_last_error.argtypes = []
        L.pf_version.restype = ctypes.c_char_p
        L.pf_version.argtypes = []
        L.pf_tile_count.restype = _I32
        L.pf_tile_count.argtypes = []
        L.pf_tile_name.restype = ctypes.c_char_p
        L.pf_tile_name.argtypes = [_I32]
        L.pf_normalize.restype = ctypes.c_int
        L.pf_normalize.argtypes = [_P, _I64, _I32, _P, _I32, _P]
        L.pf_build_index.restype = ctypes.c_int
        L.pf_build_index.argtypes = [_P, _I64, _I32, _U64, ctypes.POINTER(pf_build_opts), _I32, _P,
                                     ctypes.POINTER(_P)]
        L.pf_read_bandwidth.restype = ctypes.c_int
        L.pf_read_bandwidth.argtypes = [_U64, _I32, ctypes.POINTER(_D), _P]
        L.pf_random_read_rate.restype = ctypes.c_int
        L.pf_random_read_rate.argtypes = [_U64, _I32, ctypes.POINTER(_D), _P]
        L.pf_plan_index.restype = ctypes.c_int
        L.pf_plan_index.argtypes = [_I64, _I32, _U64, ctypes.POINTER(pf_build_opts), ctypes.POINTER(_I32),
                                    ctypes.POINTER(_U64)]
        L.pf_search.restype = ctypes.c_int
        L.pf_search.argtypes = [_P, _P, _I64, _I32, _D, _P, _P, _P, _I32, _P]
        L.pf_search_ex.restype = ctypes.c_int
        L.pf_search_ex.argtypes = [_P, _P, _I64, _I32, _D, ctypes.POINTER(pf_search_opts), _P, _P, _P,
                                   _I32, _P]
        L.pf_search_noalloc.restype = ctypes.c_int
        L.pf_search_noalloc.argtypes = [_P, _P, _I64, _I32, _D, _P, _P, _P, _P]
        L.pf_search_batch.restype = ctypes.c_int
        L.pf_search_batch.argtypes = [_P, _P, _I64, _P, _P, _I32, ctypes.POINTER(pf_search_opts), _P, _P, _P,
                                      _P, _I32, _I32, _P]
        L.pf_hash.restype = ctypes.c_int
        L.pf_hash.argtypes = [_P, _P, _I64, _P, _P, _I32, _P]
        L.pf_export.restype = ctypes.c_int
        L.pf_export.argtypes = [_P, _I32, _P, _I64, _I32, _P]
        L.pf_index_info.restype = ctypes.c_int
        L.pf_index_info.argtypes = [_P, ctypes.POINTER(pf_info)]
        L.pf_last_timing.restype = ctypes.c_int
        L.pf_last_timing.argtypes = [_P, ctypes.POINTER(pf_timing)]
        L.pf_free_index.restype = None
        L.pf_free_index.argtypes = [_P]
        L.pf_sched_create.restype = ctypes.c_int
        L.pf_sched_create.argtypes = [_U64, ctypes.POINTER(_P)]
        L.pf_sched_free.restype = None
        L.pf_sched_free.argtypes = [_P]
        L.pf_sched_params.restype = ctypes.c_int
        L.pf_sched_params.argtypes = [_P, _P, _I32]
        L.pf_features.restype = ctypes.c_int
        L.pf_features.argtypes = [_P, _P, _I64, _P, _P, _I32, _D, _P, _I32, _P]
        L.pf_sched_predict.restype = ctypes.c_int
        L.pf_sched_predict.argtypes = [_P, _P, _I64, _P, _I32, _P]
        L.pf_sched_grad.restype = ctypes.c_int
        L.pf_sched_grad.argtypes = [_P, _P, _P, _I64, _P, ctypes.POINTER(_D), _I32, _P]
        L.pf_sched_train.restype = ctypes.c_int
        L.pf_sched_train.argtypes = [_P, _P, _P, _I64, _I32, _I32, ctypes.c_float, _U64, _P, _I32, _P]
        L.pf_sched_save.restype = ctypes.c_int
        L.pf_sched_save.argtypes = [_P, ctypes.c_char_p]
        L.pf_sched_load.restype = ctypes.c_int
        L.pf_sched_load.argtypes = [_P, ctypes.c_char_p]
        L.pf_index_set_scheduler.restype = ctypes.c_int
        L.pf_index_set_scheduler.argtypes = [_P, _P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PF_OK:
        raise PfError(rc, lib().pf_last_error().decode())


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _buf(a):
    """(pointer, mem, stream) of a contiguous numpy array or torch tensor."""
    if a is None:
        return None, PF_HOST, None
    if _is_torch(a):
        import torch

        assert a.is_contiguous()
        if a.is_cuda:
            return ctypes.c_void_p(a.data_ptr()), PF_DEVICE, ctypes.c_void_p(
                torch.cuda.current_stream(a.device).cuda_stream)
        return ctypes.c_void_p(a.data_ptr()), PF_HOST, None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p), PF_HOST, None


def _empty_like_input(x, shape, np_dtype, torch_dtype):
    if _is_torch(x):
        import torch

        return torch.empty(shape, dtype=torch_dtype, device=x.device)
    return np.empty(shape, dtype=np_dtype)


def _f32(x):
    if _is_torch(x):
        import torch

        return x.to(torch.float32).contiguous()
    return np.ascontiguousarray(x, dtype=np.float32)


def pf_version() -> str:
    return lib().pf_version().decode()


def pf_tile_count() -> int:
    return int(lib().pf_tile_count())


def pf_tile_name(t: int) -> str:
    return lib().pf_tile_name(t).decode()


def pf_normalize(x):
    x = _f32(x)
    out = _empty_like_input(x, tuple(x.shape), np.float32, x.dtype if _is_torch(x) else None)
    px, mem, st = _buf(x)
    po, _, _ = _buf(out)
    _check(lib().pf_normalize(px, x.shape[0], x.shape[1], po, mem, st))
    return out


def pf_read_bandwidth(nbytes: int = 4 << 30, reps: int = 5) -> float:
    """GB/s of a plain read-only streaming kernel on the current device (measurement aid)."""
    g = _D()
    _check(lib().pf_read_bandwidth(int(nbytes), int(reps), ctypes.byref(g), None))
    return float(g.value)


def pf_random_read_rate(nbytes: int = 4 << 30, reps: int = 5) -> float:
    """Scattered 4-byte loads per second on the current device (measurement aid)."""
    g = _D()
    _check(lib().pf_random_read_rate(int(nbytes), int(reps), ctypes.byref(g), None))
    return float(g.value)


def pf_plan_index(n: int, d: int, budget: int, K: int = 24, M: int = 32, L: int | None = None, pool: int = 0,
                  family: int = PF_FAMILY_HP, pos_bytes: int = 0, prefix_bits: int = 0):
    """(L, device bytes) that pf_build_index would use (host only, no device call)."""
    opts = pf_build_opts(0, K, M, PF_HASH_BF16X3, int(L or 0), int(pool), int(family), int(pos_bytes),
                         int(prefix_bits))
    nl, nb = _I32(), _U64()
    _check(lib().pf_plan_index(int(n), int(d), int(budget), ctypes.byref(opts), ctypes.byref(nl),
                               ctypes.byref(nb)))
    return int(nl.value), int(nb.value)


@dataclass
class SearchResult:
    ids: object
    ips: object
    stats: object  # (m, 7) int64: stop_level, c_scan, c_pass, c_rerank, c_exact, c_upper, c_q8
    wave_us: object = None  # (m,) int64: microseconds each query occupied its wave

    @property
    def stop_level(self):
        return self.stats[:, 0]


def _stats_view(raw):
    """pf_query_stats array (m x 56 bytes) as (m, 7) int64 columns (the first holds the
    stop level; the wave time, in its upper 32 bits, is split off by _wave_us)."""
    if _is_torch(raw):
        s = raw.clone()
        s[:, 0] = s[:, 0] & 0xFFFFFFFF
        return s
    s = raw.copy()
    s[:, 0] &= 0xFFFFFFFF
    return s


def _wave_us(raw):
    return raw[:, 0] >> 32


class Index:
    """An index over the rows of `points` (numpy on the host or a torch device tensor)."""

    def __init__(self, points, budget: int, seed: int = 42, K: int = 24, M: int = 32,
                 hash_mode: int = PF_HASH_BF16X3, L: int | None = None, pool: int = 0,
                 family: int = PF_FAMILY_HP, pos_bytes: int = 0, prefix_bits: int = 0):
        pts = _f32(points)
        n, d = pts.shape
        opts = pf_build_opts(seed, K, M, hash_mode, int(L or 0), int(pool), int(family), int(pos_bytes),
                             int(prefix_bits))
        pp, mem, st = _buf(pts)
        h = ctypes.c_void_p()
        _check(lib().pf_build_index(pp, n, d, int(budget), ctypes.byref(opts), mem, st, ctypes.byref(h)))
        self._h = h
        self.n, self.d = n, d
        info = self.info()
        self.L, self.K, self.M, self.P, self.pool = info.L, info.K, info.M, info.P, info.pool
        self.family = info.family
        self.pos_bytes = info.pos_bytes
        dp = 1
        while dp < d:
            dp <<= 1
        self.cp_ell = dp.bit_length()  # log2(2 d')

    def close(self):
        if getattr(self, "_h", None):
            lib().pf_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> pf_info:
        i = pf_info()
        _check(lib().pf_index_info(self._h, ctypes.byref(i)))
        return i

    def last_timing(self) -> pf_timing:
        t = pf_timing()
        _check(lib().pf_last_timing(self._h, ctypes.byref(t)))
        return t

    def search(self, queries, k: int, recall: float, eps: float = 0.0, B: int = 12,
               rule: int = PF_RULE_FILTER, filter: bool = True, timing: bool = False,
               want_ips: bool = True, want_stats: bool = True, prefilter: bool = True,
               tile: int = None, groups: int = 0, test_entries: int = 0) -> SearchResult:
        """tile: kernel tile shape index (None: the default shape); groups: stopping tests per
        level (0: the library's default); test_entries: entries read between two of a level's
        tests (0: the library's default, negative: a test after every group)."""
        q = _f32(queries)
        m = q.shape[0]
        ids = _empty_like_input(q, (m, k), np.int32, _torch_dtype("int32"))
        ips = _empty_like_input(q, (m, k), np.float32, _torch_dtype("float32")) if want_ips else None
        st = _empty_like_input(q, (m, 7), np.int64, _torch_dtype("int64")) if want_stats else None
        opts = pf_search_opts(eps, B, rule, 0 if filter else 1, 1 if timing else 0, 0 if prefilter else 1,
                              0 if tile is None else tile + 1, int(groups), int(test_entries))
        pq, mem, stream = _buf(q)
        _check(lib().pf_search_ex(self._h, pq, m, k, recall, ctypes.byref(opts), _buf(ids)[0],
                                  _buf(ips)[0], _buf(st)[0], mem, stream))
        return SearchResult(ids, ips, _stats_view(st) if st is not None else None,
                            _wave_us(st) if st is not None else None)

    def search_noalloc(self, queries, k: int, recall: float, out_ids, out_ips=None, stats=None) -> None:
        """pf_search_noalloc: device tensors only; the caller provides the outputs (ids m x k
        int32, ips m x k float32, stats m x 7 int64, the last two optional)."""
        assert _is_torch(queries) and queries.is_cuda and queries.dtype == _torch_dtype("float32")
        pq, _, stream = _buf(queries)
        _check(lib().pf_search_noalloc(self._h, pq, queries.shape[0], int(k), float(recall), _buf(out_ids)[0],
                                       _buf(out_ips)[0], _buf(stats)[0], stream))

    def search_batch(self, queries, ks, recalls, kmax: int, order=None, learned: bool = False,
                     autotune: bool = False, eps: float = 0.0, B: int = 12, rule: int = PF_RULE_FILTER,
                     filter: bool = True, timing: bool = False, prefilter: bool = True,
                     tile: int = None, groups: int = 0, test_entries: int = 0) -> SearchResult:
        """One persistent launch over all queries with per-query k and recall (work queue);
        tile: kernel tile shape index (None: the autotuned or cached shape); groups and
        test_entries as for search."""
        q = _f32(queries)
        m = q.shape[0]
        torch_in = _is_torch(q)

        def arr(a, np_dt, t_dt):
            if a is None:
                return None
            if torch_in:
                import torch

                return torch.as_tensor(a, dtype=getattr(torch, t_dt), device=q.device).contiguous()
            return np.ascontiguousarray(a, dtype=np_dt)

        ks_a = arr(ks, np.int32, "int32")
        rec_a = arr(recalls, np.float64, "float64")
        ord_a = arr(order, np.int32, "int32")
        ids = _empty_like_input(q, (m, kmax), np.int32, _torch_dtype("int32"))
        ips = _empty_like_input(q, (m, kmax), np.float32, _torch_dtype("float32"))
        st = _empty_like_input(q, (m, 7), np.int64, _torch_dtype("int64"))
        opts = pf_search_opts(eps, B, rule, 0 if filter else 1, 1 if timing else 0, 0 if prefilter else 1,
                              0 if tile is None else tile + 1, int(groups), int(test_entries))
        flags = (PF_BATCH_LEARNED if learned else 0) | (PF_BATCH_AUTOTUNE if autotune else 0)
        pq, mem, stream = _buf(q)
        _check(lib().pf_search_batch(self._h, pq, m, _buf(ks_a)[0], _buf(rec_a)[0], kmax, ctypes.byref(opts),
                                     _buf(ord_a)[0], _buf(ids)[0], _buf(ips)[0], _buf(st)[0], flags, mem,
                                     stream))
        return SearchResult(ids, ips, _stats_view(st), _wave_us(st))

    def hash(self, x):
        x = _f32(x)
        m = x.shape[0]
        codes = _empty_like_input(x, (self.L, m), np.uint32, _torch_dtype("int32"))
        sk = _empty_like_input(x, (self.M, m), np.uint64, _torch_dtype("int64"))
        px, mem, st = _buf(x)
        _check(lib().pf_hash(self._h, px, m, _buf(codes)[0], _buf(sk)[0], mem, st))
        return codes, sk

    def features(self, x, ks=None, recalls=None, k: int = 10, recall: float = 0.9):
        """Scheduler features (m x 98 FP32) of the rows x under this index, for per-query
        k / recall arrays (same memory as x) or the constants k / recall."""
        x = _f32(x)
        m = x.shape[0]
        torch_in = _is_torch(x)

        def arr(a, np_dt, t_dt):
            if a is None:
                return None
            if torch_in:
                import torch

                return torch.as_tensor(a, dtype=getattr(torch, t_dt), device=x.device).contiguous()
            return np.ascontiguousarray(a, dtype=np_dt)

        ks_a, rec_a = arr(ks, np.int32, "int32"), arr(recalls, np.float64, "float64")
        f = _empty_like_input(x, (m, PF_SCHED_IN), np.float32, _torch_dtype("float32"))
        px, mem, st = _buf(x)
        _check(lib().pf_features(self._h, px, m, _buf(ks_a)[0], _buf(rec_a)[0], int(k), float(recall),
                                 _buf(f)[0], mem, st))
        return f

    def set_scheduler(self, sched):
        _check(lib().pf_index_set_scheduler(self._h, sched._h if sched is not None else None))
        self._sched = sched

    _EXPORT = {
        PF_EXPORT_POINTS: (np.float32, lambda s: (s.n, s.d)),
        PF_EXPORT_HYPERPLANES: (np.float32, lambda s: ((0 if s.family == PF_FAMILY_FHTCP else (s.pool or s.L * s.K))
                                                        + 64 * s.M, s.d)),
        PF_EXPORT_CODES: (np.uint32, lambda s: (s.L, s.n)),
        PF_EXPORT_IDX: (np.uint32, lambda s: (s.L, s.n)),
        PF_EXPORT_SKETCHES: (np.uint64, lambda s: (s.L, s.n)),
        PF_EXPORT_OFFSETS: (np.uint32, lambda s: (s.L, (1 << s.P) + 1)),
        PF_EXPORT_POOL_SEL: (np.int32, lambda s: (s.L, s.K)),
        PF_EXPORT_CP_TABLE: (np.float64, lambda s: (41, s.cp_ell + 1)),
        PF_EXPORT_ROWS8: (np.uint8, lambda s: (s.n, 8 + 4 * ((s.d + 3) // 4))),
    }

    def export(self, what: int, device: bool = False):
        """A copy of an index structure: numpy on the host, or a torch tensor on the current
        device when device=True (written on torch's current stream)."""
        dt, shp = self._EXPORT[what]
        if device:
            import torch

            out = torch.empty(shp(self), dtype=getattr(torch, np.dtype(dt).name), device="cuda")
            pq, _, stream = _buf(out)
            _check(lib().pf_export(self._h, what, pq, out.numel() * out.element_size(), PF_DEVICE, stream))
            return out
        out = np.empty(shp(self), dtype=dt)
        _check(lib().pf_export(self._h, what, _buf(out)[0], out.nbytes, PF_HOST, None))
        return out


def _torch_dtype(name: str):
    try:
        import torch

        return getattr(torch, name)
    except Exception:  # numpy-only callers never use it
        return None


class Scheduler:
    """The learned query-cost model (98 -> 128 -> 128 -> 2 MLP) trained by the library."""

    def __init__(self, seed: int = 1):
        h = ctypes.c_void_p()
        _check(lib().pf_sched_create(seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pf_sched_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        p = np.empty(PF_SCHED_PARAMS, dtype=np.float32)
        _check(lib().pf_sched_params(self._h, _buf(p)[0], 1))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == PF_SCHED_PARAMS
        _check(lib().pf_sched_params(self._h, _buf(p)[0], 0))

    def predict(self, feat):
        f = _f32(feat)
        out = _empty_like_input(f, (f.shape[0], PF_SCHED_OUT), np.float32, _torch_dtype("float32"))
        pf_, mem, st = _buf(f)
        _check(lib().pf_sched_predict(self._h, pf_, f.shape[0], _buf(out)[0], mem, st))
        return out

    def grad(self, feat, target):
        f, t = _f32(feat), _f32(target)
        g = np.empty(PF_SCHED_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        if _is_torch(f):
            import torch

            gd = torch.empty(PF_SCHED_PARAMS, dtype=torch.float32, device=f.device)
            _check(lib().pf_sched_grad(self._h, _buf(f)[0], _buf(t)[0], f.shape[0], _buf(gd)[0],
                                       ctypes.byref(loss), PF_DEVICE, _buf(f)[2]))
            return gd, loss.value
        _check(lib().pf_sched_grad(self._h, _buf(f)[0], _buf(t)[0], f.shape[0], _buf(g)[0], ctypes.byref(loss),
                                   PF_HOST, None))
        return g, loss.value

    def train(self, feat, target, epochs: int = 10, batch: int = 1024, lr: float = 1e-3, seed: int = 7):
        f, t = _f32(feat), _f32(target)
        losses = np.empty(epochs, dtype=np.float32)
        pf_, mem, st = _buf(f)
        _check(lib().pf_sched_train(self._h, pf_, _buf(t)[0], f.shape[0], epochs, batch, lr, seed,
                                    _buf(losses)[0], mem, st))
        return losses

    def save(self, path: str):
        _check(lib().pf_sched_save(self._h, path.encode()))

    def load(self, path: str):
        _check(lib().pf_sched_load(self._h, path.encode()))
