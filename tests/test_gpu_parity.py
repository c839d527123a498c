"""Parity of the gfx950 library with the CPU oracle (needs an MI355X).

Bar: bit-exact for normalised vectors, hash bits, sorted tables, prefix tables,
table-local sketches, returned ids, FP32 inner products (one fixed summation order on
both sides) and the per-query counters; queries whose FP64 filter threshold or stopping
test came within 1e-9 of flipping are reported by the oracle and excluded (the two
sides use different libm implementations there).
"""
import numpy as np
import pytest

import oracle
import paper_1906_12211_amd as pf
import workloads
from prefix_tables import check_offsets

pytestmark = pytest.mark.gpu


def _build_both(X, budget=0, L=None, seed=42, K=24, M=32, hash_mode=pf.PF_HASH_BF16X3, pos_bytes=0,
                prefix_bits=0):
    print(f"[build] n={len(X)} d={X.shape[1]} L={L} budget={budget} K={K} M={M} mode={hash_mode} "
          f"pos_bytes={pos_bytes} prefix_bits={prefix_bits}", flush=True)
    g = pf.Index(X, budget, seed=seed, K=K, M=M, hash_mode=hash_mode, L=L, pos_bytes=pos_bytes,
                 prefix_bits=prefix_bits)
    o = oracle.OracleIndex(X, budget, seed=seed, K=K, M=M, L=g.L)
    return g, o


def _assert_index_equal(g, o):
    assert (g.L, g.K, g.M) == (o.L, o.K, o.M)
    assert np.array_equal(g.export(pf.PF_EXPORT_POINTS), o.points), "normalised points"
    assert np.array_equal(g.export(pf.PF_EXPORT_HYPERPLANES), o.hp), "hyperplanes"
    gc, gi = g.export(pf.PF_EXPORT_CODES), g.export(pf.PF_EXPORT_IDX)
    bad = np.argwhere(gc != o.tcode)
    assert bad.size == 0, f"{len(bad)} code mismatches, first {bad[:5]}"
    assert np.array_equal(gi, o.tidx), "table order"
    assert check_offsets(g.export(pf.PF_EXPORT_OFFSETS), o, g.P) == 0, "prefix tables"
    assert np.array_equal(g.export(pf.PF_EXPORT_SKETCHES), o.tsk), "table-local sketches"


def _assert_search_equal(gr, orr, label=""):
    ok = orr.boundary == 0
    print(f"[search {label}] boundary cases: {int((~ok).sum())} of {len(ok)}", flush=True)
    st = gr.stats
    for name, gv, ov in [("stop_level", st[:, 0], orr.stop_level), ("c_scan", st[:, 1], orr.c_scan),
                         ("c_pass", st[:, 2], orr.c_pass), ("c_rerank", st[:, 3], orr.c_rerank)]:
        bad = np.nonzero((gv != ov) & ok)[0]
        assert bad.size == 0, f"{label} {name}: {bad.size} mismatches, q={bad[:5]} gpu={gv[bad[:5]]} oracle={ov[bad[:5]]}"
    bad = np.nonzero(np.any(gr.ids != orr.ids, axis=1) & ok)[0]
    assert bad.size == 0, f"{label} ids differ for {bad.size} queries, first {bad[:5]}"
    # bounds only rule candidates out: c_exact <= c_upper <= c_rerank, c_q8 <= c_rerank
    assert np.all((st[:, 4] >= 0) & (st[:, 4] <= st[:, 5]) & (st[:, 5] <= st[:, 3])), f"{label} c_exact/c_upper"
    assert np.all((st[:, 6] >= 0) & (st[:, 6] <= st[:, 3])), f"{label} c_q8"
    assert np.array_equal(gr.ips[ok].view(np.uint32), orr.ips[ok].view(np.uint32)), f"{label} ips"
    assert ok.mean() > 0.99


def test_normalize_bit_exact():
    for (n, d) in [(1, 1), (7, 3), (513, 17), (1000, 64), (257, 100), (64, 256), (5, 1000)]:
        X = workloads.gaussian_unit(n, d, 100 + d) * np.float32(1.7)
        X[0] *= np.float32(1e-3)
        print(f"[normalize] n={n} d={d}", flush=True)
        assert np.array_equal(pf.pf_normalize(X), oracle.normalize(X))


def test_normalize_rejects_bad_rows():
    X = workloads.gaussian_unit(10, 8, 1)
    X[4] = 0
    with pytest.raises(pf.PfError) as e:
        pf.pf_normalize(X)
    assert e.value.code == pf.PF_EINVAL


@pytest.mark.parametrize("mode", [pf.PF_HASH_BF16X3, pf.PF_HASH_FP64])
def test_build_small_bit_exact(mode):
    X = workloads.gaussian_unit(3000, 64, 7)
    g, o = _build_both(X, L=20, seed=7, hash_mode=mode)
    _assert_index_equal(g, o)


@pytest.mark.parametrize("n,d,K,M,L", [(4097, 17, 24, 3, 9), (50, 3, 8, 1, 5), (1200, 100, 13, 2, 7),
                                       (900, 33, 32, 1, 3), (4096, 130, 24, 2, 4), (700, 300, 20, 1, 3),
                                       (1000, 128, 24, 2, 5), (333, 129, 24, 1, 3), (515, 256, 24, 2, 3),
                                       (300, 257, 24, 1, 2)])
def test_build_shapes_bit_exact(n, d, K, M, L):
    """ragged tiles, d not a multiple of 4 / 16, K below and at the 13-bit prefix,
    K = 32 (no padding bits), d above 256 (32-row GEMM tiles), and d = 128 / 129 / 256 / 257
    at the bounds of the GEMM kernel that keeps the rows in registers (8 or 16 k steps)"""
    X = workloads.gaussian_unit(n, d, n + d)
    g, o = _build_both(X, L=L, seed=n, K=K, M=M)
    _assert_index_equal(g, o)


def test_hash_queries_bit_exact():
    X = workloads.gaussian_unit(2000, 100, 3)
    Q = workloads.gaussian_unit(777, 100, 4)
    g, o = _build_both(X, L=15, seed=11, M=4)
    gc, gs = g.hash(Q)
    oc, os_ = oracle.hash_codes(oracle.normalize(Q), o.hp, o.L, o.K, o.M)
    assert np.array_equal(gc, oc)
    assert np.array_equal(gs, os_)


@pytest.mark.parametrize("pos_bytes,want_L", [(0, 331), (3, 350)])
def test_config1_parity(pos_bytes, want_L):
    """gauss-10k-d64, 64 MiB budget -> L = 331 (every resident byte charged; 350 with 3-byte
    table positions), 1000 queries, k = 10, recall .9; the index's device bytes are the
    planned ones and fit the budget"""
    c = workloads.config(1)
    g, o = _build_both(c["points"], budget=c["budget"], pos_bytes=pos_bytes)
    assert (g.L, g.pos_bytes, g.P) == (want_L, pos_bytes or 4, 13)
    info = g.info()
    assert info.bytes_device == info.bytes_budget_rule == pf.pf_plan_index(10_000, 64, c["budget"],
                                                                            pos_bytes=pos_bytes)[1]
    assert info.bytes_device <= c["budget"]
    _assert_index_equal(g, o)
    gr = g.search(c["queries"], 10, 0.9)
    orr = o.search(c["queries"], 10, 0.9)
    _assert_search_equal(gr, orr, "config1")


@pytest.mark.parametrize("n,L", [(997, 1), (998, 3), (999, 5), (1000, 7), (4093, 9)])
def test_table_positions_any_count(n, L):
    """3-byte table positions for every remainder of L n modulo 4 (the last packed group
    partly filled), against 4-byte positions of the same index and the oracle's tables;
    the searches agree too."""
    X = workloads.gaussian_unit(n, 40, 31)
    Q = workloads.gaussian_unit(64, 40, 32)
    g3, o = _build_both(X, L=L, seed=n, pos_bytes=3)
    g4 = pf.Index(X, 0, seed=n, L=L, pos_bytes=4)
    assert (g3.pos_bytes, g4.pos_bytes) == (3, 4)
    _assert_index_equal(g3, o)
    assert np.array_equal(g4.export(pf.PF_EXPORT_IDX), o.tidx)
    for g in (g3, g4):  # widened on the device into device memory, too
        assert np.array_equal(g.export(pf.PF_EXPORT_IDX, device=True).cpu().numpy(), o.tidx)
    assert g4.info().bytes_device - g3.info().bytes_device == L * n
    r3, r4 = g3.search(Q, 10, 0.9), g4.search(Q, 10, 0.9)
    assert np.array_equal(r3.ids, r4.ids) and np.array_equal(r3.stats[:, :4], r4.stats[:, :4])
    _assert_search_equal(r3, o.search(Q, 10, 0.9), f"positions n={n} L={L}")


@pytest.mark.parametrize("K,P,suffix", [(24, 13, 2), (24, 14, 2), (24, 16, 1), (24, 17, 1), (24, 24, 0),
                                         (20, 13, 1), (21, 13, 1), (22, 13, 2), (32, 16, 2), (32, 15, 4),
                                         (32, 24, 1), (14, 14, 0)])
def test_prefix_widths(K, P, suffix):
    """Every prefix width the index may take, on a small ragged index: the exported prefix
    table against its definition over the oracle's codes, the codes rebuilt from prefix
    and low bits (8-, 16- or 32-bit, or none), and the search (levels at and above P read
    the prefix table, deeper ones the range kernels over the low bits)."""
    X = workloads.gaussian_unit(3001, 24, 41)
    Q = workloads.gaussian_unit(50, 24, 42)
    g, o = _build_both(X, L=7, seed=K * 100 + P, K=K, prefix_bits=P)
    assert g.P == P
    per = pf.pf_plan_index(3001, 24, 0, K=K, L=2, prefix_bits=P)[1] - pf.pf_plan_index(3001, 24, 0, K=K, L=1,
                                                                                        prefix_bits=P)[1]
    assert per == (8 + 4 + suffix) * 3001 + 4 * ((1 << P) + 1) + 4 * K * 24 + 32 * (4 * 32 + 8)
    _assert_index_equal(g, o)
    for k, rec in [(1, 0.9), (10, 0.9), (10, 0.99)]:
        _assert_search_equal(g.search(Q, k, rec), o.search(Q, k, rec), f"P={P} K={K} k={k}")


@pytest.mark.parametrize("k,recall,kw", [
    (1, 0.9, {}), (10, 0.5, {}), (10, 0.99, {}), (37, 0.9, {}), (10, 0.9, {"B": 1}), (10, 0.9, {"B": 512}),
    (10, 0.9, {"filter": False}), (10, 0.9, {"rule": pf.PF_RULE_ALG1}), (10, 0.9, {"eps": 0.1}),
    (10, 0.9, {"rule": pf.PF_RULE_EXACT}), (10, 0.8, {"rule": pf.PF_RULE_EXACT, "eps": 0.3}),
    (5, 1.0, {}), (128, 0.7, {}), (10, 0.9, {"prefilter": False}), (10, 1.0, {"prefilter": False}),
    (10, 0.9, {"groups": 1}), (10, 0.9, {"groups": 4}), (10, 0.9, {"groups": 40}), (1, 0.99, {"groups": 3, "B": 1}),
    (10, 0.9, {"groups": 7, "rule": pf.PF_RULE_EXACT}), (5, 0.99, {"groups": 13, "rule": pf.PF_RULE_ALG1}),
    (37, 0.8, {"groups": 40, "rule": pf.PF_RULE_EXACT, "eps": 0.2}),
    (10, 0.9, {"test_entries": -1}), (10, 0.9, {"test_entries": 1}), (10, 0.9, {"test_entries": 300}),
    (1, 0.99, {"test_entries": 5000}), (10, 0.9, {"test_entries": 700, "groups": 7}),
    (37, 0.8, {"test_entries": 2000, "rule": pf.PF_RULE_EXACT, "groups": 40}),
    (5, 0.9, {"test_entries": 10 ** 7, "B": 1}),
])
def test_search_variants(k, recall, kw):
    X = workloads.gaussian_unit(5000, 48, 21)
    Q = workloads.gaussian_unit(300, 48, 22)
    g, o = _build_both(X, L=40, seed=5)
    okw = dict(kw)
    if "filter" in okw:
        okw["filter_on"] = okw.pop("filter")
    okw.pop("prefilter", None)
    if okw.get("test_entries", 0) < 0:
        okw["test_entries"] = 0  # the library's negative value: a test after every group
    gr = g.search(Q, k, recall, **kw)
    orr = o.search(Q, k, recall, **okw)
    _assert_search_equal(gr, orr, f"k={k} r={recall} {kw}")
    if kw.get("prefilter", True) is False:
        assert np.array_equal(gr.stats[:, 4], gr.stats[:, 3]) and np.array_equal(gr.stats[:, 5], gr.stats[:, 3])
        assert np.all(gr.stats[:, 6] == 0)


@pytest.mark.parametrize("d", [48, 100, 128, 200, 300])
def test_prefilter_exact_and_effective(d):
    """The upper-plane bound only decides which inner products are computed: ids, inner
    products and counters equal the oracle's with it on and off, for every row-length
    specialisation, and it rules most candidates out."""
    X = workloads.gaussian_unit(6000, d, 300 + d)
    Q = workloads.gaussian_unit(200, d, 400 + d)
    g, o = _build_both(X, L=30, seed=d)
    orr = o.search(Q, 10, 0.9)
    on = g.search(Q, 10, 0.9)
    off = g.search(Q, 10, 0.9, prefilter=False)
    _assert_search_equal(on, orr, f"prefilter on d={d}")
    _assert_search_equal(off, orr, f"prefilter off d={d}")
    assert np.array_equal(off.stats[:, 4], off.stats[:, 3])
    frac = on.stats[:, 4].sum() / on.stats[:, 3].sum()
    up = on.stats[:, 5].sum() / on.stats[:, 3].sum()
    q8 = on.stats[:, 6].sum() / on.stats[:, 3].sum()
    print(f"[prefilter d={d}] of re-ranked: 8-bit bounds {q8:.4f}, upper planes read {up:.4f}, "
          f"exact inner products {frac:.4f}", flush=True)
    assert frac < 0.5 and up < 0.5 and q8 > 0.5


def test_rows8_summaries_and_bound():
    """The 8-bit row summaries follow their definition (FP32 scale max|x_i| / 127 of the row,
    or of all rows where the header cannot share the codes' line (d = 124, 128, 256 here),
    int8 codes rint(x_i / s), sum of |codes|; IEEE FP32 division), and the bound the re-rank
    takes from them, s t (C + h (A + B) + dpad h^2) with the query coded the same way and,
    in the shared-scale layout, A the largest sum of any row, dominates the FP64 inner
    product on every pair tried, with a slack of a few 1e-2."""
    for d in (5, 100, 124, 128, 256, 300):
        X = workloads.gaussian_unit(3000, d, 700 + d)
        X[:50, : d // 2] = 0.0
        g = pf.Index(X, 0, seed=7, L=4)
        rows = g.export(pf.PF_EXPORT_ROWS8)
        dpad = 4 * ((d + 3) // 4)
        assert rows.shape == (3000, 8 + dpad)
        Xn = g.export(pf.PF_EXPORT_POINTS)
        inline = 8 + dpad <= (dpad + 127) // 128 * 128
        if inline:
            s = np.abs(Xn).max(1).astype(np.float32) / np.float32(127)
        else:
            s = np.full(len(Xn), np.float32(np.abs(Xn).max()) / np.float32(127), dtype=np.float32)
        c = np.clip(np.rint(Xn / s[:, None]), -127, 127).astype(np.int64)
        assert np.array_equal(rows[:, :4].copy().view(np.float32)[:, 0], s), f"d={d} scale"
        assert np.array_equal(rows[:, 4:8].copy().view(np.int32)[:, 0], np.abs(c).sum(1)), f"d={d} sum"
        assert np.array_equal(rows[:, 8:8 + d].view(np.int8).astype(np.int64), c), f"d={d} codes"
        assert not rows[:, 8 + d:].any(), f"d={d} padding"
        Q = oracle.normalize(workloads.gaussian_unit(200, d, 800 + d))
        t = np.abs(Q).max(1).astype(np.float32) / np.float32(127)
        b = np.clip(np.rint(Q / t[:, None]), -127, 127).astype(np.int64)
        h = 0.5 + 2.0 ** -16
        C = b @ c.T
        A = np.abs(c).sum(1) if inline else np.full(len(c), np.abs(c).sum(1).max())
        ub = (s[None, :].astype(np.float64) * t[:, None]) * (C + h * (A[None, :] + np.abs(b).sum(1)[:, None])
                                                          + dpad * h * h)
        ip = Q.astype(np.float64) @ Xn.astype(np.float64).T
        slack = ub - ip
        print(f"[rows8 d={d} inline={inline}] bound slack min {slack.min():.2e} mean {slack.mean():.3e} max {slack.max():.3e}",
              flush=True)
        assert slack.min() >= 0.0 and slack.mean() < 0.1


def test_prefilter_spiky_rows():
    """Rows dominated by one coordinate (the 8-bit codes of the others round to zero) and
    queries along the same axes: candidates' inner products differ by less than the 8-bit
    bound's slack, so every bound stage is exercised on near-ties."""
    rng = np.random.default_rng(901)
    n, d = 8000, 100
    X = (np.float32(1e-3) * rng.standard_normal((n, d))).astype(np.float32)
    axes = rng.integers(0, 8, size=n)
    X[np.arange(n), axes] += np.float32(1.0)
    X[: n // 4] += np.float32(0.02) * workloads.gaussian_unit(n // 4, d, 902)
    Q = (np.float32(1e-3) * rng.standard_normal((120, d))).astype(np.float32)
    Q[np.arange(120), rng.integers(0, 8, size=120)] += np.float32(1.0)
    g, o = _build_both(X, L=20, seed=903)
    for k, rec in [(1, 0.9), (10, 0.9), (40, 0.99)]:
        _assert_search_equal(g.search(Q, k, rec), o.search(Q, k, rec), f"spiky k={k}")


def test_prefilter_low_bits_and_subnormals():
    """Points that differ only in the lower 16 bits of their coordinates (identical upper
    planes, so the bound cannot separate them), exact zeros and subnormal coordinates."""
    rng = np.random.default_rng(501)
    d = 64
    base = workloads.gaussian_unit(40, d, 502)
    X = [workloads.gaussian_unit(3000, d, 503)]
    for b in base:
        cp = np.repeat(b[None, :], 25, 0).view(np.uint32).copy()
        cp ^= rng.integers(0, 1 << 12, size=cp.shape, dtype=np.uint32)  # low bits only
        X.append(cp.view(np.float32))
    X = np.concatenate(X)
    X[:200, :8] = 0.0
    X[200:400, 8:16] = np.float32(3e-39)  # subnormal before and after normalisation
    Q = (base + np.float32(0.05) * workloads.gaussian_unit(40, d, 504)).astype(np.float32)
    g, o = _build_both(X, L=24, seed=505)
    for k, rec in [(1, 0.9), (10, 0.9), (30, 0.99)]:
        _assert_search_equal(g.search(Q, k, rec), o.search(Q, k, rec), f"low bits k={k}")


def test_large_prefix_buckets():
    """Clusters of near-identical points fill single 13-bit prefix buckets with about
    4,000 (both sides of the 4,080-entry limit of the 16-lane range count) up to 12,000
    entries (binary-searched ranges), around a Gaussian background."""
    d = 32
    rng = np.random.default_rng(601)
    centers = workloads.gaussian_unit(4, d, 602)
    parts = [workloads.gaussian_unit(4000, d, 603)]
    for c, size in zip(centers, [3900, 4200, 6000, 12000]):
        parts.append((c[None, :] + np.float32(2e-3) * rng.standard_normal((size, d))).astype(np.float32))
    X = np.concatenate(parts)
    Q = np.concatenate([(centers + np.float32(1e-2) * rng.standard_normal((4, d))).astype(np.float32)
                        for _ in range(8)] + [workloads.gaussian_unit(32, d, 604)])
    g, o = _build_both(X, L=16, seed=606)
    off = g.export(pf.PF_EXPORT_OFFSETS)[:, ::1 << (g.P - 13)]
    sizes = np.diff(off.astype(np.int64), axis=1)
    print(f"[buckets] largest 13-bit buckets {np.sort(sizes.ravel())[-6:]}", flush=True)
    assert sizes.max() > 4080 and ((sizes > 3000) & (sizes <= 4080)).any()
    for k, rec in [(1, 0.9), (10, 0.9), (50, 0.99)]:
        _assert_search_equal(g.search(Q, k, rec), o.search(Q, k, rec), f"large buckets k={k}")
        ks = np.full(len(Q), k, np.int32)
        recs = np.full(len(Q), rec)
        oids, oips, ost, obd = _oracle_per_query(o, Q, ks, recs, k)
        _assert_batch_equal(g.search_batch(Q, ks, recs, k), oids, oips, ost, obd, f"large buckets batch k={k}")


@pytest.mark.parametrize("P", [13, 16])
def test_range_group_widths(P):
    """2.2 M points: with 13-bit prefix tables a bucket averages 268 entries and the range
    counts run on 16-lane groups, with 16-bit tables (33 entries) on 8-lane groups; the walk
    (ranges through c_scan, ids, inner products) equals the oracle's either way."""
    X = workloads.gaussian_unit(2_200_000, 16, 961)
    Q = workloads.gaussian_unit(64, 16, 962)
    g, o = _build_both(X, L=4, seed=963, M=1, prefix_bits=P)
    assert g.P == P
    for k, rec in [(1, 0.9), (10, 0.9)]:
        _assert_search_equal(g.search(Q, k, rec), o.search(Q, k, rec), f"P={P} k={k}")


def test_linear_scan_equals_bruteforce():
    """recall 1: every query walks to level 0 and returns the exact k-NN (Lemma 1)."""
    X = workloads.gaussian_unit(3000, 32, 31)
    Q = workloads.gaussian_unit(100, 32, 32)
    g = pf.Index(X, 0, seed=3, L=8)
    r = g.search(Q, 10, 1.0)
    assert np.all(r.stats[:, 0] == 0)
    assert np.all(r.stats[:, 3] == r.stats[:, 2] + len(X))
    ids, _ = oracle.bruteforce(oracle.normalize(X), oracle.normalize(Q), 10)
    assert np.mean(np.all(r.ids == ids, axis=1)) > 0.95


def test_small_n_and_k_equals_n():
    X = workloads.gaussian_unit(40, 6, 41)
    Q = workloads.gaussian_unit(20, 6, 42)
    g, o = _build_both(X, L=6, seed=9)
    _assert_search_equal(g.search(Q, 40, 0.9), o.search(Q, 40, 0.9), "k=n")
    _assert_search_equal(g.search(Q, 1, 0.6), o.search(Q, 1, 0.6), "n=40 k=1")


def test_device_tensors_path():
    torch = pytest.importorskip("torch")
    X = workloads.gaussian_unit(4000, 64, 51)
    Q = workloads.gaussian_unit(200, 64, 52)
    g = pf.Index(torch.from_numpy(X).cuda(), 0, seed=13, L=30)
    o = oracle.OracleIndex(X, 0, seed=13, L=30)
    _assert_index_equal(g, o)
    r = g.search(torch.from_numpy(Q).cuda(), 10, 0.9)
    torch.cuda.synchronize()
    gr = pf.SearchResult(r.ids.cpu().numpy(), r.ips.cpu().numpy(), r.stats.cpu().numpy())
    _assert_search_equal(gr, o.search(Q, 10, 0.9), "device tensors")


def test_errors():
    X = workloads.gaussian_unit(100, 8, 61)
    with pytest.raises(pf.PfError) as e:
        pf.Index(X, 1000)
    assert e.value.code == pf.PF_EBUDGET
    bad = X.copy()
    bad[7] = np.nan
    with pytest.raises(pf.PfError) as e:
        pf.Index(bad, 0, L=4)
    assert e.value.code == pf.PF_EINVAL
    g = pf.Index(X, 0, L=4)
    for k, rec in [(0, 0.9), (101, 0.9), (10, 0.0), (10, 1.5)]:
        with pytest.raises(pf.PfError) as e:
            g.search(X[:3], k, rec)
        assert e.value.code == pf.PF_EINVAL
    q = X[:3].copy()
    q[1] = 0
    with pytest.raises(pf.PfError) as e:
        g.search(q, 5, 0.9)
    assert e.value.code == pf.PF_EINVAL
    # the index still answers after the errors
    r = g.search(X[:3], 5, 0.9)
    assert np.all(r.ids[:, 0] == np.arange(3))


def _oracle_per_query(o, Q, ks, recalls, kmax, groups=None):
    """Oracle answers for per-query (k, recall): one oracle call per distinct pair."""
    m = len(Q)
    ids = np.full((m, kmax), -1, dtype=np.int32)
    ips = np.full((m, kmax), -np.inf, dtype=np.float32)
    st = np.zeros((m, 4), dtype=np.int64)
    bd = np.zeros(m, dtype=np.int32)
    for k in np.unique(ks):
        for rec in np.unique(recalls):
            sel = np.nonzero((ks == k) & (recalls == rec))[0]
            if len(sel) == 0:
                continue
            r = o.search(Q[sel], int(k), float(rec), groups=groups)
            ids[sel, :k] = r.ids
            ips[sel, :k] = r.ips
            st[sel] = np.stack([r.stop_level, r.c_scan, r.c_pass, r.c_rerank], 1)
            bd[sel] = r.boundary
    return ids, ips, st, bd


def _assert_batch_equal(gr, oids, oips, ost, obd, label):
    ok = obd == 0
    print(f"[batch {label}] boundary cases: {int((~ok).sum())} of {len(ok)}", flush=True)
    assert np.array_equal(gr.stats[ok][:, :4], ost[ok]), label + " stats"
    assert np.array_equal(gr.ids[ok], oids[ok]), label + " ids"
    assert np.array_equal(gr.ips[ok].view(np.uint32), oips[ok].view(np.uint32)), label + " ips"
    assert ok.mean() > 0.99


def test_batch_per_query_params_and_order():
    """Persistent batched search: per-query k and recall, work queue in any order gives the
    oracle's answers (the order only changes which wave answers which query)."""
    X = workloads.gaussian_unit(6000, 40, 81)
    Q = workloads.gaussian_unit(700, 40, 82)
    rng = np.random.default_rng(83)
    ks = rng.choice(np.array([1, 10, 100], dtype=np.int32), size=len(Q))
    recalls = rng.choice(np.array([0.5, 0.9, 0.99]), size=len(Q))
    g, o = _build_both(X, L=50, seed=17)
    oids, oips, ost, obd = _oracle_per_query(o, Q, ks, recalls, 100)
    _assert_batch_equal(g.search_batch(Q, ks, recalls, 100), oids, oips, ost, obd, "fifo")
    order = rng.permutation(len(Q)).astype(np.int32)
    _assert_batch_equal(g.search_batch(Q, ks, recalls, 100, order=order), oids, oips, ost, obd, "shuffled")
    _assert_batch_equal(g.search_batch(Q, ks, recalls, 100, autotune=True, timing=True), oids, oips, ost, obd,
                        "autotuned")
    t = g.last_timing()
    assert 0 <= t.tile < pf.pf_tile_count() and t.waves_per_cu >= 1
    # the stopping test after each of 6 groups of tables, every tile shape's kernel
    gids, gips, gst, gbd = _oracle_per_query(o, Q, ks, recalls, 100, groups=6)
    for tile in range(pf.pf_tile_count()):
        _assert_batch_equal(g.search_batch(Q, ks, recalls, 100, groups=6, tile=tile), gids, gips, gst, gbd,
                            f"groups 6 tile {pf.pf_tile_name(tile)}")
    with pytest.raises(pf.PfError):
        g.search_batch(Q, ks, recalls, 100, groups=51)
    with pytest.raises(pf.PfError):
        g.search_batch(Q, ks, recalls, 100, order=np.zeros(len(Q), dtype=np.int32))
    bad = ks.copy()
    bad[3] = 101
    with pytest.raises(pf.PfError):
        g.search_batch(Q, bad, recalls, 100)


def test_index_buffers_reused_across_call_sizes():
    """An index keeps its per-call device buffers (query rows, codes, decision tables, queue,
    outputs) and grows them on demand: calls that shrink and grow m, k and the number of
    distinct recalls, with hashing in between, each give the oracle's answers."""
    X = workloads.gaussian_unit(5000, 56, 91)
    Q = workloads.gaussian_unit(900, 56, 92)
    rng = np.random.default_rng(93)
    g, o = _build_both(X, L=36, seed=19)
    calls = [("batch", 600, 100, [0.5, 0.9, 0.99]), ("single", 40, 10, [0.9]), ("hash", 900, 0, []),
             ("batch", 150, 10, [0.8]), ("single", 900, 1, [0.7]), ("batch", 7, 37, [0.6, 0.95]),
             ("single", 300, 100, [0.99])]
    for kind, m, kmax, recs in calls:
        print(f"[call] {kind} m={m} kmax={kmax} recalls={recs}", flush=True)
        Qm = Q[:m]
        if kind == "hash":
            gc, gs = g.hash(Qm)
            oc, os_ = oracle.hash_codes(oracle.normalize(Qm), o.hp, o.L, o.K, o.M)
            assert np.array_equal(gc, oc) and np.array_equal(gs, os_)
        elif kind == "single":
            _assert_search_equal(g.search(Qm, kmax, recs[0]), o.search(Qm, kmax, recs[0]), f"m={m} k={kmax}")
        else:
            ks = rng.choice(np.unique(np.array([1, max(1, kmax // 3), kmax], dtype=np.int32)), size=m)
            recalls = rng.choice(np.array(recs), size=m)
            oids, oips, ost, obd = _oracle_per_query(o, Qm, ks, recalls, kmax)
            _assert_batch_equal(g.search_batch(Qm, ks, recalls, kmax), oids, oips, ost, obd, f"m={m} kmax={kmax}")


@pytest.mark.parametrize("d", [40, 100, 128, 200, 256, 300, 384])
def test_every_tile_shape(d):
    """Every built kernel tile shape (sketch loads per lane, rows in flight, register cap,
    point ids read with every sketch or only for passing entries) at every row-length
    specialisation (d = 40, 100, 200, 300: one, two, four and any number of 64-float
    chunks; d = 128, 256: the kernels for summary rows without header, one shared scale;
    d = 384: any length with the headers read from their own array) gives the oracle's
    answers, single and batched."""
    X = workloads.gaussian_unit(3000, d, 300 + d)
    Q = workloads.gaussian_unit(160, d, 400 + d)
    rng = np.random.default_rng(d)
    ks = rng.choice(np.array([1, 10, 40], dtype=np.int32), size=len(Q))
    recalls = rng.choice(np.array([0.7, 0.95]), size=len(Q))
    g, o = _build_both(X, L=40, seed=23)
    oids, oips, ost, obd = _oracle_per_query(o, Q, ks, recalls, 40)
    r10 = o.search(Q, 10, 0.9)
    ok10 = r10.boundary == 0
    names = [pf.pf_tile_name(t) for t in range(pf.pf_tile_count())]
    assert len(set(names)) == len(names) and pf.pf_tile_name(len(names)) == "?"
    for t, name in enumerate(names):
        print(f"[tile] d={d} shape {t} {name}", flush=True)
        _assert_batch_equal(g.search_batch(Q, ks, recalls, 40, tile=t, timing=True), oids, oips, ost, obd,
                            f"tile {name}")
        assert g.last_timing().tile == t
        r = g.search(Q, 10, 0.9, tile=t)
        assert np.array_equal(r.ids[ok10], r10.ids[ok10]), name
        assert np.array_equal(r.ips[ok10].view(np.uint32), r10.ips[ok10].view(np.uint32)), name
    with pytest.raises(pf.PfError):
        g.search(Q, 10, 0.9, tile=len(names))


def test_tune_cache_file(tmp_path, monkeypatch):
    """The autotuner's choice is written to the JSON-lines file named by PF_TUNE_CACHE and
    read back by a fresh index of the same shape; an entry whose shape name does not match
    this build's shape table is ignored (the default shape is used)."""
    import json

    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("PF_TUNE_CACHE", str(cache))
    X = workloads.gaussian_unit(4000, 32, 951)
    Q = workloads.gaussian_unit(300, 32, 952)
    ks = np.full(len(Q), 10, np.int32)
    rec = np.full(len(Q), 0.9)
    g = pf.Index(X, 0, seed=9, L=20)
    g.search_batch(Q, ks, rec, 10, autotune=True, timing=True)
    tuned = g.last_timing()
    entry = json.loads(cache.read_text().splitlines()[-1])
    assert entry["tile"] == tuned.tile and entry["waves"] == tuned.waves_per_cu
    assert entry["name"] == pf.pf_tile_name(tuned.tile)
    g2 = pf.Index(X, 0, seed=9, L=20)
    g2.search_batch(Q, ks, rec, 10, timing=True)
    assert (g2.last_timing().tile, g2.last_timing().waves_per_cu) == (tuned.tile, tuned.waves_per_cu)
    # a stale entry: the index now names another shape
    other = (tuned.tile + 1) % pf.pf_tile_count()
    entry.update(tile=other, waves=1)
    cache.write_text(json.dumps(entry) + "\n")
    g3 = pf.Index(X, 0, seed=9, L=20)
    r3 = g3.search_batch(Q, ks, rec, 10, timing=True)
    assert g3.last_timing().waves_per_cu != 1  # the stale entry was not used
    o = oracle.OracleIndex(X, 0, seed=9, L=20)
    oids, oips, ost, obd = _oracle_per_query(o, Q, ks, rec, 10)
    _assert_batch_equal(r3, oids, oips, ost, obd, "after a stale cache entry")
    # an index of the same shape with 3-byte positions runs other kernels: its own entry
    g4 = pf.Index(X, 0, seed=9, L=20, pos_bytes=3)
    g4.search_batch(Q, ks, rec, 10, autotune=True, timing=True)
    keys = [json.loads(line)["key"] for line in cache.read_text().splitlines()]
    assert len(set(keys)) == 2 and any(k.endswith("|p3") for k in keys), keys


def test_batch_device_tensors():
    torch = pytest.importorskip("torch")
    X = workloads.gaussian_unit(3000, 100, 91)
    Q = workloads.gaussian_unit(300, 100, 92)
    rng = np.random.default_rng(93)
    ks = rng.choice(np.array([1, 10, 20], dtype=np.int32), size=len(Q))
    recalls = rng.choice(np.array([0.6, 0.9]), size=len(Q))
    g, o = _build_both(X, L=30, seed=19)
    oids, oips, ost, obd = _oracle_per_query(o, Q, ks, recalls, 20)
    r = g.search_batch(torch.from_numpy(Q).cuda(), torch.from_numpy(ks).cuda(), torch.from_numpy(recalls).cuda(), 20)
    torch.cuda.synchronize()
    gr = pf.SearchResult(r.ids.cpu().numpy(), r.ips.cpu().numpy(), r.stats.cpu().numpy())
    _assert_batch_equal(gr, oids, oips, ost, obd, "device")


def _build_pool(X, L, pool, seed=42, K=24, M=32, hash_mode=pf.PF_HASH_BF16X3, budget=0):
    print(f"[build pool] n={len(X)} d={X.shape[1]} L={L} pool={pool} K={K} M={M} mode={hash_mode}", flush=True)
    g = pf.Index(X, budget, seed=seed, K=K, M=M, hash_mode=hash_mode, L=L, pool=pool)
    o = oracle.OracleIndex(X, budget, seed=seed, K=K, M=M, L=g.L, pool=pool)
    return g, o


@pytest.mark.parametrize("n,d,L,pool,K,M,mode", [(3000, 64, 20, 256, 24, 32, pf.PF_HASH_BF16X3),
                                                 (2500, 100, 40, 3072, 24, 4, pf.PF_HASH_BF16X3),
                                                 (1200, 33, 9, 64, 13, 2, pf.PF_HASH_FP64),
                                                 (900, 300, 5, 32, 32, 1, pf.PF_HASH_BF16X3)])
def test_pool_build_bit_exact(n, d, L, pool, K, M, mode):
    """Pooling (Sec. 3.2): pool and sketch hyperplanes, each table's sampled functions,
    codes gathered from the pool bits, sorted tables, prefix tables and sketches."""
    X = workloads.gaussian_unit(n, d, n + pool)
    g, o = _build_pool(X, L, pool, seed=n + d, K=K, M=M, hash_mode=mode)
    assert g.pool == pool
    assert np.array_equal(g.export(pf.PF_EXPORT_POOL_SEL), o.sel), "pool selection"
    _assert_index_equal(g, o)


def test_pool_search_parity():
    X = workloads.gaussian_unit(6000, 48, 61)
    Q = workloads.gaussian_unit(300, 48, 62)
    g, o = _build_pool(X, 40, 512, seed=63)
    for k, rec, kw in [(10, 0.9, {"rule": pf.PF_RULE_POOL}), (1, 0.5, {"rule": pf.PF_RULE_POOL}),
                       (10, 0.9, {}), (20, 0.99, {"rule": pf.PF_RULE_EXACT}),
                       (10, 0.9, {"rule": pf.PF_RULE_POOL, "filter": False})]:
        okw = dict(kw)
        if "filter" in okw:
            okw["filter_on"] = okw.pop("filter")
        _assert_search_equal(g.search(Q, k, rec, **kw), o.search(Q, k, rec, **okw), f"pool k={k} {kw}")
    # the pooled budget rule, and the POOL rule refused on an index without a pool
    gb = pf.Index(X, 64 << 20, seed=63, pool=3072)
    info = gb.info()
    assert (gb.L, info.bytes_device) == pf.pf_plan_index(len(X), 48, 64 << 20, pool=3072)
    assert info.bytes_device <= 64 << 20
    plain = pf.Index(X[:500], 0, L=4)
    with pytest.raises(pf.PfError):
        plain.search(Q[:5], 5, 0.9, rule=pf.PF_RULE_POOL)
    with pytest.raises(pf.PfError):
        pf.Index(X[:500], 0, L=4, pool=40)


@pytest.mark.parametrize("n,d,L,K,M", [(3000, 100, 12, 24, 4), (2000, 64, 10, 24, 2), (800, 5, 6, 13, 1),
                                       (700, 300, 4, 32, 1)])
def test_cp_build_bit_exact(n, d, L, K, M):
    """FHT cross-polytope codes (Sec. 2.2, 4.3): the FP64 rotations on the GPU give the
    oracle's values, hence its codes and tables; the Monte Carlo table is the oracle's."""
    X = workloads.gaussian_unit(n, d, 5 * n + d)
    print(f"[build cp] n={n} d={d} L={L} K={K} M={M}", flush=True)
    g = pf.Index(X, 0, seed=d, K=K, M=M, L=L, family=pf.PF_FAMILY_FHTCP)
    o = oracle.OracleIndex(X, 0, seed=d, K=K, M=M, L=L, cp=True)
    assert g.family == pf.PF_FAMILY_FHTCP
    assert np.array_equal(g.export(pf.PF_EXPORT_CP_TABLE), o.cptab), "collision table"
    _assert_index_equal(g, o)


def test_cp_search_parity():
    X = workloads.gaussian_unit(6000, 100, 71)
    Q = workloads.gaussian_unit(300, 100, 72)
    print("[build cp] n=6000 d=100 L=30", flush=True)
    g = pf.Index(X, 0, seed=73, L=30, family=pf.PF_FAMILY_FHTCP)
    o = oracle.OracleIndex(X, 0, seed=73, L=30, cp=True)
    for k, rec, kw in [(10, 0.9, {}), (10, 0.9, {"rule": pf.PF_RULE_EXACT}), (1, 0.5, {"rule": pf.PF_RULE_ALG1}),
                       (20, 0.99, {"filter": False, "rule": pf.PF_RULE_EXACT})]:
        okw = dict(kw)
        if "filter" in okw:
            okw["filter_on"] = okw.pop("filter")
        _assert_search_equal(g.search(Q, k, rec, **kw), o.search(Q, k, rec, **okw), f"cp k={k} {kw}")
    with pytest.raises(pf.PfError):
        g.search(Q[:4], 5, 0.9, rule=pf.PF_RULE_POOL)
    gb = pf.Index(X, 64 << 20, seed=73, family=pf.PF_FAMILY_FHTCP)
    info = gb.info()
    assert (gb.L, info.bytes_device) == pf.pf_plan_index(len(X), 100, 64 << 20, family=pf.PF_FAMILY_FHTCP)
    assert info.bytes_device <= 64 << 20


def test_edge_cases():
    """Empty batches, a single point, identical points (every code and inner product tied:
    order by position), queries equal to data points, the largest k, the table cap."""
    X = workloads.gaussian_unit(500, 16, 201)
    g = pf.Index(X, 0, seed=3, L=8)
    r = g.search(np.zeros((0, 16), dtype=np.float32), 5, 0.9)
    assert r.ids.shape == (0, 5)
    rb = g.search_batch(np.zeros((0, 16), dtype=np.float32), np.zeros(0, np.int32), np.zeros(0), 5)
    assert rb.ids.shape == (0, 5)
    # one point
    one = pf.Index(X[:1], 0, seed=3, L=3)
    r = one.search(X[:4], 1, 0.9)
    assert np.all(r.ids == 0)
    # identical points: all ties, ids ascending
    same = np.repeat(X[:1], 300, axis=0)
    gs, os_ = _build_both(same, L=6, seed=4)
    _assert_search_equal(gs.search(X[:20], 7, 0.9), os_.search(X[:20], 7, 0.9), "identical points")
    assert np.all(gs.search(X[:20], 7, 0.9).ids == np.arange(7))
    # queries that are data points come back first with inner product 1 (up to rounding)
    r = g.search(X[:50], 3, 0.99)
    assert np.all(r.ids[:, 0] == np.arange(50))
    # the largest k (PF_MAX_K) in a batch with mixed k, and k > PF_MAX_K refused
    Xb = workloads.gaussian_unit(3000, 24, 202)
    gb, ob = _build_both(Xb, L=12, seed=5)
    Q = workloads.gaussian_unit(40, 24, 203)
    ks = np.where(np.arange(40) % 2 == 0, 256, 1).astype(np.int32)
    rec = np.full(40, 0.9)
    oids, oips, ost, obd = _oracle_per_query(ob, Q, ks, rec, 256)
    _assert_batch_equal(gb.search_batch(Q, ks, rec, 256), oids, oips, ost, obd, "k=256")
    with pytest.raises(pf.PfError):
        gb.search(Q, 257, 0.9)
    # a budget for more than 512 tables is capped at 512
    cap = pf.Index(X[:200], 1 << 40, seed=6)
    assert cap.L == 512


def test_max_dimension_parity():
    """d = 4096 (the largest supported): rows longer than any specialised re-rank length,
    hash reduction beyond the GEMM path (FP64 hashing), exact against the oracle."""
    X = workloads.gaussian_unit(600, 4096, 204)
    Q = workloads.gaussian_unit(20, 4096, 205)
    g, o = _build_both(X, L=6, seed=7, M=2)
    _assert_index_equal(g, o)
    _assert_search_equal(g.search(Q, 5, 0.9), o.search(Q, 5, 0.9), "d=4096")
    with pytest.raises(pf.PfError):
        pf.Index(workloads.gaussian_unit(10, 4097, 206), 0, L=2)


def test_measurement_aids_run():
    """The read-rate probes return finite positive rates (64 MiB buffers, one timed launch)."""
    gbs = pf.pf_read_bandwidth(64 << 20, 1)
    rate = pf.pf_random_read_rate(64 << 20, 1)
    print(f"[probes] streaming read {gbs:.0f} GB/s, scattered 4-byte reads {rate / 1e9:.1f} G/s", flush=True)
    assert np.isfinite(gbs) and gbs > 0
    assert np.isfinite(rate) and rate > 0
