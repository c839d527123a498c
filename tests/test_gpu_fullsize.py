"""Parity at the benchmark's full size, in the launch configuration bench.py times.

mixture-1M-d100 (n = 1,000,000, d = 100, 2 GiB -> L = 121, 10,000 queries, k = 10, recall
0.9): the GPU index against the oracle's, structure by structure (bit-exact), then the
whole query batch answered by the learned-batched path with the autotuned tile shape,
compared with the oracle on a sample of the queries (ids, FP32 inner-product bit
patterns, stop level and counters).  The mixed batch of configuration 4 (per-query k and
recall, kmax 100) is sampled the same way.  The oracle builds its own index (about 6 s
with 16 threads) and answers only the sampled queries.
"""
import numpy as np
import pytest

import oracle
import paper_1906_12211_amd as pf
import workloads
from prefix_tables import check_offsets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    torch = pytest.importorskip("torch")
    c = workloads.config(2)
    X, Q = c["points"], c["queries"]
    print(f"[fullsize] building GPU index n={len(X)} d={X.shape[1]}", flush=True)
    g = pf.Index(torch.from_numpy(X).cuda(), c["budget"], seed=workloads.INDEX_SEED)
    print(f"[fullsize] L={g.L}; building oracle index", flush=True)
    o = oracle.OracleIndex(X, c["budget"], seed=workloads.INDEX_SEED, L=g.L)
    return c, g, o


def test_fullsize_index_bit_exact(full):
    c, g, o = full
    assert g.L == o.L == 121 and g.P == 16
    info = g.info()
    assert info.bytes_device == info.bytes_budget_rule <= c["budget"]
    for what, ref, name in [(pf.PF_EXPORT_CODES, o.tcode, "codes"), (pf.PF_EXPORT_IDX, o.tidx, "positions"),
                            (pf.PF_EXPORT_SKETCHES, o.tsk, "table-local sketches"),
                            (pf.PF_EXPORT_POINTS, o.points, "normalised points")]:
        got = g.export(what)
        bad = int(np.count_nonzero(got != ref))
        print(f"[fullsize] {name}: {bad} mismatches of {ref.size}", flush=True)
        assert bad == 0, name
    bad = check_offsets(g.export(pf.PF_EXPORT_OFFSETS), o, g.P)
    print(f"[fullsize] prefix tables (P = {g.P}): {bad} mismatches", flush=True)
    assert bad == 0


def _sample(m, count, seed):
    return np.sort(np.random.default_rng(seed).choice(m, size=count, replace=False))


def test_fullsize_learned_batched_sampled(full):
    torch = pytest.importorskip("torch")
    c, g, o = full
    Q = c["queries"]
    m = len(Q)
    dev = torch.device("cuda:0")
    Qtr = workloads.queries_like(2, 4000, seed_offset=100)
    st = g.search(torch.from_numpy(Qtr).to(dev), 10, 0.9).stats.cpu().numpy()
    target = np.stack([st[:, 0], np.log2(1.0 + st[:, 1])], 1).astype(np.float32)
    s = pf.Scheduler(seed=1)
    s.train(g.features(torch.from_numpy(Qtr).to(dev)), torch.from_numpy(target).to(dev), epochs=5, batch=512,
            lr=2e-3)
    g.set_scheduler(s)
    Qd = torch.from_numpy(Q).to(dev)
    ks = torch.full((m,), 10, dtype=torch.int32, device=dev)
    rec = torch.full((m,), 0.9, dtype=torch.float64, device=dev)
    g.search_batch(Qd, ks, rec, 10, autotune=True)
    r = g.search_batch(Qd, ks, rec, 10, learned=True, timing=True)
    t = g.last_timing()
    print(f"[fullsize] learned-batched tile {t.tile} waves/CU {t.waves_per_cu}, k_search {t.search_ms:.1f} ms",
          flush=True)
    ids, ips, sts = r.ids.cpu().numpy(), r.ips.cpu().numpy(), r.stats.cpu().numpy()
    sel = _sample(m, 200, 7)
    orr = o.search(Q[sel], 10, 0.9)
    ok = orr.boundary == 0
    print(f"[fullsize] sampled {len(sel)} queries, boundary cases {int((~ok).sum())}", flush=True)
    assert ok.mean() > 0.99
    assert np.array_equal(ids[sel][ok], orr.ids[ok])
    assert np.array_equal(ips[sel][ok].view(np.uint32), orr.ips[ok].view(np.uint32))
    ost = np.stack([orr.stop_level, orr.c_scan, orr.c_pass, orr.c_rerank], 1)
    assert np.array_equal(sts[sel][ok][:, :4], ost[ok])
    # every query (not only the sample): k distinct ids, best first, 0 <= c_exact <= c_rerank
    assert np.all(np.diff(ips, axis=1) <= 0)
    srt = np.sort(ids, axis=1)
    assert np.all(srt[:, 1:] != srt[:, :-1]) and ids.min() >= 0 and ids.max() < len(c["points"])
    assert np.all((sts[:, 4] >= 0) & (sts[:, 4] <= sts[:, 3]))


def test_fullsize_mixed_batch_sampled(full):
    torch = pytest.importorskip("torch")
    c, g, o = full
    Q, ks, rec = workloads.mixed_queries(100_000)
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    r = g.search_batch(to(Q), to(ks), to(rec), 100, autotune=True)
    ids, ips, sts = r.ids.cpu().numpy(), r.ips.cpu().numpy(), r.stats.cpu().numpy()
    sel = _sample(len(Q), 180, 8)
    checked = 0
    for k in (1, 10, 100):
        for rc in (0.5, 0.9, 0.99):
            s = sel[(ks[sel] == k) & (rec[sel] == rc)]
            if len(s) == 0:
                continue
            orr = o.search(Q[s], k, rc)
            ok = orr.boundary == 0
            assert np.array_equal(ids[s][ok][:, :k], orr.ids[ok]), (k, rc)
            assert np.all(ids[s][:, k:] == -1)
            assert np.array_equal(ips[s][ok][:, :k].view(np.uint32), orr.ips[ok].view(np.uint32)), (k, rc)
            ost = np.stack([orr.stop_level, orr.c_scan, orr.c_pass, orr.c_rerank], 1)
            assert np.array_equal(sts[s][ok][:, :4], ost[ok]), (k, rc)
            checked += int(ok.sum())
    print(f"[fullsize] mixed batch: {checked} sampled queries equal to the oracle", flush=True)
    assert checked >= 170
