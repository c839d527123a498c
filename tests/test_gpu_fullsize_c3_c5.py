"""Parity at full size for the planted instance and the 10 M-point configuration, in the
launch configuration bench.py times.

planted-1M-d256 (n = 1,000,000 uniform unit vectors in d = 256 with planted neighbours,
10,000 queries, 2 GiB -> L = 64, k = 1, recall 0.5 / 0.9 / 0.99) and mixture-10M-d128
(n = 10,000,000, d = 128, 100,000 clusters, 16 GiB -> L = 82, 100,000 queries, k = 10, recall
0.9, the learned-batched path): the oracle builds its own index from the same seeded points
(in a thread, while the GPU works; the C library releases the interpreter lock), every
structure is compared bit for bit, and a sample of the batch answered by the GPU is compared
with the oracle's answers (ids, FP32 inner-product bit patterns, stop level, counters).
"""
import threading
import time

import numpy as np
import pytest

import oracle
import paper_1906_12211_amd as pf
import workloads
from prefix_tables import check_offsets

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]


def _oracle_in_thread(X, budget, L):
    box = {}

    def run():
        t0 = time.time()
        box["o"] = oracle.OracleIndex(X, budget, seed=workloads.INDEX_SEED, L=L)
        box["s"] = time.time() - t0

    th = threading.Thread(target=run)
    th.start()
    return th, box


def _structures_equal(g, o, label):
    for what, name in [(pf.PF_EXPORT_POINTS, "points"), (pf.PF_EXPORT_CODES, "tcode"), (pf.PF_EXPORT_IDX, "tidx"),
                       (pf.PF_EXPORT_SKETCHES, "tsk")]:
        got = g.export(what)
        ref = getattr(o, name)
        bad = int(np.count_nonzero(got != ref))
        print(f"[{label}] {name}: {bad} mismatches of {ref.size}", flush=True)
        assert bad == 0, f"{label} {name}"
        del got
    bad = check_offsets(g.export(pf.PF_EXPORT_OFFSETS), o, g.P)
    print(f"[{label}] off (P = {g.P}): {bad} mismatches", flush=True)
    assert bad == 0, f"{label} off"


def _sampled_equal(ids, ips, sts, sel, orr, k, label):
    ok = orr.boundary == 0
    print(f"[{label}] {len(sel)} sampled queries, {int((~ok).sum())} boundary cases", flush=True)
    assert ok.mean() > 0.97, label
    assert np.array_equal(ids[sel][ok][:, :k], orr.ids[ok]), label
    assert np.array_equal(ips[sel][ok][:, :k].view(np.uint32), orr.ips[ok].view(np.uint32)), label
    ost = np.stack([orr.stop_level, orr.c_scan, orr.c_pass, orr.c_rerank], 1)
    assert np.array_equal(sts[sel][ok][:, :4], ost[ok]), label


def _batch_properties(ids, ips, sts, n):
    """Every query, not only the sample: distinct ids in range, best first, counters ordered."""
    assert np.all(np.diff(ips, axis=1) <= 0)
    srt = np.sort(ids, axis=1)
    assert np.all(srt[:, 1:] != srt[:, :-1]) and ids.min() >= 0 and ids.max() < n
    assert np.all((sts[:, 4] >= 0) & (sts[:, 4] <= sts[:, 3]) & (sts[:, 2] <= sts[:, 1]))


@pytest.fixture(scope="module")
def planted():
    torch = pytest.importorskip("torch")
    c = workloads.config(3)
    X = c["points"]
    L, nbytes = pf.pf_plan_index(len(X), X.shape[1], c["budget"])
    print(f"[planted full] n={len(X)} d={X.shape[1]} L={L}; oracle index in a thread", flush=True)
    th, box = _oracle_in_thread(X, c["budget"], L)
    g = pf.Index(torch.from_numpy(X).cuda(), c["budget"], seed=workloads.INDEX_SEED)
    assert (g.L, g.info().bytes_device) == (L, nbytes) and nbytes <= c["budget"]
    Qd = torch.from_numpy(c["queries"]).cuda()
    m = len(Qd)
    ks = torch.ones((m,), dtype=torch.int32, device="cuda")
    res = {}
    for rec in (0.5, 0.9, 0.99):
        rc = torch.full((m,), rec, dtype=torch.float64, device="cuda")
        g.search_batch(Qd, ks, rc, 1, autotune=True)
        r = g.search_batch(Qd, ks, rc, 1, timing=True)
        res[rec] = (r.ids.cpu().numpy(), r.ips.cpu().numpy(), r.stats.cpu().numpy())
        print(f"[planted full] recall {rec}: batched k_search {g.last_timing().search_ms:.1f} ms", flush=True)
    th.join()
    print(f"[planted full] oracle index built in {box['s']:.0f} s", flush=True)
    return c, g, box["o"], res


def test_planted_fullsize_index_bit_exact(planted):
    c, g, o, _ = planted
    _structures_equal(g, o, "planted full")


def test_planted_fullsize_batched_sampled(planted):
    c, g, o, res = planted
    Q, pid = c["queries"], c["planted"]
    sel = np.sort(np.random.default_rng(31).choice(len(Q), size=100, replace=False))
    for rec, (ids, ips, sts) in res.items():
        orr = o.search(Q[sel], 1, rec)
        _sampled_equal(ids, ips, sts, sel, orr, 1, f"planted full recall {rec}")
        _batch_properties(ids, ips, sts, len(c["points"]))
        hit = float(np.mean(ids[:, 0] == pid))
        print(f"[planted full] recall {rec}: planted neighbour found for {hit:.4f}", flush=True)
        assert hit >= rec


@pytest.fixture(scope="module")
def c5():
    torch = pytest.importorskip("torch")
    c = workloads.config(5, with_train=False)
    X, Q = c["points"], c["queries"]
    n, d = X.shape
    L, nbytes = pf.pf_plan_index(n, d, c["budget"])
    print(f"[c5 full] n={n} d={d} L={L}; oracle index in a thread", flush=True)
    th, box = _oracle_in_thread(X, c["budget"], L)
    g = pf.Index(torch.from_numpy(X).cuda(), c["budget"], seed=workloads.INDEX_SEED)
    assert (g.L, g.info().bytes_device) == (L, nbytes) and nbytes <= c["budget"]
    # the learned-batched launch: scheduler trained on traces of other queries of the mixture
    Qtr = torch.from_numpy(workloads.queries_like(5, 100_000, seed_offset=100)).cuda()
    st = g.search(Qtr, 10, 0.9).stats.cpu().numpy()
    target = np.stack([st[:, 0], np.log2(1.0 + st[:, 1])], 1).astype(np.float32)
    s = pf.Scheduler(seed=5)
    s.train(g.features(Qtr), torch.from_numpy(target).cuda(), epochs=3, batch=1024, lr=2e-3)
    g.set_scheduler(s)
    del Qtr
    m = len(Q)
    Qd = torch.from_numpy(Q).cuda()
    ks = torch.full((m,), 10, dtype=torch.int32, device="cuda")
    rc = torch.full((m,), 0.9, dtype=torch.float64, device="cuda")
    g.search_batch(Qd, ks, rc, 10, autotune=True)
    r = g.search_batch(Qd, ks, rc, 10, learned=True, timing=True)
    t = g.last_timing()
    print(f"[c5 full] learned-batched tile {pf.pf_tile_name(t.tile)} waves/CU {t.waves_per_cu}, "
          f"k_search {t.search_ms:.0f} ms", flush=True)
    res = (r.ids.cpu().numpy(), r.ips.cpu().numpy(), r.stats.cpu().numpy())
    th.join()
    print(f"[c5 full] oracle index built in {box['s']:.0f} s", flush=True)
    return c, g, box["o"], res


def test_c5_fullsize_index_bit_exact(c5):
    c, g, o, _ = c5
    _structures_equal(g, o, "c5 full")


def test_c5_fullsize_learned_batched_sampled(c5):
    c, g, o, (ids, ips, sts) = c5
    Q = c["queries"]
    sel = np.sort(np.random.default_rng(32).choice(len(Q), size=100, replace=False))
    orr = o.search(Q[sel], 10, 0.9)
    _sampled_equal(ids, ips, sts, sel, orr, 10, "c5 full")
    _batch_properties(ids, ips, sts, len(c["points"]))
