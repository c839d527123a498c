"""The other workloads of the evaluation on the GPU: the planted instance (configuration
3: one neighbour at exactly 30 degrees per query, 2,000 shared decoys near 60 degrees,
uniform background) and the paper's synthetic data set (Sec. 5, "Synthetic Dataset":
x_n is every query's nearest neighbour).  At small scale the answers equal the oracle's;
at full scale the planted / known neighbour is found at least as often as requested."""
import numpy as np
import pytest

import oracle
import paper_1906_12211_amd as pf
import workloads

pytestmark = pytest.mark.gpu


def _equal(gr, orr, label):
    ok = orr.boundary == 0
    assert ok.mean() > 0.99, label
    assert np.array_equal(gr.ids[ok], orr.ids[ok]), label
    assert np.array_equal(gr.ips[ok].view(np.uint32), orr.ips[ok].view(np.uint32)), label
    ost = np.stack([orr.stop_level, orr.c_scan, orr.c_pass, orr.c_rerank], 1)
    assert np.array_equal(gr.stats[ok][:, :4], ost[ok]), label


def test_planted_small_equals_oracle():
    c = workloads.config(3, scale=0.05)
    X, Q = c["points"], c["queries"]
    print(f"[planted small] n={len(X)} d={X.shape[1]} queries={len(Q)}", flush=True)
    g = pf.Index(X, 0, seed=workloads.INDEX_SEED, L=40)
    o = oracle.OracleIndex(X, 0, seed=workloads.INDEX_SEED, L=40)
    for rec in (0.5, 0.9, 0.99):
        _equal(g.search(Q, 1, rec), o.search(Q, 1, rec), f"planted small recall {rec}")


def test_planted_full_recall():
    torch = pytest.importorskip("torch")
    c = workloads.config(3)
    X, Q, pid = c["points"], c["queries"], c["planted"]
    g = pf.Index(torch.from_numpy(X).cuda(), c["budget"], seed=workloads.INDEX_SEED)
    print(f"[planted] n={len(X)} d={X.shape[1]} L={g.L} queries={len(Q)}", flush=True)
    assert g.L == 64 and g.info().bytes_device <= c["budget"]
    Qd = torch.from_numpy(Q).cuda()
    for rec in (0.5, 0.9, 0.99):
        r = g.search(Qd, 1, rec, timing=True)
        ids = r.ids.cpu().numpy()[:, 0]
        st = r.stats.cpu().numpy()
        hit = float(np.mean(ids == pid))
        print(f"[planted] recall target {rec}: planted neighbour found for {hit:.4f}; mean stop level "
              f"{st[:, 0].mean():.2f}, mean scanned {st[:, 1].mean():.0f}, k_search "
              f"{g.last_timing().search_ms:.1f} ms", flush=True)
        assert hit >= rec


def test_paper_synthetic_small_equals_oracle():
    X, Q = workloads.paper_synthetic(30_000, 50, 200, 77)
    g = pf.Index(X, 0, seed=5, L=30)
    o = oracle.OracleIndex(X, 0, seed=5, L=30)
    for k, rec in ((1, 0.9), (10, 0.9), (1, 0.5)):
        _equal(g.search(Q, k, rec), o.search(Q, k, rec), f"paper synthetic k={k} recall {rec}")


def test_paper_synthetic_full_finds_xn():
    """n = 1,000,000 in 3 x 100 dimensions, 1,000 queries, 2 GiB: x_n (the last row) is the
    nearest neighbour of every query; the paper's robustness case."""
    torch = pytest.importorskip("torch")
    X, Q = workloads.paper_synthetic(1_000_000, 100, 1000, 78)
    g = pf.Index(torch.from_numpy(X).cuda(), 2 << 30, seed=workloads.INDEX_SEED)
    print(f"[paper synthetic] n={len(X)} d={X.shape[1]} L={g.L}", flush=True)
    Qd = torch.from_numpy(Q).cuda()
    for rec in (0.5, 0.9, 0.99):
        r = g.search(Qd, 1, rec, timing=True)
        ids = r.ids.cpu().numpy()[:, 0]
        st = r.stats.cpu().numpy()
        hit = float(np.mean(ids == len(X) - 1))
        print(f"[paper synthetic] recall target {rec}: x_n found for {hit:.4f}; mean stop level "
              f"{st[:, 0].mean():.2f}, k_search {g.last_timing().search_ms:.1f} ms", flush=True)
        assert hit >= rec
