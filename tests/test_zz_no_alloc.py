"""pf_search_noalloc, the entry point for callers that cannot allocate device memory,
against pf_search on the same index and queries: ids, FP32 inner-product bit patterns and
per-query statistics equal, on two calls in a row (the second smaller, so the shared
scratch array holds the first call's contents), for a plain, a pooled and a short-code
(K <= 13: no prefix ranges) index and indexes with 3-byte positions and with a 16-bit prefix
table (8-bit code suffixes); oversize batches and bad rows are refused."""
import numpy as np
import pytest

import paper_1906_12211_amd as pf
import workloads

pytestmark = pytest.mark.gpu


def _noalloc(g, Qd, k, recall):
    torch = pytest.importorskip("torch")
    m = Qd.shape[0]
    ids = torch.full((m, k), -7, dtype=torch.int32, device="cuda")
    ips = torch.full((m, k), float("nan"), dtype=torch.float32, device="cuda")
    st = torch.zeros((m, 7), dtype=torch.int64, device="cuda")
    g.search_noalloc(Qd, k, recall, ids, ips, st)
    st = st.cpu().numpy()
    st[:, 0] &= 0xFFFFFFFF
    return ids.cpu().numpy(), ips.cpu().numpy(), st


def _same(g, Qd, k, recall, label):
    ref = g.search(Qd, k, recall)
    ids, ips, st = _noalloc(g, Qd, k, recall)
    assert np.array_equal(ids, ref.ids.cpu().numpy()), label
    assert np.array_equal(ips.view(np.uint32), ref.ips.cpu().numpy().view(np.uint32)), label
    assert np.array_equal(st, ref.stats.cpu().numpy()), label
    print(f"[noalloc] {label}: {Qd.shape[0]} queries equal to pf_search; stop levels "
          f"{np.unique(st[:, 0]).tolist()}", flush=True)


@pytest.mark.parametrize("kw", [dict(L=40), dict(L=24, pool=512), dict(L=30, K=12), dict(L=40, pos_bytes=3),
                                dict(L=40, prefix_bits=16)])
def test_noalloc_equals_search_on_two_calls(kw):
    torch = pytest.importorskip("torch")
    X = workloads.gaussian_unit(20_000, 100, 301)
    print(f"[noalloc] index {kw}", flush=True)
    g = pf.Index(torch.from_numpy(X).cuda(), 0, seed=9, **kw)
    Q1 = torch.from_numpy(workloads.gaussian_unit(3000, 100, 302)).cuda()
    Q2 = torch.from_numpy(workloads.gaussian_unit(700, 100, 303)).cuda()
    _same(g, Q1, 10, 0.9, f"{kw} first call")
    _same(g, Q2, 5, 0.99, f"{kw} second, smaller call")


def test_noalloc_refuses_oversize_batch_and_bad_rows():
    torch = pytest.importorskip("torch")
    X = workloads.gaussian_unit(5000, 100, 311)
    g = pf.Index(torch.from_numpy(X).cuda(), 0, seed=9, L=40)
    big = torch.from_numpy(workloads.gaussian_unit(200_000, 100, 312)).cuda()
    out = torch.empty((200_000, 10), dtype=torch.int32, device="cuda")
    with pytest.raises(pf.PfError) as e:
        g.search_noalloc(big, 10, 0.9, out)
    assert e.value.code == pf.PF_EUNSUPPORTED and "scratch" in str(e.value)
    Q = torch.from_numpy(workloads.gaussian_unit(50, 100, 313)).cuda()
    Q[17] = 0.0
    with pytest.raises(pf.PfError) as e:
        g.search_noalloc(Q, 10, 0.9, out[:50])
    assert e.value.code == pf.PF_EINVAL and "row 17" in str(e.value)
    # the index still answers correctly afterwards
    _same(g, Q[18:], 10, 0.9, "after refused calls")
