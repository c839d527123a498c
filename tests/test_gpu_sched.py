"""Learned scheduler on the GPU: features, forward pass and gradients against the FP64
reference (oracle/mlp.py), training on traces of the plain method, and the learned queue
order (results must not change, predicted cost must track the real one)."""
import numpy as np
import pytest

import oracle
import paper_1906_12211_amd as pf
import workloads
from oracle import mlp

pytestmark = pytest.mark.gpu


def test_features_match_reference():
    X = workloads.gaussian_unit(5000, 32, 101)
    Q = workloads.gaussian_unit(300, 32, 102)
    g = pf.Index(X, 0, seed=21, L=40)
    o = oracle.OracleIndex(X, 0, seed=21, L=40)
    qc, qs = oracle.hash_codes(oracle.normalize(Q), o.hp, o.L, o.K, o.M)
    P = min(13, o.K)
    b = qc >> (o.K - P)
    sizes = np.stack([o.off[j, b[j] + 1] - o.off[j, b[j]] for j in range(32)], 1)
    ref = mlp.features(qs[0], sizes)
    got = g.features(Q)
    assert np.array_equal(got[:, :64], ref[:, :64])
    assert np.allclose(got[:, 64:], ref[:, 64:], rtol=1e-6, atol=1e-6)


def test_forward_and_gradient_match_fp64_reference():
    rng = np.random.default_rng(5)
    s = pf.Scheduler(seed=3)
    p = (rng.standard_normal(pf.PF_SCHED_PARAMS) * 0.05).astype(np.float32)
    s.set_params(p)
    assert np.array_equal(s.params(), p)
    x = rng.standard_normal((257, 96)).astype(np.float32)
    t = rng.standard_normal((257, 2)).astype(np.float32)
    y_ref, _ = mlp.forward(p.astype(np.float64), x)
    y = s.predict(x)
    assert np.allclose(y, y_ref, rtol=1e-5, atol=1e-5)
    g, loss = s.grad(x, t)
    loss_ref, g_ref = mlp.loss_and_grad(p.astype(np.float64), x, t)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"[grad] relative error {rel:.2e}", flush=True)
    assert rel <= 1e-4
    assert np.allclose(g, g_ref, rtol=1e-3, atol=1e-6 * np.abs(g_ref).max())


def test_training_learns_query_cost_and_keeps_results(tmp_path):
    # tight clusters (easy queries) plus uniform queries (hard ones): costs differ by orders
    d, n = 48, 40000
    cen = workloads.mixture_centers(400, d, 111)
    X = np.concatenate([workloads.mixture(n // 2, d, cen, 0.3, 112, sigma_mode="norm"),
                        workloads.gaussian_unit(n // 2, d, 113)])
    def queries(seed, m):
        return np.concatenate([workloads.mixture(m // 2, d, cen, 0.3, seed, sigma_mode="norm"),
                               workloads.gaussian_unit(m - m // 2, d, seed + 1)])
    Qtr, Qte = queries(120, 4000), queries(130, 1000)
    g = pf.Index(X, 0, seed=23, L=60)
    rtr = g.search(Qtr, 10, 0.9)
    target = np.stack([rtr.stats[:, 0], np.log2(1.0 + rtr.stats[:, 1])], 1).astype(np.float32)
    s = pf.Scheduler(seed=4)
    losses = s.train(g.features(Qtr), target, epochs=30, batch=256, lr=2e-3)
    print(f"[train] loss {losses[0]:.3f} -> {losses[-1]:.3f}", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    rte = g.search(Qte, 10, 0.9)
    pred = s.predict(g.features(Qte))[:, 1]
    actual = np.log2(1.0 + rte.stats[:, 1])
    rank = lambda v: np.argsort(np.argsort(v))
    rho = np.corrcoef(rank(pred), rank(actual))[0, 1]
    print(f"[test] Spearman rho(predicted, actual log2 scan) = {rho:.3f}", flush=True)
    assert rho > 0.5
    g.set_scheduler(s)
    ks = np.full(len(Qte), 10, dtype=np.int32)
    rec = np.full(len(Qte), 0.9)
    rl = g.search_batch(Qte, ks, rec, 10, learned=True)
    rf = g.search_batch(Qte, ks, rec, 10)
    assert np.array_equal(rl.ids, rte.ids) and np.array_equal(rf.ids, rte.ids)
    assert np.array_equal(rl.stats[:, :4], rte.stats[:, :4])
    path = str(tmp_path / "sched.bin")
    s.save(path)
    s2 = pf.Scheduler(seed=99)
    s2.load(path)
    assert np.array_equal(s2.params(), s.params())
