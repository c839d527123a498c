"""Throughput of the adaptive k-NN query path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (default): mixture-1M-d100 -- n = 1,000,000 unit vectors in d = 100 drawn from
a mixture of 10,000 Gaussian clusters (centres uniform on the sphere, sigma = 0.3 per
coordinate, then normalised), 10,000 queries from the same mixture, k = 10, recall 0.9,
memory budget 2 GiB (L = 108 tables of K = 24 bits, M = 32 sketches).

The index is built once (its device time is reported as build_ms) and stays resident
in HBM with the queries; one timed step answers the whole batch of queries: query
normalisation, hashing, prefix ranges and the adaptive search kernel.
Four query paths are timed on the same batch: the plain search (static query slots),
the persistent batched search with a FIFO work queue (with every re-ranked vector read
from both 16-bit planes, and with the upper-plane bound first), and the learned-batched
search (work queue ordered longest-predicted-first by the scheduler network, trained
first on traces of the plain method for other queries of the same distribution).
`value` is the learned-batched rate; the others are reported beside it.
Prints one JSON line.  The roofline entry is for the search kernel in the learned-batched
path, whose average launch duration is measured with HIP events on the launch stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1906_12211_amd as pf  # noqa: E402
import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "queries/sec at k=10, recall≥0.9: learned-batched vs plain GPU; filter HBM GB/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_mixture-1M-d100_traffic.json")
SEARCH_SRC = os.path.join(ROOT, "paper_1906_12211_amd", "csrc", "k_search.hip")


def algorithmic_bytes(stats: np.ndarray, d: int, k: int, L: int, K: int) -> float:
    """Bytes the method must move for the queries of one launch of the search kernel:
    8 B per scanned table-local sketch, 4 B per position of a passing entry, the 8-bit
    summary (8 + d B, or d B where the rows share one scale and carry no header: 8 + dpad
    bytes would take another 128-byte line) of every candidate bounded from it, the upper
    16-bit plane (2d B)
    of every candidate whose upper plane was read and the lower plane (2d B) of those
    whose exact inner product was needed, the query (4d) and its result (8k), and the
    two range bounds (8 B) of every table at every visited level."""
    stop = stats[:, 0].astype(np.float64)
    dpad = 4 * ((d + 3) // 4)
    hdr = 8.0 if 8 + dpad <= (dpad + 127) // 128 * 128 else 0.0
    per_q = (8.0 * stats[:, 1] + 4.0 * stats[:, 2] + (hdr + d) * stats[:, 6] + 2.0 * d * (stats[:, 5] + stats[:, 4])
             + 4.0 * d
             + 8.0 * k + 8.0 * L * (K + 1 - np.maximum(stop, 1)))
    return float(per_q.sum())


HOST_MARK = b"// ====================================================================== host side"


def search_device_sha(src: bytes = None) -> str:
    """Fingerprint of the search kernel's device code: k_search.hip up to its host-side
    section, without comments and blank space, so that host-only and comment edits keep
    the counters valid."""
    if src is None:
        src = open(SEARCH_SRC, "rb").read()
    code = src.split(HOST_MARK)[0].decode()
    code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
    code = re.sub(r"//[^\n]*", " ", code)
    code = " ".join(code.split())
    return hashlib.sha256(code.encode()).hexdigest()


def plain_gather_bytes(stats: np.ndarray, d: int, k: int, L: int) -> float:
    """The same launch counted as if every re-ranked candidate's FP32 vector were gathered
    (4d B), with the prefix-table reads (4L), sketches (8 B per scanned entry), positions
    of passing entries (4 B), the query and the result: the bytes a re-rank without the
    8-bit and 16-bit bounds would move (reported beside the roofline, not in it)."""
    per_q = 4.0 * L + 8.0 * stats[:, 1] + 4.0 * stats[:, 2] + 4.0 * d * stats[:, 3] + 4.0 * d + 8.0 * k
    return float(per_q.sum())


def traffic_entry(tile_name: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current search kernel source with the tile shape this run launched."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("k_search_device_sha256") != search_device_sha() or t.get("tile_name") != tile_name:
        return None
    return t.get("bytes_per_launch")


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(points, queries, budget, k, recall, seconds):
    """The oracle, as it stands, on the host cores over a bounded sample of the queries."""
    import oracle

    t0 = time.time()
    ix = oracle.OracleIndex(points, budget, seed=workloads.INDEX_SEED)
    build_s = time.time() - t0
    log(f"oracle index built in {build_s:.1f} s")
    done, el, chunk = 0, 0.0, 64
    while done < len(queries) and el < seconds:
        q = queries[done:done + chunk]
        t = time.time()
        ix.search(q, k, recall)
        el += time.time() - t
        done += len(q)
        chunk = min(2048, chunk * 2)
    cores = oracle.num_threads()
    # one thread, one query at a time (the paper's single-core setting), on a smaller sample
    oracle.set_threads(1)
    n1, el1 = 0, 0.0
    while n1 < len(queries) and el1 < seconds / 4:
        q = queries[n1:n1 + 16]
        t = time.time()
        ix.search(q, k, recall)
        el1 += time.time() - t
        n1 += len(q)
    oracle.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": done / el, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"first {done} of {len(queries)} queries of the same workload on the oracle's "
                      f"own index (oracle build {build_s:.1f} s, not timed)",
            "seconds": el, "single_thread_qps": n1 / el1, "single_thread_sample": n1,
            "host_cpu": model, "host_nproc": os.cpu_count()}


def mixed_batch(ix, dev, args):
    """Configuration 4 on the same index: 100,000 queries, half from the mixture and half
    uniform, with per-query k in {1, 10, 100} and recall in {0.5, 0.9, 0.99}, answered by
    the persistent batched search under four queue orders: as given (FIFO), the learned
    order (longest predicted first; network trained on traces of the plain method for
    another batch of the same distribution), the order of the true costs (the plain
    method's scanned-entry counts of this batch; a bound no predictor can beat) and the
    reverse of the learned order (shortest predicted first)."""
    import torch

    m = max(1, int(round(100_000 * args.scale)))
    Q, ks, rec = workloads.mixed_queries(m)
    Qt, kst, rect = workloads.mixed_queries(max(1, int(round(m * args.train_frac))), seed_offset=100)
    kmax = 100
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Qd, ksd, recd = to(Q), to(ks), to(rec)
    Qtd, kstd, rectd = to(Qt), to(kst), to(rect)
    t0 = time.perf_counter()
    st = ix.search_batch(Qtd, kstd, rectd, kmax).stats.cpu().numpy()
    target = np.stack([st[:, 0], np.log2(1.0 + st[:, 1])], 1).astype(np.float32)
    sched = pf.Scheduler(seed=2)
    losses = sched.train(ix.features(Qtd, kstd, rectd), to(target), epochs=20, batch=512, lr=2e-3)
    ix.set_scheduler(sched)
    train_s = time.perf_counter() - t0
    log(f"mixed batch: scheduler trained on {len(Qt)} traces in {train_s:.1f} s, "
        f"loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    ix.search_batch(Qd, ksd, recd, kmax, autotune=True)
    base = ix.search_batch(Qd, ksd, recd, kmax)
    cost = np.log2(1.0 + base.stats.cpu().numpy()[:, 1])
    pred = sched.predict(ix.features(Qd, ksd, recd)).cpu().numpy()[:, 1]
    rank = lambda v: np.argsort(np.argsort(v))
    rho = float(np.corrcoef(rank(pred), rank(cost))[0, 1])
    lpt_true = np.argsort(-cost, kind="stable").astype(np.int32)
    spt_pred = np.argsort(pred, kind="stable").astype(np.int32)
    orders = {
        "fifo": dict(),
        "learned": dict(learned=True),
        "true_cost_lpt": dict(order=to(lpt_true)),
        "shortest_predicted_first": dict(order=to(spt_pred)),
    }
    out = {}
    steps = max(1, min(args.steps, 5))
    for name, kw in orders.items():
        for _ in range(max(1, min(args.warmup, 2))):
            r = ix.search_batch(Qd, ksd, recd, kmax, timing=True, **kw)
        torch.cuda.synchronize()
        ks_ms = []
        t = time.perf_counter()
        for _ in range(steps):
            r = ix.search_batch(Qd, ksd, recd, kmax, timing=True, **kw)
            ks_ms.append(ix.last_timing().search_ms)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps * 1e3
        same = bool(torch.equal(r.ids, base.ids))
        out[name] = {"ms_per_step": wall, "qps": m / (wall / 1e3), "search_kernel_ms": float(np.mean(ks_ms)),
                     "ids_equal_fifo": same}
        log(f"mixed batch {name}: {wall:.2f} ms/step, search kernel {np.mean(ks_ms):.2f} ms, ids equal {same}")
    t = ix.last_timing()
    sb = base.stats.cpu().numpy()
    return {"workload": "mixed-100k-on-1M-d100", "queries": m, "kmax": kmax, "steps": steps,
            "orders": out,
            "learned_vs_fifo": out["fifo"]["search_kernel_ms"] / out["learned"]["search_kernel_ms"],
            "spearman_pred_vs_true_cost": rho,
            "scheduler": {"train_queries": int(len(Qt)), "train_s": train_s, "loss_first": float(losses[0]),
                          "loss_last": float(losses[-1])},
            "tile": {"tile": t.tile, "waves_per_cu": t.waves_per_cu},
            "mean_counts": {"c_scan": float(sb[:, 1].mean()), "c_pass": float(sb[:, 2].mean()),
                            "c_upper": float(sb[:, 5].mean()), "c_exact": float(sb[:, 4].mean())},
            "cost_spread_log2_scan": {"p10": float(np.percentile(cost, 10)), "p50": float(np.percentile(cost, 50)),
                                      "p90": float(np.percentile(cost, 90)), "max": float(cost.max())}}


def exact_topk_gpu(Xd, Qd, k: int, extra: int = 8):
    """Exact k-NN ids (ip desc, id asc) of normalised device rows Qd over Xd: every inner
    product in FP64 on the GPU (the FP32 library GEMM is not used: its rounding reorders
    the near-tied neighbours of large, nearly uniform point sets), the best k + extra per
    query ordered on the host."""
    import torch

    Xd64 = None
    out = np.empty((Qd.shape[0], k), dtype=np.int64)
    step = max(1, int(2e9 // (8 * Xd.shape[0])))
    for s in range(0, Qd.shape[0], step):
        q = Qd[s:s + step].double()
        G = torch.empty((q.shape[0], Xd.shape[0]), dtype=torch.float64, device=Xd.device)
        for c0 in range(0, Xd.shape[0], 1 << 22):
            G[:, c0:c0 + (1 << 22)] = q @ Xd[c0:c0 + (1 << 22)].double().T
        v, ix = torch.topk(G, k + extra, dim=1)
        v, ix = v.cpu().numpy(), ix.cpu().numpy()
        del G
        for t in range(len(q)):
            out[s + t] = ix[t][np.lexsort((ix[t], -v[t]))[:k]]
    return out


def paper_synthetic(dev):
    """The paper's synthetic set (Sec. 5): 1,000,000 points in 3 x 100 dimensions whose last
    row is every query's nearest neighbour, 1,000 queries, 2 GiB, k = 1: per recall target
    the fraction of queries that return it, the stop levels and the search time (plain
    single launch and batched work queue)."""
    import torch

    X, Q = workloads.paper_synthetic(1_000_000, 100, 1000, 78)
    Xd = torch.from_numpy(X).to(dev)
    ix = pf.Index(Xd, 2 << 30, seed=workloads.INDEX_SEED)
    del Xd
    info = ix.info()
    m = len(Q)
    Qd = torch.from_numpy(Q).to(dev)
    out = {"workload": "paper-synthetic-1M-3x100", "n": len(X), "d": X.shape[1], "queries": m, "k": 1,
           "L": info.L, "build_ms": info.build_ms, "targets": {}}
    for rec in (0.5, 0.9, 0.99):
        ks = torch.ones((m,), dtype=torch.int32, device=dev)
        rc = torch.full((m,), rec, dtype=torch.float64, device=dev)
        ix.search(Qd, 1, rec)
        plain = []
        for _ in range(3):
            r = ix.search(Qd, 1, rec, timing=True)
            plain.append(ix.last_timing().search_ms)
        ix.search_batch(Qd, ks, rc, 1, autotune=True)
        batched = []
        for _ in range(3):
            rb = ix.search_batch(Qd, ks, rc, 1, timing=True)
            batched.append(ix.last_timing().search_ms)
        hit = float(np.mean(r.ids.cpu().numpy()[:, 0] == len(X) - 1))
        hit_b = float(np.mean(rb.ids.cpu().numpy()[:, 0] == len(X) - 1))
        st = r.stats.cpu().numpy()
        out["targets"][str(rec)] = {"x_n_found": hit, "x_n_found_batched": hit_b,
                                    "mean_stop_level": float(st[:, 0].mean()),
                                    "mean_c_scan": float(st[:, 1].mean()),
                                    "search_kernel_ms_plain": float(np.mean(plain)),
                                    "search_kernel_ms_batched": float(np.mean(batched))}
        log(f"paper synthetic, recall {rec}: x_n found {hit:.4f}, kernel {np.mean(plain):.2f} ms plain, "
            f"{np.mean(batched):.2f} ms batched")
    return out


def cp_index(X, Q, k, recall, budget, dev, truth_ids):
    """The same workload on an index whose table codes are FHT cross-polytope values
    (Sec. 2.2, 4.3; the sketches stay hyperplane bits): build time (the FP64 rotations),
    query hashing time, and the batched search under the default rule."""
    import torch

    Xd = torch.from_numpy(X).to(dev)
    ix = pf.Index(Xd, budget, seed=workloads.INDEX_SEED, family=pf.PF_FAMILY_FHTCP)
    del Xd
    info = ix.info()
    m = len(Q)
    Qd = torch.from_numpy(Q).to(dev)
    ks = torch.full((m,), k, dtype=torch.int32, device=dev)
    rec = torch.full((m,), recall, dtype=torch.float64, device=dev)
    ix.search_batch(Qd, ks, rec, k, autotune=True)
    r = ix.search_batch(Qd, ks, rec, k, timing=True)
    ts = []
    for _ in range(3):
        r = ix.search_batch(Qd, ks, rec, k, timing=True)
        t = ix.last_timing()
        ts.append((t.hash_ms, t.search_ms, t.total_ms))
    ids = r.ids.cpu().numpy()[:len(truth_ids)]
    st = r.stats.cpu().numpy()
    recm = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(ids, truth_ids)]))
    out = {"family": "fht-cross-polytope", "L": info.L, "build_ms": info.build_ms,
           "normalize+hash_ms": float(np.mean([a for a, _, _ in ts])),
           "search_kernel_ms": float(np.mean([b for _, b, _ in ts])),
           "qps": m / (float(np.mean([c for _, _, c in ts])) / 1e3), "recall_measured": recm,
           "mean_counts": {"c_scan": float(st[:, 1].mean()), "c_pass": float(st[:, 2].mean())},
           "stop_level_hist": np.bincount(st[:, 0], minlength=info.K + 1).tolist()}
    log(f"cross-polytope index: build {info.build_ms:.0f} ms, search kernel {out['search_kernel_ms']:.2f} ms, "
        f"recall {recm:.4f}")
    return out


def pooled_index(X, Q, k, recall, budget, dev, truth_ids):
    """The same workload on an index built with pooling (Sec. 3.2: 3,072 shared functions,
    each table sampling its 24): build time, query hashing time, and the batched search
    under the default stopping rule and under Algorithm 3's test."""
    import torch

    Xd = torch.from_numpy(X).to(dev)
    ix = pf.Index(Xd, budget, seed=workloads.INDEX_SEED, pool=3072)
    del Xd
    info = ix.info()
    m = len(Q)
    Qd = torch.from_numpy(Q).to(dev)
    ks = torch.full((m,), k, dtype=torch.int32, device=dev)
    rec = torch.full((m,), recall, dtype=torch.float64, device=dev)
    ix.search_batch(Qd, ks, rec, k, autotune=True)
    out = {"pool": 3072, "L": info.L, "build_ms": info.build_ms}
    for name, rule in (("default_rule", pf.PF_RULE_FILTER), ("algorithm3_rule", pf.PF_RULE_POOL)):
        r = ix.search_batch(Qd, ks, rec, k, rule=rule, timing=True)
        ts = []
        for _ in range(3):
            r = ix.search_batch(Qd, ks, rec, k, rule=rule, timing=True)
            t = ix.last_timing()
            ts.append((t.hash_ms, t.search_ms, t.total_ms))
        ids = r.ids.cpu().numpy()[:len(truth_ids)]
        recm = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(ids, truth_ids)]))
        out[name] = {"normalize+hash_ms": float(np.mean([a for a, _, _ in ts])),
                     "search_kernel_ms": float(np.mean([b for _, b, _ in ts])),
                     "qps": m / (float(np.mean([c for _, _, c in ts])) / 1e3), "recall_measured": recm}
        log(f"pooled index, {name}: search kernel {out[name]['search_kernel_ms']:.2f} ms, recall {recm:.4f}")
    return out


def workload_c5(args):
    """Configuration 5: n = 10,000,000 clustered unit vectors in d = 128 (100,000 clusters),
    16 GiB budget; the scheduler is trained on 1,000,000 plain-method traces and the three
    query paths are timed on 100,000 further queries (k = 10, recall 0.9)."""
    import torch

    dev = torch.device("cuda:0")
    log("generating mixture-10M-d128")
    c = workloads.config(5, scale=args.scale)
    X, Qtr, Q = c["points"], c["train_queries"], c["queries"]
    n, d = X.shape
    m = len(Q)
    k, recall = c["k"], c["recall"]
    Xd = torch.from_numpy(X).to(dev)
    del X
    ix = pf.Index(Xd, c["budget"], seed=workloads.INDEX_SEED)
    info = ix.info()
    log(f"index built: L={info.L} device build {info.build_ms:.1f} ms, {info.bytes_device / 2**30:.2f} GiB")
    t0 = time.perf_counter()
    Qtrd = torch.from_numpy(Qtr).to(dev)
    ks_t = torch.full((len(Qtr),), k, dtype=torch.int32, device=dev)
    rec_t = torch.full((len(Qtr),), recall, dtype=torch.float64, device=dev)
    st = ix.search_batch(Qtrd, ks_t, rec_t, k).stats.cpu().numpy()
    trace_s = time.perf_counter() - t0
    target = np.stack([st[:, 0], np.log2(1.0 + st[:, 1])], 1).astype(np.float32)
    sched = pf.Scheduler(seed=5)
    t0 = time.perf_counter()
    losses = sched.train(ix.features(Qtrd), torch.from_numpy(target).to(dev), epochs=5, batch=1024, lr=2e-3)
    train_s = time.perf_counter() - t0
    ix.set_scheduler(sched)
    del Qtrd
    log(f"{len(Qtr)} traces in {trace_s:.1f} s; scheduler trained in {train_s:.1f} s, "
        f"loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    Qd = torch.from_numpy(Q).to(dev)
    ks_d = torch.full((m,), k, dtype=torch.int32, device=dev)
    rec_d = torch.full((m,), recall, dtype=torch.float64, device=dev)
    ix.search_batch(Qd, ks_d, rec_d, k, autotune=True)
    modes = {
        "plain": lambda: ix.search(Qd, k, recall, timing=True),
        "batched_fifo": lambda: ix.search_batch(Qd, ks_d, rec_d, k, timing=True),
        "learned_batched": lambda: ix.search_batch(Qd, ks_d, rec_d, k, learned=True, timing=True),
    }
    res = {}
    steps = max(1, min(args.steps, 5))
    for name, fn in modes.items():
        r = fn()
        torch.cuda.synchronize()
        ks_ms = []
        t = time.perf_counter()
        for _ in range(steps):
            r = fn()
            ks_ms.append(ix.last_timing().search_ms)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps * 1e3
        res[name] = {"ms_per_step": wall, "qps": m / (wall / 1e3), "search_kernel_ms": float(np.mean(ks_ms)),
                     "r": r}
        log(f"{name}: {wall:.2f} ms/step, search kernel {np.mean(ks_ms):.2f} ms")
    r = res["learned_batched"].pop("r")
    for v in res.values():
        v.pop("r", None)
    stats = r.stats.cpu().numpy()
    cost = np.log2(1.0 + stats[:, 1])
    pred = sched.predict(ix.features(Qd)).cpu().numpy()[:, 1]
    rank = lambda v: np.argsort(np.argsort(v))
    ns = min(args.recall_sample, m)
    Xn = torch.from_numpy(ix.export(pf.PF_EXPORT_POINTS)).to(dev)
    Qn = torch.from_numpy(pf.pf_normalize(Q[:ns])).to(dev)
    truth = exact_topk_gpu(Xn, Qn, k)
    del Xn
    ids = r.ids.cpu().numpy()
    rec = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(ids[:ns], truth)]))
    log(f"recall {rec:.4f} on {ns} queries")
    A = algorithmic_bytes(stats, d, k, info.L, info.K)
    kms = res["learned_batched"]["search_kernel_ms"]
    achieved = A / (kms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": res["learned_batched"]["qps"], "unit": "queries/s", "n_gpus": 1,
        "steps": steps, "warmup": 1, "ms_per_step": res["learned_batched"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": c["name"], "n": n, "d": d, "queries": m, "k": k, "recall_target": recall,
                   "budget_bytes": c["budget"], "L": info.L, "K": info.K, "M": info.M, "B": 12,
                   "train_traces": len(Qtr), "path": "learned_batched"},
        "paths": res,
        "learned_vs_plain": res["plain"]["ms_per_step"] / res["learned_batched"]["ms_per_step"],
        "learned_vs_fifo": res["batched_fifo"]["search_kernel_ms"] / kms,
        "scheduler": {"trace_s": trace_s, "train_s": train_s, "loss_first": float(losses[0]),
                      "loss_last": float(losses[-1]),
                      "spearman_pred_vs_true_cost": float(np.corrcoef(rank(pred), rank(cost))[0, 1])},
        "recall_measured": rec, "recall_sample": ns, "build_ms": info.build_ms,
        "bytes_device": info.bytes_device,
        "stop_level_hist": np.bincount(stats[:, 0], minlength=info.K + 1).tolist(),
        "mean_counts": {"c_scan": float(stats[:, 1].mean()), "c_pass": float(stats[:, 2].mean()),
                        "c_rerank": float(stats[:, 3].mean()), "c_q8": float(stats[:, 6].mean()),
                        "c_upper": float(stats[:, 5].mean()), "c_exact": float(stats[:, 4].mean())},
        "roofline": {"kernel": "k_search", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": A, "avg_launch_ms": kms,
                     "fp32_gather_bytes_per_launch": plain_gather_bytes(stats, d, k, info.L)},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink n and m (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--recall-sample", type=int, default=1000)
    ap.add_argument("--paths", default="plain,batched_fifo_both_planes,batched_fifo,learned_batched",
                    help="query paths to time (comma separated); the last one is the headline")
    ap.add_argument("--train-frac", type=float, default=2.0,
                    help="scheduler training queries as a multiple of the benchmark query count")
    ap.add_argument("--no-pool", action="store_true",
                    help="skip the pooled, cross-polytope and paper-synthetic measurements")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed 100,000-query batch (per-query k and recall, queue orders)")
    ap.add_argument("--workload", default="mixture-1M-d100", choices=["mixture-1M-d100", "mixture-10M-d128"],
                    help="mixture-10M-d128: the learned scheduler's 10 M-point configuration (separate line)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration) and exit")
    ap.add_argument("--compare-tiles", default="",
                    help="only run the batched search of the benchmark workload with each listed tile "
                         "shape (comma-separated indexes), twice in turn, and exit (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the search path runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe_mib:
        # a plain device-to-device copy of known size: what FETCH_SIZE / WRITE_SIZE read
        # for it calibrates the counters of the search kernel
        x = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4}))
        return

    if args.workload == "mixture-10M-d128":
        workload_c5(args)
        return

    if args.compare_tiles:
        tiles = [int(t) for t in args.compare_tiles.split(",")]
        c = workloads.config(2, scale=args.scale)
        ix = pf.Index(torch.from_numpy(c["points"]).cuda(), c["budget"], seed=workloads.INDEX_SEED)
        Qd = torch.from_numpy(c["queries"]).cuda()
        ks = torch.full((len(Qd),), c["k"], dtype=torch.int32, device="cuda")
        rc = torch.full((len(Qd),), c["recall"], dtype=torch.float64, device="cuda")
        for t in tiles + tiles:
            ix.search_batch(Qd, ks, rc, c["k"], timing=True, tile=t)
            print(json.dumps({"tile": t, "name": pf.pf_tile_name(t), "search_ms": ix.last_timing().search_ms}),
                  flush=True)
        return

    log("generating workload")
    c = workloads.config(2, scale=args.scale)
    X, Q, k, recall, budget = c["points"], c["queries"], c["k"], c["recall"], c["budget"]
    n, d = X.shape
    m = len(Q)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    torch.cuda.synchronize()
    ix = pf.Index(Xd, budget, seed=workloads.INDEX_SEED)
    info = ix.info()
    del Xd
    log(f"index built: L={info.L} device build {info.build_ms:.1f} ms")

    # learned scheduler: traces of the plain method on training queries from the same
    # distribution (their own seed), features, training on the GPU (not timed)
    t0 = time.perf_counter()
    Qtr = workloads.queries_like(2, max(1, int(round(m * args.train_frac))), seed_offset=100)
    rtr = ix.search(torch.from_numpy(Qtr).to(dev), k, recall)
    st_tr = rtr.stats.cpu().numpy()
    target = np.stack([st_tr[:, 0], np.log2(1.0 + st_tr[:, 1])], 1).astype(np.float32)
    sched = pf.Scheduler(seed=1)
    losses = sched.train(ix.features(torch.from_numpy(Qtr).to(dev)), torch.from_numpy(target).to(dev),
                         epochs=20, batch=512, lr=2e-3)
    ix.set_scheduler(sched)
    train_s = time.perf_counter() - t0
    log(f"scheduler trained on {len(Qtr)} traces in {train_s:.1f} s, loss {losses[0]:.3f} -> {losses[-1]:.3f}")

    ks_d = torch.full((m,), k, dtype=torch.int32, device=dev)
    rec_d = torch.full((m,), recall, dtype=torch.float64, device=dev)
    modes = {
        "plain": lambda: ix.search(Qd, k, recall, timing=True),
        "batched_fifo": lambda: ix.search_batch(Qd, ks_d, rec_d, k, timing=True),
        "batched_fifo_both_planes": lambda: ix.search_batch(Qd, ks_d, rec_d, k, timing=True, prefilter=False),
        "learned_batched": lambda: ix.search_batch(Qd, ks_d, rec_d, k, learned=True, timing=True),
    }
    ix.search_batch(Qd, ks_d, rec_d, k, autotune=True)  # pick the batched tile shape once
    res = {}
    wanted = [p for p in args.paths.split(",") if p]
    for name in wanted:
        fn = modes[name]
        for _ in range(args.warmup):
            r = fn()
        torch.cuda.synchronize()
        search_ms, hash_ms, ranges_ms, order_ms = [], [], [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = fn()
            tm = ix.last_timing()
            search_ms.append(tm.search_ms)
            hash_ms.append(tm.hash_ms)
            ranges_ms.append(tm.ranges_ms)
            order_ms.append(tm.order_ms)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[name] = dict(r=r, ms=wall / args.steps * 1e3, search_ms=search_ms, hash_ms=hash_ms,
                         ranges_ms=ranges_ms, order_ms=order_ms, tile=tm.tile, waves=tm.waves_per_cu)
        log(f"{name}: {res[name]['ms']:.3f} ms/step, search kernel {np.mean(search_ms):.3f} ms")
    head = res[wanted[-1]]
    r = head["r"]
    ms_per_step = head["ms"]
    qps = m / (ms_per_step / 1e3)
    search_ms, hash_ms, ranges_ms, order_ms = head["search_ms"], head["hash_ms"], head["ranges_ms"], head["order_ms"]
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")
    stats = r.stats.cpu().numpy()
    ids = r.ids.cpu().numpy()
    ns = min(args.recall_sample, m)
    Xn = torch.from_numpy(ix.export(pf.PF_EXPORT_POINTS)).to(dev)
    Qn = torch.from_numpy(pf.pf_normalize(Q[:ns])).to(dev)
    truth = exact_topk_gpu(Xn, Qn, k)
    del Xn
    rec = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(ids[:ns], truth)]))

    A = algorithmic_bytes(stats, d, k, info.L, info.K)
    avg_search_ms = float(np.mean(search_ms))
    achieved = A / (avg_search_ms * 1e-3) / 1e9
    tr = traffic_entry(pf.pf_tile_name(head["tile"]))
    line = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": c["name"], "n": n, "d": d, "queries": m, "k": k, "recall_target": recall,
                   "budget_bytes": budget, "L": info.L, "K": info.K, "M": info.M, "B": 12,
                   "path": wanted[-1]},
        "paths_qps": {name: m / (v["ms"] / 1e3) for name, v in res.items()},
        "paths_search_kernel_ms": {name: float(np.mean(v["search_ms"])) for name, v in res.items()},
        "learned_vs_plain": (res["learned_batched"]["ms"] and res["plain"]["ms"] / res["learned_batched"]["ms"])
        if "plain" in res and "learned_batched" in res else None,
        "batched_tile": {"tile": head["tile"], "name": pf.pf_tile_name(head["tile"]), "waves_per_cu": head["waves"]},
        "scheduler": {"train_queries": int(len(Qtr)), "train_s": train_s, "loss_first": float(losses[0]),
                      "loss_last": float(losses[-1])},
        "recall_measured": rec,
        "recall_sample": ns,
        "build_ms": info.build_ms,
        "phase_ms": {"normalize+hash": float(np.mean(hash_ms)), "ranges": float(np.mean(ranges_ms)),
                     "queue_order": float(np.mean(order_ms)), "search": avg_search_ms},
        "stop_level_hist": np.bincount(stats[:, 0], minlength=info.K + 1).tolist(),
        "mean_counts": {"c_scan": float(stats[:, 1].mean()), "c_pass": float(stats[:, 2].mean()),
                        "c_rerank": float(stats[:, 3].mean()), "c_q8": float(stats[:, 6].mean()),
                        "c_upper": float(stats[:, 5].mean()), "c_exact": float(stats[:, 4].mean())},
        "roofline": {"kernel": "k_search", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": tr,
                     "algorithmic_bytes_per_launch": A, "avg_launch_ms": avg_search_ms,
                     "fp32_gather_bytes_per_launch": plain_gather_bytes(stats, d, k, info.L)},
        "cpu_baseline": None,
    }
    log(f"recall {rec:.4f} on {ns} queries")
    line["mixed_batch"] = None if args.no_mixed else mixed_batch(ix, dev, args)
    if not args.no_pool:
        del ix
        line["pooled_index"] = pooled_index(X, Q, k, recall, budget, dev, truth)
        line["cross_polytope_index"] = cp_index(X, Q, k, recall, budget, dev, truth)
        line["paper_synthetic"] = paper_synthetic(dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(X, Q, budget, k, recall, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
