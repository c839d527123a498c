"""Throughput of the adaptive k-NN query path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--legs LIST] [--extras]

Headline workload (`value`): mixture-10M-d128 -- n = 10,000,000 unit vectors in d = 128 drawn
from a mixture of 100,000 Gaussian clusters (centres uniform on the sphere, sigma = 0.3 per
coordinate, then normalised), memory budget 16 GiB (every resident byte charged: L = 82
tables of K = 24 bits, M = 32 sketches); a scheduler network is trained on 1,000,000 traces of
the plain method, then 100,000 further queries are answered at k = 10, recall 0.9 by the
learned-batched path (persistent kernel, work queue ordered longest-predicted-first).  One
step is the whole query path over the batch (normalisation, hashing, decision tables, prefix
ranges, queue order, search) with the queries already in HBM; W untimed and K timed steps.

Printed: one JSON line.  Beside the headline it carries, as named legs (fewer steps each):
the same batch by the plain method and by the batched FIFO and true-cost-ordered queues; the
paper's own stopping rule (Lemma 1, epsilon slack of Sec. 5.1) at epsilon 0, 0.1, 0.2, 0.5;
the same workload on an index with 3-byte table positions (more tables for the budget);
the noise-norm reading of sigma (clusters of cosine about 0.9) for the same configuration;
mixture-1M-d100 (1 M x 100, 10,000 queries, 2 GiB) under both readings; the planted instance
(1 M x 256, k = 1, recall 0.5 / 0.9 / 0.99); and the mixed batch (100,000 queries with
per-query k and recall) with its measured recall per (k, recall) against exact k-NN.
`roofline` is for the search kernel of the headline path: algorithmic bytes per launch over
its HIP-event launch time, against 8 TB/s and against the read rate of a plain streaming
kernel measured on the same device; `cpu_baseline` times the CPU oracle on a bounded sample
of the headline batch (its index is built in a child process while the GPU legs run).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1906_12211_amd as pf  # noqa: E402
import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "queries/sec at k=10, recall≥0.9: learned-batched vs plain GPU; filter HBM GB/s"
HEADLINE = "mixture-10M-d128"
SEARCH_SRC = os.path.join(ROOT, "paper_1906_12211_amd", "csrc", "k_search.hip")
DEFAULT_LEGS = "c5_paths,paper_rule,c5_pos3,c5_norm,c2,c2_norm,c3,c4"


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"search_{workload}_traffic.json")


def algorithmic_bytes(stats: np.ndarray, d: int, k: int, L: int, K: int, posb: int = 4) -> float:
    """Bytes the method must move for the queries of one launch of the search kernel:
    8 B per scanned table-local sketch, posb B (3 or 4) per table position of a passing
    entry, the 8-bit
    summary (8 + d B, or d B where the rows share one scale and carry no header: 8 + dpad
    bytes would take another 128-byte line) of every candidate bounded from it, the upper
    16-bit plane (2d B)
    of every candidate whose upper plane was read and the lower plane (2d B) of those
    whose exact inner product was needed, the query (4d) and its result (8k), and the
    two range bounds (8 B) of every table at every visited level."""
    stop = stats[:, 0].astype(np.float64)
    dpad = 4 * ((d + 3) // 4)
    hdr = 8.0 if 8 + dpad <= (dpad + 127) // 128 * 128 else 0.0
    per_q = (8.0 * stats[:, 1] + float(posb) * stats[:, 2] + (hdr + d) * stats[:, 6] + 2.0 * d * (stats[:, 5] + stats[:, 4])
             + 4.0 * d
             + 8.0 * k + 8.0 * L * (K + 1 - np.maximum(stop, 1)))
    return float(per_q.sum())


def line_model_bytes(stats: np.ndarray, d: int, k: int, L: int, K: int, line: int = 128,
                     posb: int = 4) -> float:
    """The algorithmic bytes with each passing entry's posb-byte position priced as the
    memory system moves it: a scattered read brings in the whole line (line / posb
    consecutive positions of the table) that holds it, so a query pays, per line of its
    scanned entries, one line if any of them passes -- expected (c_scan / (line / posb))
    (1 - (1 - c_pass / c_scan)^(line / posb)) lines with passes spread independently --
    instead of posb B per passing entry."""
    per = line / posb
    scan = np.maximum(stats[:, 1].astype(np.float64), 1.0)
    frac = np.clip(stats[:, 2] / scan, 0.0, 1.0)
    lines = stats[:, 1] / per * (1.0 - (1.0 - frac) ** per)
    return (algorithmic_bytes(stats, d, k, L, K, posb)
            + float((line * lines - float(posb) * stats[:, 2]).sum()))


def filter_bytes(stats: np.ndarray, posb: int = 4) -> float:
    """The filter's share of the algorithmic bytes: 8 B per scanned sketch and posb B per
    position of a passing entry."""
    return float((8.0 * stats[:, 1] + float(posb) * stats[:, 2]).sum())


def plain_gather_bytes(stats: np.ndarray, d: int, k: int, L: int, posb: int = 4) -> float:
    """The same launch counted as if every re-ranked candidate's FP32 vector were gathered
    (4d B), with the prefix-table reads (4L), sketches (8 B per scanned entry), positions
    of passing entries (posb B), the query and the result: the bytes a re-rank without the
    8-bit and 16-bit bounds would move (reported beside the roofline, not in it)."""
    per_q = (4.0 * L + 8.0 * stats[:, 1] + float(posb) * stats[:, 2] + 4.0 * d * stats[:, 3] + 4.0 * d
             + 8.0 * k)
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


def traffic_entry(workload: str, tile_name: str, L: int, pos_bytes: int, prefix_bits: int, groups: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this workload,
    if it was taken on the current search kernel source, with the tile shape, table count,
    table layout (position and prefix widths) and stopping-test groups this run launched."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if (t.get("k_search_device_sha256") != search_device_sha() or t.get("tile_name") != tile_name
            or t.get("L") != L or t.get("pos_bytes") != pos_bytes or t.get("prefix_bits") != prefix_bits
            or t.get("groups") != groups):
        return None
    return t.get("bytes_per_launch")


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return model


# ------------------------------------------------------------------ CPU baseline (child)
def cpu_worker(cfg: int, L: int, seconds: float, build_threads: int):
    """Child process: generate the headline workload, build the oracle's index at the
    GPU's table count with `build_threads` threads (while the parent times the GPU), print
    "ready", wait for "go" on stdin, then time the oracle on the first queries of the
    headline batch with every host thread (and one thread on a smaller sample)."""
    import oracle

    c = workloads.config(cfg, with_train=False)
    total = oracle.num_threads()
    oracle.set_threads(max(1, min(build_threads, total)))
    t0 = time.time()
    ix = oracle.OracleIndex(c["points"], c["budget"], seed=workloads.INDEX_SEED, L=L)
    build_s = time.time() - t0
    del c["points"]
    print(json.dumps({"ready": True, "build_s": build_s}), flush=True)
    sys.stdin.readline()
    oracle.set_threads(total)
    Q, k, recall = c["queries"], c["k"], c["recall"]
    done, el, chunk = 0, 0.0, 32
    while done < len(Q) and el < seconds:
        q = Q[done:done + chunk]
        t = time.time()
        ix.search(q, k, recall)
        el += time.time() - t
        done += len(q)
        chunk = min(1024, chunk * 2)
    oracle.set_threads(1)
    n1, el1 = 0, 0.0
    while n1 < len(Q) and el1 < seconds / 4:
        q = Q[n1:n1 + 4]
        t = time.time()
        ix.search(q, k, recall)
        el1 += time.time() - t
        n1 += len(q)
    print(json.dumps({"value": done / el, "unit": "queries/s", "cores": total, "kind": "oracle",
                      "sample": f"first {done} of {len(Q)} queries of the {c['name']} batch on the oracle's own "
                                f"index (n = {ix.n:,}, L = {L}; built in {build_s:.0f} s with {build_threads} "
                                f"threads while the GPU legs ran, not timed)",
                      "seconds": el, "single_thread_qps": n1 / el1, "single_thread_sample": n1,
                      "host_cpu": host_cpu(), "host_nproc": os.cpu_count(), "oracle_build_s": build_s}),
          flush=True)


class CpuBaseline:
    def __init__(self, cfg: int, L: int, seconds: float):
        threads = max(1, (os.cpu_count() or 4) - 4)
        self.p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(cfg),
                                   "--cpu-L", str(L), "--cpu-seconds", str(seconds),
                                   "--cpu-build-threads", str(threads)],
                                  stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
        log(f"oracle index for the CPU baseline: building in a child process ({threads} threads)")

    def result(self):
        ready = json.loads(self.p.stdout.readline() or "{}")
        if not ready.get("ready"):
            self.p.kill()
            raise RuntimeError("CPU baseline worker failed")
        log(f"oracle index was built in {ready['build_s']:.0f} s; timing the oracle")
        self.p.stdin.write("go\n")
        self.p.stdin.flush()
        out = json.loads(self.p.stdout.readline())
        self.p.wait()
        return out


# ------------------------------------------------------------------ helpers
def timed(fn, ix, warmup: int, steps: int):
    """Run fn warmup + steps times; returns (wall ms per timed step, per-phase mean ms of the
    timed steps from the library's HIP events, last result)."""
    import torch

    r = None
    for _ in range(warmup):
        r = fn()
    torch.cuda.synchronize()
    ph = {"normalize+hash": [], "ranges": [], "queue_order": [], "search": []}
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fn()
        t = ix.last_timing()
        ph["normalize+hash"].append(t.hash_ms)
        ph["ranges"].append(t.ranges_ms)
        ph["queue_order"].append(t.order_ms)
        ph["search"].append(t.search_ms)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    return wall, {k: float(np.mean(v)) for k, v in ph.items()}, r


def exact_topk_gpu(Xd, Qd, k: int, extra: int = 8):
    """Exact k-NN ids (ip desc, id asc) of normalised device rows Qd over Xd: every inner
    product in FP64 on the GPU (the FP32 library GEMM is not used: its rounding reorders
    the near-tied neighbours of large, nearly uniform point sets), the best k + extra per
    query ordered on the host."""
    import torch

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


def truth_of(ix, Q, k: int, dev):
    """Exact top-k of the normalised queries Q over the index's normalised points (exported
    once per index and kept on the device beside it)."""
    import torch

    if getattr(ix, "_bench_points", None) is None:
        ix._bench_points = torch.from_numpy(ix.export(pf.PF_EXPORT_POINTS)).to(dev)
    Qn = torch.from_numpy(pf.pf_normalize(np.ascontiguousarray(Q))).to(dev)
    return exact_topk_gpu(ix._bench_points, Qn, k)


def recall_of(ids: np.ndarray, truth: np.ndarray, k: int) -> float:
    return float(np.mean([len(set(a[:k]) & set(b[:k])) / k for a, b in zip(ids, truth)]))


def counts(st: np.ndarray) -> dict:
    return {"c_scan": float(st[:, 1].mean()), "c_pass": float(st[:, 2].mean()), "c_rerank": float(st[:, 3].mean()),
            "c_q8": float(st[:, 6].mean()), "c_upper": float(st[:, 5].mean()), "c_exact": float(st[:, 4].mean())}


def wave_busy(ix, r) -> dict:
    """How much of the persistent launch's wave-time did queries fill: W = the sum of the
    queries' wave times, S = the query waves launched, T = the launch time.  With the work
    conserved, no queue order can finish before W / S, so T / (W / S) - 1 bounds what any
    order (learned or not) could gain over this one."""
    t = ix.last_timing()
    W = float(r.wave_us.cpu().numpy().astype(np.float64).sum())
    S, T = float(t.slots), float(t.search_ms) * 1e3
    frac = W / (S * T) if S > 0 and T > 0 else float("nan")
    return {"slots": int(t.slots), "busy_fraction": frac, "order_gain_bound": 1.0 / frac - 1.0}


def spearman(a, b) -> float:
    rk = lambda v: np.argsort(np.argsort(v, kind="stable"), kind="stable")
    return float(np.corrcoef(rk(a), rk(b))[0, 1])


def train_scheduler(ix, Qtr, k, recall, dev, seed, epochs, batch, chunk=100_000):
    """Traces of the plain method on the training queries (in chunks of `chunk`, so that the
    index's call buffers stay at the evaluation batch's size), then training on the GPU."""
    import torch

    t0 = time.perf_counter()
    st, feats = [], []
    for s in range(0, len(Qtr), chunk):
        q = torch.from_numpy(Qtr[s:s + chunk]).to(dev)
        st.append(ix.search(q, k, recall).stats.cpu().numpy())
        feats.append(ix.features(q, k=k, recall=recall))
    st = np.concatenate(st)
    feat = torch.cat(feats)
    trace_s = time.perf_counter() - t0
    target = np.stack([st[:, 0], np.log2(1.0 + st[:, 1])], 1).astype(np.float32)
    sched = pf.Scheduler(seed=seed)
    t0 = time.perf_counter()
    losses = sched.train(feat, torch.from_numpy(target).to(dev), epochs=epochs, batch=batch, lr=2e-3)
    train_s = time.perf_counter() - t0
    ix.set_scheduler(sched)
    del feat
    return sched, {"traces": int(len(Qtr)), "trace_s": trace_s, "train_s": train_s,
                   "loss_first": float(losses[0]), "loss_last": float(losses[-1])}


def order_paths(ix, Qd, k, recall, sched, dev, steps, warmup=1):
    """The batch under the plain method (static slots) and the batched queue in FIFO,
    learned and true-cost (longest scanned first; a bound no predictor can beat) order."""
    import torch

    m = Qd.shape[0]
    ks = torch.full((m,), k, dtype=torch.int32, device=dev)
    rc = torch.full((m,), recall, dtype=torch.float64, device=dev)
    base = ix.search_batch(Qd, ks, rc, k, timing=True)
    bst = base.stats.cpu().numpy()
    busy = wave_busy(ix, base)
    lpt = torch.from_numpy(np.argsort(-bst[:, 1], kind="stable").astype(np.int32)).to(dev)
    modes = {
        "plain": lambda: ix.search(Qd, k, recall, timing=True),
        "batched_fifo": lambda: ix.search_batch(Qd, ks, rc, k, timing=True),
        "learned_batched": lambda: ix.search_batch(Qd, ks, rc, k, learned=True, timing=True),
        "true_cost_lpt": lambda: ix.search_batch(Qd, ks, rc, k, order=lpt, timing=True),
    }
    out = {}
    for name, fn in modes.items():
        wall, ph, r = timed(fn, ix, warmup, steps)
        out[name] = {"ms_per_step": wall, "qps": m / (wall / 1e3), "search_kernel_ms": ph["search"],
                     "phase_ms": ph, "ids_equal_fifo": bool(torch.equal(r.ids, base.ids))}
        log(f"  {name}: {wall:.2f} ms/step, phases " + ", ".join(f"{a} {b:.2f}" for a, b in ph.items()))
    pred = sched.predict(ix.features(Qd, k=k, recall=recall)).cpu().numpy()[:, 1]
    cost = np.log2(1.0 + bst[:, 1])
    extra = {"learned_vs_plain": out["plain"]["ms_per_step"] / out["learned_batched"]["ms_per_step"],
             "fifo_wave_busy": busy,
             "learned_vs_fifo": out["batched_fifo"]["search_kernel_ms"] / out["learned_batched"]["search_kernel_ms"],
             "true_lpt_vs_fifo": out["batched_fifo"]["search_kernel_ms"] / out["true_cost_lpt"]["search_kernel_ms"],
             "spearman_pred_vs_true_cost": spearman(pred, cost),
             "cost_spread_log2_scan": {p: float(np.percentile(cost, q)) for p, q in
                                       (("p1", 1), ("p10", 10), ("p50", 50), ("p90", 90), ("p99", 99))},
             "stop_level_hist": np.bincount(bst[:, 0], minlength=ix.K + 1).tolist(),
             "mean_counts": counts(bst)}
    return out, extra, base


WORKLOADS = {"mixture-10M-d128": 5, "mixture-1M-d100": 2}


# ------------------------------------------------------------------ headline
def headline(args, dev):
    """The learned-batched path on configuration 5 (or, for counter runs, configuration 2)."""
    import torch

    cfg = WORKLOADS[args.workload]
    log(f"generating {args.workload}")
    t0 = time.perf_counter()
    c = workloads.config(cfg)
    Qtr = c.pop("train_queries") if cfg == 5 else workloads.queries_like(2, 20_000, seed_offset=100)
    if args.train_queries:
        Qtr = Qtr[:args.train_queries]
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    X, Q = c.pop("points"), c["queries"]
    n, d = X.shape
    m, k, recall = len(Q), c["k"], c["recall"]
    ix = pf.Index(torch.from_numpy(X).to(dev), c["budget"], seed=workloads.INDEX_SEED, pos_bytes=args.pos_bytes,
                  prefix_bits=args.prefix_bits)
    del X
    info = ix.info()
    log(f"index built: L={info.L}, {info.bytes_device / 2**30:.2f} GiB on the device "
        f"(budget {c['budget'] / 2**30:.0f} GiB), device build {info.build_ms:.0f} ms")
    sched, sch = train_scheduler(ix, Qtr, k, recall, dev, seed=cfg, epochs=5 if cfg == 5 else 20,
                                 batch=1024 if cfg == 5 else 512)
    del Qtr
    log(f"scheduler: {sch['traces']} traces in {sch['trace_s']:.1f} s, trained in {sch['train_s']:.1f} s, "
        f"loss {sch['loss_first']:.3f} -> {sch['loss_last']:.3f}")
    Qd = torch.from_numpy(Q).to(dev)
    ks = torch.full((m,), k, dtype=torch.int32, device=dev)
    rc = torch.full((m,), recall, dtype=torch.float64, device=dev)
    ix.search_batch(Qd, ks, rc, k, autotune=True)
    fn = lambda: ix.search_batch(Qd, ks, rc, k, learned=True, timing=True)
    # the headline: W untimed and K timed steps of the learned-batched path
    wall, ph, r = timed(fn, ix, args.warmup, args.steps)
    qps = m / (wall / 1e3)
    log(f"learned-batched: {wall:.1f} ms/step ({qps:.0f} queries/s), search kernel {ph['search']:.1f} ms")
    tile = ix.last_timing().tile
    waves = ix.last_timing().waves_per_cu
    busy = wave_busy(ix, r)
    stats = r.stats.cpu().numpy()
    ids = r.ids.cpu().numpy()
    ns = min(args.recall_sample, m)
    truth = truth_of(ix, Q[:ns], k, dev)
    rec = recall_of(ids[:ns], truth, k)
    log(f"recall {rec:.4f} on {ns} queries")
    A = algorithmic_bytes(stats, d, k, info.L, info.K, info.pos_bytes)
    F = filter_bytes(stats, info.pos_bytes)
    kms = ph["search"]
    achieved = A / (kms * 1e-3) / 1e9
    read_gbs = pf.pf_read_bandwidth(4 << 30, 5)
    log(f"read-only streaming kernel: {read_gbs:.0f} GB/s")
    rr = pf.pf_random_read_rate(4 << 30, 3)
    log(f"scattered 4-byte reads: {rr / 1e9:.1f} G/s, each the streaming bandwidth of {read_gbs * 1e9 / rr:.0f} bytes")
    tname = pf.pf_tile_name(tile)
    line = {
        "metric": METRIC, "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "queries": m, "k": k, "recall_target": recall,
                   "groups": int(ix.last_timing().groups),
                   "budget_bytes": c["budget"], "L": info.L, "K": info.K, "M": info.M, "B": 12,
                   "pos_bytes": info.pos_bytes, "prefix_bits": info.P,
                   "sigma_reading": "per coordinate", "train_traces": sch["traces"], "path": "learned_batched"},
        "recall_measured": rec, "recall_sample": ns,
        "bytes_device": info.bytes_device, "build_ms": info.build_ms,
        "phase_ms": ph,
        "batched_tile": {"tile": tile, "name": tname, "waves_per_cu": waves},
        "wave_busy": busy,
        "scheduler": sch,
        "stop_level_hist": np.bincount(stats[:, 0], minlength=info.K + 1).tolist(),
        "mean_counts": counts(stats),
        "filter_gbs": F / (kms * 1e-3) / 1e9,
        "filter_share_of_bytes": F / A,
        "roofline": {"kernel": "k_search", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_entry(args.workload, tname, info.L, info.pos_bytes, info.P,
                                             int(ix.last_timing().groups)),
                     "measured_read_gbs": read_gbs, "frac_of_measured_read": achieved / read_gbs,
                     "algorithmic_bytes_per_launch": A, "avg_launch_ms": kms, "queries_per_launch": m,
                     "fp32_gather_bytes_per_launch": plain_gather_bytes(stats, d, k, info.L, info.pos_bytes),
                     "line_model_bytes_per_launch": line_model_bytes(stats, d, k, info.L, info.K,
                                                                     posb=info.pos_bytes),
                     "scattered_4b_reads_per_s": rr, "bytes_per_scattered_read": read_gbs * 1e9 / rr},
        "cpu_baseline": None,
    }
    tr = line["roofline"]["traffic"]
    if tr:
        line["roofline"]["traffic_gbs"] = tr / (kms * 1e-3) / 1e9
        # algorithmic bytes over the bytes the counters saw move (the cache-line waste)
        line["roofline"]["useful_over_moved"] = A / tr
    legs = set(args.legs.split(",")) if args.legs else set()
    steps2 = max(1, min(3, args.steps))
    if "c5_paths" in legs:
        log("headline batch under the other query paths")
        paths, extra, _ = order_paths(ix, Qd, k, recall, sched, dev, steps2)
        line["paths"] = paths
        line.update({"learned_vs_plain": paths["plain"]["ms_per_step"] / wall,
                     "learned_vs_fifo": paths["batched_fifo"]["search_kernel_ms"] / kms,
                     "true_lpt_vs_fifo": extra["true_lpt_vs_fifo"],
                     "spearman_pred_vs_true_cost": extra["spearman_pred_vs_true_cost"],
                     "cost_spread_log2_scan": extra["cost_spread_log2_scan"]})
    if "paper_rule" in legs:
        line["paper_rule"] = paper_rule(ix, Qd, Q[:ns], truth, k, recall, dev)
    del ix, sched, Qd
    torch.cuda.empty_cache()
    return line


def paper_rule(ix, Qd, Qs, truth, k, recall, dev):
    """The paper's own method on the headline batch: Lemma 1's bound (1 - p^i)^L <= delta,
    tested once all repetitions of a round are inspected (Sec. 4.1), with the filter
    threshold (1 + eps) 64 theta_k / pi of Sec. 5.1, eps from the sweep {0, 0.1, 0.2, 0.5};
    the smallest eps whose measured recall reaches the target is the paper's operating
    point."""
    import torch

    m = Qd.shape[0]
    ks = torch.full((m,), k, dtype=torch.int32, device=dev)
    rc = torch.full((m,), recall, dtype=torch.float64, device=dev)
    out = {"rule": "PF_RULE_EXACT (Lemma 1, filter not accounted), tested once per round (Sec. 4.1)", "sweep": {}}
    chosen = None
    for eps in (0.0, 0.1, 0.2, 0.5):
        fn = lambda: ix.search_batch(Qd, ks, rc, k, rule=pf.PF_RULE_EXACT, eps=eps, groups=1, learned=True,
                                     timing=True)
        wall, ph, r = timed(fn, ix, 0, 1)
        rec = recall_of(r.ids.cpu().numpy()[:len(truth)], truth, k)
        st = r.stats.cpu().numpy()
        out["sweep"][str(eps)] = {"qps": m / (wall / 1e3), "ms_per_step": wall, "search_kernel_ms": ph["search"],
                                  "recall_measured": rec, "mean_stop_level": float(st[:, 0].mean()),
                                  "mean_c_scan": float(st[:, 1].mean())}
        log(f"  paper rule eps {eps}: {m / (wall / 1e3):.0f} queries/s, kernel {ph['search']:.1f} ms, recall {rec:.4f}")
        if chosen is None and rec >= recall:
            chosen = eps
            break  # the sweep stops at the smallest epsilon that reaches the target
    out["eps_reaching_target"] = chosen
    if chosen is not None:
        out["at_target"] = dict(out["sweep"][str(chosen)], eps=chosen)
    return out


# ------------------------------------------------------------------ legs
def leg_positions3(args, dev):
    """The headline workload on an index whose table positions are stored in 3 bytes
    (pos_bytes = 3): the budget buys more tables, each passing entry's position read moves
    a line of 42 positions instead of 32, and every position read is an unaligned load;
    batched FIFO order (learned order = FIFO on this batch)."""
    import torch

    c = workloads.config(5, with_train=False)
    X, Q = c.pop("points"), c["queries"]
    m, k, recall = len(Q), c["k"], c["recall"]
    ix = pf.Index(torch.from_numpy(X).to(dev), c["budget"], seed=workloads.INDEX_SEED, pos_bytes=3)
    del X
    info = ix.info()
    Qd = torch.from_numpy(Q).to(dev)
    ks = torch.full((m,), k, dtype=torch.int32, device=dev)
    rc = torch.full((m,), recall, dtype=torch.float64, device=dev)
    ix.search_batch(Qd, ks, rc, k, autotune=True)
    wall, ph, r = timed(lambda: ix.search_batch(Qd, ks, rc, k, timing=True), ix, 1, max(1, min(3, args.steps)))
    st = r.stats.cpu().numpy()
    ns = min(1000, m)
    rec = recall_of(r.ids.cpu().numpy()[:ns], truth_of(ix, Q[:ns], k, dev), k)
    t = ix.last_timing()
    out = {"workload": c["name"], "pos_bytes": info.pos_bytes, "prefix_bits": info.P, "L": info.L,
           "bytes_device": info.bytes_device, "qps": m / (wall / 1e3), "ms_per_step": wall,
           "search_kernel_ms": ph["search"], "phase_ms": ph, "recall_measured": rec, "recall_sample": ns,
           "batched_tile": {"tile": t.tile, "name": pf.pf_tile_name(t.tile), "waves_per_cu": t.waves_per_cu},
           "algorithmic_gbs": algorithmic_bytes(st, info.d, k, info.L, info.K, info.pos_bytes) / (ph["search"] * 1e-3) / 1e9,
           "stop_level_hist": np.bincount(st[:, 0], minlength=info.K + 1).tolist(), "mean_counts": counts(st)}
    log(f"3-byte positions: L={info.L}, {out['qps']:.0f} queries/s (batched FIFO), search kernel "
        f"{ph['search']:.1f} ms, recall {rec:.4f}")
    del ix, Qd
    torch.cuda.empty_cache()
    return out


def leg_mixture(cfg, sigma_mode, args, dev, ntrain):
    """Configuration 2 or 5 under a sigma reading: learned-batched, FIFO, plain and true-cost
    order on its own index, with the scheduler trained on `ntrain` traces."""
    import torch

    t0 = time.perf_counter()
    c = workloads.config(cfg, sigma_mode=sigma_mode, with_train=False)
    Qtr = workloads.queries_like(cfg, ntrain, seed_offset=100, sigma_mode=sigma_mode)
    X, Q = c.pop("points"), c["queries"]
    n, d = X.shape
    m, k, recall = len(Q), c["k"], c["recall"]
    ix = pf.Index(torch.from_numpy(X).to(dev), c["budget"], seed=workloads.INDEX_SEED)
    del X
    info = ix.info()
    log(f"{c['name']} ({sigma_mode}): L={info.L}, generated and built in {time.perf_counter() - t0:.1f} s")
    sched, sch = train_scheduler(ix, Qtr, k, recall, dev, seed=cfg, epochs=20 if ntrain <= 50_000 else 5,
                                 batch=512 if ntrain <= 50_000 else 1024)
    Qd = torch.from_numpy(Q).to(dev)
    m_ = Qd.shape[0]
    ks = torch.full((m_,), k, dtype=torch.int32, device=dev)
    rc = torch.full((m_,), recall, dtype=torch.float64, device=dev)
    ix.search_batch(Qd, ks, rc, k, autotune=True)
    paths, extra, base = order_paths(ix, Qd, k, recall, sched, dev, max(1, min(3, args.steps)))
    ns = min(1000, m)
    truth = truth_of(ix, Q[:ns], k, dev)
    rec = recall_of(base.ids.cpu().numpy()[:ns], truth, k)
    st = base.stats.cpu().numpy()
    t = ix.last_timing()
    out = {"workload": c["name"], "sigma_reading": "per coordinate" if sigma_mode == "coord" else "noise norm",
           "n": n, "d": d, "queries": m, "L": info.L, "bytes_device": info.bytes_device, "paths": paths,
           "scheduler": sch, "recall_measured": rec, "recall_sample": ns,
           "batched_tile": {"tile": t.tile, "name": pf.pf_tile_name(t.tile), "waves_per_cu": t.waves_per_cu},
           "algorithmic_gbs": algorithmic_bytes(st, d, k, info.L, info.K, info.pos_bytes)
           / (paths["learned_batched"]["search_kernel_ms"] * 1e-3) / 1e9}
    out.update(extra)
    log(f"{c['name']} ({sigma_mode}): recall {rec:.4f}; learned/fifo {extra['learned_vs_fifo']:.3f}, "
        f"true-LPT/fifo {extra['true_lpt_vs_fifo']:.3f}, rho {extra['spearman_pred_vs_true_cost']:.2f}")
    return out, ix, sched


def leg_planted(args, dev):
    """Configuration 3: 1 M uniform unit vectors in d = 256 with planted neighbours (100 groups
    of 100 queries, 2,000 decoys near 60 degrees per group, one neighbour at 30 degrees per
    query), 2 GiB, k = 1: per recall target the planted-neighbour hit rate, stop levels and
    the batched search's rate."""
    import torch

    c = workloads.config(3)
    X, Q, pid = c["points"], c["queries"], c["planted"]
    ix = pf.Index(torch.from_numpy(X).to(dev), c["budget"], seed=workloads.INDEX_SEED)
    del X
    info = ix.info()
    m = len(Q)
    Qd = torch.from_numpy(Q).to(dev)
    ks = torch.ones((m,), dtype=torch.int32, device=dev)
    out = {"workload": c["name"], "n": info.n, "d": info.d, "queries": m, "k": 1, "L": info.L,
           "bytes_device": info.bytes_device, "targets": {}}
    for rec in (0.5, 0.9, 0.99):
        rc = torch.full((m,), rec, dtype=torch.float64, device=dev)
        ix.search_batch(Qd, ks, rc, 1, autotune=True)
        wall, ph, r = timed(lambda: ix.search_batch(Qd, ks, rc, 1, timing=True), ix, 1, max(1, min(3, args.steps)))
        st = r.stats.cpu().numpy()
        hit = float(np.mean(r.ids.cpu().numpy()[:, 0] == pid))
        out["targets"][str(rec)] = {"qps": m / (wall / 1e3), "ms_per_step": wall, "search_kernel_ms": ph["search"],
                                    "planted_found": hit, "mean_stop_level": float(st[:, 0].mean()),
                                    "stop_level_hist": np.bincount(st[:, 0], minlength=info.K + 1).tolist(),
                                    "mean_counts": counts(st)}
        log(f"planted, recall {rec}: {m / (wall / 1e3):.0f} queries/s, planted found {hit:.4f}, "
            f"mean stop level {st[:, 0].mean():.2f}")
    del ix
    torch.cuda.empty_cache()
    return out


def leg_mixed(ix, args, dev):
    """Configuration 4 on mixture-1M-d100's index: 100,000 queries, half from the mixture and
    half uniform, per-query k in {1, 10, 100} and recall in {0.5, 0.9, 0.99}; the queue in
    FIFO, learned (network trained on traces of another batch of the same distribution),
    true-cost and shortest-predicted-first order; measured recall per (k, recall) against
    exact k-NN on a sample."""
    import torch

    m = 100_000
    Q, ks, rec = workloads.mixed_queries(m)
    Qt, kst, rect = workloads.mixed_queries(200_000, seed_offset=100)
    kmax = 100
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Qd, ksd, recd = to(Q), to(ks), to(rec)
    t0 = time.perf_counter()
    st, feats = [], []
    for s in range(0, len(Qt), m):
        q, kk, rr = to(Qt[s:s + m]), to(kst[s:s + m]), to(rect[s:s + m])
        st.append(ix.search_batch(q, kk, rr, kmax).stats.cpu().numpy())
        feats.append(ix.features(q, kk, rr))
    st = np.concatenate(st)
    target = np.stack([st[:, 0], np.log2(1.0 + st[:, 1])], 1).astype(np.float32)
    sched = pf.Scheduler(seed=2)
    losses = sched.train(torch.cat(feats), to(target), epochs=20, batch=512, lr=2e-3)
    ix.set_scheduler(sched)
    train_s = time.perf_counter() - t0
    ix.search_batch(Qd, ksd, recd, kmax, autotune=True)
    base = ix.search_batch(Qd, ksd, recd, kmax)
    bst = base.stats.cpu().numpy()
    cost = np.log2(1.0 + bst[:, 1])
    pred = sched.predict(ix.features(Qd, ksd, recd)).cpu().numpy()[:, 1]
    orders = {"fifo": dict(), "learned": dict(learned=True),
              "true_cost_lpt": dict(order=to(np.argsort(-cost, kind="stable").astype(np.int32))),
              "shortest_predicted_first": dict(order=to(np.argsort(pred, kind="stable").astype(np.int32)))}
    out = {}
    for name, kw in orders.items():
        wall, ph, r = timed(lambda: ix.search_batch(Qd, ksd, recd, kmax, timing=True, **kw), ix, 1,
                            max(1, min(3, args.steps)))
        out[name] = {"ms_per_step": wall, "qps": m / (wall / 1e3), "search_kernel_ms": ph["search"],
                     "ids_equal_fifo": bool(torch.equal(r.ids, base.ids))}
        log(f"mixed batch {name}: {wall:.2f} ms/step, search kernel {ph['search']:.2f} ms")
    # measured recall per (k, recall) against exact k-NN, on a stratified sample
    ids = base.ids.cpu().numpy()
    rng = np.random.default_rng(44)
    per = {}
    for k in (1, 10, 100):
        for rc in (0.5, 0.9, 0.99):
            sel = np.flatnonzero((ks == k) & (rec == rc))
            sel = np.sort(rng.choice(sel, size=min(300, len(sel)), replace=False))
            truth = truth_of(ix, Q[sel], k, dev)
            per[f"k{k}_r{rc}"] = {"recall_measured": recall_of(ids[sel], truth, k), "sample": int(len(sel)),
                                  "mean_stop_level": float(bst[sel, 0].mean())}
    worst = min(v["recall_measured"] - float(key.split("_r")[1]) for key, v in per.items())
    log("mixed batch recall per (k, recall): " + ", ".join(f"{a} {v['recall_measured']:.3f}" for a, v in per.items()))
    return {"workload": "mixed-100k-on-1M-d100", "queries": m, "kmax": kmax, "orders": out,
            "learned_vs_fifo": out["fifo"]["search_kernel_ms"] / out["learned"]["search_kernel_ms"],
            "true_lpt_vs_fifo": out["fifo"]["search_kernel_ms"] / out["true_cost_lpt"]["search_kernel_ms"],
            "spearman_pred_vs_true_cost": spearman(pred, cost),
            "scheduler": {"train_queries": int(len(Qt)), "train_s": train_s, "loss_first": float(losses[0]),
                          "loss_last": float(losses[-1])},
            "recall_by_k_and_target": per, "min_recall_margin": worst,
            "mean_counts": counts(bst),
            "cost_spread_log2_scan": {p: float(np.percentile(cost, q)) for p, q in
                                      (("p10", 10), ("p50", 50), ("p90", 90), ("max", 100))}}


def leg_extras(dev, k, recall):
    """Index options on mixture-1M-d100 (pooling, FHT cross-polytope codes) and the paper's
    synthetic set."""
    import torch

    c = workloads.config(2, with_train=False)
    X, Q, budget = c["points"], c["queries"], c["budget"]
    out = {}
    for name, kw in (("pooled_index", dict(pool=3072)), ("cross_polytope_index", dict(family=pf.PF_FAMILY_FHTCP))):
        ix = pf.Index(torch.from_numpy(X).to(dev), budget, seed=workloads.INDEX_SEED, **kw)
        info = ix.info()
        m = len(Q)
        Qd = torch.from_numpy(Q).to(dev)
        ks = torch.full((m,), k, dtype=torch.int32, device=dev)
        rc = torch.full((m,), recall, dtype=torch.float64, device=dev)
        truth = truth_of(ix, Q[:1000], k, dev)
        ix.search_batch(Qd, ks, rc, k, autotune=True)
        res = {"L": info.L, "build_ms": info.build_ms}
        rules = [("default_rule", pf.PF_RULE_FILTER)] + ([("algorithm3_rule", pf.PF_RULE_POOL)] if "pool" in kw else [])
        for rname, rule in rules:
            wall, ph, r = timed(lambda: ix.search_batch(Qd, ks, rc, k, rule=rule, timing=True), ix, 1, 3)
            res[rname] = {"qps": m / (wall / 1e3), "search_kernel_ms": ph["search"],
                          "normalize+hash_ms": ph["normalize+hash"],
                          "recall_measured": recall_of(r.ids.cpu().numpy()[:1000], truth, k)}
            log(f"{name} {rname}: kernel {ph['search']:.2f} ms, recall {res[rname]['recall_measured']:.4f}")
        out[name] = res
        del ix
        torch.cuda.empty_cache()
    X, Q = workloads.paper_synthetic(1_000_000, 100, 1000, 78)
    ix = pf.Index(torch.from_numpy(X).to(dev), 2 << 30, seed=workloads.INDEX_SEED)
    m = len(Q)
    Qd = torch.from_numpy(Q).to(dev)
    ks = torch.ones((m,), dtype=torch.int32, device=dev)
    syn = {"workload": "paper-synthetic-1M-3x100", "L": ix.L, "targets": {}}
    for rec in (0.5, 0.9, 0.99):
        rc = torch.full((m,), rec, dtype=torch.float64, device=dev)
        ix.search_batch(Qd, ks, rc, 1, autotune=True)
        wall, ph, r = timed(lambda: ix.search_batch(Qd, ks, rc, 1, timing=True), ix, 1, 3)
        st = r.stats.cpu().numpy()
        syn["targets"][str(rec)] = {"x_n_found": float(np.mean(r.ids.cpu().numpy()[:, 0] == len(X) - 1)),
                                    "mean_stop_level": float(st[:, 0].mean()), "search_kernel_ms": ph["search"]}
    out["paper_synthetic"] = syn
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--recall-sample", type=int, default=1000)
    ap.add_argument("--legs", default=DEFAULT_LEGS,
                    help="secondary measurements (comma separated; '' for none): " + DEFAULT_LEGS)
    ap.add_argument("--extras", action="store_true",
                    help="also the pooled and cross-polytope indexes and the paper's synthetic set")
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(WORKLOADS),
                    help="headline workload (mixture-1M-d100: for counter runs of configuration 2)")
    ap.add_argument("--pos-bytes", type=int, default=0, choices=(0, 3, 4),
                    help="table position width of the headline index (0: the library's default)")
    ap.add_argument("--prefix-bits", type=int, default=0,
                    help="prefix table width of the headline index (0: the library's default)")
    ap.add_argument("--train-queries", type=int, default=0,
                    help="train the scheduler on only this many traces (counter runs; 0 = the configuration's)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration) and exit")
    ap.add_argument("--random-read-probe", action="store_true",
                    help="only run the scattered 4-byte read probe (for counter calibration) and exit")
    ap.add_argument("--cpu-worker", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-L", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-build-threads", type=int, default=12, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker, args.cpu_L, args.cpu_seconds, args.cpu_build_threads)
        return
    if args.gpus != 1:
        print(f"bench.py: the search path runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
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
    if args.random_read_probe:
        # scattered 4-byte reads (plain and non-temporal, one warm-up and one timed launch
        # each): what FETCH_SIZE reads per load for them prices the search kernel's reads of
        # passing entries' positions
        rate = pf.pf_random_read_rate(4 << 30, 1)
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        print(json.dumps({"random_read_loads_per_launch": cus * 64 * 256 * 64, "loads_per_s": rate}))
        return

    dev = torch.device("cuda:0")
    t_start = time.perf_counter()
    cpu = None
    if not args.no_cpu_baseline:
        cfg = WORKLOADS[args.workload]
        n, d = (10_000_000, 128) if cfg == 5 else (1_000_000, 100)
        L, _ = pf.pf_plan_index(n, d, 16 << 30 if cfg == 5 else 2 << 30, pos_bytes=args.pos_bytes,
                                prefix_bits=args.prefix_bits)
        cpu = CpuBaseline(cfg, L, args.cpu_seconds)
    line = headline(args, dev)
    legs = set(args.legs.split(",")) if args.legs else set()
    if args.workload != HEADLINE:
        legs -= {"c2", "c5_norm", "c5_pos3"}
    if "c5_pos3" in legs:
        line["c5_pos3"] = leg_positions3(args, dev)
    if "c5_norm" in legs:
        out, ix, _ = leg_mixture(5, "norm", args, dev, 200_000)
        line["c5_noise_norm"] = out
        del ix
        torch.cuda.empty_cache()
    c2ix = None
    if "c2" in legs:
        line["c2"], c2ix, _ = leg_mixture(2, "coord", args, dev, 20_000)
    if "c4" in legs:
        if c2ix is None:
            c2 = workloads.config(2, with_train=False)
            c2ix = pf.Index(torch.from_numpy(c2["points"]).to(dev), c2["budget"], seed=workloads.INDEX_SEED)
        line["c4_mixed"] = leg_mixed(c2ix, args, dev)
    del c2ix
    torch.cuda.empty_cache()
    if "c2_norm" in legs:
        out, ix, _ = leg_mixture(2, "norm", args, dev, 20_000)
        line["c2_noise_norm"] = out
        del ix
        torch.cuda.empty_cache()
    if "c3" in legs:
        line["c3_planted"] = leg_planted(args, dev)
    if args.extras:
        line["extras"] = leg_extras(dev, 10, 0.9)
    if cpu is not None:
        line["cpu_baseline"] = cpu.result()
        line["gpu_vs_cpu_oracle"] = line["value"] / line["cpu_baseline"]["value"]
    line["bench_wall_s"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
