"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws input vectors only (numpy PCG64); it holds none of the search
method's arithmetic.  Every workload is a plain function of its seeds.

Workloads (all FP32, rows are points):
  gaussian_unit   i.i.d. N(0, I_d) rows, L2-normalised (uniform on the sphere).
  mixture         clustered rows: centres uniform on the sphere, x = c + sigma * g with
                  g ~ N(0, I_d) (sigma per coordinate, the literal reading), then
                  normalised.  sigma_mode="norm" instead scales the noise to norm sigma
                  (x = c + sigma * g / sqrt(d)), which makes clusters tight.
  planted         uniform background, groups of queries, each with one neighbour at
                  exactly 30 degrees and shared decoys near 60 degrees.
  paper_synthetic the 3d-dimensional instance of the paper's evaluation (Sec. 5,
                  "Synthetic Dataset"): x_i = (0, y_i, z_i), x_n = (v, w, 0),
                  q_i = (v, 0, r_i); x_n is the nearest neighbour of every query.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

DATA_SEED = 1000
QUERY_SEED = 2000
CENTER_SEED = 3000
INDEX_SEED = 42


def _unit_rows(a: np.ndarray) -> np.ndarray:
    a = a.astype(np.float64, copy=False)
    nrm = np.linalg.norm(a, axis=1, keepdims=True)
    return (a / nrm).astype(np.float32)


_CHUNK = 1 << 17


def _chunked(n: int, d: int, seed: int, fn) -> np.ndarray:
    """Rows [s, s + _CHUNK) come from their own PCG64 stream (child s / _CHUNK of the seed's
    SeedSequence), so that chunks are drawn in parallel threads and the result does not
    depend on the thread count."""
    out = np.empty((n, d), dtype=np.float32)
    starts = list(range(0, n, _CHUNK))
    kids = np.random.SeedSequence(seed).spawn(len(starts))

    def one(i):
        s = starts[i]
        e = min(n, s + _CHUNK)
        out[s:e] = fn(np.random.default_rng(kids[i]), e - s)

    if len(starts) <= 1:
        for i in range(len(starts)):
            one(i)
    else:
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1, len(starts))) as ex:
            list(ex.map(one, range(len(starts))))
    return out


def gaussian_unit(n: int, d: int, seed: int) -> np.ndarray:
    return _chunked(n, d, seed, lambda r, c: _unit_rows(r.standard_normal((c, d), dtype=np.float32)))


def mixture_centers(n_clusters: int, d: int, seed: int) -> np.ndarray:
    return gaussian_unit(n_clusters, d, seed)


def mixture(n: int, d: int, centers: np.ndarray, sigma: float, seed: int,
            sigma_mode: str = "coord") -> np.ndarray:
    scale = sigma if sigma_mode == "coord" else sigma / np.sqrt(d)

    def fn(r, c):
        lab = r.integers(0, centers.shape[0], size=c)
        g = r.standard_normal((c, d), dtype=np.float32)
        return _unit_rows(centers[lab] + np.float32(scale) * g)

    return _chunked(n, d, seed, fn)


def planted(n: int, d: int, n_groups: int, per_group: int, decoys: int, seed: int):
    """Uniform background with planted structure.

    Group g has a unit vector v_g; its queries are q = (v_g + r)/|v_g + r| with r a unit
    vector orthogonal to v_g; decoys D = (v_g + u)/|.| with u a random unit vector
    orthogonal to v_g (about 60 degrees from the group's queries); each query gets one
    planted neighbour at exactly 30 degrees.  Returns (points, queries, planted_ids).
    """
    rng = np.random.default_rng(seed)
    X = gaussian_unit(n, d, seed + 1)
    m = n_groups * per_group
    Q = np.empty((m, d), dtype=np.float32)
    ids = rng.permutation(n)[: n_groups * (decoys + per_group)]
    plant_ids = np.empty(m, dtype=np.int64)
    t = 0
    for g in range(n_groups):
        v = rng.standard_normal(d)
        v /= np.linalg.norm(v)

        def orth(a):
            a = a - np.outer(a @ v, v) if a.ndim == 2 else a - (a @ v) * v
            return a / np.linalg.norm(a, axis=-1, keepdims=True)

        dec_ids = ids[t: t + decoys]
        t += decoys
        u = orth(rng.standard_normal((decoys, d)))
        X[dec_ids] = _unit_rows(v[None, :] + u)
        for s in range(per_group):
            r = orth(rng.standard_normal(d))
            q = (v + r) / np.linalg.norm(v + r)
            w = rng.standard_normal(d)
            w = w - (w @ q) * q
            w /= np.linalg.norm(w)
            x = np.cos(np.pi / 6) * q + np.sin(np.pi / 6) * w
            pid = ids[t]
            t += 1
            X[pid] = x.astype(np.float32)
            Q[g * per_group + s] = q.astype(np.float32)
            plant_ids[g * per_group + s] = pid
    return X, Q, plant_ids


def paper_synthetic(n: int, d: int, m: int, seed: int):
    """Returns (points (n x 3d), queries (m x 3d)); row n-1 is every query's neighbour."""
    rng = np.random.default_rng(seed)
    s = np.float32(np.sqrt(1.0 / (2 * d)))
    X = np.zeros((n, 3 * d), dtype=np.float32)
    for a in range(0, n - 1, 1 << 18):
        b = min(n - 1, a + (1 << 18))
        X[a:b, d: 2 * d] = rng.standard_normal((b - a, d), dtype=np.float32) * s
        X[a:b, 2 * d:] = rng.standard_normal((b - a, d), dtype=np.float32) * s
    v = rng.standard_normal(d).astype(np.float32) * s
    w = rng.standard_normal(d).astype(np.float32) * s
    X[n - 1, :d] = v
    X[n - 1, d: 2 * d] = w
    Q = np.zeros((m, 3 * d), dtype=np.float32)
    Q[:, :d] = v
    r = rng.standard_normal((m, d))
    r = r / np.linalg.norm(r, axis=1, keepdims=True) * np.sqrt(0.5)
    Q[:, 2 * d:] = r.astype(np.float32)
    return X, Q


# ------------------------------------------------------------------ the five configurations
def config(c: int, scale: float = 1.0, sigma_mode: str = "coord", query_seed_offset: int = 0,
           with_train: bool = True):
    """Points, queries and parameters of configuration c (1..5).

    scale < 1 shrinks n and the query count (for quick tests); sizes otherwise as
    stated in the workload descriptions.  with_train=False leaves out configuration 5's
    1,000,000 training queries.
    """
    def sz(v):
        return max(1, int(round(v * scale)))

    if c == 1:
        n, d, m = sz(10_000), 64, sz(1_000)
        return dict(points=gaussian_unit(n, d, DATA_SEED + 1),
                    queries=gaussian_unit(m, d, QUERY_SEED + 1 + query_seed_offset),
                    k=10, recall=0.9, budget=64 << 20, name="gauss-10k-d64")
    if c == 2:
        n, d, m = sz(1_000_000), 100, sz(10_000)
        cen = mixture_centers(10_000, d, CENTER_SEED + 2)
        return dict(points=mixture(n, d, cen, 0.3, DATA_SEED + 2, sigma_mode),
                    queries=mixture(m, d, cen, 0.3, QUERY_SEED + 2 + query_seed_offset, sigma_mode),
                    k=10, recall=0.9, budget=2 << 30, name="mixture-1M-d100")
    if c == 3:
        n, d = sz(1_000_000), 256
        groups = max(1, sz(100))
        X, Q, pid = planted(n, d, groups, 100, min(2000, n // (4 * groups)), DATA_SEED + 3)
        return dict(points=X, queries=Q, planted=pid, k=1, recall=0.9, budget=2 << 30,
                    name="planted-1M-d256")
    if c == 4:
        n, d = sz(1_000_000), 100
        cen = mixture_centers(10_000, d, CENTER_SEED + 2)
        X = mixture(n, d, cen, 0.3, DATA_SEED + 2, sigma_mode)
        Q, ks, recalls = mixed_queries(sz(100_000), 0, sigma_mode)
        return dict(points=X, queries=Q, ks=ks, recalls=recalls, k=100, budget=2 << 30,
                    name="mixed-100k-on-1M-d100")
    if c == 5:
        n, d = sz(10_000_000), 128
        cen = mixture_centers(100_000, d, CENTER_SEED + 5)
        out = dict(points=mixture(n, d, cen, 0.3, DATA_SEED + 5, sigma_mode),
                   queries=mixture(sz(100_000), d, cen, 0.3, QUERY_SEED + 50, sigma_mode),
                   k=10, recall=0.9, budget=16 << 30, name="mixture-10M-d128")
        if with_train:
            out["train_queries"] = mixture(sz(1_000_000), d, cen, 0.3, QUERY_SEED + 5, sigma_mode)
        return out
    raise ValueError(c)


def queries_like(c: int, m: int, seed_offset: int = 100, sigma_mode: str = "coord") -> np.ndarray:
    """m further queries of configuration c's query distribution (configs 1, 2, 5), drawn
    with their own seed (query seed + seed_offset); used as training traces."""
    if c == 1:
        return gaussian_unit(m, 64, QUERY_SEED + 1 + seed_offset)
    if c == 2:
        cen = mixture_centers(10_000, 100, CENTER_SEED + 2)
        return mixture(m, 100, cen, 0.3, QUERY_SEED + 2 + seed_offset, sigma_mode)
    if c == 5:
        cen = mixture_centers(100_000, 128, CENTER_SEED + 5)
        return mixture(m, 128, cen, 0.3, QUERY_SEED + 5 + seed_offset, sigma_mode)
    raise ValueError(c)


def mixed_queries(m: int, seed_offset: int = 0, sigma_mode: str = "coord"):
    """Configuration 4's batch (its points are configuration 2's): half the queries from
    configuration 2's mixture, half i.i.d. Gaussian then normalised (d = 100), shuffled,
    with per-query k in {1, 10, 100} and recall in {0.5, 0.9, 0.99} drawn uniformly.
    seed_offset > 0 draws another batch of the same distribution (training traces)."""
    d = 100
    cen = mixture_centers(10_000, d, CENTER_SEED + 2)
    qa = mixture(m // 2, d, cen, 0.3, QUERY_SEED + 4 + seed_offset, sigma_mode)
    qb = gaussian_unit(m - m // 2, d, QUERY_SEED + 40 + seed_offset)
    Q = np.concatenate([qa, qb])
    rng = np.random.default_rng(QUERY_SEED + 41 + seed_offset)
    perm = rng.permutation(m)
    ks = rng.choice(np.array([1, 10, 100], dtype=np.int32), size=m)
    recalls = rng.choice(np.array([0.5, 0.9, 0.99]), size=m)
    return Q[perm], ks, recalls
