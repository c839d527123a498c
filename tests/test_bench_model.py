"""The benchmark's byte models (host only): the algorithmic bytes of a launch from the
kernel's per-query counters, and the same bytes with each passing entry's position
priced as the 128-byte line a scattered read brings in."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _stats(rows):
    """rows of (stop, c_scan, c_pass, c_q8, c_upper, c_exact) -> the kernel's stats layout"""
    st = np.zeros((len(rows), 7), dtype=np.int64)
    for i, (stop, scan, npass, q8, upper, exact) in enumerate(rows):
        st[i, 0], st[i, 1], st[i, 2], st[i, 3] = stop, scan, npass, npass
        st[i, 6], st[i, 5], st[i, 4] = q8, upper, exact
    return st


def test_algorithmic_bytes_term_by_term():
    d, k, L, K = 128, 10, 76, 24
    st = _stats([(6, 1000, 40, 40, 3, 2)])
    # d = 128: rows share one scale, no header; 19 visited levels (K + 1 - 6)
    want = 8 * 1000 + 4 * 40 + 128 * 40 + 2 * 128 * (3 + 2) + 4 * 128 + 8 * k + 8 * L * 19
    assert bench.algorithmic_bytes(st, d, k, L, K) == want
    # d = 100: an 8-byte header in front of the codes in the same line
    st = _stats([(0, 10, 1, 1, 0, 0)])
    want = 8 * 10 + 4 + 108 + 4 * 100 + 8 * k + 8 * L * 24
    assert bench.algorithmic_bytes(st, 100, k, L, K) == want


def test_line_model_limits():
    d, k, L, K = 128, 10, 76, 24
    for npass in (0, 3200):  # nothing passes / everything passes
        st = _stats([(6, 3200, npass, npass, 0, 0)])
        assert abs(bench.line_model_bytes(st, d, k, L, K) - bench.algorithmic_bytes(st, d, k, L, K)) < 1e-6
    # one passing entry per 32 scanned, all in distinct lines at most: never more than a line each
    st = _stats([(6, 3200, 100, 100, 0, 0)])
    extra = bench.line_model_bytes(st, d, k, L, K) - bench.algorithmic_bytes(st, d, k, L, K)
    assert 0 < extra <= 100 * (128 - 4)


def test_line_model_against_simulated_lines():
    """Expected lines touched when each entry passes independently with probability f, against
    counting them on random pass patterns."""
    rng = np.random.default_rng(7)
    scan, f = 32 * 4096, 0.037
    hits = rng.random((20, scan)) < f
    lines = hits.reshape(20, -1, 32).any(axis=2).sum(axis=1).mean()
    npass = hits.sum(axis=1).mean()
    st = _stats([(6, scan, int(round(npass)), int(round(npass)), 0, 0)])
    model = bench.line_model_bytes(st, 128, 10, 76, 24) - bench.algorithmic_bytes(st, 128, 10, 76, 24)
    simulated = 128 * lines - 4 * npass
    assert abs(model - simulated) <= 0.01 * simulated


def test_three_byte_positions():
    """3-byte positions: posb B per passing entry in the algorithmic bytes, and 128 / 3
    positions per line in the line model, against counting the lines that the 8-byte read
    of each passing entry (the two words from the one holding its first byte) touches on
    random pass patterns; the model ignores the reads that cross into the next line."""
    d, k, L, K = 128, 10, 82, 24
    st = _stats([(6, 1000, 40, 40, 3, 2)])
    assert bench.algorithmic_bytes(st, d, k, L, K, 3) == bench.algorithmic_bytes(st, d, k, L, K) - 40
    assert bench.filter_bytes(st, 3) == 8 * 1000 + 3 * 40
    rng = np.random.default_rng(11)
    scan, f = 3 * 32 * 4096, 0.037
    first = 4 * ((3 * np.arange(scan)) // 4)
    simulated, npass_all = [], []
    for _ in range(10):
        hit = rng.random(scan) < f
        lines = np.union1d(first[hit] // 128, (first[hit] + 7) // 128)
        simulated.append(128 * lines.size - 3 * hit.sum())
        npass_all.append(hit.sum())
    npass = int(round(np.mean(npass_all)))
    st = _stats([(6, scan, npass, npass, 0, 0)])
    model = bench.line_model_bytes(st, d, k, L, K, posb=3) - bench.algorithmic_bytes(st, d, k, L, K, 3)
    assert -0.01 * np.mean(simulated) <= np.mean(simulated) - model <= 0.05 * np.mean(simulated)
