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


def test_traffic_summary_only_for_its_own_launch(tmp_path, monkeypatch):
    """The committed counter summary is reported only for the launch it was taken on: the
    same search-kernel source, tile shape, table count, position and prefix widths and
    stopping-test groups; any difference gives no traffic figure."""
    import json

    entry = {"k_search_device_sha256": bench.search_device_sha(), "tile_name": "ept8-u4q8-o4-late-nts", "L": 82,
             "pos_bytes": 4, "prefix_bits": 16, "groups": 16, "bytes_per_launch": 1.25e13}
    monkeypatch.setattr(bench, "traffic_file", lambda w: str(tmp_path / f"{w}.json"))
    (tmp_path / "w.json").write_text(json.dumps(entry))
    args = ("w", "ept8-u4q8-o4-late-nts", 82, 4, 16, 16)
    assert bench.traffic_entry(*args) == 1.25e13
    for i, other in ((1, "ept8-u8"), (2, 88), (3, 3), (4, 13), (5, 64)):
        changed = list(args)
        changed[i] = other
        assert bench.traffic_entry(*changed) is None, i
    assert bench.traffic_entry("missing", *args[1:]) is None
    stale = dict(entry, k_search_device_sha256="0" * 64)
    (tmp_path / "w.json").write_text(json.dumps(stale))
    assert bench.traffic_entry(*args) is None
