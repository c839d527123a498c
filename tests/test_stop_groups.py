"""The stopping test inside a level (Algorithm 1 tests after every repetition; Sec. 4.1
once per level): with the repetitions of a level split into G consecutive groups and the
test after each group, the failure bound counts the repetitions done at prefix length i
and the rest at i + 1.  Pins: the identities that tie the partial bound to the per-level
one, its monotonicity, the walk's reduction to the per-level walk at G = 1, and Lemma 1's
per-neighbour guarantee measured over independent index seeds at G = L and G = 3."""
import math

import numpy as np
import pytest

import workloads


RULES = ("RULE_EXACT", "RULE_FILTER", "RULE_ALG1")


def test_partial_bound_at_full_level_is_the_level_bound(oracle_mod):
    """a = L (every repetition at level i) is the per-level test, for every rule."""
    for ipk in (0.2, 0.5, 0.8, 0.93):
        for L, M in ((108, 32), (20, 4), (7, 3)):
            for i in (1, 5, 13, 24):
                for rule in RULES:
                    for T in (64, 30, 10):
                        a, ma = oracle_mod.stop(ipk, i, L, 0.1, getattr(oracle_mod, rule), M=M, tau_int=T)
                        b, mb = oracle_mod.stop_partial(ipk, i, L, L, 24, 0.1, getattr(oracle_mod, rule), M=M,
                                                        tau_int=T)
                        assert a == b and ma == mb


def test_partial_bound_with_no_repetition_done_is_the_previous_level(oracle_mod):
    """a = 0 below the first level: every repetition is still at level i + 1, so the
    bound equals the per-level bound of level i + 1 (exact and filter-aware rules); at the
    first level (i = K) nothing has been taken and the bound is 1 (never stops)."""
    for ipk in (0.3, 0.7, 0.9):
        for L, M in ((40, 32), (20, 4), (9, 9)):
            for i in (1, 6, 12, 23):
                for rule in ("RULE_EXACT", "RULE_FILTER"):
                    for T in (64, 25):
                        a, ma = oracle_mod.stop(ipk, i + 1, L, 0.2, getattr(oracle_mod, rule), M=M, tau_int=T)
                        b, mb = oracle_mod.stop_partial(ipk, i, 0, L, 24, 0.2, getattr(oracle_mod, rule), M=M,
                                                        tau_int=T)
                        assert a == b and abs(ma - mb) <= 1e-12 * (1 + abs(ma))
            s, m = oracle_mod.stop_partial(ipk, 24, 0, L, 24, 0.2, oracle_mod.RULE_EXACT)
            assert not s and abs(m - (-math.log(0.2))) < 1e-15


def test_partial_bound_falls_as_repetitions_move_to_the_shorter_prefix(oracle_mod):
    """A repetition at prefix length i collides with probability p^i > p^(i+1), so every
    repetition that reaches level i lowers the failure bound: the margin is non-increasing
    in a, and so is Algorithm 1's (a p^i grows)."""
    for ipk in (0.25, 0.6, 0.85):
        for L, M in ((30, 8), (17, 17)):
            for i in (3, 10, 18):
                for rule in RULES:
                    ms = [oracle_mod.stop_partial(ipk, i, a, L, 24, 0.1, getattr(oracle_mod, rule), M=M,
                                                  tau_int=40)[1] for a in range(L + 1)]
                    assert all(b <= a + 1e-12 * (1 + abs(a)) for a, b in zip(ms, ms[1:])), (ipk, L, i, rule)


def test_walk_with_groups_stops_no_later(oracle_mod):
    """The default is G = 16.  With G > 1 the test also runs inside a level, on the
    top-k of the entries taken so far, and its last group's test is the per-level one, so
    a query stops at the same point or earlier: never more entries scanned, and a stop
    level at least as high."""
    X = workloads.gaussian_unit(3000, 24, 31)
    Q = workloads.gaussian_unit(60, 24, 32)
    ix = oracle_mod.OracleIndex(X, budget=0, L=24, seed=7, M=4)
    for rule in (oracle_mod.RULE_FILTER, oracle_mod.RULE_EXACT, oracle_mod.RULE_ALG1):
        base = ix.search(Q, 10, 0.9, rule=rule, groups=1, test_entries=0)
        dflt = ix.search(Q, 10, 0.9, rule=rule, test_entries=0)
        assert np.array_equal(dflt.c_scan, ix.search(Q, 10, 0.9, rule=rule, groups=16, test_entries=0).c_scan)
        assert np.all(dflt.c_scan <= base.c_scan)
        earlier = 0
        for G in (2, 5, 24):
            r = ix.search(Q, 10, 0.9, rule=rule, groups=G, test_entries=0)
            assert np.all(r.c_scan <= base.c_scan) and np.all(r.stop_level >= base.stop_level)
            earlier += int(np.sum(r.c_scan < base.c_scan))
        if rule != oracle_mod.RULE_ALG1:
            assert earlier > 0  # the test inside a level does stop some queries earlier
    with pytest.raises(ValueError):
        ix.search(Q, 10, 0.9, groups=25)


@pytest.mark.parametrize("G,T", [(6, 0), (3, 0), (6, 40)])
def test_lemma1_guarantee_with_groups_statistical(oracle_mod, G, T):
    """Lemma 1 with the test after each group of repetitions (G = L: after every repetition,
    as Algorithm 1 writes it), or after a group once T entries were read since the previous
    test: each of the k true nearest neighbours is returned with probability at least
    1 - delta over 300 independent index seeds (filter off), within 4 sigma."""
    X = workloads.gaussian_unit(400, 8, 21)
    Q = workloads.gaussian_unit(4, 8, 22)
    k, recall = 3, 0.8
    true_ids, _ = oracle_mod.bruteforce(oracle_mod.normalize(X), oracle_mod.normalize(Q), k)
    seeds = 300
    hits = np.zeros((len(Q), k))
    scans = []
    for s in range(seeds):
        ix = oracle_mod.OracleIndex(X, budget=0, L=6, seed=1000 + s, M=1)
        r = ix.search(Q, k, recall, rule=oracle_mod.RULE_EXACT, filter_on=False, groups=G, test_entries=T)
        scans.append(r.c_scan)
        for t in range(len(Q)):
            hits[t] += np.isin(true_ids[t], r.ids[t])
    rate = hits / seeds
    delta = 1 - recall
    sd = math.sqrt(delta * (1 - delta) / seeds)
    assert np.all(rate >= 1 - delta - 4 * sd), rate
    assert np.mean(np.concatenate(scans) < 400) > 0.5  # not a linear scan


def test_lemma1_guarantee_filter_rule_after_every_repetition(oracle_mod):
    """The filter-aware bound with the test after every repetition (G = L = 20, four
    sketches): the per-neighbour guarantee holds with the sketch filter on (300 seeds)."""
    X = workloads.gaussian_unit(400, 32, 71)
    Q = workloads.gaussian_unit(4, 32, 72)
    k, recall = 3, 0.8
    true_ids, _ = oracle_mod.bruteforce(oracle_mod.normalize(X), oracle_mod.normalize(Q), k)
    seeds = 300
    hits = np.zeros((len(Q), k))
    for s in range(seeds):
        ix = oracle_mod.OracleIndex(X, budget=0, L=20, seed=5000 + s, M=4)
        r = ix.search(Q, k, recall, rule=oracle_mod.RULE_FILTER, filter_on=True, groups=20, test_entries=0)
        for t in range(len(Q)):
            hits[t] += np.isin(true_ids[t], r.ids[t])
    rate = hits / seeds
    delta = 1 - recall
    sd = math.sqrt(delta * (1 - delta) / seeds)
    assert np.all(rate >= 1 - delta - 4 * sd), rate


def test_partial_bound_when_a_point_coincides_with_the_query(oracle_mod):
    """ip_k = 1 (the k-th neighbour coincides with the query): every repetition holds it,
    p^l = 1 at every prefix length, so the failure bound is 0 as soon as one repetition has
    taken a level -- repetition counts of zero add nothing (never 0 * log 0)."""
    for L, M in ((40, 32), (20, 4)):
        for i in (1, 12, 23):
            for a in (1, 5, L - 1, L):
                for rule in ("RULE_EXACT", "RULE_FILTER"):
                    s, m = oracle_mod.stop_partial(1.0, i, a, L, 24, 0.1, getattr(oracle_mod, rule), M=M, tau_int=30)
                    assert s and m == -math.inf, (L, i, a, rule)


def test_test_entries_schedule(oracle_mod):
    """The stopping test after a group only once T entries were read since the level's
    previous test (and always after the level's last group): T = 0 is the test after every
    group; a T above any level's entries leaves only the last group's test, which is the
    test once per level (groups = 1) and gives the same walk; any T tests at a subset of
    the every-group points and a superset of the per-level ones, and the walk up to a
    common point is the same, so a query scans at least the every-group count and at most
    the per-level count, and some T lies strictly between."""
    X = workloads.gaussian_unit(4000, 24, 41)
    Q = workloads.gaussian_unit(80, 24, 42)
    ix = oracle_mod.OracleIndex(X, budget=0, L=24, seed=9, M=4)
    for rule in (oracle_mod.RULE_FILTER, oracle_mod.RULE_EXACT):
        every = ix.search(Q, 10, 0.9, rule=rule, test_entries=0)
        level = ix.search(Q, 10, 0.9, rule=rule, groups=1, test_entries=0)
        huge = ix.search(Q, 10, 0.9, rule=rule, test_entries=4000 * 24 + 1)
        for a, b in ((huge, level),):
            assert np.array_equal(a.ids, b.ids) and np.array_equal(a.c_scan, b.c_scan)
            assert np.array_equal(a.stop_level, b.stop_level) and np.array_equal(a.c_pass, b.c_pass)
        between = 0
        for T in (1, 50, 300, 1024, 5000):
            r = ix.search(Q, 10, 0.9, rule=rule, test_entries=T)
            assert np.all(every.c_scan <= r.c_scan) and np.all(r.c_scan <= level.c_scan), (rule, T)
            assert np.all(r.stop_level <= every.stop_level) and np.all(r.stop_level >= level.stop_level)
            between += int(np.sum((every.c_scan < r.c_scan) & (r.c_scan < level.c_scan)))
        assert between > 0
    with pytest.raises(ValueError):
        ix.search(Q, 10, 0.9, test_entries=-1)
