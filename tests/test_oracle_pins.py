"""Pins of the CPU oracle against facts the paper and mathematics fix (no GPU).

Each test names the passage it pins and the kind of pin: closed form, special case,
textbook routine, brute force, error bound, or a statistical guarantee.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------- generator
def test_splitmix64_published_stream(oracle_mod):
    """Published first outputs of SplitMix64 from seed 0 (generator's reference code)."""
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [oracle_mod.splitmix64(0, s) for s in range(3)] == vals


def test_hyperplanes_are_standard_normal(oracle_mod):
    """Sec. 2.2: every coordinate of a hyperplane is an independent N(0,1) draw.
    Statistical pin: moments and a Kolmogorov-Smirnov test over 10^6 draws; a wrong
    Box-Muller constant (e.g. a dropped factor 2) moves the variance by 50%."""
    a = oracle_mod.hyperplanes(7, 1000, 1000).astype(np.float64).ravel()
    N = a.size
    assert abs(a.mean()) < 5 / math.sqrt(N)
    assert abs(a.var() - 1.0) < 5 * math.sqrt(2.0 / N)
    assert abs(stats.kurtosis(a, fisher=False) - 3.0) < 5 * math.sqrt(24.0 / N)
    assert stats.kstest(a[:200_000], "norm").pvalue > 1e-4
    # coordinates of one row are uncorrelated
    r = np.corrcoef(a[:-1], a[1:])[0, 1]
    assert abs(r) < 5 / math.sqrt(N)
    # deterministic in the seed, different across seeds
    assert np.array_equal(oracle_mod.hyperplanes(7, 3, 5), oracle_mod.hyperplanes(7, 3, 5))
    assert not np.array_equal(oracle_mod.hyperplanes(7, 3, 5), oracle_mod.hyperplanes(8, 3, 5))


# ----------------------------------------------------------------------- normalisation
def test_normalize(oracle_mod):
    """Sec. 4.2 (vector storage): rows become unit vectors; zero rows are rejected."""
    x = workloads.gaussian_unit(500, 37, 5) * np.float32(3.7)
    y = oracle_mod.normalize(x)
    ref = (x.astype(np.float64) / np.linalg.norm(x.astype(np.float64), axis=1, keepdims=True))
    # FP64 quotient rounded once: within half an ulp of the FP64 value (plus FP64 noise)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(y - ref) <= 0.5 * ulp + 1e-15)
    assert np.allclose(np.linalg.norm(y.astype(np.float64), axis=1), 1.0, atol=1e-6)
    bad = x.copy()
    bad[3] = 0
    with pytest.raises(ValueError):
        oracle_mod.normalize(bad)
    bad[3] = np.nan
    with pytest.raises(ValueError):
        oracle_mod.normalize(bad)


# ----------------------------------------------------------------------- budget -> L
def test_num_tables_budget(oracle_mod):
    """Sec. 1 / Sec. 5.2: the memory budget alone fixes L; the index (vectors, hash
    functions, tables) must fit.  Closed form: bytes(L) <= budget < bytes(L + 1)."""
    def bytes_for(n, d, K, M, L):
        P = min(13, K)
        return 4 * n * d + 4 * 64 * M * d + L * (16 * n + 4 * (2 ** P + 1) + 4 * K * d)

    for (n, d, budget) in [(10_000, 64, 64 << 20), (1_000_000, 100, 2 << 30),
                           (1_000_000, 256, 2 << 30), (10_000_000, 128, 16 << 30), (1000, 8, 1 << 22)]:
        L = oracle_mod.num_tables(n, d, budget)
        assert bytes_for(n, d, 24, 32, L) <= budget < bytes_for(n, d, 24, 32, L + 1)
    assert oracle_mod.num_tables(10_000, 64, 64 << 20) == 321
    assert oracle_mod.num_tables(1_000_000, 100, 2 << 30) == 108
    assert oracle_mod.num_tables(1000, 8, 1000) == 0


# ----------------------------------------------------------------------- hashing
def _angle(a, b):
    """Angle between two rows, stable near 0 and pi: 2 asin(|a - b| / 2) of unit rows."""
    a = a.astype(np.float64) / np.linalg.norm(a.astype(np.float64))
    b = b.astype(np.float64) / np.linalg.norm(b.astype(np.float64))
    return 2.0 * math.asin(min(1.0, np.linalg.norm(a - b) / 2.0))


def _angle_pair(d, theta, seed=0):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(d)
    u /= np.linalg.norm(u)
    w = rng.standard_normal(d)
    w -= (w @ u) * u
    w /= np.linalg.norm(w)
    x = u
    y = math.cos(theta) * u + math.sin(theta) * w
    return np.stack([x, y]).astype(np.float32)


@pytest.mark.parametrize("deg", [0, 30, 60, 90, 120, 180])
def test_hp_collision_probability(oracle_mod, deg):
    """Sec. 2.2 / Sec. 4.3: a random-hyperplane bit collides with probability
    1 - theta/pi (Charikar).  Closed form, 5 sigma over ~10^6 functions."""
    d, K, L, M = 16, 24, 41_667, 1
    pts = oracle_mod.normalize(_angle_pair(d, math.radians(deg)))
    theta = _angle(pts[0], pts[1])
    hp = oracle_mod.hyperplanes(11 + deg, L * K + 64 * M, d)
    codes, _ = oracle_mod.hash_codes(pts, hp, L, K, M)
    diff = np.unpackbits((codes[:, 0] ^ codes[:, 1]).view(np.uint8)).sum()
    N = L * K
    p = 1 - theta / math.pi
    same = 1 - diff / N
    sd = math.sqrt(max(p * (1 - p), 1e-12) / N)
    assert abs(same - p) <= 5 * sd + 1e-12


def test_hash_bit_layout_special_cases(oracle_mod):
    """Sec. 2.2: bit = 1 iff <a, x> >= 0 (so a projection of exactly 0 gives 1).
    Sec. 4.2: codes are bitstrings sorted lexicographically, h_{1,j} leading.
    Special case with a hand-computed answer: axis-aligned hyperplanes."""
    d, K, L, M = 2, 3, 2, 1
    x = np.array([[1.0, 0.0]], dtype=np.float32)
    hp = np.zeros((L * K + 64 * M, d), dtype=np.float32)
    # table 0: h1 = +e0 (1), h2 = -e0 (0), h3 = e1 (projection 0 -> 1)  => 0b101
    hp[0] = [1, 0]
    hp[1] = [-1, 0]
    hp[2] = [0, 1]
    # table 1: h1 = -e0 (0), h2 = -e0 (0), h3 = +e0 (1)                    => 0b001
    hp[3] = [-1, 0]
    hp[4] = [-1, 0]
    hp[5] = [1, 0]
    # sketch bits: bit b = 1 iff b is even (hyperplane +e0), odd bits use -e0
    for b in range(64):
        hp[L * K + b] = [1, 0] if b % 2 == 0 else [-1, 0]
    codes, sk = oracle_mod.hash_codes(x, hp, L, K, M)
    assert codes[0, 0] == 0b101 and codes[1, 0] == 0b001
    assert int(sk[0, 0]) == 0x5555555555555555


@pytest.mark.parametrize("deg", [30, 60, 90])
def test_sketch_expected_hamming(oracle_mod, deg):
    """Sec. 5.1 footnote (read as the probability that bits differ): the expected
    Hamming distance of two 64-bit sketches at angle theta is 64 theta / pi."""
    d, K, L, M = 16, 24, 1, 15_625
    pts = oracle_mod.normalize(_angle_pair(d, math.radians(deg), seed=3))
    theta = _angle(pts[0], pts[1])
    hp = oracle_mod.hyperplanes(100 + deg, L * K + 64 * M, d)
    _, sk = oracle_mod.hash_codes(pts, hp, L, K, M)
    h = np.unpackbits((sk[:, 0] ^ sk[:, 1]).view(np.uint8)).reshape(M, 64).sum(1)
    mean = 64 * theta / math.pi
    sd = math.sqrt(64 * (theta / math.pi) * (1 - theta / math.pi) / M)
    assert abs(h.mean() - mean) <= 5 * sd


def test_tau_closed_form(oracle_mod):
    """Sec. 4.2 / Sec. 5.1: tau = (1 + eps) 64 arccos(ip_k) / pi at known angles."""
    assert oracle_mod.tau(1.0) == 0.0
    assert abs(oracle_mod.tau(0.0) - 32.0) < 1e-12
    assert abs(oracle_mod.tau(-1.0) - 64.0) < 1e-12
    assert abs(oracle_mod.tau(0.5) - 64.0 / 3.0) < 1e-6
    c30 = float(np.float32(math.cos(math.pi / 6)))
    assert abs(oracle_mod.tau(c30) - 64.0 / 6.0) < 1e-5
    assert abs(oracle_mod.tau(0.5, 0.1) - 1.1 * 64.0 / 3.0) < 1e-6
    # out-of-range FP32 inner products are clamped (rounding can exceed 1 slightly)
    assert oracle_mod.tau(1.0000001) == 0.0


# ----------------------------------------------------------------------- tables
def test_sorted_tables_textbook(oracle_mod):
    """Sec. 4.1 / 4.2: repetition j is the array of (code, position) sorted by code;
    equal codes by position.  Textbook pin: numpy's stable argsort.  Prefix table:
    brute-force counts of entries whose leading 13 bits are below p."""
    rng = np.random.default_rng(0)
    L, n, K = 5, 3000, 24
    codes = rng.integers(0, 1 << 12, size=(L, n), dtype=np.uint32) << 12  # many ties
    codes |= rng.integers(0, 4, size=(L, n), dtype=np.uint32)
    tcode, tidx, off = oracle_mod.build_tables(codes, K)
    for j in range(L):
        perm = np.argsort(codes[j], kind="stable")
        assert np.array_equal(tidx[j], perm.astype(np.uint32))
        assert np.array_equal(tcode[j], codes[j][perm])
        top = codes[j] >> (K - 13)
        for p in list(range(0, 40)) + [4095, 4096, 4097, 8191, 8192]:
            assert off[j, p] == np.count_nonzero(top < p)


def test_table_sketches_permute_sketches(oracle_mod):
    """Sec. 4.2: repetition j reads sketch sigma(j) of each candidate; the table-local
    copy is that sketch array permuted by the table order (multiset preserved)."""
    rng = np.random.default_rng(1)
    L, M, n = 7, 3, 500
    sk = rng.integers(0, 2 ** 63, size=(M, n), dtype=np.uint64)
    tidx = np.stack([rng.permutation(n).astype(np.uint32) for _ in range(L)])
    tsk = oracle_mod.table_sketches(tidx, sk)
    for j in range(L):
        assert np.array_equal(np.sort(tsk[j]), np.sort(sk[j % M]))
        e = rng.integers(0, n, 20)
        assert np.array_equal(tsk[j, e], sk[j % M, tidx[j, e]])


# ----------------------------------------------------------------------- inner product
@pytest.mark.parametrize("d", [1, 3, 4, 17, 64, 100, 256, 300])
def test_ip32_error_bound(oracle_mod, d):
    """Re-rank inner product in FP32: error within Higham's bound
    |fl(x.q) - x.q| <= gamma_d * sum |x_i q_i|, gamma_d = d u / (1 - d u), u = 2^-24,
    against the exact rational value of the FP32 inputs."""
    rng = np.random.default_rng(d)
    u = 2.0 ** -24
    g = d * u / (1 - d * u)
    for _ in range(20):
        x = rng.standard_normal(d).astype(np.float32)
        q = rng.standard_normal(d).astype(np.float32)
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, q))
        bound = g * float(np.sum(np.abs(x.astype(np.float64) * q)))
        assert abs(float(Fraction(oracle_mod.ip32(x, q)) - exact)) <= bound
        assert abs(oracle_mod.ip64(x, q) - float(exact)) <= 1e-12 * (1 + bound)


def test_ip32_short_vectors_are_sequential_sums(oracle_mod):
    """Special case: with d <= 4 only partial 0 is used, so the FP32 result is the
    plain left-to-right FP32 sum of FP32 products."""
    rng = np.random.default_rng(5)
    for d in (1, 2, 3, 4):
        for _ in range(50):
            x = rng.standard_normal(d).astype(np.float32)
            q = rng.standard_normal(d).astype(np.float32)
            s = np.float32(0)
            for a, b in zip(x, q):
                s = np.float32(s + np.float32(a * b))
            assert oracle_mod.ip32(x, q) == float(s)


# ----------------------------------------------------------------------- stopping rule
@pytest.mark.parametrize("rule", ["exact", "alg1"])
def test_stop_rule_closed_form(oracle_mod, rule):
    """Lemma 1: failure after L repetitions at level i is at most (1 - p^i)^L.
    Exact rule: stop iff (1 - p^i)^L <= delta, whose solution in i is
    i <= ln(1 - delta^(1/L)) / ln p.  Algorithm 1's test L >= ln(1/delta)/p^i solves to
    i <= ln(ln(1/delta)/L) / ln p.  Both closed forms checked on a grid."""
    for ipk in (0.3, 0.378, 0.5, 0.8, 0.9, 0.95):
        ipf = float(np.float32(ipk))
        p = 1 - math.acos(ipf) / math.pi
        for L in (2, 10, 69, 100, 108, 321):
            for delta in (0.5, 0.1, 0.01, 0.001):
                if rule == "exact":
                    istar = math.log(1 - delta ** (1.0 / L)) / math.log(p)
                else:
                    istar = math.log(math.log(1 / delta) / L) / math.log(p)
                for i in range(1, 25):
                    if abs(i - istar) < 1e-6:
                        continue
                    r = oracle_mod.RULE_EXACT if rule == "exact" else oracle_mod.RULE_ALG1
                    got, _ = oracle_mod.stop(ipf, i, L, delta, r)
                    assert got == (i <= istar), (ipk, L, delta, i, istar)


def test_exact_rule_never_later_than_alg1(oracle_mod):
    """(1 - x)^L <= exp(-L x): whenever Algorithm 1's test fires the exact bound holds."""
    for ipk in np.linspace(-0.5, 0.99, 40):
        for L in (1, 3, 10, 100):
            for delta in (0.5, 0.2, 0.05):
                for i in range(1, 25):
                    a1, _ = oracle_mod.stop(float(ipk), i, L, delta, oracle_mod.RULE_ALG1)
                    ex, _ = oracle_mod.stop(float(ipk), i, L, delta, oracle_mod.RULE_EXACT)
                    assert ex or not a1


# ----------------------------------------------------------------------- search
@pytest.fixture(scope="module")
def small_index(oracle_mod):
    X = workloads.gaussian_unit(2000, 16, 11)
    Q = workloads.gaussian_unit(60, 16, 12)
    ix = oracle_mod.OracleIndex(X, budget=0, L=30, seed=5)
    return ix, Q


def test_bruteforce_textbook(oracle_mod, small_index):
    """Exact k-NN: numpy lexsort on (-ip, id) of FP64 inner products."""
    ix, Q = small_index
    qn = oracle_mod.normalize(Q)
    ids, ips = oracle_mod.bruteforce(ix.points, qn, 7)
    G = qn.astype(np.float64) @ ix.points.astype(np.float64).T
    for t in range(len(qn)):
        order = np.lexsort((np.arange(ix.n), -G[t]))[:7]
        assert np.array_equal(ids[t], order)
        assert np.allclose(ips[t], G[t, order], atol=1e-12)


def test_ranges_match_bruteforce_prefix_sets(oracle_mod, small_index):
    """Sec. 3.1 / 4.2: at level i the entries colliding with q on the first i functions
    form one contiguous range [lo_i, hi_i) of the sorted array, nested in i.
    Brute force: count entries of each table by prefix comparison."""
    ix, Q = small_index
    r = ix.search(Q[:1], 5, 1.0, trace=True)  # recall 1: walks every level
    qn = oracle_mod.normalize(Q[:1])
    qc, _ = oracle_mod.hash_codes(qn, ix.hp, ix.L, ix.K, ix.M)
    K = ix.K
    for j in range(ix.L):
        prev = None
        for i in range(K, 0, -1):
            pre = ix.tcode[j] >> (K - i)
            qp = int(qc[j, 0]) >> (K - i)
            lo, hi = int(np.count_nonzero(pre < qp)), int(np.count_nonzero(pre <= qp))
            assert (r.trace[i, j, 0], r.trace[i, j, 1]) == (lo, hi)
            assert np.all(pre[lo:hi] == qp)
            if prev:
                assert lo <= prev[0] and hi >= prev[1]
            prev = (lo, hi)


def test_segment_rule_B1_gives_Pi_sets(oracle_mod, small_index):
    """App. C: B = 1 considers only points with a matching prefix, i.e. after level i
    the consumed window is exactly S_{i,j}(q) and the new entries are Pi_{i,j}(q)."""
    ix, Q = small_index
    r = ix.search(Q[:1], 5, 1.0, B=1, trace=True)
    for i in range(ix.K, 0, -1):
        assert np.array_equal(r.trace[i, :, 2], r.trace[i, :, 0])
        assert np.array_equal(r.trace[i, :, 3], r.trace[i, :, 1])


def test_segment_rule_B12_superset(oracle_mod, small_index):
    """Sec. 4.2 / App. C: with B = 12 every access takes whole segments, so the window
    covers S_{i,j}(q), grows by multiples of B (unless clipped at the array ends),
    and never grows when the level adds no matching entry."""
    ix, Q = small_index
    r = ix.search(Q[:1], 5, 1.0, B=12, trace=True)
    n = ix.n
    for j in range(ix.L):
        prev = None
        for i in range(ix.K, 0, -1):
            lo, hi, clo, chi = r.trace[i, j]
            assert clo <= lo and chi >= hi
            if prev is not None:
                pclo, pchi = prev
                dl, dr = pclo - clo, chi - pchi
                assert dl % 12 == 0 or clo == 0
                assert dr % 12 == 0 or chi == n
                if pclo <= lo:
                    assert dl == 0
                if pchi >= hi:
                    assert dr == 0
            prev = (clo, chi)


@pytest.mark.parametrize("k", [1, 5, 17])
def test_linear_scan_is_exact(oracle_mod, small_index, k):
    """Lemma 1, case i = 0: the query degrades to a linear scan and reports the true
    k-NN.  recall = 1 means delta = 0, which no level can satisfy."""
    ix, Q = small_index
    r = ix.search(Q, k, 1.0)
    ids, ips = oracle_mod.bruteforce(ix.points, oracle_mod.normalize(Q), k)
    assert np.all(r.stop_level == 0)
    assert np.all(r.c_rerank == r.c_pass + ix.n)
    # the FP32 ordering may swap two neighbours whose FP64 ips differ by less than
    # the FP32 error bound; compare as sets and check that any swap is such a tie
    for t in range(len(Q)):
        if not np.array_equal(r.ids[t], ids[t]):
            assert set(r.ids[t]) == set(ids[t]) or np.min(np.abs(np.diff(ips[t]))) < 1e-6
    assert np.mean([np.array_equal(a, b) for a, b in zip(r.ids, ids)]) > 0.95


def test_results_sorted_distinct_and_exact_ips(oracle_mod, small_index):
    """Output contract: k distinct points ordered by (ip desc, id asc); each ip is the
    canonical FP32 inner product of that point with the normalised query."""
    ix, Q = small_index
    r = ix.search(Q, 8, 0.7)
    qn = oracle_mod.normalize(Q)
    for t in range(len(Q)):
        assert len(set(r.ids[t])) == 8
        for s in range(8):
            assert r.ips[t, s] == np.float32(oracle_mod.ip32(ix.points[r.ids[t, s]], qn[t]))
            if s:
                a, b = (r.ips[t, s - 1], r.ids[t, s - 1]), (r.ips[t, s], r.ids[t, s])
                assert a[0] > b[0] or (a[0] == b[0] and a[1] < b[1])
    assert np.all(r.c_pass <= r.c_scan)
    assert np.all(r.c_rerank == r.c_pass + np.where(r.stop_level == 0, ix.n, 0))


@pytest.mark.parametrize("B", [1, 12])
def test_lemma1_guarantee_statistical(oracle_mod, B):
    """Lemma 1: each of the k true nearest neighbours is returned with probability at
    least 1 - delta.  Statistical pin over 300 independent index seeds (filter off, as
    the lemma covers Algorithm 1 without sketches): the hit rate of every true
    neighbour is at least 1 - delta - 4 sigma."""
    X = workloads.gaussian_unit(400, 8, 21)
    Q = workloads.gaussian_unit(4, 8, 22)
    k, recall = 3, 0.8
    qn = oracle_mod.normalize(Q)
    true_ids, _ = oracle_mod.bruteforce(oracle_mod.normalize(X), qn, k)
    seeds = 300
    hits = np.zeros((len(Q), k))
    levels = []
    for s in range(seeds):
        ix = oracle_mod.OracleIndex(X, budget=0, L=6, seed=1000 + s, M=1)
        r = ix.search(Q, k, recall, B=B, filter_on=False)
        levels.append(r.stop_level)
        for t in range(len(Q)):
            hits[t] += np.isin(true_ids[t], r.ids[t])
    rate = hits / seeds
    delta = 1 - recall
    sd = math.sqrt(delta * (1 - delta) / seeds)
    assert np.all(rate >= 1 - delta - 4 * sd), rate
    # the instance is not trivial: queries stop above the linear scan
    assert np.mean(np.concatenate(levels) > 0) > 0.5


def test_paper_synthetic_known_answer(oracle_mod):
    """Sec. 5 (synthetic dataset): x_n is the nearest neighbour of every query, and the
    search at recall .9 finds it for at least 90% of queries minus sampling slack."""
    X, Q = workloads.paper_synthetic(3000, 100, 40, seed=9)
    qn = oracle_mod.normalize(Q)
    ids, _ = oracle_mod.bruteforce(oracle_mod.normalize(X), qn, 1)
    assert np.all(ids[:, 0] == len(X) - 1)
    ix = oracle_mod.OracleIndex(X, budget=0, L=40, seed=3)
    r = ix.search(Q, 1, 0.9)
    assert np.mean(r.ids[:, 0] == len(X) - 1) >= 0.9 - 4 * math.sqrt(0.09 / 40)


# ----------------------------------------------------------------------- filter-aware bound
def test_binom_cdf_matches_scipy(oracle_mod):
    """Pass probability of the sketch filter: the Binomial(64, t) CDF (library routine)."""
    for t in (1e-3, 0.05, 0.2, 0.3333, 0.366, 0.5, 0.77, 0.999):
        for T in (-1, 0, 1, 10, 21, 23, 32, 50, 63, 64):
            assert abs(oracle_mod.binom_cdf64(t, T) - stats.binom.cdf(T, 64, t)) < 1e-12, (t, T)
    assert oracle_mod.binom_cdf64(0.0, 0) == 1.0
    assert oracle_mod.binom_cdf64(1.0, 63) == 0.0


def test_filter_rule_without_filtering_is_the_exact_rule(oracle_mod):
    """Special case: threshold 64 passes everything (q = 1), and the bound collapses to
    (1 - p^i)^L whatever the sketch grouping."""
    for ipk in (0.2, 0.41, 0.8, 0.95):
        for L, M in ((108, 32), (10, 32), (321, 32), (7, 3)):
            for delta in (0.5, 0.1, 0.01):
                for i in range(1, 25):
                    a, ma = oracle_mod.stop(ipk, i, L, delta, oracle_mod.RULE_EXACT)
                    b, mb = oracle_mod.stop(ipk, i, L, delta, oracle_mod.RULE_FILTER, M=M, tau_int=64)
                    assert a == b and abs(ma - mb) < 1e-9 * (1 + abs(ma))


def test_filter_rule_closed_form_independent_sketches(oracle_mod):
    """With one sketch per table (M >= L) the bound is (1 - q p^i)^L <= delta, solved in
    closed form as i <= ln((1 - delta^(1/L)) / q) / ln p, q from scipy's binomial CDF."""
    for ipk in (0.3, 0.41, 0.6, 0.9):
        ipf = float(np.float32(ipk))
        theta = math.acos(ipf)
        p = 1 - theta / math.pi
        for T in (10, 20, 23, 30, 40):
            q = stats.binom.cdf(T, 64, theta / math.pi)
            for L in (5, 20, 60):
                for delta in (0.5, 0.1, 0.01):
                    arg = (1 - delta ** (1.0 / L)) / q
                    istar = math.log(arg) / math.log(p) if arg < 1 else -1
                    for i in range(1, 25):
                        if abs(i - istar) < 1e-6:
                            continue
                        got, _ = oracle_mod.stop(ipf, i, L, delta, oracle_mod.RULE_FILTER, M=64, tau_int=T)
                        assert got == (i <= istar), (ipk, T, L, delta, i, istar)


def test_filter_rule_shared_sketches_stop_no_earlier(oracle_mod):
    """Invariant: tables that share a sketch fail the filter together, so grouping L
    tables onto M < L sketches can only weaken the bound (stop at the same level or
    later than with independent sketches), and always stops later than ignoring the
    filter when q < 1."""
    for ipk in (0.3, 0.41, 0.7):
        for T in (15, 23, 35):
            for L, M in ((108, 32), (40, 8), (10, 3)):
                for delta in (0.1, 0.01):
                    for i in range(1, 25):
                        grp, _ = oracle_mod.stop(ipk, i, L, delta, oracle_mod.RULE_FILTER, M=M, tau_int=T)
                        ind, _ = oracle_mod.stop(ipk, i, L, delta, oracle_mod.RULE_FILTER, M=L, tau_int=T)
                        exact, _ = oracle_mod.stop(ipk, i, L, delta, oracle_mod.RULE_EXACT)
                        assert (not grp) or ind
                        assert (not ind) or exact


def test_lemma1_guarantee_with_filter_statistical(oracle_mod):
    """Lemma 1 with the sketch filter on and the filter-aware bound: each of the k true
    neighbours is returned with probability at least 1 - delta (300 independent index
    seeds; neighbours at 60-70 degrees, so the filter often rejects a true neighbour it
    sees; four sketches shared by twenty tables).  Negative control: the bound without
    the filter's misses (the paper's rule) falls visibly short on the same instance."""
    X = workloads.gaussian_unit(400, 32, 71)
    Q = workloads.gaussian_unit(4, 32, 72)
    k, recall = 3, 0.8
    qn = oracle_mod.normalize(Q)
    true_ids, _ = oracle_mod.bruteforce(oracle_mod.normalize(X), qn, k)
    seeds = 300
    hits = np.zeros((len(Q), k))
    hits_paper = np.zeros((len(Q), k))
    levels = []
    for s in range(seeds):
        ix = oracle_mod.OracleIndex(X, budget=0, L=20, seed=5000 + s, M=4)
        r = ix.search(Q, k, recall, rule=oracle_mod.RULE_FILTER, filter_on=True)
        rp = ix.search(Q, k, recall, rule=oracle_mod.RULE_EXACT, filter_on=True)
        levels.append(r.stop_level)
        for t in range(len(Q)):
            hits[t] += np.isin(true_ids[t], r.ids[t])
            hits_paper[t] += np.isin(true_ids[t], rp.ids[t])
    rate = hits / seeds
    delta = 1 - recall
    sd = math.sqrt(delta * (1 - delta) / seeds)
    assert np.all(rate >= 1 - delta - 4 * sd), rate
    assert np.all(np.concatenate(levels) > 0)
    assert (hits_paper / seeds).min() < rate.min() - 0.05


# ----------------------------------------------------------------------- scheduler network
def test_mlp_gradient_finite_differences():
    """The FP64 reference gradient of the scheduler network against central finite
    differences (closed form of the derivative, relative error <= 1e-6)."""
    from oracle import mlp

    rng = np.random.default_rng(3)
    p = rng.standard_normal(mlp.NPARAMS) * 0.1
    x = rng.standard_normal((20, mlp.IN))
    t = rng.standard_normal((20, mlp.OUT))
    loss, g = mlp.loss_and_grad(p, x, t)
    idx = np.concatenate([rng.choice(mlp.NPARAMS, 200, replace=False), [mlp.NPARAMS - 1, mlp.NPARAMS - 2]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, t)[0] - mlp.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])
    assert mlp.NPARAMS == 29442


def test_scheduler_features_special_case():
    """Features: sketch bits as +1/-1 in bit order, log2(1 + bucket size) per table."""
    from oracle import mlp

    f = mlp.features(np.array([0b1011], dtype=np.uint64), np.array([[0, 1, 3, 7]]))
    assert list(f[0, :5]) == [1.0, 1.0, -1.0, 1.0, -1.0]
    assert np.all(f[0, 5:64] == -1.0)
    assert list(f[0, 64:68]) == [0.0, 1.0, 2.0, 3.0]
    assert np.all(f[0, 68:96] == 0.0)
    assert f.shape == (1, 98)
    # log2 k and log2(1/delta): k = 10, recall 0.9 by default; powers of two exactly
    assert abs(f[0, 96] - 3.321928094887362) < 1e-15 and abs(f[0, 97] - 3.321928094887362) < 1e-12
    g = mlp.features(np.zeros(3, dtype=np.uint64), np.zeros((3, 32)), ks=[1, 64, 256],
                     recalls=[0.5, 0.75, 1.0])
    assert list(g[:, 96]) == [0.0, 6.0, 8.0] and list(g[:, 97]) == [1.0, 2.0, 40.0]


# ----------------------------------------------------------------------- pooling (Sec. 3.2, App. B)
def test_pool_budget_closed_form(oracle_mod):
    """With a pool of m functions the budget counts the m shared hyperplanes once and K
    pool indices per trie: closed-form L at two configurations (hand-computed)."""
    # n 10,000, d 64, 64 MiB, m 3072: fixed = 2,560,000 + 524,288 + 786,432; per = 160,000 + 32,772 + 96
    assert oracle_mod.num_tables(10_000, 64, 64 << 20, pool=3072) == (67_108_864 - 3_870_720) // 192_868 == 327
    # n 1,000,000, d 100, 2 GiB: fixed = 400,000,000 + 819,200 + 1,228,800; per = 16,000,000 + 32,772 + 96
    assert oracle_mod.num_tables(1_000_000, 100, 2 << 30, pool=3072) == 1_745_435_648 // 16_032_868 == 108


def test_pool_selection_is_a_uniform_subset(oracle_mod):
    """Each trie's K functions are distinct pool indices, every position of the sample is
    uniform over the pool and every ordered pair of positions uniform over distinct pairs
    (chi-square over 30,000 tries, m = 12, K = 4), and K = m gives permutations."""
    m, K, L = 12, 4, 30_000
    sel = oracle_mod.pool_select(11, m, L, K)
    assert sel.min() >= 0 and sel.max() < m
    assert all(len(set(r)) == K for r in sel[:2000])
    assert np.all(np.sort(sel, axis=1)[:, 1:] != np.sort(sel, axis=1)[:, :-1])
    for t in range(K):
        cnt = np.bincount(sel[:, t], minlength=m)
        assert stats.chisquare(cnt).pvalue > 1e-4, (t, cnt)
    pair = sel[:, 0] * m + sel[:, 2]
    cnt = np.bincount(pair, minlength=m * m).reshape(m, m)
    assert np.all(np.diag(cnt) == 0)
    off = cnt[~np.eye(m, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-4
    perm = oracle_mod.pool_select(3, 7, 50, 7)
    assert np.all(np.sort(perm, axis=1) == np.arange(7))
    with pytest.raises(ValueError):
        oracle_mod.pool_select(3, 5, 2, 6)


def test_pool_codes_are_pool_bits(oracle_mod):
    """Bit s of trie j's code (most significant first) is [<a, x> >= 0] for the pool
    hyperplane a = pool[sel[j][s-1]], recomputed here with numpy in FP64; sketches use the
    rows after the pool."""
    m, K, L, M, d = 96, 10, 7, 2, 20
    hp = oracle_mod.hyperplanes(8, m + 64 * M, d)
    sel = oracle_mod.pool_select(8, m, L, K)
    x = oracle_mod.normalize(workloads.gaussian_unit(300, d, 9))
    codes, sk = oracle_mod.hash_codes(x, hp, L, K, M, sel)
    proj = x.astype(np.float64) @ hp.astype(np.float64).T
    bits = proj >= 0
    for j in range(L):
        want = np.zeros(len(x), dtype=np.uint64)
        for s in range(K):
            want |= bits[:, sel[j, s]].astype(np.uint64) << np.uint64(K - 1 - s)
        assert np.array_equal(codes[j].astype(np.uint64), want)
    for mm in range(M):
        want = np.zeros(len(x), dtype=np.uint64)
        for b in range(64):
            want |= bits[:, m + 64 * mm + b].astype(np.uint64) << np.uint64(b)
        assert np.array_equal(sk[mm], want)


def test_pool_prefix_collision_probability(oracle_mod):
    """A trie's i-bit prefix under pooling collides with probability p^i (distinct pool
    functions; over the random pool, each agrees with probability p = 1 - theta/pi):
    pairs at 45 degrees, 400 pools of 256 functions, 24 tries each, i = 1..4."""
    d, K, L, m = 16, 8, 24, 256
    rng = np.random.default_rng(21)
    q = rng.standard_normal(d)
    q /= np.linalg.norm(q)
    w = rng.standard_normal(d)
    w -= (w @ q) * q
    w /= np.linalg.norm(w)
    x = np.cos(np.pi / 4) * q + np.sin(np.pi / 4) * w
    pts = np.stack([q, x]).astype(np.float32)
    p = 1 - 0.25
    agree = np.zeros(4)
    total = 0
    for s in range(400):
        hp = oracle_mod.hyperplanes(100 + s, m + 64, d)
        sel = oracle_mod.pool_select(100 + s, m, L, K)
        codes, _ = oracle_mod.hash_codes(pts, hp, L, K, 1, sel)
        for i in range(1, 5):
            agree[i - 1] += np.sum((codes[:, 0] >> (K - i)) == (codes[:, 1] >> (K - i)))
        total += L
    rate = agree / total
    for i in range(1, 5):
        sd = math.sqrt(p ** i * (1 - p ** i) / total) * 4  # pools make the trials dependent
        assert abs(rate[i - 1] - p ** i) < 4 * sd + 0.01, (i, rate[i - 1], p ** i)


def test_pool_stop_rule_closed_form(oracle_mod):
    """Algorithm 3's test L p^i >= 2 and m >= 5 i^2 / p at ip = 0 (p = 1/2 exactly):
    with L = 16 the first condition holds for i <= 3; m = 3072 allows i <= 17 and m = 40
    only i <= 2.  delta plays no part."""
    for delta in (0.9, 0.5, 0.01):
        for i in range(1, 25):
            got, _ = oracle_mod.stop(0.0, i, 16, delta, oracle_mod.RULE_POOL, pool=3072)
            assert got == (i <= 3), i
            got, _ = oracle_mod.stop(0.0, i, 16, delta, oracle_mod.RULE_POOL, pool=40)
            assert got == (i <= 2), i
    # larger ip, p = 1 - acos(ip)/pi; L = 100: L p^i >= 2 iff i <= ln(50)/ln(1/p)
    for ipk in (0.3, 0.6, 0.9):
        p = 1 - math.acos(float(np.float32(ipk))) / math.pi
        for i in range(1, 25):
            want = 100 * p ** i >= 2 and 3072 * p >= 5 * i * i
            got, _ = oracle_mod.stop(ipk, i, 100, 0.1, oracle_mod.RULE_POOL, pool=3072)
            assert got == want, (ipk, i)


def test_pool_guarantee_statistical(oracle_mod):
    """Appendix B: with pooling and Algorithm 3's test each true neighbour is found with
    probability at least 1/2 (filter off; 200 index seeds, pool of 64 functions so that
    the pool condition binds at deep levels)."""
    X = workloads.gaussian_unit(400, 32, 81)
    Q = workloads.gaussian_unit(4, 32, 82)
    k = 3
    true_ids, _ = oracle_mod.bruteforce(oracle_mod.normalize(X), oracle_mod.normalize(Q), k)
    seeds = 200
    hits = np.zeros((len(Q), k))
    for s in range(seeds):
        ix = oracle_mod.OracleIndex(X, budget=0, L=12, seed=7000 + s, M=2, pool=64)
        r = ix.search(Q, k, 0.5, rule=oracle_mod.RULE_POOL, filter_on=False)
        for t in range(len(Q)):
            hits[t] += np.isin(true_ids[t], r.ids[t])
    rate = hits / seeds
    assert np.all(rate >= 0.5 - 4 * math.sqrt(0.25 / seeds)), rate


# ----------------------------------------------------------------------- FHT cross-polytope (Sec. 2.2, 4.3)
def _cp_signs(oracle_mod, sseed, fn, dp):
    return np.array([[-1.0 if oracle_mod.splitmix64(sseed, (fn * 3 + k) * dp + c) >> 63 else 1.0
                      for c in range(dp)] for k in range(3)])


def test_cp_value_is_argmax_of_rotation(oracle_mod):
    """A function's value is s d' + i for i = argmax |H D3 H D2 H D1 x| and s the sign
    there, recomputed with scipy's Hadamard matrix (a dense product, not the transform)."""
    from scipy.linalg import hadamard

    for d in (100, 64, 5):
        dp, ell = oracle_mod.cp_dims(d)
        assert dp == 1 << (ell - 1) and dp >= d > dp // 2
        H = hadamard(dp).astype(np.float64)
        X = oracle_mod.normalize(workloads.gaussian_unit(40, d, d))
        for fn in (0, 7, 123):
            D = _cp_signs(oracle_mod, 9 + 3, fn, dp)
            for x in X:
                y = np.zeros(dp)
                y[:d] = x
                for k in range(3):
                    y = H @ (D[k] * y)
                i = int(np.argmax(np.abs(y)))
                assert oracle_mod.cp_value(x, 9, fn) == (dp if y[i] < 0 else 0) + i


def test_cp_code_layout(oracle_mod):
    """A table's K-bit code is the first K bits of its functions' values concatenated,
    function 1 first (ell = 8 for d = 100: three values; ell = 7 for d = 64: four values,
    the last cut after 3 bits)."""
    for d, ell, c in ((100, 8, 3), (64, 7, 4)):
        X = oracle_mod.normalize(workloads.gaussian_unit(30, d, 3 * d))
        codes = oracle_mod.cp_hash(X, 5, 4, 24)
        for i, x in enumerate(X):
            for j in range(4):
                cat = 0
                for f in range(c):
                    cat = (cat << ell) | oracle_mod.cp_value(x, 5, j * c + f)
                assert codes[j, i] == cat >> (c * ell - 24)


def test_cp_table_recount_and_special_values(oracle_mod):
    """The Monte Carlo table recounted here from single function values (stream seed + 2,
    the pair e_1 and (alpha, sqrt(1 - alpha^2))), then made non-decreasing in alpha;
    tab[g][0] = 1, identical points always collide, antipodal points never agree in the
    sign bit."""
    d, seed, R = 20, 3, 60
    dp, ell = oracle_mod.cp_dims(d)
    lib = oracle_mod.lib()
    tab = np.empty((41, ell + 1))
    lib.oracle_cp_table(seed, d, R, tab.ctypes.data_as(__import__("ctypes").c_void_p))
    raw = np.zeros((41, ell + 1))
    for g in range(41):
        a = -1.0 + 0.05 * g
        x = np.zeros(dp, dtype=np.float32)
        y = np.zeros(dp, dtype=np.float32)
        x[0], y[0], y[1] = 1.0, np.float32(a), np.float32(math.sqrt(max(0.0, 1 - a * a)))
        for r in range(R):
            vx, vy = oracle_mod.cp_value(x, seed - 1, r), oracle_mod.cp_value(y, seed - 1, r)
            for b in range(ell + 1):
                raw[g, b] += (vx >> (ell - b)) == (vy >> (ell - b))
    raw /= R
    want = np.minimum.accumulate(raw[::-1], axis=0)[::-1]
    assert np.array_equal(tab, want)
    full = oracle_mod.cp_table(42, 100)
    assert np.all(full[:, 0] == 1.0) and np.all(full[40] == 1.0) and np.all(full[0, 1:] == 0.0)
    assert np.all(np.diff(full, axis=0) >= 0) and np.all(np.diff(full, axis=1) <= 0)


def test_cp_prob_lookup(oracle_mod):
    """P(i) = tab[g][ell]^a * tab[g][b], i = a ell + b, g = floor((ip + 1) * 20): hand cases."""
    tab = oracle_mod.cp_table(42, 100)
    ell = tab.shape[1] - 1
    for ip, g in ((0.337, 26), (-1.0, 0), (1.0, 40), (0.0, 20), (-0.26, 14)):
        ipf = float(np.float32(ip))
        for i in (0, 1, 5, 8, 13, 19, 24):
            a, b = divmod(i, ell)
            assert abs(oracle_mod.cp_prob(tab, ipf, i) - tab[g, ell] ** a * tab[g, b]) <= 1e-15, (ip, i)


def test_cp_budget_closed_form(oracle_mod):
    """FHT-CP tables store three d'-bit sign vectors per function: n 1,000,000, d 100 (d' 128,
    ell 8, three functions), 2 GiB: per table 16,000,000 + 32,772 + 144 bytes."""
    assert oracle_mod.num_tables(1_000_000, 100, 2 << 30, cp=True) == \
        (2_147_483_648 - 400_000_000 - 819_200) // 16_032_916 == 108


def test_cp_lemma1_guarantee_statistical(oracle_mod):
    """Lemma 1 with FHT cross-polytope codes and the Monte Carlo collision tables (filter
    off, the paper's bound): each true neighbour found with probability at least
    1 - delta, up to the tables' sampling error (150 index seeds)."""
    X = workloads.gaussian_unit(500, 24, 91)
    Q = workloads.gaussian_unit(3, 24, 92)
    k, recall = 3, 0.8
    true_ids, _ = oracle_mod.bruteforce(oracle_mod.normalize(X), oracle_mod.normalize(Q), k)
    seeds = 150
    hits = np.zeros((len(Q), k))
    for s in range(seeds):
        ix = oracle_mod.OracleIndex(X, 0, seed=9000 + s, L=10, M=2, cp=True)
        r = ix.search(Q, k, recall, rule=oracle_mod.RULE_EXACT, filter_on=False)
        for t in range(len(Q)):
            hits[t] += np.isin(true_ids[t], r.ids[t])
    rate = hits / seeds
    sd = math.sqrt(0.2 * 0.8 / seeds)
    assert np.all(rate >= 0.8 - 4 * sd - 0.03), rate
