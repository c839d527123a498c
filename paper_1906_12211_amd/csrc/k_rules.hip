// Decision tables of the adaptive query (Algorithm 1 with the stopping bound of Lemma 1,
// Sec. 3.1; filter threshold of Sec. 5.1; Algorithm 3 for pooled indexes, App. B).
#include "pf_device.h"
#include "pf_internal.h"

namespace pf {

// The FP64 decisions of a round -- the integer filter threshold and the stopping test
// -- depend on the query only through the FP32 k-th inner product ip_k, and both are
// monotone in it.  A small kernel bisects, over the ordered FP32 values in [-1, 1], the
// boundaries at which they change (FP64 evaluation, as in the definitions below), so
// the search kernel decides by FP32 comparisons:
//   tauv[h]  (h = 0..64): largest ip with T(ip) >= h, T(ip) = floor((1+eps) 64 theta/pi)
//                         clipped to [-1, 64]; +2 if even ip = 1 has T >= h, -2 if none
//   stopw[d][i-1][g][T+1]: smallest ip at which level i, after group g of the G groups of
//                         repetitions, with filter threshold T stops for the d-th
//                         distinct delta; -2 if every ip stops, +2 if none
static constexpr double kPi = 3.14159265358979323846264338327950288;

__device__ int tau_of(float ip, double eps) {
    double v = (double)ip;
    v = v > 1.0 ? 1.0 : (v < -1.0 ? -1.0 : v);
    const double ft = floor((1.0 + eps) * 64.0 * acos(v) / kPi);
    return ft >= 64.0 ? 64 : (ft < -1.0 ? -1 : (int)ft);
}

// P[Binomial(64, t) <= T]: probability that a point at angle t*pi passes a sketch
// filter of integer threshold T (each of the 64 random-hyperplane bits differs with
// probability t); C(64,h) by the recurrence C(64,h+1) = C(64,h) (64-h)/(h+1).
__device__ double binom_cdf64(double t, int T) {
    if (T < 0) return 0.0;
    if (T >= 64 || t <= 0.0) return 1.0;
    if (t >= 1.0) return 0.0;
    const double lt = log(t), l1t = log1p(-t);
    double c = 1.0, s = 0.0;
    for (int h = 0; h <= T; ++h) {
        s = s + c * exp((double)h * lt + (double)(64 - h) * l1t);
        c = c * (double)(64 - h) / (double)(h + 1);
    }
    return s < 1.0 ? s : 1.0;
}

// Stopping test once the first a of the L repetitions have taken level i and the rest
// are still at level i + 1 (nothing taken yet when i = K); a = L after the whole level
// (Sec. 4.1), a < L after repetition a as Algorithm 1 writes it.  A repetition at prefix
// length l holds a point at angle theta with probability p^l.  EXACT: failure bound of
// Lemma 1, a log1p(-p^i) + (L - a) log1p(-p^(i+1)) <= ln(delta).  ALG1: Algorithm 1's test
// a p^i >= ln(1/delta).  FILTER: Lemma 1 with the sketch filter -- a true neighbour at
// angle <= theta_k is missed only if, for each sketch s, its sketch fails the filter
// (pass probability >= q = P[Bin(64, theta_k/pi) <= T], the threshold only shrinks over
// levels) or none of the tables reading sketch s (j mod M = s; g_i of them at level i,
// g_1 at level i + 1) holds it in its window; each factor
// 1 - q + q (1 - p^i)^{g_i} (1 - p^(i+1))^{g_1} is evaluated without cancellation.
// p = 1 - theta_k/pi, FP64.
// Collision probability of an i-bit prefix under FHT cross-polytope codes (Sec. 4.3): the
// Monte Carlo table at the similarity rounded down to the grid -1, -0.95, ..., 1, with
// i = a ell + b: tab[g][ell]^a tab[g][b].
__device__ double cp_prob(const double *tab, int ell, float ip, int i) {
    const double gv = floor(((double)ip + 1.0) * 20.0);
    const int g = gv < 0.0 ? 0 : (gv > 40.0 ? 40 : (int)gv);
    const double *row = tab + (int64_t)g * (ell + 1);
    const int a = i / ell, b = i % ell;
    const double full = a > 0 ? exp((double)a * log(row[ell])) : 1.0;
    return full * row[b];
}

// POOL: Algorithm 3's test (pooling, App. B): a p^i >= 2 and pool p >= 5 i^2.
// cptab != nullptr: p^i is the cross-polytope table's prefix probability.
__device__ bool stop_of(float ip, int i, int a, int K, int T, double lndelta, int rule, int L, int M, int pool,
                        const double *cptab, int ell) {
    double v = (double)ip;
    v = v > 1.0 ? 1.0 : (v < -1.0 ? -1.0 : v);
    const double theta = acos(v);
    const double lnp = log1p(-theta / kPi);
    const double pw = cptab ? cp_prob(cptab, ell, ip, i) : exp((double)i * lnp);
    const bool deeper = a < L && i < K;
    const double pw1 = !deeper ? 0.0 : (cptab ? cp_prob(cptab, ell, ip, i + 1) : exp((double)(i + 1) * lnp));
    if (rule == PF_RULE_POOL)
        return (double)a * pw >= 2.0 && (double)pool * (1.0 - theta / kPi) >= 5.0 * (double)i * (double)i;
    if (rule == PF_RULE_ALG1) return (double)a * pw >= -lndelta;
    const double l1p = log1p(-pw), l1p1 = deeper ? log1p(-pw1) : 0.0;
    // (a count of zero repetitions contributes nothing, also where log1p(-p^l) is -inf at p = 1)
    if (rule == PF_RULE_EXACT)
        return (a > 0 ? (double)a * l1p : 0.0) + (L - a > 0 ? (double)(L - a) * l1p1 : 0.0) <= lndelta;
    const double q = binom_cdf64(theta / kPi, T);
    double term = 0.0;
    for (int s = 0; s < M && s < L; ++s) {
        const int g = L / M + (s < L % M ? 1 : 0);
        const int gi = a / M + (s < a % M ? 1 : 0);
        const double e = (gi > 0 ? (double)gi * l1p : 0.0) + (g - gi > 0 ? (double)(g - gi) * l1p1 : 0.0);
        const double x = q * expm1(e);
        term = term + ((x > -0.5) ? log1p(x) : log((1.0 - q) + q * exp(e)));
    }
    return term <= lndelta;
}

__global__ __launch_bounds__(64) void k_rule_tables(const double *__restrict__ lndeltas, int32_t ndelta,
                                                    double eps, int32_t rule, int32_t L, int32_t M,
                                                    int32_t K, int32_t G, int32_t pool,
                                                    const double *__restrict__ cptab, int32_t ell,
                                                    float *__restrict__ tauv, float *__restrict__ stopw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t olo = ord_of(-1.0f), ohi = ord_of(1.0f);
    if (t < 65) {
        const int h = (int)t;
        float v;
        if (tau_of(1.0f, eps) >= h) {
            v = 2.0f;
        } else if (tau_of(-1.0f, eps) < h) {
            v = -2.0f;
        } else {
            uint32_t lo = olo, hi = ohi; // T(lo) >= h, T(hi) < h
            while (hi - lo > 1) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (tau_of(float_of(mid), eps) >= h)
                    lo = mid;
                else
                    hi = mid;
            }
            v = float_of(lo);
        }
        tauv[h] = v;
        return;
    }
    const int64_t e = t - 65;
    const int64_t per_delta = (int64_t)K * G * kTauCols;
    if (e >= (int64_t)ndelta * per_delta) return;
    const int32_t dl = (int32_t)(e / per_delta);
    const int32_t rem = (int32_t)(e - (int64_t)dl * per_delta);
    const int32_t i = rem / (G * kTauCols) + 1;
    const int32_t g = (rem / kTauCols) % G;
    const int32_t T = rem % kTauCols - 1;
    const int32_t a = (int32_t)((int64_t)(g + 1) * L / G); // repetitions done at level i
    const double lnd = lndeltas[dl];
    float w;
    if (stop_of(-1.0f, i, a, K, T, lnd, rule, L, M, pool, cptab, ell)) {
        w = -2.0f;
    } else if (!stop_of(1.0f, i, a, K, T, lnd, rule, L, M, pool, cptab, ell)) {
        w = 2.0f;
    } else {
        uint32_t lo = olo, hi = ohi; // stop(lo) false, stop(hi) true
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (stop_of(float_of(mid), i, a, K, T, lnd, rule, L, M, pool, cptab, ell))
                hi = mid;
            else
                lo = mid;
        }
        w = float_of(hi);
    }
    stopw[e] = w;
}

void launch_rule_tables(const double *lndeltas_dev, int32_t ndelta, double eps, int32_t rule, int32_t L,
                        int32_t M, int32_t K, int32_t G, int32_t pool, const double *cptab, int32_t ell,
                        float *tauv, float *stopw, hipStream_t s) {
    const int64_t total = 65 + (int64_t)ndelta * K * G * kTauCols;
    hipLaunchKernelGGL(k_rule_tables, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, lndeltas_dev, ndelta,
                       eps, rule, L, M, K, G, pool, cptab, ell, tauv, stopw);
    PF_HIP(hipGetLastError());
}

int32_t rule_table_cols() { return kTauCols; }

// 16 groups (about 5 to 8 tables each at the budgets measured): the test inside a level
// lets most queries stop before the level's end, and flushing the top-k 16 times per level
// costs little against a level's work
int32_t default_groups(int32_t L) { return L < 16 ? L : 16; }

int32_t test_entries_of(int32_t opt) { return opt == 0 ? 256 : (opt < 0 ? 0 : opt); }

} // namespace pf
