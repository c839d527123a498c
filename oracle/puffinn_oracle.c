/*
 * puffinn_oracle.c -- plain, slow CPU oracle for the adaptive k-NN query path of
 * PUFFINN (Aumueller, Christiani, Pagh, Vesterli; "PUFFINN: Parameterless and
 * Universally Fast FInding of Nearest Neighbors", ESA 2019).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  The GPU library never calls, links or
 * includes anything from here, and this file includes nothing from the GPU library.
 *
 * Every function below follows a passage of the paper; where the paper is silent or
 * ambiguous the reading taken is stated next to the code.  Floating point: hash
 * projections, norms, collision probabilities, the filter threshold and the stopping
 * bound are evaluated in FP64; the re-rank inner product is FP32 in one fixed
 * summation order (see oracle_ip32) so that an FP32 implementation can match it bit
 * for bit; an FP64 inner product is returned beside it for error reporting.
 *
 * Parity pins (what this code is checked against, in the CPU tests): the collision
 * probability 1 - theta/pi of random-hyperplane bits, the expected sketch Hamming
 * distance 64 theta/pi, textbook sorting, brute-force prefix counts, the B = 1 special
 * case of the segment rule, the closed-form solution of the stopping inequality, exact
 * k-NN in the linear-scan case (recall 1), the Higham error bound of the FP32 inner
 * product, and the per-neighbour guarantee of Lemma 1 measured over many index seeds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-3)

#define OR_RULE_FILTER 0 /* the bound of Lemma 1 with the sketch filter's misses included */
#define OR_RULE_EXACT 1  /* L * log1p(-p^i) <= ln(delta): the bound in the proof of Lemma 1 */
#define OR_RULE_ALG1 2   /* L >= ln(1/delta) / p^i: the test printed in Algorithm 1 */
#define OR_RULE_POOL 3   /* L p^i >= 2 and m >= 5 i^2 / p: Algorithm 3 (pooling, delta <= 1/2) */

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------------------
 * Random hyperplanes (Sec. 2.2, random-hyperplane LSH: every coordinate of a is an
 * independent standard normal).  The paper fixes no generator.  Both the oracle and
 * the GPU library implement the same published counter-based generator, SplitMix64
 * (Steele, Lea, Flood, OOPSLA 2014), each from its definition, feeding the Box-Muller
 * transform (Box, Muller 1958) in FP64:
 *   output s of the stream seeded with `seed` is mix(seed + (s+1) * 0x9E3779B97F4A7C15)
 *   element (r, c) of a d-column matrix uses t = r*d + c, outputs z1 = 2t, z2 = 2t+1
 *   u1 = ((z1 >> 11) + 1) * 2^-53 in (0,1],  u2 = (z2 >> 11) * 2^-53 in [0,1)
 *   a  = float( sqrt(-2 log u1) * cos(2 pi u2) )
 * ---------------------------------------------------------------------------------- */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t s) {
    uint64_t z = seed + (s + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void oracle_hyperplanes(uint64_t seed, int64_t rows, int32_t d, float *out) {
    for (int64_t r = 0; r < rows; ++r) {
        for (int32_t c = 0; c < d; ++c) {
            uint64_t t = (uint64_t)r * (uint64_t)d + (uint64_t)c;
            uint64_t z1 = oracle_splitmix64(seed, 2u * t);
            uint64_t z2 = oracle_splitmix64(seed, 2u * t + 1u);
            double u1 = ((double)(z1 >> 11) + 1.0) * 0x1.0p-53;
            double u2 = (double)(z2 >> 11) * 0x1.0p-53;
            double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
            out[r * (int64_t)d + c] = (float)g;
        }
    }
}

/* ------------------------------------------------------------------------------------
 * Vector storage (Sec. 4.2, "Vector storage"): every data and query vector is
 * normalised to unit length.  The squared norm is summed in FP64 in index order, the
 * square root and the division are FP64, and each quotient is rounded once to FP32.
 * Returns -1 when every row is usable, else the index of the first row whose norm is
 * zero or not finite (such a row has no direction, so it cannot be placed on the
 * sphere).
 * ---------------------------------------------------------------------------------- */
int64_t oracle_normalize(float *x, int64_t n, int32_t d) {
    for (int64_t i = 0; i < n; ++i) {
        float *row = x + i * (int64_t)d;
        double s = 0.0;
        for (int32_t c = 0; c < d; ++c) s += (double)row[c] * (double)row[c];
        double nrm = sqrt(s);
        if (!(nrm > 0.0) || !isfinite(nrm)) return i;
        for (int32_t c = 0; c < d; ++c) row[c] = (float)((double)row[c] / nrm);
    }
    return -1;
}

/* ------------------------------------------------------------------------------------
 * Index size (Sec. 1 and Sec. 5.2: the user gives only the memory the index may use,
 * and that size counts the data set and the hash functions).  Resident bytes:
 *   fixed     = 4 n d            (FP32 vectors) + 4 (64 M) d (sketch hyperplanes)
 *             + 4 m d            (with pooling: the m pool hyperplanes, shared)
 *   per table = 16 n             (u32 code, u32 position, u64 table-local sketch)
 *             + 4 (2^P + 1)      (prefix-position table, P = min(13, K))
 *             + 4 K d            (independent functions: the K hyperplanes of the table)
 *               or 4 K           (pooling: the indices of its K pool functions)
 *               or 3 c d' / 8    (FHT cross-polytope: c functions of three d'-bit sign vectors)
 * L = floor((budget - fixed) / per_table); 0 when the budget holds no table.
 * pool = m (0: independent functions, Alg. 1).
 * ---------------------------------------------------------------------------------- */
int32_t oracle_cp_dims(int32_t d, int32_t *dprime, int32_t *ell);

int64_t oracle_num_tables(int64_t n, int32_t d, int32_t K, int32_t M, int32_t pool, int32_t cp, uint64_t budget) {
    int32_t P = K < 13 ? K : 13;
    uint64_t fixed = 4ull * (uint64_t)n * (uint64_t)d + 4ull * 64ull * (uint64_t)M * (uint64_t)d +
                     4ull * (uint64_t)(pool > 0 ? pool : 0) * (uint64_t)d;
    uint64_t fn_bytes = pool > 0 ? 4ull * (uint64_t)K : 4ull * (uint64_t)K * (uint64_t)d;
    if (cp) {
        /* FHT cross-polytope: c = ceil(K / ell) functions, three sign vectors of d' bits each */
        int32_t dp, ell;
        oracle_cp_dims(d, &dp, &ell);
        fn_bytes = (uint64_t)((K + ell - 1) / ell) * 3ull * (uint64_t)dp / 8ull;
    }
    uint64_t per = 16ull * (uint64_t)n + 4ull * ((1ull << P) + 1ull) + fn_bytes;
    if (budget <= fixed) return 0;
    return (int64_t)((budget - fixed) / per);
}

/* ------------------------------------------------------------------------------------
 * Pooling (Sec. 3.2 "Pooling", App. B, Algorithm 3): a pool of m independent hash
 * functions is shared by the tries, and each trie independently samples a random
 * subset of K of them (without replacement).  sel[j*K + t] is the pool index of
 * h_{t+1,j}.  The draws come from the SplitMix64 stream seeded with seed + 1 (the
 * hyperplanes use the stream seeded with seed): for trie j a fresh array a = 0..m-1 is
 * shuffled by the first K steps of Fisher-Yates (Knuth's Algorithm P), step t taking
 * u = t + (z mod (m - t)) with z the output j*K + t, swapping a[t] and a[u], and
 * selecting a[t].  Returns OR_EINVAL when m < K.
 * ---------------------------------------------------------------------------------- */
int oracle_pool_select(uint64_t seed, int32_t pool, int32_t L, int32_t K, int32_t *sel) {
    if (pool < K || K < 1 || L < 1) return OR_EINVAL;
    int32_t *a = (int32_t *)malloc((size_t)pool * sizeof(int32_t));
    if (!a) return OR_ENOMEM;
    for (int32_t j = 0; j < L; ++j) {
        for (int32_t r = 0; r < pool; ++r) a[r] = r;
        for (int32_t t = 0; t < K; ++t) {
            const uint64_t z = oracle_splitmix64(seed + 1u, (uint64_t)j * (uint64_t)K + (uint64_t)t);
            const int32_t u = t + (int32_t)(z % (uint64_t)(pool - t));
            const int32_t tmp = a[t];
            a[t] = a[u];
            a[u] = tmp;
            sel[(int64_t)j * K + t] = a[t];
        }
    }
    free(a);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------
 * Hashing (Sec. 2.2): bit = 1 iff <a, x> >= 0.  The projection is the FP64 sum of the
 * (exact) FP64 products a_c * x_c taken in index order c = 0..d-1.
 * Layout of the hyperplane matrix: row j*K + (s-1) is h_{s,j} (s = 1..K) of table j;
 * rows L*K + 64 m + b are the bits b = 0..63 of sketch m (Sec. 4.2, "Filtering
 * candidate points": M sketches of 64 bits from random-hyperplane LSH).
 * Codes: the K-bit code of table j is the bitstring h_{1,j} .. h_{K,j} read with h_{1,j}
 * as its most significant bit (Sec. 4.2 views the hash code as a bitstring and sorts
 * it lexicographically, so the first function is the leading character).
 * Output layouts: codes[j][i] (u32), sketches[m][i] (u64, bit b = hyperplane b).
 * Four rows are accumulated side by side only to keep four independent FP64 chains in
 * flight; each row's sum is still the plain sequential one.
 * ---------------------------------------------------------------------------------- */
static double dot64(const float *a, const float *x, int32_t d) {
    double s = 0.0;
    for (int32_t c = 0; c < d; ++c) s += (double)a[c] * (double)x[c];
    return s;
}

/* projections of x onto the rows r0 .. r0+cnt-1 (cnt <= 4) of hp */
static void dot64_rows(const float *hp, int64_t r0, int cnt, const float *x, int32_t d, double *out) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const float *a0 = hp + r0 * d;
    const float *a1 = cnt > 1 ? a0 + d : a0, *a2 = cnt > 2 ? a0 + 2 * d : a0, *a3 = cnt > 3 ? a0 + 3 * d : a0;
    for (int32_t c = 0; c < d; ++c) {
        const double xc = (double)x[c];
        s0 += (double)a0[c] * xc;
        s1 += (double)a1[c] * xc;
        s2 += (double)a2[c] * xc;
        s3 += (double)a3[c] * xc;
    }
    out[0] = s0, out[1] = s1, out[2] = s2, out[3] = s3;
}

/* With pooling (sel != NULL) the hyperplane rows are the pool functions 0..pool-1, then
 * the sketch bits pool + 64 m + b, and bit s of table j is pool function sel[j*K + s-1]. */
void oracle_hash(const float *x, int64_t n, int32_t d, const float *hp, int32_t L, int32_t K,
                 int32_t M, const int32_t *sel, int32_t pool, uint32_t *codes, uint64_t *sketches) {
    const int64_t srow = sel ? (int64_t)pool : (int64_t)L * K;
    const int64_t rows = srow + 64 * (int64_t)M;
#pragma omp parallel
    {
        uint8_t *bit = (uint8_t *)malloc((size_t)rows);
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const float *xi = x + i * (int64_t)d;
            for (int64_t r = 0; r < rows; r += 4) {
                double p[4];
                const int cnt = rows - r < 4 ? (int)(rows - r) : 4;
                dot64_rows(hp, r, cnt, xi, d, p);
                for (int t = 0; t < cnt; ++t) bit[r + t] = p[t] >= 0.0;
            }
            for (int32_t j = 0; j < L; ++j) {
                uint32_t code = 0;
                for (int32_t s = 0; s < K; ++s) {
                    const int64_t row = sel ? (int64_t)sel[(int64_t)j * K + s] : (int64_t)j * K + s;
                    if (bit[row]) code |= 1u << (K - 1 - s);
                }
                codes[(int64_t)j * n + i] = code;
            }
            for (int32_t m = 0; m < M; ++m) {
                uint64_t sk = 0;
                for (int32_t b = 0; b < 64; ++b)
                    if (bit[srow + 64 * m + b]) sk |= 1ull << b;
                sketches[(int64_t)m * n + i] = sk;
            }
        }
        free(bit);
    }
}

/* ------------------------------------------------------------------------------------
 * Cross-polytope LSH with the pseudorandom rotation of three Hadamard transforms (Sec.
 * 2.2; Sec. 4.3 "Supported LSH Functions"; Andoni et al. 2015).  A function rotates x,
 * zero padded to d' = the smallest power of two >= d, by y = H D3 H D2 H D1 x (H the
 * Walsh-Hadamard matrix, unnormalised -- scaling does not move the argmax; D_k random
 * +-1 diagonals) and maps it to the closest of the 2d' signed basis vectors: index
 * i = argmax |y_i| (the smallest i on ties) and sign s = [y_i < 0].  Its value is the
 * ell = log2(2 d')-bit string v = s d' + i, the sign as the most significant bit (a
 * reading: the paper drops the last bit when the prefix shrinks; with the sign last,
 * antipodal points would collide once the sign is dropped and the collision
 * probability would not grow with similarity, which the stopping argument needs).
 * A table's K-bit code is the first K bits of the concatenation of its c = ceil(K/ell)
 * functions' values, function 1 first.
 * Signs: D_k[c] of function fn is -1 when the top bit of output (3 fn + k) d' + c of the
 * SplitMix64 stream seeded with sseed is set; the index uses seed + 3 (fn = j c + f for
 * function f of table j) and the Monte Carlo tables seed + 2.
 * The transform is FP64: butterflies for h = 1, 2, 4, ... replace (y[j], y[j+h]), bit h of
 * j clear, by (a + b, a - b) -- one fixed set of operations, so a GPU following it gets
 * the same bits.
 * ---------------------------------------------------------------------------------- */
#define OR_CP_GRID 41 /* tabulated similarities alpha_g = -1 + 0.05 g, g = 0..40 */

int32_t oracle_cp_dims(int32_t d, int32_t *dprime, int32_t *ell) {
    int32_t dp = 1, l = 1;
    while (dp < d) dp <<= 1, ++l;
    if (dprime) *dprime = dp;
    if (ell) *ell = l; /* log2(2 dp) */
    return dp;
}

static void fht64(double *y, int32_t dp) {
    for (int32_t h = 1; h < dp; h <<= 1)
        for (int32_t j = 0; j < dp; ++j)
            if (!(j & h)) {
                const double a = y[j], b = y[j + h];
                y[j] = a + b;
                y[j + h] = a - b;
            }
}

static uint32_t cp_value(const float *x, int32_t d, int32_t dp, uint64_t sseed, uint64_t fn, double *y) {
    for (int32_t c = 0; c < dp; ++c) y[c] = c < d ? (double)x[c] : 0.0;
    for (int32_t k = 0; k < 3; ++k) {
        for (int32_t c = 0; c < dp; ++c)
            if (oracle_splitmix64(sseed, (fn * 3u + (uint64_t)k) * (uint64_t)dp + (uint64_t)c) >> 63) y[c] = -y[c];
        fht64(y, dp);
    }
    int32_t best = 0;
    for (int32_t c = 1; c < dp; ++c)
        if (fabs(y[c]) > fabs(y[best])) best = c;
    return (uint32_t)((y[best] < 0.0 ? dp : 0) + best);
}

/* value of CP function fn (stream seed + 3) at x; exported for the tests */
uint32_t oracle_cp_value(const float *x, int32_t d, uint64_t seed, uint64_t fn) {
    int32_t dp;
    oracle_cp_dims(d, &dp, NULL);
    double *y = (double *)malloc((size_t)dp * sizeof(double));
    const uint32_t v = cp_value(x, d, dp, seed + 3u, fn, y);
    free(y);
    return v;
}

/* codes[j][i] of the rows x under FHT-CP tables (K-bit codes, see above) */
void oracle_cp_hash(const float *x, int64_t n, int32_t d, uint64_t seed, int32_t L, int32_t K, uint32_t *codes) {
    int32_t dp, ell;
    oracle_cp_dims(d, &dp, &ell);
    const int32_t c = (K + ell - 1) / ell;
#pragma omp parallel
    {
        double *y = (double *)malloc((size_t)dp * sizeof(double));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            for (int32_t j = 0; j < L; ++j) {
                uint64_t cat = 0;
                for (int32_t f = 0; f < c; ++f)
                    cat = (cat << ell) | cp_value(x + i * (int64_t)d, d, dp, seed + 3u, (uint64_t)j * c + f, y);
                codes[(int64_t)j * n + i] = (uint32_t)(cat >> (c * ell - K));
            }
        }
        free(y);
    }
}

/* Monte Carlo collision table (Sec. 4.3 "Estimating Collision Probabilities"): for each
 * alpha_g the pair x = e_1, y = (alpha, sqrt(1 - alpha^2), 0, ...) is hashed by R random
 * functions (stream seed + 2, fn = 0..R-1) and tab[g][b] is the fraction whose values
 * agree in their first b bits (tab[g][0] = 1).  The estimate is then made non-decreasing
 * in alpha by taking, at each g, the minimum over all g' >= g (a lower bound is what the
 * stopping rule needs, and the rule's argument needs monotonicity). */
void oracle_cp_table(uint64_t seed, int32_t d, int32_t R, double *tab) {
    int32_t dp, ell;
    oracle_cp_dims(d, &dp, &ell);
    float *px = (float *)calloc((size_t)dp, sizeof(float)), *py = (float *)calloc((size_t)dp, sizeof(float));
    double *y = (double *)malloc((size_t)dp * sizeof(double));
    for (int32_t g = 0; g < OR_CP_GRID; ++g) {
        const double alpha = -1.0 + 0.05 * (double)g;
        px[0] = 1.0f;
        py[0] = (float)alpha;
        py[1] = (float)sqrt(fmax(0.0, 1.0 - alpha * alpha));
        double *row = tab + (int64_t)g * (ell + 1);
        int64_t cnt[33] = {0};
        for (int32_t r = 0; r < R; ++r) {
            const uint32_t vx = cp_value(px, dp, dp, seed + 2u, (uint64_t)r, y);
            const uint32_t vy = cp_value(py, dp, dp, seed + 2u, (uint64_t)r, y);
            for (int32_t b = 1; b <= ell; ++b)
                if ((vx >> (ell - b)) == (vy >> (ell - b))) ++cnt[b];
        }
        row[0] = 1.0;
        for (int32_t b = 1; b <= ell; ++b) row[b] = (double)cnt[b] / (double)R;
    }
    for (int32_t g = OR_CP_GRID - 2; g >= 0; --g)
        for (int32_t b = 0; b <= ell; ++b) {
            double *a = tab + (int64_t)g * (ell + 1), *up = tab + (int64_t)(g + 1) * (ell + 1);
            if (up[b] < a[b]) a[b] = up[b];
        }
    free(px), free(py), free(y);
}

/* Collision probability of an i-bit prefix at inner product ip under FHT-CP: the
 * similarity is rounded down to the grid (g = floor((ip + 1) * 20), clamped to 0..40,
 * FP64), and with i = a ell + b the a whole functions and the first b bits of the next
 * one must agree: P = tab[g][ell]^a * tab[g][b], the power as exp(a log tab). */
double oracle_cp_prob(const double *tab, int32_t ell, float ip, int32_t i) {
    double gv = floor(((double)ip + 1.0) * 20.0);
    int32_t g = gv < 0.0 ? 0 : (gv > 40.0 ? 40 : (int32_t)gv);
    const double *row = tab + (int64_t)g * (ell + 1);
    const int32_t a = i / ell, b = i % ell;
    const double full = a > 0 ? exp((double)a * log(row[ell])) : 1.0;
    return full * row[b];
}

/* ------------------------------------------------------------------------------------
 * LSH forest as sorted arrays (Sec. 4.1 and Sec. 4.2, "Retrieving candidate points"):
 * repetition j is the array of (code, position) pairs sorted by code.  Equal codes
 * are ordered by position (the paper leaves ties open; this makes the array unique).
 * The prefix-position table (13-bit prefixes tabulated to speed up the search):
 *   off[j][p] = number of entries whose leading P bits are < p, p = 0..2^P.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    uint32_t code;
    uint32_t pos;
} or_pair;

static int cmp_pair(const void *a, const void *b) {
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return 0;
}

int oracle_build_tables(const uint32_t *codes, int64_t n, int32_t L, int32_t K, uint32_t *tcode,
                        uint32_t *tidx, uint32_t *off) {
    int32_t P = K < 13 ? K : 13;
    int64_t np = (int64_t)1 << P;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < L; ++j) {
        or_pair *v = (or_pair *)malloc((size_t)n * sizeof(or_pair));
        if (!v) {
            err = 1;
            continue;
        }
        for (int64_t i = 0; i < n; ++i) {
            v[i].code = codes[(int64_t)j * n + i];
            v[i].pos = (uint32_t)i;
        }
        qsort(v, (size_t)n, sizeof(or_pair), cmp_pair);
        for (int64_t e = 0; e < n; ++e) {
            tcode[(int64_t)j * n + e] = v[e].code;
            tidx[(int64_t)j * n + e] = v[e].pos;
        }
        free(v);
        uint32_t *o = off + (int64_t)j * (np + 1);
        int64_t *cnt = (int64_t *)calloc((size_t)np, sizeof(int64_t));
        if (!cnt) {
            err = 1;
            continue;
        }
        for (int64_t e = 0; e < n; ++e) cnt[tcode[(int64_t)j * n + e] >> (K - P)]++;
        int64_t run = 0;
        for (int64_t p = 0; p < np; ++p) {
            o[p] = (uint32_t)run;
            run += cnt[p];
        }
        o[np] = (uint32_t)run;
        free(cnt);
    }
    return err ? OR_ENOMEM : OR_OK;
}

/* Sketch chosen for repetition j: Sec. 4.2 ("Filtering candidate points") lets each
 * repetition pick one of the M sketches by a fixed scrambling of its index.  The sketch
 * hyperplanes are independent, so any fixed map is equivalent in distribution; this
 * oracle takes sigma(j) = j mod M and stores, per table, the sketch of each sorted entry. */
void oracle_table_sketches(const uint32_t *tidx, const uint64_t *sketches, int64_t n, int32_t L,
                           int32_t M, uint64_t *tsk) {
    for (int32_t j = 0; j < L; ++j) {
        const uint64_t *s = sketches + (int64_t)(j % M) * n;
        for (int64_t e = 0; e < n; ++e) tsk[(int64_t)j * n + e] = s[tidx[(int64_t)j * n + e]];
    }
}

/* ------------------------------------------------------------------------------------
 * Re-rank inner product (Sec. 4.2, "Computing distances": the exact distance of every
 * candidate that passes the filter).  On unit vectors the inner product orders
 * neighbours (Sec. 2.2, angular distance).  FP32, one fixed order so that results are
 * reproducible bit for bit by any FP32 implementation that follows it:
 *   partial r (r = 0..15) sums the FP32-rounded products x_i*q_i over the indices
 *   i = 64t + 4r + c (t >= 0, c = 0..3, i < d) in increasing i, every add rounded to
 *   FP32 and no fused multiply-add; then s_r <- s_r + s_{r xor h} for h = 8, 4, 2, 1
 *   (all r at once), and the result is s_0.
 * ---------------------------------------------------------------------------------- */
float oracle_ip32(const float *x, const float *q, int32_t d) {
    float s[16], t[16];
    for (int r = 0; r < 16; ++r) s[r] = 0.0f;
    for (int32_t i = 0; i < d; ++i) {
        int r = (i & 63) >> 2;
        float prod = x[i] * q[i];
        s[r] = s[r] + prod;
    }
    for (int h = 8; h >= 1; h >>= 1) {
        for (int r = 0; r < 16; ++r) t[r] = s[r] + s[r ^ h];
        for (int r = 0; r < 16; ++r) s[r] = t[r];
    }
    return s[0];
}

double oracle_ip64(const float *x, const float *q, int32_t d) { return dot64(x, q, d); }

/* ------------------------------------------------------------------------------------
 * Collision probability of random-hyperplane LSH at inner product ip (Sec. 4.3 notes a
 * closed form exists; it is Charikar's p = 1 - theta/pi, theta = arccos(ip)), FP64.
 * ---------------------------------------------------------------------------------- */
static double clamp1(double v) { return v > 1.0 ? 1.0 : (v < -1.0 ? -1.0 : v); }

double oracle_collision_prob(float ip) { return 1.0 - acos(clamp1((double)ip)) / OR_PI; }

/* Filter threshold (Sec. 4.2 "Filtering candidate points" and Sec. 5.1): a candidate
 * passes when the Hamming distance of its sketch to the query's sketch is at most
 * tau = (1 + eps) * (expected Hamming distance at the current k-th inner product).
 * The expected distance of 64 random-hyperplane bits at angle theta is
 * 64 * Pr[bits differ] = 64 theta / pi.  (The paper's footnote says "collide"; with
 * that reading near neighbours would get tau near 64 and nothing would be filtered,
 * so the differ-probability is taken.)  eps = 0 is the paper's setting. */
double oracle_tau(float ip_k, double eps) {
    return (1.0 + eps) * 64.0 * acos(clamp1((double)ip_k)) / OR_PI;
}

/* Probability that two points at angle theta = t * pi pass the sketch filter, i.e. that
 * the Hamming distance of their 64-bit sketches (a Binomial(64, t) variable, each
 * random-hyperplane bit differing with probability t) is at most T:
 *   sum_{h=0..T} C(64,h) t^h (1-t)^(64-h),
 * with C(64,h) built by the recurrence C(64,h+1) = C(64,h) (64-h)/(h+1) in FP64. */
double oracle_binom_cdf64(double t, int32_t T) {
    if (T < 0) return 0.0;
    if (T >= 64 || t <= 0.0) return 1.0;
    if (t >= 1.0) return 0.0;
    const double lt = log(t), l1t = log1p(-t);
    double c = 1.0, s = 0.0;
    for (int32_t h = 0; h <= T; ++h) {
        s += c * exp((double)h * lt + (double)(64 - h) * l1t);
        c = c * (double)(64 - h) / (double)(h + 1);
    }
    return s < 1.0 ? s : 1.0;
}

/* Stopping test once the first a of the L repetitions have taken level i's entries and
 * the other L - a are still at level i + 1 (none taken yet when i = K); a = L is the test
 * after all repetitions of the level have been inspected (Sec. 4.1), a < L the test that
 * Algorithm 1 makes after each repetition j = a.  Each repetition contributes the
 * collision probability of its own prefix length: p^i for the first a, p^(i+1) for the
 * rest (the windows of Lemma 1's proof are independent across repetitions).
 * OR_RULE_EXACT stops when the failure bound of Lemma 1's proof, (1 - p^i)^L, is at
 * most delta, evaluated as L * log1p(-p^i) <= ln(delta) with ln p = log1p(-theta/pi)
 * and p^i = exp(i ln p).  OR_RULE_ALG1 stops when L >= ln(1/delta) / p^i, the test
 * written in Algorithm 1 (it implies the exact bound, so it never stops earlier).
 * OR_RULE_FILTER extends the bound to the sketch filter (Sec. 4.2), which the proof
 * of Lemma 1 does not cover: a true neighbour x (angle <= theta_k) is missed only if,
 * for every sketch s, either x's sketch s fails the filter or none of the g_s tables
 * reading sketch s (tables j with j mod M = s) holds x in its window at level i.  Table
 * windows and sketches use independent hyperplanes; the threshold never grows from
 * level to level, so x passes sketch s with probability at least
 * q = P[Binomial(64, theta_k/pi) <= T], T the integer threshold of level i.  Hence the
 * failure probability is at most prod_s (1 - q + q (1 - p^i)^{g_s}).  Each factor is
 * evaluated without cancellation: with a = g_s log1p(-p^i) and x = q expm1(a), the log
 * of the factor is log1p(x) when x > -1/2, else log((1 - q) + q exp(a)) (two
 * non-negative terms).  The test is sum_s log(factor_s) <= ln(delta).  With q = 1 (no
 * filtering) this is the exact rule.
 * OR_RULE_POOL is the test of Algorithm 3 (pooling; App. B proves failure probability at
 * most 1/2 with it, for any delta): after all L tries, stop when the expected number of
 * collisions with the k-th neighbour is at least two, L p^i >= 2, and the pool is large
 * enough for Cantelli's inequality, pool >= 5 i^2 / p (evaluated as pool p >= 5 i^2).
 * delta is not used.  With FHT cross-polytope codes (cptab != NULL) p^i is replaced by
 * the tabulated collision probability of the i-bit prefix (oracle_cp_prob); the filter's
 * q stays the hyperplane sketches' own.  *margin receives the signed distance of the two sides (term -
 * threshold; for OR_RULE_POOL minus the smaller of the two slacks), <= 0 to stop. */
int oracle_stop_partial(float ip_k, int32_t i, int32_t a, int32_t L, int32_t M, int32_t K, double delta,
                        int32_t rule, int32_t tau_int, int32_t pool, const double *cptab, int32_t ell,
                        double *margin) {
    double theta = acos(clamp1((double)ip_k));
    double lnp = log1p(-theta / OR_PI);
    /* collision probability of an i-bit prefix: p^i for hyperplane bits, the Monte Carlo
       table for FHT cross-polytope codes (cptab != NULL) */
    double pi_ = cptab ? oracle_cp_prob(cptab, ell, ip_k, i) : exp((double)i * lnp);
    /* the tables after the first a are at level i + 1 (nothing taken yet when i = K) */
    const int32_t rest = L - a;
    const int deeper = rest > 0 && i < K;
    double pi1 = 0.0;
    if (deeper) pi1 = cptab ? oracle_cp_prob(cptab, ell, ip_k, i + 1) : exp((double)(i + 1) * lnp);
    double lnd = log(delta);
    if (rule == OR_RULE_POOL) {
        /* Algorithm 3's test counts the tries inspected at the current prefix length */
        const double p = 1.0 - theta / OR_PI;
        const double sa = (double)a * pi_ - 2.0, sb = (double)pool * p - 5.0 * (double)i * (double)i;
        const double slack = sa < sb ? sa : sb;
        if (margin) *margin = -slack;
        return slack >= 0.0;
    }
    if (rule == OR_RULE_ALG1) {
        /* Algorithm 1's test with j = a repetitions done at prefix length i: j p^i >= -ln(delta) */
        double lhs = (double)a * pi_;
        if (margin) *margin = -lnd - lhs;
        return lhs >= -lnd;
    }
    const double l1p = log1p(-pi_), l1p1 = deeper ? log1p(-pi1) : 0.0;
    if (rule == OR_RULE_FILTER) {
        const double q = oracle_binom_cdf64(theta / OR_PI, tau_int);
        double term = 0.0;
        for (int32_t s = 0; s < M && s < L; ++s) {
            /* tables j = s, s + M, ... read sketch s: those below a are at level i */
            const int32_t g = L / M + (s < L % M ? 1 : 0);
            const int32_t gi = a / M + (s < a % M ? 1 : 0);
            /* (a count of zero contributes nothing, also where log1p(-p^l) = -inf at p = 1) */
            const double e = (gi > 0 ? (double)gi * l1p : 0.0) + (g - gi > 0 ? (double)(g - gi) * l1p1 : 0.0);
            const double x = q * expm1(e);
            term += (x > -0.5) ? log1p(x) : log((1.0 - q) + q * exp(e));
        }
        if (margin) *margin = term - lnd;
        return term <= lnd;
    }
    double term = (a > 0 ? (double)a * l1p : 0.0) + (rest > 0 ? (double)rest * l1p1 : 0.0);
    if (margin) *margin = term - lnd;
    return term <= lnd;
}

int oracle_stop(float ip_k, int32_t i, int32_t L, int32_t M, double delta, int32_t rule,
                int32_t tau_int, int32_t pool, const double *cptab, int32_t ell, double *margin) {
    return oracle_stop_partial(ip_k, i, L, L, M, i, delta, rule, tau_int, pool, cptab, ell, margin);
}

/* ------------------------------------------------------------------------------------
 * The adaptive query (Algorithm 1, adaptive-kNN(q, k, delta), realised on sorted arrays
 * as in Sec. 4.1-4.2).  Readings taken where the paper leaves freedom:
 *  - rounds are level-synchronous: in level i every repetition j = 1..L contributes its
 *    new entries, with the stopping test after each of `groups` consecutive groups of
 *    repetitions (once per level, as in Sec. 4.1, when groups = 1); with test_entries =
 *    T > 0 the test after a group is taken only when at least T entries were read since
 *    the level's previous test, or the group is the level's last; groups without entries
 *    that directly follow a tested group are tested with it (they add nothing, so the
 *    k-th inner product is the same).  T = 0 tests after every group;
 *  - the filter threshold tau_i is fixed for the whole level from the top-k as it stood
 *    before the level (64, i.e. no filtering, while fewer than k points are known);
 *  - retrieval (Sec. 4.2 and App. C): per repetition a consumed window [c_lo, c_hi)
 *    starts empty at the insertion point of the query's code; at level i it grows by
 *    whole segments of B entries to the left while the entry just left of it shares the
 *    query's i-bit prefix, and to the right likewise, clipped to [0, n).  B = 1 gives
 *    exactly the sets Pi_{i,j}(q) of Sec. 3.1;
 *  - every entry that passes the filter has its distance computed and enters the
 *    accumulator (Sec. 4.1), which de-duplicates (Sec. 4.2, "Computing distances"): the
 *    top-k holds distinct points, a point seen in several repetitions counts once;
 *  - the top-k is ordered by (inner product descending, position ascending);
 *  - level 0 is a linear scan (Lemma 1: at i = 0 the query degrades to a linear scan):
 *    every point is re-ranked, unfiltered, and the exact top-k is returned.
 * Counters: c_scan = entries taken from the arrays, c_pass = entries that passed the
 * filter (with multiplicity), c_rerank = distance computations (c_pass, plus n when
 * the linear scan runs).
 * ---------------------------------------------------------------------------------- */
typedef struct {
    float ip;
    double ip64;
    int32_t id;
} or_cand;

static int cmp_cand(const void *a, const void *b) {
    const or_cand *x = (const or_cand *)a, *y = (const or_cand *)b;
    if (x->ip > y->ip) return -1;
    if (x->ip < y->ip) return 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

typedef struct {
    or_cand *v;
    int64_t len, cap;
} or_list;

static int list_push(or_list *l, or_cand c) {
    if (l->len == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 1024;
        or_cand *nv = (or_cand *)realloc(l->v, (size_t)nc * sizeof(or_cand));
        if (!nv) return OR_ENOMEM;
        l->v = nv;
        l->cap = nc;
    }
    l->v[l->len++] = c;
    return OR_OK;
}

/* number of entries of the sorted array tc[0..n) whose leading i bits (of K) are
 * smaller than those of the query code qc (below = 1) or at most those (below = 0) */
static int64_t prefix_bound(const uint32_t *tc, int64_t n, int32_t K, int32_t i, uint32_t qc,
                            int below) {
    uint64_t qp = (uint64_t)qc >> (K - i);
    int64_t lo = 0, hi = n; /* first e with pre(tc[e]) >= qp (below) or > qp (!below) */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        uint64_t ep = (uint64_t)tc[mid] >> (K - i);
        int go_right = below ? (ep < qp) : (ep <= qp);
        if (go_right)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

typedef struct {
    const float *points;
    int64_t n;
    int32_t d;
    const uint32_t *tcode, *tidx;
    const uint64_t *tsk;
    int32_t L, K, M;
    int32_t pool; /* pool size m for OR_RULE_POOL (0: independent functions) */
    const double *cptab; /* FHT cross-polytope collision table (NULL: hyperplane codes) */
    int32_t ell;
} or_index;

/* trace (optional, one query): per level i (row i of K+1) and table j:
 * [0] lo_i [1] hi_i [2] c_lo after level i [3] c_hi after level i
 * ltrace (optional, the same query): per level i, row i of K+1 rows of OR_LT_W int64:
 * [0] the filter threshold the level used (64: no filtering), -2 when the level was not
 *     reached, -1 for the linear scan; [1] the set of point ids among the level's new
 *     entries, [2] the set among those that passed the filter, [6] the set of the top-k
 *     after the level, each as a bit mask (bit x for point x; meaningful for n <= 64);
 *     [3] c_scan, [4] c_pass, [5] c_rerank after the level; [7] 1 when the query stopped
 *     there. */
#define OR_LT_W 8
/* bit x of a trace mask (x < 64), formed unsigned so that bit 63 is no signed overflow */
static int64_t or_bit(int64_t x) { return (int64_t)((uint64_t)1 << x); }
/* top <- best k distinct points of top u fresh (the accumulator's flush): sort by
 * (ip desc, id asc); copies of one point carry the same inner product, so they are
 * adjacent and all but the first are dropped. */
static int accumulate(or_list *top, const or_list *fresh, int32_t k) {
    for (int64_t t = 0; t < fresh->len; ++t)
        if (list_push(top, fresh->v[t])) return OR_ENOMEM;
    if (top->len > 1) /* (an empty list may have no storage yet: qsort needs a non-null array) */
        qsort(top->v, (size_t)top->len, sizeof(or_cand), cmp_cand);
    int64_t w = 0;
    for (int64_t t = 0; t < top->len && w < k; ++t)
        if (w == 0 || top->v[t].id != top->v[w - 1].id) top->v[w++] = top->v[t];
    top->len = w;
    return OR_OK;
}

static int walk_one(const or_index *ix, const float *q, const uint32_t *qcode, const uint64_t *qsk,
                    int32_t k, double delta, double eps, int32_t B, int32_t rule, int32_t filter_on,
                    int32_t groups, int32_t test_entries, int64_t *clo, int64_t *chi, or_list *top,
                    or_list *fresh,
                    int32_t *stop_level, int64_t *cnt, int32_t *boundary, int64_t *trace,
                    int64_t *ltrace) {
    const int64_t n = ix->n;
    const int32_t L = ix->L, K = ix->K, d = ix->d;
    top->len = 0;
    cnt[0] = cnt[1] = cnt[2] = 0;
    *boundary = 0;
    if (ltrace)
        for (int32_t i = 0; i <= K; ++i) {
            memset(ltrace + (int64_t)i * OR_LT_W, 0, OR_LT_W * sizeof(int64_t));
            ltrace[(int64_t)i * OR_LT_W] = -2;
        }
    for (int32_t j = 0; j < L; ++j) {
        int64_t lk = prefix_bound(ix->tcode + (int64_t)j * n, n, K, K, qcode[j], 1);
        clo[j] = chi[j] = lk;
    }
    for (int32_t i = K; i >= 1; --i) {
        /* threshold fixed for the level, from the top-k before it */
        double tau = 64.0;
        int32_t tau_int = 64;
        if (filter_on && top->len == k) {
            tau = oracle_tau(top->v[k - 1].ip, eps);
            double fr = tau - floor(tau);
            if (fr < 1e-9 || fr > 1.0 - 1e-9) *boundary = 1;
            tau_int = tau >= 64.0 ? 64 : (tau < -1.0 ? -1 : (int32_t)floor(tau));
        }
        int64_t *lt = ltrace ? ltrace + (int64_t)i * OR_LT_W : NULL;
        if (lt) lt[0] = tau_int;
        /* the repetitions in `groups` consecutive groups; the stopping test after a group
           once test_entries entries were read since the level's previous test (always after
           the last group, and after a group without entries that follows a tested one) */
        int64_t since = 0;
        int prev_tested = 0;
        for (int32_t gi = 0; gi < groups; ++gi) {
        const int32_t j0 = (int32_t)((int64_t)gi * L / groups), j1 = (int32_t)((int64_t)(gi + 1) * L / groups);
        const int64_t scanned_before = cnt[0];
        fresh->len = 0;
        for (int32_t j = j0; j < j1; ++j) {
            const uint32_t *tc = ix->tcode + (int64_t)j * n;
            const uint32_t *ti = ix->tidx + (int64_t)j * n;
            const uint64_t *ts = ix->tsk + (int64_t)j * n;
            const uint64_t qs = qsk[j % ix->M];
            int64_t lo_i = prefix_bound(tc, n, K, i, qcode[j], 1);
            int64_t hi_i = prefix_bound(tc, n, K, i, qcode[j], 0);
            if (trace) {
                trace[((int64_t)i * L + j) * 4 + 0] = lo_i;
                trace[((int64_t)i * L + j) * 4 + 1] = hi_i;
            }
            /* new entries of this repetition at this level: whole segments outward */
            int64_t seg[2][2];
            int nseg = 0;
            if (clo[j] > lo_i) {
                int64_t a = clo[j];
                while (a > lo_i) a = a - B > 0 ? a - B : 0;
                seg[nseg][0] = a;
                seg[nseg][1] = clo[j];
                ++nseg;
                clo[j] = a;
            }
            if (chi[j] < hi_i) {
                int64_t b = chi[j];
                while (b < hi_i) b = b + B < n ? b + B : n;
                seg[nseg][0] = chi[j];
                seg[nseg][1] = b;
                ++nseg;
                chi[j] = b;
            }
            if (trace) {
                trace[((int64_t)i * L + j) * 4 + 2] = clo[j];
                trace[((int64_t)i * L + j) * 4 + 3] = chi[j];
            }
            for (int s = 0; s < nseg; ++s) {
                for (int64_t e = seg[s][0]; e < seg[s][1]; ++e) {
                    cnt[0]++;
                    int h = __builtin_popcountll(ts[e] ^ qs);
                    if (lt && ti[e] < 64) lt[1] |= or_bit(ti[e]);
                    if ((double)h > tau) continue;
                    cnt[1]++;
                    cnt[2]++;
                    uint32_t x = ti[e];
                    if (lt && x < 64) lt[2] |= or_bit(x);
                    const float *px = ix->points + (int64_t)x * d;
                    or_cand c = {oracle_ip32(px, q, d), oracle_ip64(px, q, d), (int32_t)x};
                    if (list_push(fresh, c)) return OR_ENOMEM;
                }
            }
        }
        if (accumulate(top, fresh, k)) return OR_ENOMEM;
        const int64_t read = cnt[0] - scanned_before;
        since += read;
        const int tested = since >= test_entries || gi == groups - 1 || (read == 0 && prev_tested);
        prev_tested = tested;
        if (!tested) continue;
        since = 0;
        if (lt) {
            lt[3] = cnt[0], lt[4] = cnt[1], lt[5] = cnt[2];
            for (int64_t t = 0; t < top->len; ++t)
                if (top->v[t].id < 64) lt[6] |= or_bit(top->v[t].id);
        }
        if (top->len == k) {
            double margin;
            int stop = oracle_stop_partial(top->v[k - 1].ip, i, j1, L, ix->M, K, delta, rule, tau_int, ix->pool,
                                           ix->cptab, ix->ell, &margin);
            if (fabs(margin) < 1e-9 * (1.0 + fabs(log(delta)))) *boundary = 1;
            if (ix->cptab) {
                /* the table lookup changes cell at grid points of the similarity */
                const double gv = ((double)top->v[k - 1].ip + 1.0) * 20.0;
                if (fabs(gv - floor(gv + 0.5)) < 1e-9) *boundary = 1;
            }
            if (stop) {
                *stop_level = i;
                if (lt) lt[7] = 1;
                return OR_OK;
            }
        }
        }
    }
    /* level 0: linear scan, every point re-ranked */
    fresh->len = 0;
    for (int64_t x = 0; x < n; ++x) {
        cnt[2]++;
        const float *px = ix->points + x * d;
        or_cand c = {oracle_ip32(px, q, d), oracle_ip64(px, q, d), (int32_t)x};
        if (list_push(fresh, c)) return OR_ENOMEM;
    }
    if (accumulate(top, fresh, k)) return OR_ENOMEM;
    if (ltrace) {
        int64_t *lt = ltrace;
        lt[0] = -1;
        for (int64_t x = 0; x < n && x < 64; ++x) lt[1] |= or_bit(x);
        lt[2] = lt[1];
        lt[3] = cnt[0], lt[4] = cnt[1], lt[5] = cnt[2];
        for (int64_t t = 0; t < top->len; ++t)
            if (top->v[t].id < 64) lt[6] |= or_bit(top->v[t].id);
        lt[7] = 1;
    }
    *stop_level = 0;
    return OR_OK;
}

/* Search m queries.  `queries` are raw rows (normalised here), `points` are the
 * normalised data rows, hp the hyperplanes, (tcode, tidx, tsk) the L sorted tables.
 * recall in (0,1] gives delta = 1 - recall (Sec. 2.1: expected recall (1 - delta)).
 * sel / pool: the tries' pool functions (NULL / 0 for independent functions); pool is
 * also the m of OR_RULE_POOL.  cptab != NULL: FHT cross-polytope codes with seed cp_seed
 * and that collision table (hp then holds the sketch hyperplanes only).
 * Outputs per query: ids[k], ips[k] (FP32 order above), ips64[k], stop level, the three
 * counters, and boundary = 1 when a decision came within 1e-9 of flipping (a test of an
 * FP32 ip against an FP64 threshold computed with a different libm may then differ).
 * trace (nullable) records the walk of query 0 only: (K+1) x L x 4 int64; ltrace
 * (nullable) the same query's levels, (K+1) x OR_LT_W int64 (see walk_one).
 * groups (1..L): the repetitions of a level are taken in `groups` consecutive groups,
 * group g holding repetitions floor(g L / groups) .. floor((g+1) L / groups) - 1, and the
 * stopping test (oracle_stop_partial, a = the repetitions done) runs after each group: 1
 * is the test once per level of Sec. 4.1, L the test after every repetition of
 * Algorithm 1.  test_entries (>= 0): a group's test is skipped while fewer entries than
 * that were read since the level's previous test (see walk_one; 0 tests after every
 * group).  The filter threshold stays fixed for the whole level.
 * Returns 0, OR_EINVAL (bad arguments or a zero / non-finite query row), OR_ENOMEM. */
int oracle_search(const float *points, int64_t n, int32_t d, const float *hp, const uint32_t *tcode,
                  const uint32_t *tidx, const uint64_t *tsk, int32_t L, int32_t K, int32_t M,
                  const int32_t *sel, int32_t pool, const double *cptab, uint64_t cp_seed,
                  const float *queries, int64_t m, int32_t k, double recall, double eps, int32_t B,
                  int32_t rule, int32_t filter_on, int32_t groups, int32_t test_entries, int32_t *ids, float *ips,
                  double *ips64, int32_t *stop_level, int64_t *c_scan, int64_t *c_pass, int64_t *c_rerank,
                  int32_t *boundary, int64_t *trace, int64_t *ltrace) {
    if (n < 1 || d < 1 || L < 1 || K < 1 || K > 32 || M < 1 || m < 0 || k < 1 || k > n || B < 1 || groups < 1 ||
        groups > L || test_entries < 0)
        return OR_EINVAL;
    if (rule == OR_RULE_POOL && (pool < 1 || cptab)) return OR_EINVAL;
    if (!(recall > 0.0 && recall <= 1.0)) return OR_EINVAL;
    float *qn = (float *)malloc((size_t)(m > 0 ? m : 1) * (size_t)d * sizeof(float));
    uint32_t *qc = (uint32_t *)malloc((size_t)(m > 0 ? m : 1) * (size_t)L * sizeof(uint32_t));
    uint64_t *qs = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * (size_t)M * sizeof(uint64_t));
    if (!qn || !qc || !qs) {
        free(qn), free(qc), free(qs);
        return OR_ENOMEM;
    }
    memcpy(qn, queries, (size_t)m * (size_t)d * sizeof(float));
    if (oracle_normalize(qn, m, d) >= 0) {
        free(qn), free(qc), free(qs);
        return OR_EINVAL;
    }
    /* query codes: table-major like the data codes */
    int32_t ell = 0;
    if (cptab) {
        /* FHT cross-polytope codes; hp then holds only the 64 M sketch hyperplanes */
        oracle_cp_dims(d, NULL, &ell);
        oracle_cp_hash(qn, m, d, cp_seed, L, K, qc);
        oracle_hash(qn, m, d, hp, 0, K, M, NULL, 0, NULL, qs);
    } else {
        oracle_hash(qn, m, d, hp, L, K, M, sel, pool, qc, qs);
    }
    or_index ix = {points, n, d, tcode, tidx, tsk, L, K, M, pool, cptab, ell};
    const double delta = 1.0 - recall;
    int err = OR_OK;
#pragma omp parallel
    {
        int64_t *clo = (int64_t *)malloc((size_t)L * sizeof(int64_t));
        int64_t *chi = (int64_t *)malloc((size_t)L * sizeof(int64_t));
        uint32_t *mycode = (uint32_t *)malloc((size_t)L * sizeof(uint32_t));
        uint64_t *mysk = (uint64_t *)malloc((size_t)M * sizeof(uint64_t));
        or_list top = {0, 0, 0}, fresh = {0, 0, 0};
        if (!clo || !chi || !mycode || !mysk) err = OR_ENOMEM;
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < m; ++t) {
            if (err) continue;
            for (int32_t j = 0; j < L; ++j) mycode[j] = qc[(int64_t)j * m + t];
            for (int32_t s = 0; s < M; ++s) mysk[s] = qs[(int64_t)s * m + t];
            int64_t cnt[3];
            int32_t sl = 0, bd = 0;
            int rc = walk_one(&ix, qn + t * d, mycode, mysk, k, delta, eps, B, rule, filter_on, groups, test_entries,
                              clo, chi, &top, &fresh, &sl, cnt, &bd, t == 0 ? trace : NULL,
                              t == 0 ? ltrace : NULL);
            if (rc) {
                err = rc;
                continue;
            }
            for (int32_t r = 0; r < k; ++r) {
                ids[t * k + r] = top.v[r].id;
                if (ips) ips[t * k + r] = top.v[r].ip;
                if (ips64) ips64[t * k + r] = top.v[r].ip64;
            }
            if (stop_level) stop_level[t] = sl;
            if (c_scan) c_scan[t] = cnt[0];
            if (c_pass) c_pass[t] = cnt[1];
            if (c_rerank) c_rerank[t] = cnt[2];
            if (boundary) boundary[t] = bd;
        }
        free(clo), free(chi), free(mycode), free(mysk);
        free(top.v), free(fresh.v);
    }
    free(qn), free(qc), free(qs);
    return err;
}

/* ------------------------------------------------------------------------------------
 * Exact k-NN by brute force (the problem of Sec. 2.1 with delta = 0): FP64 inner
 * products of the normalised rows, ordered by (inner product descending, position
 * ascending).  `points` and `queries` must already be normalised.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    double ip;
    int32_t id;
} or_bf;

static int cmp_bf(const void *a, const void *b) {
    const or_bf *x = (const or_bf *)a, *y = (const or_bf *)b;
    if (x->ip > y->ip) return -1;
    if (x->ip < y->ip) return 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

int oracle_bruteforce(const float *points, int64_t n, int32_t d, const float *queries, int64_t m,
                      int32_t k, int32_t *ids, double *ips64) {
    if (k < 1 || k > n) return OR_EINVAL;
    int err = OR_OK;
#pragma omp parallel
    {
        or_bf *all = (or_bf *)malloc((size_t)n * sizeof(or_bf));
        if (!all) err = OR_ENOMEM;
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < m; ++t) {
            if (err) continue;
            for (int64_t x = 0; x < n; ++x) {
                all[x].ip = dot64(points + x * d, queries + t * d, d);
                all[x].id = (int32_t)x;
            }
            qsort(all, (size_t)n, sizeof(or_bf), cmp_bf);
            for (int32_t r = 0; r < k; ++r) {
                ids[t * k + r] = all[r].id;
                if (ips64) ips64[t * k + r] = all[r].ip;
            }
        }
        free(all);
    }
    return err;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the following oracle calls (timing only; results do not depend on it) */
void oracle_set_threads(int32_t t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
