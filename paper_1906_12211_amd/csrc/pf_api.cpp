// C-ABI of the gfx950 adaptive k-NN index (declared in include/pfhip.h): argument
// checks, device memory, the host-side hyperplane generator and hash plan, and the
// order of kernel launches for build and search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "pf_internal.h"

#define PF_API extern "C" __attribute__((visibility("default")))

namespace pf {

static thread_local std::string g_err;

void set_last_error(const std::string &msg) { g_err = msg; }

template <class F> static int guard(F &&f) {
    try {
        f();
        return PF_OK;
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return PF_ENOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return PF_EDEVICE;
    }
}

// ------------------------------------------------------------------ hyperplanes
// Random hyperplanes (Sec. 2.2: independent standard normal coordinates).  Counter-based
// SplitMix64 (Steele, Lea, Flood 2014): output s of the stream with seed S is
// mix(S + (s + 1) * 0x9E3779B97F4A7C15).  Element (r, c) of the d-column matrix uses
// outputs 2t and 2t+1, t = r d + c, in the Box-Muller transform evaluated in FP64:
// u1 = ((z1 >> 11) + 1) 2^-53, u2 = (z2 >> 11) 2^-53, a = sqrt(-2 ln u1) cos(2 pi u2).
static inline uint64_t splitmix64_at(uint64_t seed, uint64_t s) {
    uint64_t z = seed + (s + 1u) * 0x9E3779B97F4A7C15ull;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

static void make_hyperplanes(uint64_t seed, int64_t rows, int32_t d, float *out) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t r = 0; r < rows; ++r)
        for (int32_t c = 0; c < d; ++c) {
            const uint64_t t = (uint64_t)r * (uint64_t)d + (uint64_t)c;
            const uint64_t z1 = splitmix64_at(seed, 2u * t);
            const uint64_t z2 = splitmix64_at(seed, 2u * t + 1u);
            const double u1 = ((double)(z1 >> 11) + 1.0) * 0x1.0p-53;
            const double u2 = (double)(z2 >> 11) * 0x1.0p-53;
            out[r * d + c] = (float)(std::sqrt(-2.0 * std::log(u1)) * std::cos(two_pi * u2));
        }
}

static inline uint16_t bf16_rne_host(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Error bound of the split-BF16 projection (see k_hash.hip).  For one column a and a
// unit row x: the three dropped split products are at most 3.01 * 2^-16 * sum|a_i x_i|,
// and the FP32 accumulation of 3 kp exact products adds at most 1.02 * gamma_{3 kp} *
// sum|a_i x_i| (Higham's bound, gamma_m = m u / (1 - m u), u = 2^-24); sum|a_i x_i| <=
// |a| |x| and |x| <= 1.0001 after normalisation.  The bound is doubled to allow for
// truncating accumulation inside the matrix core.
static double split_bf16_bound(int32_t kp, double norm_a) {
    const double u = 0x1.0p-24;
    const double m = 3.0 * kp;
    const double gamma = m * u / (1.0 - m * u);
    return 2.0 * (3.01 * 0x1.0p-16 + 1.02 * gamma) * norm_a * 1.0001 + 1e-30 * kp;
}

static void build_plan(Index &ix, const std::vector<float> &hp) {
    HashPlan &p = ix.plan;
    p.d = ix.d;
    p.dpad = ix.dpad;
    p.kp = (ix.d + 15) / 16 * 16;
    p.L = ix.L;
    p.K = ix.K;
    p.M = ix.M;
    p.pool = ix.pool;
    // code words: the table codes (one per table), the pool bits, or none when the codes
    // are cross-polytope values computed by their own kernel
    p.cw = ix.family == PF_FAMILY_FHTCP ? 0 : (ix.pool ? ix.pool / 32 : ix.L);
    p.words = p.cw + 2 * ix.M;
    p.ncols = 32 * p.words;
    const int64_t srow = ix.family == PF_FAMILY_FHTCP ? 0
                         : (ix.pool ? (int64_t)ix.pool : (int64_t)ix.L * ix.K); // first sketch row
    std::vector<int32_t> colrow(p.ncols, -1);
    std::vector<float> beta(p.ncols, -1.0f);
    for (int32_t wb = 0; wb < p.words; ++wb)
        for (int32_t c = 0; c < 32; ++c) {
            int64_t row = -1;
            if (wb < p.cw) {
                if (ix.pool)
                    row = (int64_t)wb * 32 + c;
                else if (c < ix.K)
                    row = (int64_t)wb * ix.K + (ix.K - 1 - c);
            } else {
                const int32_t s = wb - p.cw;
                row = srow + 64 * (s >> 1) + 32 * (s & 1) + c;
            }
            colrow[wb * 32 + c] = (int32_t)row;
        }
    std::vector<uint16_t> hb((size_t)2 * p.ncols * p.kp, 0);
    for (int32_t col = 0; col < p.ncols; ++col) {
        const int64_t row = colrow[col];
        if (row < 0) continue;
        double s2 = 0.0;
        for (int32_t c = 0; c < ix.d; ++c) {
            const float v = hp[row * ix.d + c];
            s2 += (double)v * (double)v;
            const uint16_t h = bf16_rne_host(v);
            uint32_t hu = (uint32_t)h << 16;
            float hf;
            std::memcpy(&hf, &hu, 4);
            hb[(size_t)col * p.kp + c] = h;
            hb[(size_t)p.ncols * p.kp + (size_t)col * p.kp + c] = bf16_rne_host(v - hf);
        }
        beta[col] = (float)(split_bf16_bound(p.kp, std::sqrt(s2)) * (1.0 + 0x1.0p-20));
    }
    ix.hcolrow.alloc(colrow.size() * sizeof(int32_t));
    PF_HIP(hipMemcpy(ix.hcolrow.p, colrow.data(), colrow.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    ix.hbeta.alloc(beta.size() * sizeof(float));
    PF_HIP(hipMemcpy(ix.hbeta.p, beta.data(), beta.size() * sizeof(float), hipMemcpyHostToDevice));
    ix.hbf.alloc(hb.size() * sizeof(uint16_t));
    PF_HIP(hipMemcpy(ix.hbf.p, hb.data(), hb.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
}

// FHT cross-polytope: d' = the smallest power of two >= d, ell = log2(2 d') bits per value
static void cp_dims(int32_t d, int32_t &dp, int32_t &ell) {
    dp = 1;
    ell = 1;
    while (dp < d) dp <<= 1, ++ell;
}

// Budget rule: every byte the index keeps on the device, split into the part that does
// not depend on L and the bytes each table adds (Sec. 1 and Sec. 5.2: the budget covers
// the data set and the hash functions as well as the tables).  The terms mirror the
// allocations of pf_build_index and build_plan one for one:
//   fixed: the vectors as two 16-bit planes, their 8-bit summaries (+ the 8-byte headers
//          when rows share one scale), the sketch (and pool) hyperplanes, their GEMM
//          copies (BF16 hi + lo, column rows, flag bounds; 32 columns per word), the
//          cross-polytope collision table, and the padding after the positions;
//   per table: table-local sketches (8n), positions (posb n: 4 bytes, or 3 on request when
//          n <= 2^24), the low K - P bits of the sorted codes (n when K - P <= 8, 2n when
//          K - P <= 16, 4n when larger, none when K <= P), the P-bit prefix table
//          (4 (2^P + 1)), the table's K hyperplanes and their GEMM word
//          (independent functions), its K pool indices (pooling) or its cross-polytope
//          sign words.
static void budget_terms(int64_t n, int32_t d, int32_t K, int32_t M, int32_t pool, int32_t family, int32_t posb,
                         int32_t P, uint64_t &fixed, uint64_t &per) {
    const uint64_t un = (uint64_t)n, ud = (uint64_t)d;
    const int32_t dpad = (d + 3) / 4 * 4;
    int32_t hs, ls, rq, co;
    plane_strides(dpad, &hs, &ls);
    rows8_layout(dpad, &rq, &co);
    const uint64_t kp = (uint64_t)((d + 15) / 16 * 16);
    const uint64_t word = 32ull * (4ull * kp + 8ull); // hbf hi + lo, hcolrow, hbeta of 32 columns
    const bool cp = family == PF_FAMILY_FHTCP;
    fixed = 2ull * un * (uint64_t)(hs + std::max(ls, 1)) + un * (uint64_t)rq + (co == 0 ? 8ull * un : 0ull) +
            4ull * 64ull * (uint64_t)M * ud + 4ull * (uint64_t)pool * ud +
            (2ull * (uint64_t)M + (uint64_t)(pool / 32)) * word + (uint64_t)kPosPad;
    per = (8ull + (uint64_t)posb + (uint64_t)code_suffix_bytes(K, P)) * un + 4ull * ((1ull << P) + 1ull);
    if (cp) {
        int32_t dp, ell;
        cp_dims(d, dp, ell);
        fixed += 41ull * (uint64_t)(ell + 1) * 8ull;
        per += (uint64_t)((K + ell - 1) / ell) * 3ull * (uint64_t)((dp + 31) / 32) * 4ull;
    } else if (pool) {
        per += 4ull * (uint64_t)K;
    } else {
        per += 4ull * (uint64_t)K * ud + word;
    }
}

// sign bit of coordinate c of rotation round k of cross-polytope function fn: the top bit
// of output (3 fn + k) d' + c of the SplitMix64 stream seeded with sseed
static inline bool cp_sign(uint64_t sseed, uint64_t fn, int32_t k, int32_t c, int32_t dp) {
    return (splitmix64_at(sseed, (fn * 3u + (uint64_t)k) * (uint64_t)dp + (uint64_t)c) >> 63) != 0;
}

// value of one cross-polytope function on the host (Monte Carlo estimation), FP64, the
// same butterflies as the device kernel
static uint32_t cp_value_host(const std::vector<float> &x, int32_t dp, uint64_t sseed, uint64_t fn,
                              std::vector<double> &y) {
    for (int32_t c = 0; c < dp; ++c) y[c] = (double)x[c];
    for (int32_t k = 0; k < 3; ++k) {
        for (int32_t c = 0; c < dp; ++c)
            if (cp_sign(sseed, fn, k, c, dp)) y[c] = -y[c];
        for (int32_t h = 1; h < dp; h <<= 1)
            for (int32_t j = 0; j < dp; ++j)
                if (!(j & h)) {
                    const double a = y[j], b = y[j + h];
                    y[j] = a + b;
                    y[j + h] = a - b;
                }
    }
    int32_t best = 0;
    for (int32_t c = 1; c < dp; ++c)
        if (std::fabs(y[c]) > std::fabs(y[best])) best = c;
    return (uint32_t)((y[best] < 0.0 ? dp : 0) + best);
}

// Monte Carlo collision table (Sec. 4.3): at similarity alpha_g = -1 + 0.05 g the pair e_1,
// (alpha, sqrt(1 - alpha^2)) is hashed by 1,000 functions of the stream seeded with
// seed + 2; tab[g][b] = fraction agreeing in the first b bits, then made non-decreasing
// in alpha (the minimum over all g' >= g), a lower bound for the stopping rule.
static std::vector<double> cp_table_host(uint64_t seed, int32_t dp, int32_t ell) {
    constexpr int kGrid = 41, kDraws = 1000;
    std::vector<double> tab((size_t)kGrid * (ell + 1));
    std::vector<float> px(dp, 0.0f), py(dp, 0.0f);
    std::vector<double> y(dp);
    for (int g = 0; g < kGrid; ++g) {
        const double alpha = -1.0 + 0.05 * (double)g;
        px[0] = 1.0f;
        py[0] = (float)alpha;
        py[1] = (float)std::sqrt(std::fmax(0.0, 1.0 - alpha * alpha));
        std::vector<int64_t> cnt(ell + 1, 0);
        for (int r = 0; r < kDraws; ++r) {
            const uint32_t vx = cp_value_host(px, dp, seed + 2u, (uint64_t)r, y);
            const uint32_t vy = cp_value_host(py, dp, seed + 2u, (uint64_t)r, y);
            for (int b = 1; b <= ell; ++b)
                if ((vx >> (ell - b)) == (vy >> (ell - b))) ++cnt[b];
        }
        tab[(size_t)g * (ell + 1)] = 1.0;
        for (int b = 1; b <= ell; ++b) tab[(size_t)g * (ell + 1) + b] = (double)cnt[b] / (double)kDraws;
    }
    for (int g = kGrid - 2; g >= 0; --g)
        for (int b = 0; b <= ell; ++b)
            tab[(size_t)g * (ell + 1) + b] =
                std::min(tab[(size_t)g * (ell + 1) + b], tab[(size_t)(g + 1) * (ell + 1) + b]);
    return tab;
}

// Pooling (Sec. 3.2): table j's K functions, h_{t+1,j} = pool function sel[j K + t],
// drawn without replacement by the first K steps of Fisher-Yates on a fresh 0..m-1
// array; step t takes u = t + (z mod (m - t)) with z output j K + t of the SplitMix64
// stream seeded with seed + 1.
static std::vector<int32_t> pool_select(uint64_t seed, int32_t pool, int32_t L, int32_t K) {
    std::vector<int32_t> sel((size_t)L * K), a(pool);
    for (int32_t j = 0; j < L; ++j) {
        for (int32_t r = 0; r < pool; ++r) a[r] = r;
        for (int32_t t = 0; t < K; ++t) {
            const uint64_t z = splitmix64_at(seed + 1u, (uint64_t)j * (uint64_t)K + (uint64_t)t);
            const int32_t u = t + (int32_t)(z % (uint64_t)(pool - t));
            std::swap(a[t], a[u]);
            sel[(size_t)j * K + t] = a[t];
        }
    }
    return sel;
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// normalise caller rows (host or device) into dst (rows x dpad); throws PF_EINVAL on a bad row
static void normalize_into(const float *src, int64_t rows, int32_t d, int32_t mem, float *dst, int32_t dpad,
                           DevBuf &staging, DevBuf &flag, hipStream_t s) {
    const float *in = src;
    if (mem == PF_HOST) {
        staging.ensure((size_t)rows * d * sizeof(float));
        PF_HIP(hipMemcpyAsync(staging.p, src, (size_t)rows * d * sizeof(float), hipMemcpyHostToDevice, s));
        in = staging.as<float>();
    }
    flag.ensure(sizeof(unsigned long long));
    const unsigned long long init = ~0ull;
    PF_HIP(hipMemcpyAsync(flag.p, &init, sizeof(init), hipMemcpyHostToDevice, s));
    launch_normalize(in, rows, d, d, dst, dpad, flag.as<unsigned long long>(), s);
    unsigned long long bad = 0;
    PF_HIP(hipMemcpyAsync(&bad, flag.p, sizeof(bad), hipMemcpyDeviceToHost, s));
    PF_HIP(hipStreamSynchronize(s));
    if (bad != ~0ull)
        throw Error(PF_EINVAL, "row " + std::to_string(bad) + " has zero or non-finite norm");
}

} // namespace pf

using namespace pf;


PF_API const char *pf_last_error(void) { return g_err.c_str(); }
PF_API const char *pf_version(void) { return "pfhip 0.1 (gfx950)"; }

PF_API int pf_read_bandwidth(uint64_t bytes, int32_t reps, double *gbs, void *stream) {
    return guard([&] {
        PF_CHECK(gbs && bytes >= (1ull << 20) && reps >= 1, PF_EINVAL,
                 "pf_read_bandwidth: need gbs, bytes >= 1 MiB and reps >= 1");
        int dev = 0;
        PF_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        PF_HIP(hipGetDeviceProperties(&prop, dev));
        *gbs = pf::read_bandwidth_gbs(bytes, reps, prop.multiProcessorCount, as_stream(stream));
    });
}

PF_API int pf_random_read_rate(uint64_t bytes, int32_t reps, double *loads_per_s, void *stream) {
    return guard([&] {
        PF_CHECK(loads_per_s && bytes >= (1ull << 20) && reps >= 1, PF_EINVAL,
                 "pf_random_read_rate: need loads_per_s, bytes >= 1 MiB and reps >= 1");
        int dev = 0;
        PF_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        PF_HIP(hipGetDeviceProperties(&prop, dev));
        *loads_per_s = pf::random_read_rate(bytes, reps, prop.multiProcessorCount, as_stream(stream));
    });
}

PF_API int32_t pf_tile_count(void) { return pf::search_tile_count(); }

PF_API const char *pf_tile_name(int32_t t) { return pf::search_tile_name(t); }

PF_API int pf_normalize(const float *x, int64_t n, int32_t d, float *out, int32_t mem, void *stream) {
    return guard([&] {
        PF_CHECK(x && out && n >= 0 && d >= 1 && d <= PF_MAX_DIM, PF_EINVAL, "pf_normalize: bad arguments");
        PF_CHECK(mem == PF_HOST || mem == PF_DEVICE, PF_EINVAL, "pf_normalize: bad mem");
        if (n == 0) return;
        hipStream_t s = as_stream(stream);
        DevBuf staging, flag, dst;
        float *o = out;
        if (mem == PF_HOST) {
            dst.alloc((size_t)n * d * sizeof(float));
            o = dst.as<float>();
        }
        normalize_into(x, n, d, mem, o, d, staging, flag, s);
        if (mem == PF_HOST) {
            PF_HIP(hipMemcpyAsync(out, o, (size_t)n * d * sizeof(float), hipMemcpyDeviceToHost, s));
            PF_HIP(hipStreamSynchronize(s));
        }
    });
}

// Options with defaults filled in, checked, and the table count of the budget rule
// (host only; shared by pf_plan_index and pf_build_index).
struct BuildPlan {
    pf_build_opts o;
    int32_t K, M, posb, P;
    int64_t L;
    uint64_t fixed, per;
};

static BuildPlan plan_build(int64_t n, int32_t d, uint64_t budget, const pf_build_opts *opts) {
    PF_CHECK(n >= 1 && n < (1ll << 31), PF_EINVAL, "pf_build_index: n must be in [1, 2^31)");
    PF_CHECK(d >= 1 && d <= PF_MAX_DIM, PF_EINVAL, "pf_build_index: d out of range");
    BuildPlan b;
    b.o = pf_build_opts{};
    if (opts) b.o = *opts;
    const pf_build_opts &o = b.o;
    b.K = o.K ? o.K : 24;
    b.M = o.M ? o.M : 32;
    const int32_t K = b.K, M = b.M;
    PF_CHECK(K >= 1 && K <= 32, PF_EINVAL, "pf_build_index: K must be in [1, 32]");
    PF_CHECK(M >= 1 && M <= 64, PF_EINVAL, "pf_build_index: M must be in [1, 64]");
    PF_CHECK(o.hash_mode == PF_HASH_BF16X3 || o.hash_mode == PF_HASH_FP64, PF_EINVAL,
             "pf_build_index: bad hash_mode");
    PF_CHECK(o.pool == 0 || (o.pool >= K && o.pool <= 65536 && o.pool % 32 == 0), PF_EINVAL,
             "pf_build_index: pool must be 0 or a multiple of 32 in [K, 65536]");
    PF_CHECK(o.family == PF_FAMILY_HP || o.family == PF_FAMILY_FHTCP, PF_EINVAL, "pf_build_index: bad family");
    PF_CHECK(o.family == PF_FAMILY_HP || o.pool == 0, PF_EINVAL,
             "pf_build_index: pooling is implemented for hyperplane functions");
    PF_CHECK(o.pos_bytes == 0 || o.pos_bytes == 4 || (o.pos_bytes == 3 && n <= (1ll << 24)), PF_EINVAL,
             "pf_build_index: pos_bytes must be 0, 4, or 3 with n <= 2^24");
    PF_CHECK(o.prefix_bits == 0 || (o.prefix_bits >= prefix_bits_min(K) && o.prefix_bits <= prefix_bits_max(K)),
             PF_EINVAL, "pf_build_index: prefix_bits must be 0 or in [min(13, K), min(24, K)]");
    b.posb = pos_bytes_for(n, o.pos_bytes);
    b.P = o.prefix_bits ? o.prefix_bits : choose_prefix_bits(n, K);
    budget_terms(n, d, K, M, o.pool, o.family, b.posb, b.P, b.fixed, b.per);
    int64_t L = o.L_override;
    if (L <= 0) L = budget > b.fixed ? (int64_t)((budget - b.fixed) / b.per) : 0;
    PF_CHECK(L >= 1, PF_EBUDGET, "pf_build_index: the memory budget holds no table");
    L = std::min<int64_t>(L, PF_MAX_TABLES);
    // table positions, and the search's entry counters (which run up to a chunk past a
    // level's last entry), are 32-bit: a table count from the budget stops below 2^32 - 2^16
    // entries (at least one table, n < 2^31), an explicit one beyond it is refused
    const int64_t entry_cap = (int64_t)(((1ull << 32) - (1ull << 16) - 1ull) / (uint64_t)n);
    if (o.L_override <= 0) L = std::min<int64_t>(L, entry_cap);
    PF_CHECK((uint64_t)L * (uint64_t)n < (1ull << 32) - (1ull << 16), PF_EUNSUPPORTED,
             "pf_build_index: L * n must be below 2^32 - 2^16");
    b.L = L;
    return b;
}

PF_API int pf_plan_index(int64_t n, int32_t d, uint64_t budget, const pf_build_opts *opts, int32_t *L,
                         uint64_t *bytes_device) {
    return guard([&] {
        const BuildPlan b = plan_build(n, d, budget, opts);
        if (L) *L = (int32_t)b.L;
        if (bytes_device) *bytes_device = b.fixed + (uint64_t)b.L * b.per;
    });
}

PF_API int pf_build_index(const float *points, int64_t n, int32_t d, uint64_t budget,
                          const pf_build_opts *opts, int32_t mem, void *stream, pf_index **out) {
    return guard([&] {
        PF_CHECK(out && points, PF_EINVAL, "pf_build_index: null argument");
        PF_CHECK(mem == PF_HOST || mem == PF_DEVICE, PF_EINVAL, "pf_build_index: bad mem");
        const BuildPlan bp = plan_build(n, d, budget, opts);
        const pf_build_opts &o = bp.o;
        const int32_t K = bp.K, M = bp.M;
        const int64_t L = bp.L;
        const uint64_t fixed = bp.fixed, per = bp.per;

        auto ix = std::make_unique<pf_index>();
        hipStream_t s = as_stream(stream);
        PF_HIP(hipGetDevice(&ix->device));
        hipDeviceProp_t prop;
        PF_HIP(hipGetDeviceProperties(&prop, ix->device));
        ix->num_cus = prop.multiProcessorCount;
        int wall_khz = 0;
        if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, ix->device) == hipSuccess)
            ix->wall_khz = wall_khz;
        ix->n = n;
        ix->d = d;
        ix->dpad = (d + 3) / 4 * 4;
        ix->K = K;
        ix->M = M;
        ix->P = bp.P;
        ix->L = (int32_t)L;
        ix->seed = o.seed;
        ix->hash_mode = o.hash_mode;
        ix->pool = o.pool;
        ix->family = o.family;
        if (o.family == PF_FAMILY_FHTCP) {
            cp_dims(d, ix->cp_dp, ix->cp_ell);
            ix->cp_c = (K + ix->cp_ell - 1) / ix->cp_ell;
        }
        ix->bytes_rule = fixed + (uint64_t)L * per;

        hipEvent_t e0, e1;
        PF_HIP(hipEventCreate(&e0));
        PF_HIP(hipEventCreate(&e1));
        PF_HIP(hipEventRecord(e0, s));
        // a1: normalised vectors (FP32 while the index is built, then two 16-bit planes)
        DevBuf X;
        X.alloc((size_t)n * ix->dpad * sizeof(float));
        normalize_into(points, n, d, mem, X.as<float>(), ix->dpad, ix->tmp, ix->flags, s);
        ix->tmp.release();
        // a3: hyperplanes (host generator), device copies and hash plan
        const int64_t rows = (o.family == PF_FAMILY_FHTCP ? 0 : (o.pool ? (int64_t)o.pool : L * K)) + 64ll * M;
        std::vector<float> hp((size_t)rows * d);
        make_hyperplanes(o.seed, rows, d, hp.data());
        ix->hp.alloc(hp.size() * sizeof(float));
        PF_HIP(hipMemcpy(ix->hp.p, hp.data(), hp.size() * sizeof(float), hipMemcpyHostToDevice));
        if (o.family == PF_FAMILY_FHTCP) {
            // sign bits of every function's three rotations (stream seed + 3), and the
            // Monte Carlo collision table (stream seed + 2)
            const int32_t dp = ix->cp_dp, sw = (dp + 31) / 32;
            const int64_t nfn = L * (int64_t)ix->cp_c;
            std::vector<uint32_t> sg((size_t)nfn * 3 * sw, 0u);
            for (int64_t fn = 0; fn < nfn; ++fn)
                for (int32_t k = 0; k < 3; ++k)
                    for (int32_t c = 0; c < dp; ++c)
                        if (cp_sign(o.seed + 3u, (uint64_t)fn, k, c, dp))
                            sg[(size_t)(fn * 3 + k) * sw + c / 32] |= 1u << (c % 32);
            ix->cpsign.alloc(sg.size() * sizeof(uint32_t));
            PF_HIP(hipMemcpy(ix->cpsign.p, sg.data(), sg.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
            const std::vector<double> tab = cp_table_host(o.seed, dp, ix->cp_ell);
            ix->cptab.alloc(tab.size() * sizeof(double));
            PF_HIP(hipMemcpy(ix->cptab.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        }
        if (o.pool) {
            const std::vector<int32_t> sel = pool_select(o.seed, o.pool, (int32_t)L, K);
            ix->psel.alloc(sel.size() * sizeof(int32_t));
            PF_HIP(hipMemcpy(ix->psel.p, sel.data(), sel.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        }
        build_plan(*ix, hp);
        // a4/a5: codes (L x n) and sketches (M x n)
        DevBuf codes, sk, scratch;
        codes.alloc((size_t)L * n * sizeof(uint32_t));
        sk.alloc((size_t)M * n * sizeof(uint64_t));
        hash_rows(*ix, X.as<float>(), n, codes.as<uint32_t>(), sk.as<uint64_t>(), scratch, s);
        plane_strides(ix->dpad, &ix->hs, &ix->ls);
        ix->Xh.alloc((size_t)n * ix->hs * sizeof(uint16_t));
        ix->Xl.alloc((size_t)n * std::max(ix->ls, 1) * sizeof(uint16_t));
        launch_split_planes(X.as<float>(), n, ix->dpad, ix->Xh.as<uint16_t>(), ix->Xl.as<uint16_t>(), s);
        rows8_layout(ix->dpad, &ix->rq, &ix->qco);
        ix->Xq.alloc((size_t)n * ix->rq);
        if (ix->qco == 0) ix->Xqh.alloc((size_t)n * 8);
        DevBuf gmax;
        gmax.alloc(2 * sizeof(uint32_t));
        launch_rows8(X.as<float>(), n, ix->dpad, ix->Xq.as<uint8_t>(), ix->Xqh.as<uint8_t>(), gmax.as<uint32_t>(), s);
        if (ix->qco == 0) { // the common scale as the kernel computed it (row 0's header), largest sum
            PF_HIP(hipMemcpyAsync(&ix->s8, ix->Xqh.p, sizeof(float), hipMemcpyDeviceToHost, s));
            PF_HIP(hipMemcpyAsync(&ix->a8, gmax.as<uint32_t>() + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        }
        // a6: sorted tables (the full codes only while the index is built); 4-byte positions
        // are sorted into the index's array, 3-byte ones into a 4-byte array packed below
        DevBuf tcode, wide;
        tcode.alloc((size_t)L * n * sizeof(uint32_t));
        ix->posb = bp.posb;
        ix->tpos.alloc((size_t)L * n * ix->posb + (size_t)kPosPad);
        if (ix->posb != 4) wide.alloc((size_t)L * n * sizeof(uint32_t));
        uint32_t *tidx = ix->posb == 4 ? ix->tpos.as<uint32_t>() : wide.as<uint32_t>();
        sort_tables(codes.as<uint32_t>(), n, (int32_t)L, K, tcode.as<uint32_t>(), tidx, scratch, s);
        // a7: prefix tables, then the codes' low K - P bits (the prefix table holds the rest)
        ix->off.alloc((size_t)L * ((1ull << ix->P) + 1) * sizeof(uint32_t));
        prefix_tables(tcode.as<uint32_t>(), n, (int32_t)L, K, ix->P, ix->off.as<uint32_t>(), s);
        ix->sufw = code_suffix_bytes(K, ix->P);
        if (ix->sufw) {
            ix->tsuf.alloc((size_t)L * n * ix->sufw);
            code_suffixes(tcode.as<uint32_t>(), n, (int32_t)L, K, ix->P, ix->tsuf.p, s);
        }
        // a8: table-local sketches
        ix->tsk.alloc((size_t)L * n * sizeof(uint64_t));
        gather_sketches(tidx, sk.as<uint64_t>(), n, (int32_t)L, M, ix->tsk.as<uint64_t>(), s);
        // the stored positions (in place for 4 bytes) and the padding after them
        pack_positions(tidx, (int64_t)L * n, ix->posb, ix->tpos.as<uint8_t>(), s);
        PF_HIP(hipEventRecord(e1, s));
        PF_HIP(hipStreamSynchronize(s));
        float ms = 0;
        PF_HIP(hipEventElapsedTime(&ms, e0, e1));
        ix->build_ms = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *out = ix.release();
    });
}

namespace pf {
// normalise + hash rows into qX / codes / sketches held by the index
void prepare_rows_for(Index &ixr, const float *x, int64_t m, int32_t mem, hipStream_t s, float **qX,
                      uint32_t **qcode, uint64_t **qsk) {
    Index *ix = &ixr;
    ix->qX.ensure((size_t)m * ix->dpad * sizeof(float));
    normalize_into(x, m, ix->d, mem, ix->qX.as<float>(), ix->dpad, ix->tmp, ix->flags, s);
    ix->qcode.ensure((size_t)m * ix->L * sizeof(uint32_t));
    ix->qsk.ensure((size_t)m * ix->M * sizeof(uint64_t));
    hash_rows(*ix, ix->qX.as<float>(), m, ix->qcode.as<uint32_t>(), ix->qsk.as<uint64_t>(), ix->hscratch, s);
    *qX = ix->qX.as<float>();
    *qcode = ix->qcode.as<uint32_t>();
    *qsk = ix->qsk.as<uint64_t>();
}

// the longest-predicted-first queue order of m queries, written to order (device, m)
void learned_order(Index &ix, const uint32_t *qcode, const uint64_t *qsk, int64_t m, const int32_t *ks_host,
                   int32_t kconst, const double *rec_host, double recall_const, int32_t *order, hipStream_t s);

// ------------------------------------------------------------------ autotuner
// Tile shapes of the batched search kernel (sketch loads and rows in flight per lane)
// and the number of resident query waves per CU are timed on the batch itself; the
// fastest is kept per (architecture, n, d, L, kmax, position width: the two widths run
// different kernels) in memory and, when the environment variable PF_TUNE_CACHE names a
// file, in that file as JSON lines.
struct TuneChoice {
    int32_t tile = search_default_tile(), waves = 0;
    double us_per_query = 0.0;
};

static std::string tune_key(const Index &ix, int32_t kmax) {
    hipDeviceProp_t prop;
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, ix.device) == hipSuccess) arch = prop.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch = arch.substr(0, c);
    return arch + "|n" + std::to_string(ix.n) + "|d" + std::to_string(ix.d) + "|L" + std::to_string(ix.L) +
           "|k" + std::to_string(kmax) + "|p" + std::to_string(ix.posb);
}

static bool tune_cache_read(const std::string &key, TuneChoice &out) {
    const char *path = std::getenv("PF_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[256], name[64];
        TuneChoice t;
        // an entry counts only if its shape index still names the same shape in this build
        if (std::sscanf(line,
                        "{\"key\": \"%255[^\"]\", \"tile\": %d, \"waves\": %d, \"us_per_query\": %lf, \"name\": \"%63[^\"]\"",
                        k, &t.tile, &t.waves, &t.us_per_query, name) == 5 &&
            key == k && t.tile >= 0 && t.tile < search_tile_count() && std::strcmp(name, search_tile_name(t.tile)) == 0) {
            out = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void tune_cache_write(const std::string &key, const TuneChoice &t) {
    const char *path = std::getenv("PF_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"tile\": %d, \"waves\": %d, \"us_per_query\": %.6f, \"name\": \"%s\"}\n",
                 key.c_str(), t.tile, t.waves, t.us_per_query, search_tile_name(t.tile));
    std::fclose(f);
}

static TuneChoice cached_tuning(Index &ix, int32_t kmax) {
    const std::string key = tune_key(ix, kmax);
    auto it = ix.tuned.find(key);
    if (it != ix.tuned.end()) return TuneChoice{it->second.tile, it->second.waves, it->second.us};
    TuneChoice t;
    if (tune_cache_read(key, t)) ix.tuned[key] = {t.tile, t.waves, t.us_per_query};
    return t;
}

static TuneChoice autotune(Index &ix, SearchArgs a, int32_t kmax, hipStream_t s) {
    const std::string key = tune_key(ix, kmax);
    const int64_t sample = std::min<int64_t>(a.m, 8192);
    a.qstride = a.m; // query codes were computed for the whole batch
    a.m = sample;    // time the first queries of the batch (in queue order)
    hipEvent_t e0, e1;
    PF_HIP(hipEventCreate(&e0));
    PF_HIP(hipEventCreate(&e1));
    const int32_t nl = ix.K - ix.P;
    const uint32_t *rg = nl > 0 ? ix.ranges.as<uint32_t>() : nullptr;
    // microseconds per query of shape t at w resident waves per CU: the faster of two timed
    // launches after a warm-up (one launch's time varies by a few percent)
    auto time_of = [&](int32_t t, int32_t w) {
        a.tile = t;
        a.waves_per_cu = w;
        launch_search(ix, a, rg, s);
        float best_ms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            PF_HIP(hipEventRecord(e0, s));
            launch_search(ix, a, rg, s);
            PF_HIP(hipEventRecord(e1, s));
            PF_HIP(hipEventSynchronize(e1));
            float ms = 0;
            PF_HIP(hipEventElapsedTime(&ms, e0, e1));
            best_ms = rep == 0 ? ms : std::min(best_ms, ms);
        }
        return best_ms * 1e3 / (double)sample;
    };
    // every shape at its occupancy limit, then lower occupancy caps for the fastest shape
    TuneChoice best, best_default;
    best.us_per_query = 1e300;
    for (int32_t t = 0; t < search_tile_count(); ++t) {
        const int32_t w = search_waves_per_cu(ix, kmax, t);
        const double us = time_of(t, w);
        if (us < best.us_per_query) best = TuneChoice{t, w, us};
        if (t == search_default_tile()) best_default = TuneChoice{t, w, us}; // the default
    }
    const int32_t wmax = best.waves;
    for (int32_t w : {(3 * wmax) / 4, wmax / 2}) {
        if (w < 1 || w == wmax) continue;
        const double us = time_of(best.tile, w);
        if (us < best.us_per_query) best = TuneChoice{best.tile, w, us};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // another shape or occupancy cap replaces the default (the default shape at its
    // occupancy limit) only if it is clearly faster on the sample: one launch's time varies
    // by a few percent from run to run, so near-equal choices would otherwise alternate
    if (best.us_per_query > 0.95 * best_default.us_per_query) best = best_default;
    ix.tuned[key] = {best.tile, best.waves, best.us_per_query};
    tune_cache_write(key, best);
    return best;
}

struct BatchCtl {
    bool queue = false;           // device work queue instead of static slots
    const int32_t *order = nullptr; // host or device (see mem) queue order, nullable
    bool learned = false;         // order from the attached scheduler
    bool autotune = false;        // choose the tile shape by timing this batch
};

static void search_impl(pf_index *ix, const float *queries, int64_t m, const int32_t *ks, int32_t kconst,
                        int32_t kmax, const double *recalls, double recall_const, const pf_search_opts *opts,
                        int32_t *out_ids, float *out_ips, pf_query_stats *stats, int32_t mem, void *stream,
                        const BatchCtl &bc = BatchCtl()) {
    PF_CHECK(ix, PF_EINVAL, "null index");
    PF_CHECK(queries && out_ids && m >= 0, PF_EINVAL, "search: bad arguments");
    PF_CHECK(mem == PF_HOST || mem == PF_DEVICE, PF_EINVAL, "search: bad mem");
    PF_CHECK(kmax >= 1 && kmax <= PF_MAX_K && kmax <= ix->n, PF_EINVAL, "search: k must be in [1, min(n, 256)]");
    pf_search_opts o{};
    if (opts) o = *opts;
    if (o.B == 0) o.B = 12;
    PF_CHECK(o.B >= 1, PF_EINVAL, "search: B must be >= 1");
    PF_CHECK(o.rule != PF_RULE_POOL || ix->pool > 0, PF_EINVAL, "search: PF_RULE_POOL needs a pooled index");
    PF_CHECK(o.rule != PF_RULE_POOL || ix->family == PF_FAMILY_HP, PF_EINVAL,
             "search: PF_RULE_POOL is for hyperplane codes");
    PF_CHECK(o.rule == PF_RULE_FILTER || o.rule == PF_RULE_EXACT || o.rule == PF_RULE_ALG1 || o.rule == PF_RULE_POOL,
             PF_EINVAL,
             "search: bad rule");
    PF_CHECK(std::isfinite(o.eps) && o.eps > -1.0, PF_EINVAL, "search: eps must be finite and > -1");
    PF_CHECK(o.tile >= 0 && o.tile <= search_tile_count(), PF_EINVAL, "search: tile must be in [0, pf_tile_count()]");
    const int32_t G = o.groups > 0 ? o.groups : default_groups(ix->L);
    PF_CHECK(o.groups >= 0 && G <= std::min<int32_t>(ix->L, 64), PF_EINVAL,
             "search: groups must be in [0, min(L, 64)]");
    if (!recalls)
        PF_CHECK(recall_const > 0.0 && recall_const <= 1.0, PF_EINVAL, "search: recall must be in (0, 1]");
    if (m == 0) return;
    hipStream_t s = as_stream(stream);
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;

    // per-query parameters are checked on the host (copied there when device-resident)
    std::vector<int32_t> ks_host;
    std::vector<double> rec_host;
    if (ks) {
        ks_host.resize(m);
        PF_HIP(hipMemcpy(ks_host.data(), ks, (size_t)m * sizeof(int32_t),
                         mem == PF_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < m; ++i)
            PF_CHECK(ks_host[i] >= 1 && ks_host[i] <= kmax, PF_EINVAL, "search: per-query k out of [1, kmax]");
    }
    if (recalls) {
        rec_host.resize(m);
        PF_HIP(hipMemcpy(rec_host.data(), recalls, (size_t)m * sizeof(double),
                         mem == PF_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < m; ++i)
            PF_CHECK(rec_host[i] > 0.0 && rec_host[i] <= 1.0, PF_EINVAL, "search: recall must be in (0, 1]");
    }

    hipEvent_t ev[5];
    if (o.timing)
        for (auto &e : ev) PF_HIP(hipEventCreate(&e));
    if (o.timing) PF_HIP(hipEventRecord(ev[0], s));
    float *qX;
    uint32_t *qcode;
    uint64_t *qsk;
    prepare_rows_for(*ix, queries, m, mem, s, &qX, &qcode, &qsk);
    if (o.timing) PF_HIP(hipEventRecord(ev[1], s));

    // decision tables for this call's (rule, eps, distinct deltas): delta = 1 - recall
    std::vector<double> lnd;
    std::vector<int32_t> qtab_host;
    if (recalls) {
        std::vector<double> uniq(rec_host);
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        PF_CHECK(uniq.size() <= 4096, PF_EUNSUPPORTED, "search: at most 4096 distinct recall values per call");
        for (double r : uniq) lnd.push_back(std::log(1.0 - r));
        qtab_host.resize(m);
        for (int64_t i = 0; i < m; ++i)
            qtab_host[i] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), rec_host[i]) - uniq.begin());
    } else {
        lnd.push_back(std::log(1.0 - recall_const));
    }
    const int32_t cols = rule_table_cols();
    const int32_t filt = o.no_filter ? 0 : 1;
    if (ix->rule_key_rule != o.rule || ix->rule_key_eps != o.eps || ix->rule_key_filter != filt ||
        ix->rule_key_groups != G || ix->rule_key_lndeltas != lnd) {
        ix->rule_key_lndeltas.clear(); // (no call's key matches while the tables are rebuilt)
        const size_t tab_floats = 65 + (size_t)lnd.size() * ix->K * G * cols;
        const size_t dl_off = (tab_floats * sizeof(float) + 15) & ~(size_t)15;
        ix->rule_tab.ensure(dl_off + lnd.size() * sizeof(double));
        double *dl = reinterpret_cast<double *>(ix->rule_tab.as<char>() + dl_off);
        PF_HIP(hipMemcpyAsync(dl, lnd.data(), lnd.size() * sizeof(double), h2d, s));
        float *tab = ix->rule_tab.as<float>();
        launch_rule_tables(dl, (int32_t)lnd.size(), o.eps, o.rule, ix->L, ix->M, ix->K, G, ix->pool,
                           ix->family == PF_FAMILY_FHTCP ? ix->cptab.as<double>() : nullptr, ix->cp_ell, tab,
                           tab + 65, s);
        PF_HIP(hipStreamSynchronize(s));
        ix->rule_key_rule = o.rule;
        ix->rule_key_eps = o.eps;
        ix->rule_key_filter = filt;
        ix->rule_key_groups = G;
        ix->rule_key_lndeltas = lnd;
    }

    // outputs and per-query parameters on the device (the index's grow-only call buffers,
    // so that a call allocates nothing once they are large enough)
    DevBuf &dids = ix->c_ids, &dips = ix->c_ips, &dstats = ix->c_stats, &dks = ix->c_ks, &dqtab = ix->c_qtab;
    int32_t *oid = out_ids;
    float *oip = out_ips;
    pf_query_stats *ost = stats;
    if (mem == PF_HOST) {
        dids.ensure((size_t)m * kmax * sizeof(int32_t));
        oid = dids.as<int32_t>();
        if (out_ips) {
            dips.ensure((size_t)m * kmax * sizeof(float));
            oip = dips.as<float>();
        }
        if (stats) {
            dstats.ensure((size_t)m * sizeof(pf_query_stats));
            ost = dstats.as<pf_query_stats>();
        }
    }
    if (ks) {
        dks.ensure((size_t)m * sizeof(int32_t));
        PF_HIP(hipMemcpyAsync(dks.p, ks_host.data(), (size_t)m * sizeof(int32_t), h2d, s));
    }
    if (!qtab_host.empty()) {
        dqtab.ensure(qtab_host.size() * sizeof(int32_t));
        PF_HIP(hipMemcpyAsync(dqtab.p, qtab_host.data(), qtab_host.size() * sizeof(int32_t), h2d, s));
    }
    SearchArgs a;
    a.Q = qX;
    a.qcode = qcode;
    a.qsk = qsk;
    a.m = m;
    a.qstride = m;
    a.ks = ks ? dks.as<int32_t>() : nullptr;
    a.kconst = kconst;
    a.kmax = kmax;
    a.qtab = qtab_host.empty() ? nullptr : dqtab.as<int32_t>();
    a.tauv = ix->rule_tab.as<float>();
    a.stopw = ix->rule_tab.as<float>() + 65;
    a.B = o.B;
    a.groups = G;
    a.test_entries = test_entries_of(o.test_entries);
    a.filter = filt;
    a.prefilter = o.no_prefilter ? 0 : 1;
    a.queue = nullptr;
    a.order = nullptr;
    a.tile = o.tile > 0 ? o.tile - 1 : search_default_tile();
    a.waves_per_cu = 0;
    a.out_ids = oid;
    a.out_ips = oip;
    a.stats = ost;
    const int32_t nl = ix->K - ix->P;
    uint32_t *rg = nullptr;
    if (nl > 0) {
        ix->ranges.ensure((size_t)m * ix->L * nl * 2 * sizeof(uint32_t));
        rg = ix->ranges.as<uint32_t>();
    }
    launch_ranges(*ix, a, rg, s);
    if (o.timing) PF_HIP(hipEventRecord(ev[4], s));
    DevBuf &dqueue = ix->c_queue, &dorder = ix->c_order;
    if (bc.queue) {
        dqueue.ensure(64);
        a.queue = dqueue.as<unsigned int>();
        std::vector<int32_t> ord;
        if (bc.order) {
            ord.resize(m);
            PF_HIP(hipMemcpy(ord.data(), bc.order, (size_t)m * sizeof(int32_t),
                             mem == PF_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost));
        } else if (bc.learned) {
            // computed and sorted on the device; a permutation by construction
            PF_CHECK(ix->sched, PF_EINVAL, "search_batch: PF_BATCH_LEARNED needs an attached scheduler");
            dorder.ensure((size_t)m * sizeof(int32_t));
            learned_order(*ix, qcode, qsk, m, ks ? ks_host.data() : nullptr, kconst,
                          recalls ? rec_host.data() : nullptr, recall_const, dorder.as<int32_t>(), s);
            a.order = dorder.as<int32_t>();
        }
        if (!ord.empty()) {
            std::vector<char> seen(m, 0);
            for (int64_t i = 0; i < m; ++i) {
                PF_CHECK(ord[i] >= 0 && ord[i] < m && !seen[ord[i]], PF_EINVAL,
                         "search_batch: order must be a permutation of 0..m-1");
                seen[ord[i]] = 1;
            }
            dorder.ensure((size_t)m * sizeof(int32_t));
            PF_HIP(hipMemcpyAsync(dorder.p, ord.data(), (size_t)m * sizeof(int32_t), h2d, s));
            a.order = dorder.as<int32_t>();
        }
        if (o.tile == 0) {
            const TuneChoice tc = bc.autotune ? autotune(*ix, a, kmax, s) : cached_tuning(*ix, kmax);
            a.tile = tc.tile;
            a.waves_per_cu = tc.waves;
        }
    }
    if (o.timing) PF_HIP(hipEventRecord(ev[2], s));
    const int64_t slots = launch_search(*ix, a, rg, s);
    if (o.timing) PF_HIP(hipEventRecord(ev[3], s));
    if (mem == PF_HOST) {
        PF_HIP(hipMemcpyAsync(out_ids, oid, (size_t)m * kmax * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (out_ips)
            PF_HIP(hipMemcpyAsync(out_ips, oip, (size_t)m * kmax * sizeof(float), hipMemcpyDeviceToHost, s));
        if (stats)
            PF_HIP(hipMemcpyAsync(stats, ost, (size_t)m * sizeof(pf_query_stats), hipMemcpyDeviceToHost, s));
    }
    // results are complete on return, and the next call may reuse the index's buffers
    PF_HIP(hipStreamSynchronize(s));
    if (o.timing) {
        float t01, t14, t42, t23, t03;
        PF_HIP(hipEventElapsedTime(&t01, ev[0], ev[1]));
        PF_HIP(hipEventElapsedTime(&t14, ev[1], ev[4]));
        PF_HIP(hipEventElapsedTime(&t42, ev[4], ev[2]));
        PF_HIP(hipEventElapsedTime(&t23, ev[2], ev[3]));
        PF_HIP(hipEventElapsedTime(&t03, ev[0], ev[3]));
        ix->timing.normalize_ms = 0.0;
        ix->timing.hash_ms = t01;
        ix->timing.ranges_ms = t14;
        ix->timing.order_ms = t42;
        ix->timing.search_ms = t23;
        ix->timing.total_ms = t03;
        ix->timing.tile = a.tile;
        ix->timing.waves_per_cu = a.waves_per_cu;
        ix->timing.slots = slots;
        ix->timing.groups = G;
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
}
} // namespace pf

PF_API int pf_search_ex(pf_index *ix, const float *queries, int64_t m, int32_t k, double recall,
                        const pf_search_opts *opts, int32_t *out_ids, float *out_ips, pf_query_stats *stats,
                        int32_t mem, void *stream) {
    return guard([&] {
        search_impl(ix, queries, m, nullptr, k, k, nullptr, recall, opts, out_ids, out_ips, stats, mem, stream);
    });
}

PF_API int pf_search_batch(pf_index *ix, const float *queries, int64_t m, const int32_t *ks, const double *recalls,
                           int32_t kmax, const pf_search_opts *opts, const int32_t *order, int32_t *out_ids,
                           float *out_ips, pf_query_stats *stats, int32_t flags, int32_t mem, void *stream) {
    return guard([&] {
        PF_CHECK(recalls, PF_EINVAL, "pf_search_batch: recalls is required");
        PF_CHECK((flags & ~(PF_BATCH_LEARNED | PF_BATCH_AUTOTUNE)) == 0, PF_EINVAL, "pf_search_batch: bad flags");
        PF_CHECK(!(order && (flags & PF_BATCH_LEARNED)), PF_EINVAL,
                 "pf_search_batch: give an order or PF_BATCH_LEARNED, not both");
        BatchCtl bc;
        bc.queue = true;
        bc.order = order;
        bc.learned = (flags & PF_BATCH_LEARNED) != 0;
        bc.autotune = (flags & PF_BATCH_AUTOTUNE) != 0;
        search_impl(ix, queries, m, ks, kmax, kmax, recalls, 0.0, opts, out_ids, out_ips, stats, mem, stream, bc);
    });
}

PF_API int pf_search(pf_index *ix, const float *queries, int64_t m, int32_t k, double recall, int32_t *out_ids,
                     float *out_ips, pf_query_stats *stats, int32_t mem, void *stream) {
    return pf_search_ex(ix, queries, m, k, recall, nullptr, out_ids, out_ips, stats, mem, stream);
}

PF_API int pf_hash(pf_index *ix, const float *x, int64_t m, uint32_t *codes, uint64_t *sketches, int32_t mem,
                   void *stream) {
    return guard([&] {
        PF_CHECK(ix && x && m >= 0, PF_EINVAL, "pf_hash: bad arguments");
        PF_CHECK(mem == PF_HOST || mem == PF_DEVICE, PF_EINVAL, "pf_hash: bad mem");
        if (m == 0) return;
        hipStream_t s = as_stream(stream);
        float *qX;
        uint32_t *qc;
        uint64_t *qs;
        prepare_rows_for(*ix, x, m, mem, s, &qX, &qc, &qs);
        const hipMemcpyKind kind = mem == PF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        if (codes) PF_HIP(hipMemcpyAsync(codes, qc, (size_t)m * ix->L * sizeof(uint32_t), kind, s));
        if (sketches) PF_HIP(hipMemcpyAsync(sketches, qs, (size_t)m * ix->M * sizeof(uint64_t), kind, s));
        PF_HIP(hipStreamSynchronize(s));
    });
}

PF_API int pf_export(const pf_index *ix, int32_t what, void *dst, int64_t dst_bytes, int32_t mem, void *stream) {
    return guard([&] {
        PF_CHECK(ix && dst, PF_EINVAL, "pf_export: null argument");
        PF_CHECK(mem == PF_HOST || mem == PF_DEVICE, PF_EINVAL, "pf_export: bad mem");
        hipStream_t s = as_stream(stream);
        const hipMemcpyKind kind = mem == PF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        const int64_t n = ix->n;
        auto need = [&](int64_t b) {
            PF_CHECK(dst_bytes >= b, PF_EINVAL, "pf_export: destination too small");
        };
        switch (what) {
        case PF_EXPORT_POINTS: {
            need(n * ix->d * 4);
            DevBuf X;
            X.alloc((size_t)n * ix->dpad * sizeof(float));
            launch_join_planes(ix->Xh.as<uint16_t>(), ix->Xl.as<uint16_t>(), n, ix->dpad, X.as<float>(), s);
            PF_HIP(hipMemcpy2DAsync(dst, (size_t)ix->d * 4, X.p, (size_t)ix->dpad * 4, (size_t)ix->d * 4,
                                    (size_t)n, kind, s));
            PF_HIP(hipStreamSynchronize(s));
            break;
        }
        case PF_EXPORT_HYPERPLANES: {
            const int64_t b = ((ix->family == PF_FAMILY_FHTCP ? 0 : ix->pool ? (int64_t)ix->pool : (int64_t)ix->L * ix->K) +
                               64ll * ix->M) * ix->d * 4;
            need(b);
            PF_HIP(hipMemcpyAsync(dst, ix->hp.p, (size_t)b, kind, s));
            break;
        }
        case PF_EXPORT_CODES: {
            need((int64_t)ix->L * n * 4);
            DevBuf codes;
            codes.alloc((size_t)ix->L * n * 4);
            join_codes(ix->tsuf.p, ix->off.as<uint32_t>(), n, ix->L, ix->K, ix->P, codes.as<uint32_t>(), s);
            PF_HIP(hipMemcpyAsync(dst, codes.p, (size_t)ix->L * n * 4, kind, s));
            PF_HIP(hipStreamSynchronize(s));
            break;
        }
        case PF_EXPORT_IDX: {
            need((int64_t)ix->L * n * 4);
            const int64_t count = (int64_t)ix->L * n;
            if (ix->posb == 4) {
                PF_HIP(hipMemcpyAsync(dst, ix->tpos.p, (size_t)count * 4, kind, s));
            } else if (mem == PF_DEVICE) {
                unpack_positions(ix->tpos.as<uint8_t>(), count, ix->posb, static_cast<uint32_t *>(dst), s);
            } else {
                DevBuf pos;
                pos.alloc((size_t)count * 4);
                unpack_positions(ix->tpos.as<uint8_t>(), count, ix->posb, pos.as<uint32_t>(), s);
                PF_HIP(hipMemcpyAsync(dst, pos.p, (size_t)count * 4, kind, s));
                PF_HIP(hipStreamSynchronize(s));
            }
            break;
        }
        case PF_EXPORT_SKETCHES:
            need((int64_t)ix->L * n * 8);
            PF_HIP(hipMemcpyAsync(dst, ix->tsk.p, (size_t)ix->L * n * 8, kind, s));
            break;
        case PF_EXPORT_OFFSETS: {
            const int64_t b = (int64_t)ix->L * ((1ll << ix->P) + 1) * 4;
            need(b);
            PF_HIP(hipMemcpyAsync(dst, ix->off.p, (size_t)b, kind, s));
            break;
        }
        case PF_EXPORT_CP_TABLE: {
            PF_CHECK(ix->family == PF_FAMILY_FHTCP, PF_EINVAL, "pf_export: the index has no cross-polytope table");
            const int64_t b = 41ll * (ix->cp_ell + 1) * 8;
            need(b);
            PF_HIP(hipMemcpyAsync(dst, ix->cptab.p, (size_t)b, kind, s));
            break;
        }
        case PF_EXPORT_ROWS8: {
            const size_t w = 8 + (size_t)ix->dpad;
            need(n * (int64_t)w);
            char *o = static_cast<char *>(dst);
            if (ix->qco) {
                PF_HIP(hipMemcpy2DAsync(o, w, ix->Xq.p, (size_t)ix->rq, w, (size_t)n, kind, s));
            } else {
                PF_HIP(hipMemcpy2DAsync(o, w, ix->Xqh.p, 8, 8, (size_t)n, kind, s));
                PF_HIP(hipMemcpy2DAsync(o + 8, w, ix->Xq.p, (size_t)ix->rq, (size_t)ix->dpad, (size_t)n, kind, s));
            }
            break;
        }
        case PF_EXPORT_POOL_SEL: {
            PF_CHECK(ix->pool > 0, PF_EINVAL, "pf_export: the index has no pool");
            const int64_t b = (int64_t)ix->L * ix->K * 4;
            need(b);
            PF_HIP(hipMemcpyAsync(dst, ix->psel.p, (size_t)b, kind, s));
            break;
        }
        default:
            throw Error(PF_EINVAL, "pf_export: unknown structure");
        }
        PF_HIP(hipStreamSynchronize(s));
    });
}

PF_API int pf_index_info(const pf_index *ix, pf_info *info) {
    return guard([&] {
        PF_CHECK(ix && info, PF_EINVAL, "pf_index_info: null argument");
        pf_info r{};
        r.n = ix->n;
        r.d = ix->d;
        r.L = ix->L;
        r.K = ix->K;
        r.M = ix->M;
        r.P = ix->P;
        r.pool = ix->pool;
        r.family = ix->family;
        r.bytes_budget_rule = ix->bytes_rule;
        r.bytes_device = ix->Xh.bytes + ix->Xl.bytes + ix->Xq.bytes + ix->Xqh.bytes + ix->hp.bytes + ix->hcolrow.bytes + ix->hbf.bytes + ix->hbeta.bytes +
                         ix->psel.bytes + ix->cpsign.bytes + ix->cptab.bytes + ix->tsuf.bytes + ix->tpos.bytes + ix->tsk.bytes + ix->off.bytes;
        r.build_ms = ix->build_ms;
        r.pos_bytes = ix->posb;
        *info = r;
    });
}

PF_API int pf_last_timing(const pf_index *ix, pf_timing *t) {
    return guard([&] {
        PF_CHECK(ix && t, PF_EINVAL, "pf_last_timing: null argument");
        *t = ix->timing;
    });
}

PF_API void pf_free_index(pf_index *ix) { delete ix; }
