// The adaptive query (Algorithm 1, adaptive-kNN(q, k, delta)) on the sorted arrays of
// Sec. 4.1-4.2, level-synchronous: in round i (prefix length i = K .. 1) every table
// contributes the entries newly covered by its window, the window growing by whole
// segments of B entries (Sec. 4.2, App. C) while the next entry shares the query's
// i-bit prefix; candidates pass the sketch filter when popcount(sketch xor query
// sketch) <= tau (Sec. 4.2 "Filtering candidate points", tau from Sec. 5.1, fixed for
// the round); passing points not yet re-ranked get their exact FP32 inner product and
// enter the top-k; after all tables the stopping bound of Lemma 1 is tested in FP64.
// Round 0 is a linear scan.
//
// k_ranges: for every (query, table) the bounds [lo_i, hi_i) of the entries sharing the
// query's i-bit prefix for the levels i > P that the P-bit prefix table cannot answer.
// k_search: one workgroup per query slot (static slot -> query assignment).
#include "pf_internal.h"

namespace pf {

// --------------------------------------------------------------------------- ranges
static constexpr int kScanMax = 1024; // larger prefix buckets use binary searches

// one wave per (table j, query q); ranges[q][j][i - P - 1] = (lo_i, hi_i), i = P+1..K
__global__ __launch_bounds__(256) void k_ranges(const uint32_t *__restrict__ tcode,
                                                const uint32_t *__restrict__ off, int64_t n,
                                                int32_t L, int32_t K, int32_t P,
                                                const uint32_t *__restrict__ qcode, int64_t m,
                                                int64_t q0, uint32_t *__restrict__ ranges) {
    const int lane = threadIdx.x & 63;
    const int32_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t q = q0 + blockIdx.y;
    if (j >= L) return;
    const int32_t nl = K - P;
    const uint32_t qc = qcode[(int64_t)j * m + q];
    const int64_t np1 = ((int64_t)1 << P) + 1;
    const uint32_t b = qc >> (K - P);
    const uint32_t B0 = off[(int64_t)j * np1 + b];
    const uint32_t B1 = off[(int64_t)j * np1 + b + 1];
    const uint32_t *tc = tcode + (int64_t)j * n;
    uint32_t *out = ranges + ((q - q0) * L + j) * (int64_t)nl * 2;
    if (B1 - B0 <= (uint32_t)kScanMax) {
        // count over the bucket: lo_i = B0 + #{code < qc, lcp < i},
        // hi_i = B0 + #{code < qc} + #{code >= qc, lcp >= i}
        uint32_t mylo = 0, myhi = 0, nlt = 0;
        const int mylevel = P + 1 + lane; // lane < nl holds level P+1+lane
        for (uint32_t e0 = B0; e0 < B1; e0 += 64) {
            const uint32_t e = e0 + lane;
            const bool valid = e < B1;
            const uint32_t code = valid ? tc[e] : qc;
            const uint32_t x = (code ^ qc) << (32 - K);
            const int lcp = x ? __clz(x) : K;
            const bool lt = valid && code < qc;
            nlt += (uint32_t)__popcll(__ballot(lt));
            for (int i = 0; i < nl; ++i) {
                const int lev = P + 1 + i;
                const uint64_t blo = __ballot(lt && lcp < lev);
                const uint64_t bhi = __ballot(valid && !lt && lcp >= lev);
                if (lane == i) {
                    mylo += (uint32_t)__popcll(blo);
                    myhi += (uint32_t)__popcll(bhi);
                }
            }
        }
        (void)mylevel;
        if (lane < nl) {
            out[2 * lane] = B0 + mylo;
            out[2 * lane + 1] = B0 + nlt + myhi;
        }
    } else if (lane < 2 * nl) {
        // lane 2i + s: level P+1+i, s = 0 lower bound, s = 1 upper bound
        const int lev = P + 1 + (lane >> 1);
        const uint64_t pre = (uint64_t)(qc >> (K - lev));
        const uint64_t target = (lane & 1) ? ((pre + 1) << (K - lev)) : (pre << (K - lev));
        uint32_t lo = B0, hi = B1;
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if ((uint64_t)tc[mid] < target)
                lo = mid + 1;
            else
                hi = mid;
        }
        out[lane] = lo;
    }
}

void launch_ranges(const Index &ix, const SearchArgs &a, uint32_t *ranges, hipStream_t s) {
    if (ix.K <= ix.P || a.m <= 0) return;
    const int64_t chunk = 65535;
    for (int64_t q0 = 0; q0 < a.m; q0 += chunk) {
        const int64_t mq = std::min<int64_t>(chunk, a.m - q0);
        hipLaunchKernelGGL(k_ranges, dim3((ix.L + 3) / 4, (unsigned)mq), dim3(256), 0, s,
                           ix.tcode.as<uint32_t>(), ix.off.as<uint32_t>(), ix.n, ix.L, ix.K, ix.P,
                           a.qcode, a.m, q0, ranges + q0 * ix.L * (int64_t)(ix.K - ix.P) * 2);
        PF_HIP(hipGetLastError());
    }
}

// --------------------------------------------------------------------------- search
static constexpr int NT = 256;
static constexpr int EPT = 2;              // flat entries per thread per filter chunk
static constexpr int CH = NT * EPT;        // entries per filter chunk
static constexpr int RB = 256;             // re-rank once this many candidates wait
static constexpr int PCAP = CH + RB;       // pending capacity
static constexpr int CC = 1024;            // candidate buffer (power of two)
static constexpr int RCAP = 16384;         // per-slot list of re-ranked ids (for clearing)
static constexpr double kPi = 3.14159265358979323846264338327950288;

struct SearchK {
    const float *X;
    const uint32_t *tcode, *tidx, *off;
    const uint64_t *tsk;
    int64_t n;
    int32_t dpad, L, K, M, P, B;
    const float *Q;
    const uint32_t *qcode;
    const uint64_t *qsk;
    const uint32_t *ranges;
    int64_t m;
    const int32_t *ks;
    int32_t kconst, kmax;
    const double *recalls;
    double recall_const, eps;
    int32_t rule, filter;
    uint32_t *bitmap;
    int64_t bwords;
    uint32_t *rlist;
    int32_t *out_ids;
    float *out_ips;
    pf_query_stats *stats;
};

struct SearchShared {
    unsigned long long c_pass;
    long long c_scan, c_rerank;
    unsigned long long thr;
    int pend_cnt, rr_cnt, cand_cnt, top_cnt;
    int tau_int, stop;
    uint32_t wsum[4];
};

__device__ __forceinline__ uint32_t f2ord(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_ip(unsigned long long key) {
    const uint32_t o = (uint32_t)(key >> 32);
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint32_t key_id(unsigned long long key) {
    return 0xFFFFFFFFu - (uint32_t)key;
}
// larger key = better: inner product descending, then position ascending
__device__ __forceinline__ unsigned long long mkkey(float ip, uint32_t id) {
    return ((unsigned long long)f2ord(ip) << 32) | (unsigned long long)(0xFFFFFFFFu - id);
}

// Inner product in the fixed FP32 order: lane r (of a 16-lane group) sums the products
// of the elements 64 t + 4 r + c in increasing order, no fused multiply-add; the sixteen
// partial sums are combined by s_r + s_{r^8}, then ^4, ^2, ^1.  Rows are zero padded to
// dpad; zero products leave a partial sum unchanged.
__device__ __forceinline__ float dot_canon(const float *__restrict__ xrow, const float *qv, int32_t dpad,
                                           int r) {
    float s = 0.0f;
    for (int base = 4 * r; base < dpad; base += 64) {
        const float4 xv = *reinterpret_cast<const float4 *>(xrow + base);
        const float4 qq = *reinterpret_cast<const float4 *>(qv + base);
        s = s + xv.x * qq.x;
        s = s + xv.y * qq.y;
        s = s + xv.z * qq.z;
        s = s + xv.w * qq.w;
    }
    s = s + __shfl_xor(s, 8, 16);
    s = s + __shfl_xor(s, 4, 16);
    s = s + __shfl_xor(s, 2, 16);
    s = s + __shfl_xor(s, 1, 16);
    return s;
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

// Failure bound of Lemma 1 with the sketch filter (log of an upper bound on the
// probability of missing a true neighbour after level i): a true neighbour at angle
// <= theta_k is missed only if, for each sketch s, its sketch fails the filter (pass
// probability >= q, the threshold only shrinks over levels) or none of the g_s tables
// reading sketch s (j mod M = s) holds it in its window (probability (1 - p^i)^{g_s}).
// Each factor 1 - q + q (1 - p^i)^{g_s} is evaluated without cancellation.
__device__ double filter_bound(double theta, double pw, int tau_int, int L, int M) {
    const double q = binom_cdf64(theta / kPi, tau_int);
    const double l1p = log1p(-pw);
    double term = 0.0;
    for (int s = 0; s < M && s < L; ++s) {
        const int g = L / M + (s < L % M ? 1 : 0);
        const double a = (double)g * l1p;
        const double x = q * expm1(a);
        term = term + ((x > -0.5) ? log1p(x) : log((1.0 - q) + q * exp(a)));
    }
    return term;
}

// inclusive scan of a[0..N) in LDS by all NT threads
__device__ void block_scan_incl(uint32_t *a, int N, uint32_t *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int per = (N + NT - 1) / NT;
    const int s0 = tid * per, s1 = min(N, s0 + per);
    uint32_t tot = 0;
    for (int i = s0; i < s1; ++i) tot += a[i];
    uint32_t v = tot;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    uint32_t pre = v - tot;
    for (int i = 0; i < w; ++i) pre += wsum[i];
    for (int i = s0; i < s1; ++i) {
        pre += a[i];
        a[i] = pre;
    }
    __syncthreads();
}

// number of elements of the descending array arr[0..len) that are greater than key
__device__ __forceinline__ int count_greater(const unsigned long long *arr, int len,
                                             unsigned long long key) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (arr[mid] > key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// top <- best k of top u cand (cand unsorted); called by all threads
__device__ void merge_all(unsigned long long *top, unsigned long long *ntop, unsigned long long *cand,
                          SearchShared &sh, int k) {
    __syncthreads();
    const int c = sh.cand_cnt;
    if (c == 0) return;
    int P2 = 1;
    while (P2 < c) P2 <<= 1;
    for (int t = c + threadIdx.x; t < P2; t += NT) cand[t] = 0ull;
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (P2 >> 1); t += NT) {
                const int i = 2 * t - (t & (stride - 1));
                const int l = i + stride;
                const unsigned long long a = cand[i], b = cand[l];
                const bool desc = (i & size) == 0;
                if (desc ? (a < b) : (a > b)) {
                    cand[i] = b;
                    cand[l] = a;
                }
            }
            __syncthreads();
        }
    }
    const int tc = sh.top_cnt;
    const int newc = min(k, tc + c);
    for (int t = threadIdx.x; t < c; t += NT) {
        const int r = t + count_greater(top, tc, cand[t]);
        if (r < k) ntop[r] = cand[t];
    }
    for (int t = threadIdx.x; t < tc; t += NT) {
        const int r = t + count_greater(cand, c, top[t]);
        if (r < k) ntop[r] = top[t];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < newc; t += NT) top[t] = ntop[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        sh.top_cnt = newc;
        sh.cand_cnt = 0;
        sh.thr = (newc == k) ? top[k - 1] : 0ull;
    }
    __syncthreads();
}

struct Lds {
    unsigned long long *top, *ntop, *cand, *tq;
    uint32_t *pending, *rr, *clo, *chi, *qc, *segBeg, *segStart;
    float *qv;
    SearchShared *sh;
};

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

__host__ __device__ inline size_t search_lds_layout(int L, int kmax, int dpad, Lds *o, void *base) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) {
        char *p = b ? b + off : nullptr;
        off = align16(off + bytes);
        return p;
    };
    Lds l;
    l.sh = reinterpret_cast<SearchShared *>(take(sizeof(SearchShared)));
    l.top = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * kmax));
    l.ntop = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * kmax));
    l.cand = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * CC));
    l.tq = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * L));
    l.pending = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * PCAP));
    l.rr = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * PCAP));
    l.clo = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * L));
    l.chi = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * L));
    l.qc = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * L));
    l.segBeg = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * 2 * L));
    l.segStart = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * (2 * L + 1)));
    l.qv = reinterpret_cast<float *>(take(sizeof(float) * dpad));
    if (o) *o = l;
    return off;
}

__device__ __forceinline__ void level_range(const SearchK &p, int32_t j, int32_t i, uint32_t qc, int64_t q,
                                            uint32_t &lo, uint32_t &hi) {
    if (i > p.P) {
        const uint32_t *r = p.ranges + ((q * p.L + j) * (int64_t)(p.K - p.P) + (i - p.P - 1)) * 2;
        lo = r[0];
        hi = r[1];
    } else {
        const int64_t np1 = ((int64_t)1 << p.P) + 1;
        const uint32_t *o = p.off + (int64_t)j * np1;
        const uint32_t pre = (i == 0) ? 0u : (qc >> (p.K - i));
        lo = o[(int64_t)pre << (p.P - i)];
        hi = o[((int64_t)pre + 1) << (p.P - i)];
    }
}

// Re-rank the waiting candidates: position lookup, de-duplication against every point
// already re-ranked (one bit per point, per slot), inner product, top-k candidates.
__device__ void process_pending(const SearchK &p, Lds &l, int k, uint32_t *bm, uint32_t *rl) {
    SearchShared &sh = *l.sh;
    const int tid = threadIdx.x;
    const int pc = sh.pend_cnt;
    for (int t = tid; t < pc; t += NT) {
        const uint32_t x = p.tidx[l.pending[t]];
        const uint32_t bit = 1u << (x & 31u);
        const uint32_t old = atomicOr(&bm[x >> 5], bit);
        if (!(old & bit)) {
            const int r = atomicAdd(&sh.rr_cnt, 1);
            l.rr[r] = x;
        }
    }
    __syncthreads();
    const int rc = sh.rr_cnt;
    const long long done = sh.c_rerank;
    for (int t = tid; t < rc; t += NT)
        if (done + t < RCAP) rl[done + t] = l.rr[t];
    const int g = tid >> 4, r = tid & 15;
    const bool full = sh.top_cnt == k;
    const unsigned long long thr = sh.thr;
    for (int t = g; t < rc; t += NT / 16) {
        const uint32_t x = l.rr[t];
        const float ip = dot_canon(p.X + (int64_t)x * p.dpad, l.qv, p.dpad, r);
        if (r == 0) {
            const unsigned long long key = mkkey(ip, x);
            if (!full || key > thr) {
                const int c = atomicAdd(&sh.cand_cnt, 1);
                l.cand[c] = key;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        sh.c_rerank += rc;
        sh.rr_cnt = 0;
        sh.pend_cnt = 0;
    }
    __syncthreads();
}

__global__ __launch_bounds__(NT) void k_search(SearchK p) {
    extern __shared__ __align__(16) unsigned char smem[];
    Lds l;
    search_lds_layout(p.L, p.kmax, p.dpad, &l, smem);
    SearchShared &sh = *l.sh;
    const int tid = threadIdx.x;
    uint32_t *bm = p.bitmap + (int64_t)blockIdx.x * p.bwords;
    uint32_t *rl = p.rlist + (int64_t)blockIdx.x * RCAP;
    const int32_t L = p.L, K = p.K;
    const int64_t n = p.n;

    for (int64_t q = blockIdx.x; q < p.m; q += gridDim.x) {
        const int k = p.ks ? max(1, min(p.ks[q], p.kmax)) : p.kconst;
        const double recall = p.recalls ? p.recalls[q] : p.recall_const;
        const double lndelta = log(1.0 - recall);
        for (int c = tid; c < p.dpad; c += NT) l.qv[c] = p.Q[q * p.dpad + c];
        for (int32_t j = tid; j < L; j += NT) {
            const uint32_t qc = p.qcode[(int64_t)j * p.m + q];
            l.qc[j] = qc;
            l.tq[j] = p.qsk[(int64_t)(j % p.M) * p.m + q];
            uint32_t lo, hi;
            level_range(p, j, K, qc, q, lo, hi);
            l.clo[j] = lo;
            l.chi[j] = lo;
        }
        if (tid == 0) {
            sh.c_pass = 0;
            sh.c_scan = 0;
            sh.c_rerank = 0;
            sh.thr = 0;
            sh.pend_cnt = sh.rr_cnt = sh.cand_cnt = sh.top_cnt = 0;
            sh.tau_int = 64;
            sh.stop = 0;
        }
        __syncthreads();
        unsigned long long my_pass = 0;
        int stop_level = 0;
        for (int32_t i = K; i >= 1; --i) {
            // new segments of every table for this level
            for (int32_t j = tid; j < L; j += NT) {
                uint32_t lo, hi;
                level_range(p, j, i, l.qc[j], q, lo, hi);
                const uint32_t a = l.clo[j], b = l.chi[j];
                uint32_t na = a, nb = b;
                if (a > lo) {
                    const uint64_t st = ((uint64_t)(a - lo) + p.B - 1) / p.B * (uint64_t)p.B;
                    na = (a > st) ? (uint32_t)(a - st) : 0u;
                }
                if (b < hi) {
                    const uint64_t st = ((uint64_t)(hi - b) + p.B - 1) / p.B * (uint64_t)p.B;
                    const uint64_t e = (uint64_t)b + st;
                    nb = e < (uint64_t)n ? (uint32_t)e : (uint32_t)n;
                }
                l.segBeg[2 * j] = na;
                l.segBeg[2 * j + 1] = b;
                l.segStart[2 * j + 1] = a - na;
                l.segStart[2 * j + 2] = nb - b;
                l.clo[j] = na;
                l.chi[j] = nb;
            }
            if (tid == 0) l.segStart[0] = 0;
            __syncthreads();
            block_scan_incl(l.segStart + 1, 2 * L, sh.wsum);
            const uint32_t total = l.segStart[2 * L];
            const int tau = sh.tau_int;
            if (tid == 0) sh.c_scan += total;
            for (uint32_t base = 0; base < total; base += CH) {
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const uint32_t f = base + u * NT + tid;
                    if (f < total) {
                        int lo = 0, hi = 2 * L;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (l.segStart[mid] <= f)
                                lo = mid;
                            else
                                hi = mid;
                        }
                        const int32_t j = lo >> 1;
                        const uint32_t pos = l.segBeg[lo] + (f - l.segStart[lo]);
                        const uint32_t e = (uint32_t)j * (uint32_t)n + pos;
                        const int h = __popcll(p.tsk[e] ^ l.tq[j]);
                        if (h <= tau) {
                            ++my_pass;
                            const int slot = atomicAdd(&sh.pend_cnt, 1);
                            l.pending[slot] = e;
                        }
                    }
                }
                // decide from a value no thread can change until the second barrier
                __syncthreads();
                const bool proc = sh.pend_cnt >= RB || base + CH >= total;
                __syncthreads();
                if (proc) {
                    process_pending(p, l, k, bm, rl);
                    if (sh.cand_cnt > CC - PCAP) merge_all(l.top, l.ntop, l.cand, sh, k);
                }
            }
            merge_all(l.top, l.ntop, l.cand, sh, k);
            if (tid == 0) {
                int stop = 0;
                if (sh.top_cnt == k) {
                    double ipk = (double)key_ip(l.top[k - 1]);
                    ipk = ipk > 1.0 ? 1.0 : (ipk < -1.0 ? -1.0 : ipk);
                    const double theta = acos(ipk);
                    const double lnp = log1p(-theta / kPi);
                    const double pw = exp((double)i * lnp);
                    if (p.rule == PF_RULE_ALG1)
                        stop = ((double)L * pw >= -lndelta);
                    else if (p.rule == PF_RULE_EXACT)
                        stop = ((double)L * log1p(-pw) <= lndelta);
                    else
                        stop = filter_bound(theta, pw, sh.tau_int, L, p.M) <= lndelta;
                    if (p.filter) {
                        const double t = (1.0 + p.eps) * 64.0 * theta / kPi;
                        const double ft = floor(t);
                        sh.tau_int = ft >= 64.0 ? 64 : (ft < -1.0 ? -1 : (int)ft);
                    }
                }
                sh.stop = stop;
            }
            __syncthreads();
            if (sh.stop) {
                stop_level = i;
                break;
            }
        }
        if (!sh.stop) {
            // level 0: linear scan over every point not yet re-ranked
            const int g = tid >> 4, r = tid & 15;
            for (int64_t base = 0; base < n; base += 16 * 16) {
                const bool full = sh.top_cnt == k;
                const unsigned long long thr = sh.thr;
                for (int u = 0; u < 16; ++u) {
                    const int64_t x = base + u * 16 + g;
                    if (x >= n) break;
                    const uint32_t w = __hip_atomic_load(&bm[x >> 5], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    if ((w >> (x & 31)) & 1u) continue;
                    const float ip = dot_canon(p.X + x * p.dpad, l.qv, p.dpad, r);
                    if (r == 0) {
                        const unsigned long long key = mkkey(ip, (uint32_t)x);
                        if (!full || key > thr) {
                            const int c = atomicAdd(&sh.cand_cnt, 1);
                            l.cand[c] = key;
                        }
                    }
                }
                __syncthreads();
                const bool flush = sh.cand_cnt > CC - 256;
                __syncthreads();
                if (flush) merge_all(l.top, l.ntop, l.cand, sh, k);
            }
            merge_all(l.top, l.ntop, l.cand, sh, k);
            if (tid == 0) sh.c_rerank = n;
            stop_level = 0;
        }
        atomicAdd(&sh.c_pass, my_pass);
        __syncthreads();
        for (int t = tid; t < p.kmax; t += NT) {
            const int64_t o = q * p.kmax + t;
            if (t < k) {
                const unsigned long long key = l.top[t];
                p.out_ids[o] = (int32_t)key_id(key);
                if (p.out_ips) p.out_ips[o] = key_ip(key);
            } else {
                p.out_ids[o] = -1;
                if (p.out_ips) p.out_ips[o] = -INFINITY;
            }
        }
        if (tid == 0 && p.stats) {
            pf_query_stats st;
            st.stop_level = stop_level;
            st.reserved = 0;
            st.c_scan = sh.c_scan;
            st.c_pass = (int64_t)sh.c_pass;
            st.c_rerank = sh.c_rerank;
            p.stats[q] = st;
        }
        // clear this slot's de-duplication bits for the next query
        const long long nr = sh.c_rerank;
        if (sh.stop && nr <= RCAP) {
            for (long long t = tid; t < nr; t += NT) bm[rl[t] >> 5] = 0u;
        } else {
            for (int64_t t = tid; t < p.bwords; t += NT) bm[t] = 0u;
        }
        __threadfence();
        __syncthreads();
    }
}

int64_t search_slots(const Index &ix, int64_t m) {
    const int64_t per_cu = 8;
    return std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)ix.num_cus * per_cu));
}

void launch_search(Index &ix, const SearchArgs &a, const uint32_t *ranges, hipStream_t s) {
    if (a.m <= 0) return;
    const int64_t slots = search_slots(ix, a.m);
    const int64_t bwords = (ix.n + 31) / 32;
    const size_t bm_bytes = (size_t)slots * bwords * sizeof(uint32_t);
    if (ix.bitmap.bytes < bm_bytes) {
        // every query leaves its slot's bits cleared, so zero only a fresh allocation
        ix.bitmap.alloc(bm_bytes);
        launch_fill_u32(ix.bitmap.as<uint32_t>(), (int64_t)(ix.bitmap.bytes / 4), 0u, s);
    }
    ix.rlist.ensure((size_t)slots * RCAP * sizeof(uint32_t));
    SearchK p;
    p.X = ix.X.as<float>();
    p.tcode = ix.tcode.as<uint32_t>();
    p.tidx = ix.tidx.as<uint32_t>();
    p.off = ix.off.as<uint32_t>();
    p.tsk = ix.tsk.as<uint64_t>();
    p.n = ix.n;
    p.dpad = ix.dpad;
    p.L = ix.L;
    p.K = ix.K;
    p.M = ix.M;
    p.P = ix.P;
    p.B = a.B;
    p.Q = a.Q;
    p.qcode = a.qcode;
    p.qsk = a.qsk;
    p.ranges = ranges;
    p.m = a.m;
    p.ks = a.ks;
    p.kconst = a.kconst;
    p.kmax = a.kmax;
    p.recalls = a.recalls;
    p.recall_const = a.recall_const;
    p.eps = a.eps;
    p.rule = a.rule;
    p.filter = a.filter;
    p.bitmap = ix.bitmap.as<uint32_t>();
    p.bwords = bwords;
    p.rlist = ix.rlist.as<uint32_t>();
    p.out_ids = a.out_ids;
    p.out_ips = a.out_ips;
    p.stats = a.stats;
    const size_t lds = search_lds_layout(ix.L, a.kmax, ix.dpad, nullptr, nullptr);
    PF_HIP(hipFuncSetAttribute((const void *)k_search, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(k_search, dim3((unsigned)slots), dim3(NT), lds, s, p);
    PF_HIP(hipGetLastError());
}

} // namespace pf
