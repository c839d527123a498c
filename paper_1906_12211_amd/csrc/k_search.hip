// The adaptive query (Algorithm 1, adaptive-kNN(q, k, delta)) on the sorted arrays of
// Sec. 4.1-4.2, level-synchronous: in round i (prefix length i = K .. 1) every table
// contributes the entries newly covered by its window, the window growing by whole
// segments of B entries (Sec. 4.2, App. C) while the next entry shares the query's
// i-bit prefix; candidates pass the sketch filter when popcount(sketch xor query
// sketch) <= tau (Sec. 4.2 "Filtering candidate points", tau from Sec. 5.1, fixed for
// the round); passing points get their exact FP32 inner product (unless an upper bound
// of it from an 8-bit or the 16-bit copy of the row shows they cannot enter the top-k)
// and enter the top-k; after all tables the stopping bound of Lemma 1 is tested in FP64.
// The last round, i = 0, is a linear scan.  The ranges of the levels i > P (k_ranges.hip)
// and the decision tables of a round (k_rules.hip) are computed before the walk.
#include "pf_device.h"
#include "pf_internal.h"

#include <type_traits>

namespace pf {

// --------------------------------------------------------------------------- search
// One wave (a 64-lane workgroup) per query slot.  A query's whole walk -- segments,
// sketch filter, re-rank, top-k, stopping test -- runs inside its wave without
// workgroup barriers (lanes exchange data through the wave's own LDS region in program
// order, compaction by ballot), so the many query waves resident on a CU hide each
// other's memory latency.  Queries are taken either statically (slot s answers queries
// s, s + G, ...) or from a device work queue (an atomic counter, optionally through an
// order array), which balances queries of very different cost.
//
// Tile shape: EPT sketch loads in flight per lane in a filter chunk, U rows in flight
// per 16-lane group in the re-rank (UQ when bounding from the 8-bit summaries), WPE the
// query waves per SIMD the register allocation must allow (1 = no constraint), LATE:
// point ids read for passing entries only, one chunk late (else for every scanned
// entry, with its sketch); SH: the kernel is built for summary rows without header (one
// scale for all rows); NT: sketches and summary rows are read with non-temporal loads
// (streamed past the caches: neither is read again by the same query); DT = 64-float
// chunks per row (0 = any length).
static constexpr int WV = 64; // lanes per query wave
template <int EPT_, int U_, int WPE_ = 1, bool LATE_ = false, int UQ_ = U_, bool SH_ = false, int NT_ = 0>
struct Tile {
    static constexpr int EPT = EPT_;
    static constexpr int NT = NT_; // 1: sketch loads non-temporal, 2: sketch and summary-row loads
    static constexpr bool SH = SH_; // summary rows without header: one scale s8, sums up to a8
    static constexpr int U = U_;
    static constexpr int UQ = UQ_; // rows in flight per 16-lane group when bounding from 8-bit summaries
    static constexpr int WPE = WPE_;
    static constexpr bool LATE = LATE_;
    static constexpr int WCH = WV * EPT;       // entries per filter chunk
    static constexpr int RB = 128;             // re-rank once this many candidates wait
    static constexpr int UCAP = LATE ? WV : 0; // passing entries whose point id is still being read
    static constexpr int PCAP = WCH + RB + UCAP; // pending capacity
    static constexpr int CW = U >= 8 ? 256 : 128; // candidate buffer (power of two)
    static constexpr int RROWS = 4 * U;        // rows re-ranked per wave iteration
    static_assert(PCAP % WV == 0, "pending capacity must be a multiple of the wave size");
    static_assert(CW >= 4 * RROWS, "candidate buffer holds at least four re-rank slices");
};

struct SearchK {
    const uint16_t *Xh, *Xl; // upper / lower 16-bit planes of the n x dpad FP32 vectors
    int32_t hs, ls, spare;   // plane row lengths; lower halves of elements < spare sit in
                             // the upper row after its dpad upper halves
    int32_t prefilter;
    const uint8_t *Xq;  // 8-bit row summaries: rq bytes per row, int8 codes from byte qco,
    const uint8_t *Xqh; // headers (FP32 scale, int32 sum of |codes|) at the row's start
    int32_t rq, qco;    // (qco = 8) or, when qco = 0, in Xqh (8 bytes per row; every row's
    float s8;           // scale is then s8 and no row's sum exceeds a8, which kernels built
    int32_t a8;         // for that layout take instead of reading Xqh)
    const void *pos;    // table positions, PB bytes each (the kernel's parameter)
    const uint32_t *off;
    const uint64_t *tsk;
    int64_t n;
    int32_t dpad, L, K, M, P, B;
    const float *Q;
    const uint32_t *qcode;
    const uint64_t *qsk;
    const uint32_t *ranges;
    int64_t m;       // queries to answer (queue positions 0..m-1)
    int64_t qstride; // row stride of qcode / qsk (the batch size they were computed for)
    const int32_t *ks;
    int32_t kconst, kmax;
    const int32_t *qtab; // per-query row of stopw (nullable: 0)
    const float *tauv, *stopw;
    int32_t G;           // groups of repetitions per level, the stopping test after each (1..64)
    int32_t tmin;        // ... once at least tmin entries were read since the previous test
    int32_t filter;
    unsigned int *queue;  // work-queue counter (nullable: static assignment)
    const int32_t *order; // queue position -> query (nullable: identity)
    int32_t *out_ids;
    float *out_ips;
    pf_query_stats *stats;
    float us_per_tick; // microseconds per tick of the device's constant clock (wall_clock64)
};

// loads that stream past the caches when NT is set (each sketch and summary row is read
// once per query)
template <bool NT> __device__ __forceinline__ uint64_t ld_u64(const uint64_t *ptr) {
    if constexpr (NT)
        return __builtin_nontemporal_load(ptr);
    else
        return *ptr;
}
template <bool NT> __device__ __forceinline__ uint2 ld_u2(const uint8_t *ptr) {
    if constexpr (NT) {
        typedef uint32_t v2u __attribute__((ext_vector_type(2)));
        const v2u t = __builtin_nontemporal_load(reinterpret_cast<const v2u *>(ptr));
        return make_uint2(t.x, t.y);
    } else {
        return *reinterpret_cast<const uint2 *>(ptr);
    }
}

__device__ __forceinline__ float key_ip(unsigned long long key) { return float_of((uint32_t)(key >> 32)); }
__device__ __forceinline__ uint32_t key_id(unsigned long long key) { return 0xFFFFFFFFu - (uint32_t)key; }
// larger key = better: inner product descending, then position ascending
__device__ __forceinline__ unsigned long long mkkey(float ip, uint32_t id) {
    return ((unsigned long long)ord_of(ip) << 32) | (unsigned long long)(0xFFFFFFFFu - id);
}

// order this wave's LDS accesses: everything before is visible to every lane after
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// number of set bits of a wave mask in the lanes below this one (v_mbcnt)
__device__ __forceinline__ int lanes_below(uint64_t mk) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
}

// number of elements of the descending array arr[0..len) that are greater than key
__device__ __forceinline__ int count_greater(const unsigned long long *arr, int len, unsigned long long key) {
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

struct WLds {
    unsigned long long *top, *ntop, *cand, *tq;
    uint32_t *pending, *upos, *clo, *chi, *qc, *segBeg, *segStart, *segTab;
    uint32_t *qb, *qba; // query as bfloat16 pairs (round to nearest even) and their magnitudes
    uint32_t *q8;       // query int8 codes laid out like a summary row (8 zero bytes first)
    float *qv;
};

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Byte offsets of the wave's LDS arrays in the dynamic shared memory block.
struct LdsOff {
    uint32_t top, ntop, cand, tq, pending, upos, clo, chi, qc, segBeg, segStart, segTab, qb, qba, q8, qv, total;
};

// pcap, cw, ucap: the tile's pending, candidate and late-id capacities; rq: bytes of an
// 8-bit summary row
__host__ __device__ inline LdsOff search_lds_offsets(int L, int kmax, int dpad, int pcap, int cw, int ucap,
                                                     int rq) {
    LdsOff o;
    uint32_t off = 0;
    auto take = [&](size_t bytes) {
        const uint32_t at = off;
        off = (uint32_t)align16(off + bytes);
        return at;
    };
    o.top = take(sizeof(unsigned long long) * kmax);
    o.ntop = take(sizeof(unsigned long long) * kmax);
    o.cand = take(sizeof(unsigned long long) * cw);
    o.tq = take(sizeof(unsigned long long) * L);
    o.pending = take(sizeof(uint32_t) * pcap);
    o.upos = take(sizeof(uint32_t) * ucap);
    o.clo = take(sizeof(uint32_t) * L);
    o.chi = take(sizeof(uint32_t) * L);
    o.qc = take(sizeof(uint32_t) * L);
    o.segBeg = take(sizeof(uint32_t) * (2 * L + 1));
    o.segStart = take(sizeof(uint32_t) * (2 * L + 2));
    o.segTab = take(sizeof(uint32_t) * (2 * L + 1));
    o.qb = take(sizeof(uint32_t) * (dpad / 2));
    o.qba = take(sizeof(uint32_t) * (dpad / 2));
    o.q8 = take(rq);
    o.qv = take(sizeof(float) * dpad);
    o.total = off;
    return o;
}



// Per-query state kept in registers; every lane holds the same (wave-uniform) values.
struct QState {
    int k;
    int pend, cand, top;
    unsigned long long thr;
    float qt;    // query int8 scale t (q_i ~ t b_i)
    int32_t qB;  // sum_i |b_i|
    long long c_scan, c_pass, c_rerank, c_exact, c_upper, c_q8;
};

// top <- best k distinct points of top u cand[0..cand) (the accumulator's flush; cand
// unsorted): bitonic sort of the candidates, then copies of a point -- equal keys,
// since a point's inner product is the same each time it is re-ranked -- are dropped
// (adjacent in the sorted candidates, or already in the top-k), and every remaining
// element's rank in the union is its index in its own list plus the count of greater
// elements in the other.
__device__ void wave_merge(WLds &l, QState &st) {
    const int lane = threadIdx.x;
    int c = st.cand;
    if (c == 0) return;
    wsync();
    unsigned long long *cand = l.cand;
    int P2 = 1;
    while (P2 < c) P2 <<= 1;
    for (int t = c + lane; t < P2; t += WV) cand[t] = 0ull;
    wsync();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < (P2 >> 1); t += WV) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const unsigned long long a = cand[i], b = cand[j];
                const bool desc = (i & size) == 0;
                if (desc ? (a < b) : (a > b)) {
                    cand[i] = b;
                    cand[j] = a;
                }
            }
            wsync();
        }
    }
    const int tc = st.top, k = st.k;
    {
        // drop copies; in place, one 64-element block at a time (reads before writes)
        int w = 0;
        for (int t0 = 0; t0 < c; t0 += WV) {
            const int t = t0 + lane;
            unsigned long long key = 0;
            bool keep = false;
            if (t < c) {
                key = cand[t];
                keep = (t == 0 || cand[t - 1] != key);
                if (keep) {
                    const int g = count_greater(l.top, tc, key);
                    keep = !(g < tc && l.top[g] == key);
                }
            }
            wsync();
            const uint64_t mk = __ballot(keep);
            if (keep) cand[w + lanes_below(mk)] = key;
            w += __popcll(mk);
            wsync();
        }
        c = w;
    }
    const int newc = min(k, tc + c);
    for (int t = lane; t < c; t += WV) {
        const int r = t + count_greater(l.top, tc, cand[t]);
        if (r < k) l.ntop[r] = cand[t];
    }
    for (int t = lane; t < tc; t += WV) {
        const int r = t + count_greater(cand, c, l.top[t]);
        if (r < k) l.ntop[r] = l.top[t];
    }
    wsync();
    for (int t = lane; t < newc; t += WV) l.top[t] = l.ntop[t];
    wsync();
    st.top = newc;
    st.cand = 0;
    st.thr = (newc == k) ? l.top[k - 1] : 0ull;
}

// Element values of a row from its two planes: lane-local 4-element group, upper
// halves h, lower halves w, two elements per 32-bit word (element 2j in the low half).
__device__ __forceinline__ float4 join4(uint2 h, uint2 w) {
    return make_float4(__uint_as_float((h.x << 16) | (w.x & 0xFFFFu)), __uint_as_float((h.x & 0xFFFF0000u) | (w.x >> 16)),
                       __uint_as_float((h.y << 16) | (w.y & 0xFFFFu)), __uint_as_float((h.y & 0xFFFF0000u) | (w.y >> 16)));
}
__device__ __forceinline__ float4 upper4(uint2 h) {
    return make_float4(__uint_as_float(h.x << 16), __uint_as_float(h.x & 0xFFFF0000u), __uint_as_float(h.y << 16),
                       __uint_as_float(h.y & 0xFFFF0000u));
}
// Sum over the 16 lanes of a DPP row in the order s_r + s_{r^8}, then ^4, ^2, ^1, left in
// every lane.  row_ror:m hands lane r the value of lane (r + m) mod 16; after the steps
// before it that value equals lane r^m's (the values are equal within each coset of the
// bits already combined, and IEEE addition commutes), so the result is bit-identical to
// the butterfly written with exchanges of lanes r and r^m.
template <int CTRL> __device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row_sum16(float s) {
    s = s + dpp_f<0x128>(s); // row_ror:8
    s = s + dpp_f<0x124>(s); // row_ror:4
    s = s + dpp_f<0x122>(s); // row_ror:2
    s = s + dpp_f<0x121>(s); // row_ror:1
    return s;
}

// (c + a.lo * b.lo) + a.hi * b.hi on bfloat16 pairs in IEEE FP32: a bfloat16 widens to
// FP32 exactly, the product of two has at most 16 significant bits and is exact (unless
// it underflows), and each addition rounds to nearest (the library is built without
// multiply-add contraction), so the error of a chain of such steps follows from the
// documented FP32 rounding alone
__device__ __forceinline__ float dot2bf(uint32_t a, uint32_t b, float c) {
    const float a0 = __uint_as_float(a << 16), a1 = __uint_as_float(a & 0xFFFF0000u);
    const float b0 = __uint_as_float(b << 16), b1 = __uint_as_float(b & 0xFFFF0000u);
    return (c + a0 * b0) + a1 * b1;
}
// bfloat16 bits of a finite FP32 value, rounded to nearest even
__device__ __forceinline__ uint32_t bf16_rne(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// upper / lower halves of elements base .. base+3 of row id (base a multiple of 4)
__device__ __forceinline__ uint2 ld_hi(const SearchK &p, uint32_t id, int base) {
    return *reinterpret_cast<const uint2 *>(p.Xh + (int64_t)id * p.hs + base);
}
__device__ __forceinline__ uint2 ld_lo(const SearchK &p, uint32_t id, int base) {
    const uint16_t *a = base < p.spare ? p.Xh + (int64_t)id * p.hs + p.dpad + base
                                       : p.Xl + (int64_t)id * p.ls + (base - p.spare);
    return *reinterpret_cast<const uint2 *>(a);
}

// Inner products of up to U rows per 16-lane group in the fixed FP32 order: lane r sums
// the products of the elements 64 t + 4 r + c in increasing order with no fused
// multiply-add; the sixteen partial sums are combined by s_r + s_{r^8}, then ^4, ^2, ^1.
// Rows are zero padded to dpad; a zero product leaves a partial sum unchanged.
// DT > 0: rows of at most 64 DT floats, every load of the group issued before any use;
// DT = 0: any length, one 64-float chunk at a time.
template <int DT, int U>
__device__ __forceinline__ void dot_rows(const SearchK &p, const float *qv, const uint32_t *ids, int cnt, int r,
                                         float *out) {
    const int32_t dpad = p.dpad;
    float acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0f;
    if constexpr (DT > 0) {
        // rows in batches of UB, so that at most 16 (row, chunk) loads per plane are live
        constexpr int UB = (DT * U > 16) ? 16 / DT : U;
#pragma unroll
        for (int u0 = 0; u0 < U; u0 += UB) {
            uint2 hv[UB][DT], wv[UB][DT];
#pragma unroll
            for (int t = 0; t < DT; ++t) {
                const int base = 64 * t + 4 * r;
#pragma unroll
                for (int v = 0; v < UB; ++v) {
                    const bool ok = u0 + v < cnt && base < dpad;
                    hv[v][t] = ok ? ld_hi(p, ids[u0 + v], base) : make_uint2(0u, 0u);
                    wv[v][t] = ok ? ld_lo(p, ids[u0 + v], base) : make_uint2(0u, 0u);
                }
            }
#pragma unroll
            for (int t = 0; t < DT; ++t) {
                const int base = 64 * t + 4 * r;
                const float4 qq = base < dpad ? *reinterpret_cast<const float4 *>(qv + base)
                                              : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int v = 0; v < UB; ++v) {
                    const float4 xv = join4(hv[v][t], wv[v][t]);
                    acc[u0 + v] = acc[u0 + v] + xv.x * qq.x;
                    acc[u0 + v] = acc[u0 + v] + xv.y * qq.y;
                    acc[u0 + v] = acc[u0 + v] + xv.z * qq.z;
                    acc[u0 + v] = acc[u0 + v] + xv.w * qq.w;
                }
            }
        }
    } else {
        for (int base = 4 * r; base < dpad; base += 64) {
            const float4 qq = *reinterpret_cast<const float4 *>(qv + base);
            uint2 hv[U], wv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                hv[u] = u < cnt ? ld_hi(p, ids[u], base) : make_uint2(0u, 0u);
                wv[u] = u < cnt ? ld_lo(p, ids[u], base) : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float4 xv = join4(hv[u], wv[u]);
                acc[u] = acc[u] + xv.x * qq.x;
                acc[u] = acc[u] + xv.y * qq.y;
                acc[u] = acc[u] + xv.z * qq.z;
                acc[u] = acc[u] + xv.w * qq.w;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) out[u] = row_sum16(acc[u]);
}

// Upper bounds of the exact inner products of up to U rows per 16-lane group from the
// upper plane alone, with bfloat16 dot products against the query rounded to bfloat16
// (q_b, |q - q_b| <= 2^-8 |q|).  The upper half of an FP32 pattern is the value truncated
// to 8 significant bits, so |x_i - hi_i| <= 2^-7 |hi_i| (hi_i normal; a zero or subnormal
// hi_i leaves less than 2^-126).  With M = sum_i |hi_i q_b,i|,
//   |<x, q> - sum_i hi_i q_b,i| <= (2^-7 + 2^-8) M / (1 - 2^-8) + 2 d 2^-126.
// Rounding: each sum is a chain of at most 256 FP32 additions of exact products per lane
// (d <= 4096) and 4 butterfly additions, so it errs by at most gamma_260 M < 2^-15 M
// (Higham's bound, gamma_n = n u / (1 - n u), u = 2^-24); the kernel's exact FP32 inner
// product differs from <x, q> by at most gamma_260 sum |x_i q_i| < 2^-16 M (unit vectors).
// kBoundRel adds these to 0.0117647 with room to spare (0.0118800 - 0.0117647 = 1.15e-4
// > 2^-15 + 2^-16 + the relative error of M itself times 0.012), and kBoundAbs covers
// the subnormal terms, underflowed products and the two roundings of the final expression
// (|ub| <= 1.02).
constexpr float kBoundRel = 0.011880f;
constexpr float kBoundAbs = 9.5367431640625e-07f; // 2^-20
template <int DT, int U>
__device__ __forceinline__ void bound_rows(const SearchK &p, const WLds &l, const uint32_t *ids, int cnt, int r,
                                           float *ub) {
    const int32_t dpad = p.dpad;
    float acc[U], mag[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = mag[u] = 0.0f;
    if constexpr (DT > 0) {
        constexpr int UB = (DT * U > 32) ? 32 / DT : U;
#pragma unroll
        for (int u0 = 0; u0 < U; u0 += UB) {
            uint2 hv[UB][DT];
#pragma unroll
            for (int t = 0; t < DT; ++t) {
                const int base = 64 * t + 4 * r;
#pragma unroll
                for (int v = 0; v < UB; ++v)
                    hv[v][t] = (u0 + v < cnt && base < dpad) ? ld_hi(p, ids[u0 + v], base) : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int t = 0; t < DT; ++t) {
                const int base = 64 * t + 4 * r;
                const uint2 qq =
                    base < dpad ? *reinterpret_cast<const uint2 *>(l.qb + base / 2) : make_uint2(0u, 0u);
                const uint2 qa =
                    base < dpad ? *reinterpret_cast<const uint2 *>(l.qba + base / 2) : make_uint2(0u, 0u);
#pragma unroll
                for (int v = 0; v < UB; ++v) {
                    const int u = u0 + v;
                    acc[u] = dot2bf(hv[v][t].x, qq.x, acc[u]);
                    acc[u] = dot2bf(hv[v][t].y, qq.y, acc[u]);
                    mag[u] = dot2bf(hv[v][t].x & 0x7FFF7FFFu, qa.x, mag[u]);
                    mag[u] = dot2bf(hv[v][t].y & 0x7FFF7FFFu, qa.y, mag[u]);
                }
            }
        }
    } else {
        for (int base = 4 * r; base < dpad; base += 64) {
            const uint2 qq = *reinterpret_cast<const uint2 *>(l.qb + base / 2);
            const uint2 qa = *reinterpret_cast<const uint2 *>(l.qba + base / 2);
            uint2 hv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) hv[u] = u < cnt ? ld_hi(p, ids[u], base) : make_uint2(0u, 0u);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                acc[u] = dot2bf(hv[u].x, qq.x, acc[u]);
                acc[u] = dot2bf(hv[u].y, qq.y, acc[u]);
                mag[u] = dot2bf(hv[u].x & 0x7FFF7FFFu, qa.x, mag[u]);
                mag[u] = dot2bf(hv[u].y & 0x7FFF7FFFu, qa.y, mag[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) ub[u] = row_sum16(acc[u]) + row_sum16(mag[u]) * kBoundRel + kBoundAbs;
}

// The query as int8 codes for the 8-bit row summaries: t = max_i |q_i| / 127, b_i =
// rint(q_i / t) (|q_i - t b_i| <= t (1/2 + 2^-16), as for the rows), laid out like a
// summary row (byte qco + i holds b_i; bytes before qco, facing an inline header, are
// zero); st.qt = t, st.qB = sum_i |b_i|.
__device__ void query_rows8(const SearchK &p, WLds &l, QState &st) {
    const int lane = threadIdx.x;
    float mx = 0.0f;
    for (int c = lane; c < p.dpad; c += WV) mx = fmaxf(mx, fabsf(l.qv[c]));
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    const float t = mx / 127.0f;
    int32_t bsum = 0;
    for (int w = lane; w < p.rq / 4; w += WV) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int c = 4 * w - p.qco + b;
            int32_t v = 0;
            if (c >= 0 && c < p.dpad && t > 0.0f) v = (int32_t)fminf(127.0f, fmaxf(-127.0f, rintf(l.qv[c] / t)));
            bsum += v < 0 ? -v : v;
            word |= (uint32_t)(uint8_t)(int8_t)v << (8 * b);
        }
        l.q8[w] = word;
    }
    for (int o = 32; o >= 1; o >>= 1) bsum += __shfl_xor(bsum, o);
    // wave-uniform: kept in scalar registers
    st.qt = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(t)));
    st.qB = __builtin_amdgcn_readfirstlane(bsum);
}

// Integer sums of U rows over the 16 lanes of a DPP row, transposed: step S pairs lane r
// with lane r ^ m_S (m = 8, 7, 2, 1: row_ror:8, row_half_mirror, quad_perm [2,3,0,1],
// quad_perm [1,0,3,2]); while a lane holds n > 1 partial rows it keeps the half selected by
// bit 3 - S of r and adds the partner's partial of the same rows.  The four masks are
// independent over GF(2)^4, so every lane ends with the sum over all 16 lanes of row
// r / (16 / U).
template <int S> __device__ __forceinline__ int32_t dpp_step(int32_t v) {
    constexpr int ctrl = S == 0 ? 0x128 : S == 1 ? 0x141 : S == 2 ? 0x4E : 0xB1;
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, false);
}
template <int S, int N> __device__ __forceinline__ void tsum_rows(int32_t *a, int r) {
    if constexpr (S < 4) {
        if constexpr (N > 1) {
            const bool hi = (r >> (3 - S)) & 1;
#pragma unroll
            for (int j = 0; j < N / 2; ++j) {
                const int32_t keep = hi ? a[j + N / 2] : a[j];
                const int32_t send = hi ? a[j] : a[j + N / 2];
                a[j] = keep + dpp_step<S>(send);
            }
            tsum_rows<S + 1, N / 2>(a, r);
        } else {
            a[0] += dpp_step<S>(a[0]);
            tsum_rows<S + 1, 1>(a, r);
        }
    }
}

// Upper bound of the exact inner product of row r / (16 / U) of the group's U rows (in
// lane r of the group) from the 8-bit summaries; the caller passes row 0 for missing rows
// and ignores their results.  SH (rows without a header in their lines): the common
// scale p.s8 and, for A, the largest sum p.a8 of any row (the bound grows with A), so that
// no header is read.  With
// x_i = s c_i + e_i, |e_i| <= h s, q_i = t b_i + f_i, |f_i| <= h t, h = 1/2 + 2^-16,
// A = sum |c_i|, B = sum |b_i|, C = sum c_i b_i (exact, v_dot4_i32_i8):
//   <x, q> <= s t (C + h (A + B) + dpad h^2).
// The FP32 evaluation errs by less than 2^-21 (|s t C| <= 1.02, s t h (A + B) < 0.1), and
// the kernel's exact FP32 inner product exceeds <x, q> by less than 2^-16 (unit vectors,
// d <= 4096); kAbs8 = 2^-15 covers both.  Lane r of a group reads bytes 8r .. 8r + 7 of
// each 128-byte chunk of every row (an inline header faces zero query bytes) and the
// header (s, A) of the row it ends with.
constexpr float kH8 = 0.5f + 1.52587890625e-05f;
constexpr float kAbs8 = 3.0517578125e-05f;
template <int U, bool SH, bool NT>
__device__ __forceinline__ float bound8_row(const SearchK &p, const WLds &l, const uint32_t *ids, int r,
                                            float qt, int32_t qB) {
    const uint8_t *q8 = reinterpret_cast<const uint8_t *>(l.q8);
    int32_t acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0;
    static_assert(U == 2 || U == 4 || U == 8 || U == 16, "rows per group");
    const int row = r / (16 / U);
    uint32_t myid = ids[0];
#pragma unroll
    for (int u = 1; u < U; ++u)
        if (row == u) myid = ids[u];
    uint2 hdr = make_uint2(__float_as_uint(p.s8), (uint32_t)p.a8);
    if constexpr (!SH) {
        const uint8_t *hp = p.Xqh ? p.Xqh + (int64_t)myid * 8 : p.Xq + (int64_t)myid * p.rq;
        hdr = *reinterpret_cast<const uint2 *>(hp);
    }
    for (int off = 8 * r; off < p.rq; off += 128) {
        const uint2 qq = *reinterpret_cast<const uint2 *>(q8 + off);
        uint2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld_u2<NT>(p.Xq + (int64_t)ids[u] * p.rq + off);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc[u] = __builtin_amdgcn_sdot4((int)v[u].x, (int)qq.x, acc[u], false);
            acc[u] = __builtin_amdgcn_sdot4((int)v[u].y, (int)qq.y, acc[u], false);
        }
    }
    tsum_rows<0, U>(acc, r);
    const int32_t C = acc[0];
    const float sc = __uint_as_float(hdr.x);
    const int32_t A = (int32_t)hdr.y;
    const float inner = (float)C + (kH8 * (float)(A + qB) + (float)p.dpad * (kH8 * kH8));
    return (sc * qt) * inner + kAbs8;
}

// One pruning pass over ids[0..rc): rows whose bound (from the 8-bit summaries, Q8, or
// from the upper plane) is below the k-th inner product ipk could not enter the top-k;
// the rest are compacted, in order, to the front of ids.  Returns their count.
template <int DT, int U, bool Q8, bool SH = false, bool NT = false>
__device__ int prune_rows(const SearchK &p, const WLds &l, uint32_t *ids, int rc, float ipk, const QState &st) {
    constexpr int RROWS = 4 * U;
    const int lane = threadIdx.x, g = lane >> 4, r = lane & 15;
    int w = 0;
    for (int t0 = 0; t0 < rc; t0 += RROWS) {
        const int first = t0 + g * U;
        const int cnt = max(0, min(U, rc - first));
        uint32_t x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = u < cnt ? ids[first + u] : 0u;
        bool keep = false;
        uint32_t myx = x[0];
        if constexpr (Q8) {
            // row r / (16 / U) ends in lanes r; the first of them keeps it
            const float ub = bound8_row<U, SH, NT>(p, l, x, r, st.qt, st.qB);
            const int row = r / (16 / U);
#pragma unroll
            for (int u = 1; u < U; ++u)
                if (row == u) myx = x[u];
            keep = r % (16 / U) == 0 && row < cnt && ub >= ipk;
        } else {
            float ub[U];
            bound_rows<DT, U>(p, l, x, cnt, r, ub);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (r == u) {
                    keep = u < cnt && ub[u] >= ipk;
                    myx = x[u];
                }
        }
        const uint64_t mk = __ballot(keep);
        wsync();
        if (keep) ids[w + lanes_below(mk)] = myx;
        w += __popcll(mk);
        wsync();
    }
    return w;
}

// Re-rank rows ids[0..rc); candidates better than the current k-th enter the buffer,
// which is merged into the top-k whenever it could overflow.  Once the top-k is full, a
// pass over the 8-bit summaries and then one over the upper plane drop every row whose
// bound is below the k-th inner product (it could not enter the top-k), each compacting
// the rest, in order, to the front of ids; only those are read from both planes.
template <int DT, class TL>
__device__ void wave_rerank(const SearchK &p, WLds &l, uint32_t *ids, int rc, QState &st) {
    // rows of 256 floats (DT = 4) or of any length (DT = 0) take at most 4 rows per group in
    // flight: 8 would exceed the register file
    constexpr int U = (DT == 4 || DT == 0) && TL::U > 4 ? 4 : TL::U;
    constexpr int RROWS = 4 * U, CW = TL::CW;
    const int lane = threadIdx.x, g = lane >> 4, r = lane & 15;
    if (p.prefilter && st.top == st.k) {
        // 8-bit summaries first (one 128-byte line per row of up to 120 elements), then
        // the upper plane for the rows they cannot rule out
        const float ipk = key_ip(st.thr);
        st.c_q8 += rc;
        rc = prune_rows<DT, TL::UQ, true, TL::SH, (TL::NT >= 2)>(p, l, ids, rc, ipk, st);
        st.c_upper += rc;
        rc = prune_rows<DT, U, false>(p, l, ids, rc, ipk, st);
    } else {
        st.c_upper += rc;
    }
    st.c_exact += rc;
    for (int t0 = 0; t0 < rc; t0 += RROWS) {
        const int first = t0 + g * U;
        const int cnt = max(0, min(U, rc - first));
        uint32_t x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = u < cnt ? ids[first + u] : 0u;
        float ip[U];
        dot_rows<DT, U>(p, l.qv, x, cnt, r, ip);
        bool emit = false;
        unsigned long long key = 0;
        if (r < cnt) {
            float myip = ip[0];
            uint32_t myx = x[0];
#pragma unroll
            for (int u = 1; u < U; ++u)
                if (r == u) {
                    myip = ip[u];
                    myx = x[u];
                }
            key = mkkey(myip, myx);
            emit = st.top < st.k || key > st.thr;
        }
        const uint64_t mk = __ballot(emit);
        if (emit) l.cand[st.cand + lanes_below(mk)] = key;
        st.cand += __popcll(mk);
        if (st.cand > CW - RROWS) wave_merge(l, st);
    }
}

// Candidates waiting in pending[0..pend) (point positions) are re-ranked; the top-k
// merge drops points seen before.
template <int DT, class TL> __device__ void wave_process(const SearchK &p, WLds &l, QState &st) {
    wave_rerank<DT, TL>(p, l, l.pending, st.pend, st);
    st.c_rerank += st.pend;
    st.pend = 0;
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

// inclusive scan of a[0..N) in this wave's LDS
__device__ void wave_scan_incl(uint32_t *a, int N) {
    const int lane = threadIdx.x;
    const int per = (N + WV - 1) / WV;
    const int s0 = lane * per, s1 = min(N, s0 + per);
    uint32_t tot = 0;
    for (int i = s0; i < s1; ++i) tot += a[i];
    uint32_t v = tot;
    for (int o = 1; o < WV; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    uint32_t pre = v - tot;
    for (int i = s0; i < s1; ++i) {
        pre += a[i];
        a[i] = pre;
    }
    wsync();
}

template <int DT, class TL, int PB>
__global__ __launch_bounds__(WV) __attribute__((amdgpu_waves_per_eu(TL::WPE))) void k_search(SearchK p) {
    constexpr int EPT = TL::EPT, WCH = TL::WCH, RB = TL::RB, PCAP = TL::PCAP;
    extern __shared__ __align__(16) unsigned char smem[];
    // every pointer below is derived from smem by a constant-free offset only, so the
    // compiler keeps them in the LDS address space (ds_read / ds_write, counted by
    // lgkmcnt alone); a generic pointer would turn each LDS access into a flat access
    // that also waits for every global load in flight
    const LdsOff lo_ = search_lds_offsets(p.L, p.kmax, p.dpad, TL::PCAP, TL::CW, TL::UCAP, p.rq);
    WLds l;
    l.top = reinterpret_cast<unsigned long long *>(smem + lo_.top);
    l.ntop = reinterpret_cast<unsigned long long *>(smem + lo_.ntop);
    l.cand = reinterpret_cast<unsigned long long *>(smem + lo_.cand);
    l.tq = reinterpret_cast<unsigned long long *>(smem + lo_.tq);
    l.pending = reinterpret_cast<uint32_t *>(smem + lo_.pending);
    l.upos = reinterpret_cast<uint32_t *>(smem + lo_.upos);
    l.clo = reinterpret_cast<uint32_t *>(smem + lo_.clo);
    l.chi = reinterpret_cast<uint32_t *>(smem + lo_.chi);
    l.qc = reinterpret_cast<uint32_t *>(smem + lo_.qc);
    l.segBeg = reinterpret_cast<uint32_t *>(smem + lo_.segBeg);
    l.segStart = reinterpret_cast<uint32_t *>(smem + lo_.segStart);
    l.segTab = reinterpret_cast<uint32_t *>(smem + lo_.segTab);
    l.qb = reinterpret_cast<uint32_t *>(smem + lo_.qb);
    l.qba = reinterpret_cast<uint32_t *>(smem + lo_.qba);
    l.q8 = reinterpret_cast<uint32_t *>(smem + lo_.q8);
    l.qv = reinterpret_cast<float *>(smem + lo_.qv);
    const int lane = threadIdx.x;
    const int32_t L = p.L, K = p.K;
    const int64_t n = p.n;

    int64_t qi = blockIdx.x;
    if (p.queue) qi = __shfl((int64_t)(lane == 0 ? atomicAdd(p.queue, 1u) : 0u), 0);
    while (qi < p.m) {
        const int64_t q = p.order ? (int64_t)p.order[qi] : qi;
        const uint64_t t_begin = wall_clock64();
        QState st;
        st.k = p.ks ? max(1, min(p.ks[q], p.kmax)) : p.kconst;
        st.pend = st.cand = st.top = 0;
        st.thr = 0;
        st.c_scan = st.c_pass = st.c_rerank = st.c_exact = st.c_upper = st.c_q8 = 0;
        const float *stopw = p.stopw + (int64_t)(p.qtab ? p.qtab[q] : 0) * K * p.G * kTauCols;
        for (int c = lane; c < p.dpad; c += WV) l.qv[c] = p.Q[q * p.dpad + c];
        for (int c = lane; c < p.dpad / 2; c += WV) {
            const uint32_t w = bf16_rne(p.Q[q * p.dpad + 2 * c]) | (bf16_rne(p.Q[q * p.dpad + 2 * c + 1]) << 16);
            l.qb[c] = w;
            l.qba[c] = w & 0x7FFF7FFFu;
        }
        wsync();
        query_rows8(p, l, st);
        for (int32_t j = lane; j < L; j += WV) {
            const uint32_t qc = p.qcode[(int64_t)j * p.qstride + q];
            l.qc[j] = qc;
            l.tq[j] = p.qsk[(int64_t)(j % p.M) * p.qstride + q];
            uint32_t lo, hi;
            level_range(p, j, K, qc, q, lo, hi);
            l.clo[j] = lo;
            l.chi[j] = lo;
        }
        if (lane == 0) l.segStart[0] = 0;
        wsync();
        int tau = 64;
        bool stopped = false;
        int stop_level = 0;
        for (int32_t i = K; i >= 1; --i) {
            // new entries of this level: per table the whole segments of B added on the left
            // and on the right of its window; only non-empty segments are listed, in table
            // order (left before right), with their table
            uint32_t nseg = 0;
            for (int32_t j0 = 0; j0 < L; j0 += WV) {
                const int32_t j = j0 + lane;
                uint32_t a = 0, b = 0, na = 0, nb = 0;
                if (j < L) {
                    uint32_t lo, hi;
                    level_range(p, j, i, l.qc[j], q, lo, hi);
                    a = l.clo[j];
                    b = l.chi[j];
                    na = a;
                    nb = b;
                    if (a > lo) {
                        const uint64_t sz = ((uint64_t)(a - lo) + p.B - 1) / p.B * (uint64_t)p.B;
                        na = (a > sz) ? (uint32_t)(a - sz) : 0u;
                    }
                    if (b < hi) {
                        const uint64_t sz = ((uint64_t)(hi - b) + p.B - 1) / p.B * (uint64_t)p.B;
                        const uint64_t e = (uint64_t)b + sz;
                        nb = e < (uint64_t)n ? (uint32_t)e : (uint32_t)n;
                    }
                    l.clo[j] = na;
                    l.chi[j] = nb;
                }
                const bool left = na < a, right = nb > b;
                const uint64_t ml = __ballot(left), mr = __ballot(right);
                uint32_t at = nseg + (uint32_t)(lanes_below(ml) + lanes_below(mr));
                if (left) {
                    l.segBeg[at] = na;
                    l.segTab[at] = (uint32_t)j;
                    l.segStart[at + 1] = a - na;
                    ++at;
                }
                if (right) {
                    l.segBeg[at] = b;
                    l.segTab[at] = (uint32_t)j;
                    l.segStart[at + 1] = nb - b;
                }
                nseg += (uint32_t)(__popcll(ml) + __popcll(mr));
            }
            wsync();
            wave_scan_incl(l.segStart + 1, (int)nseg);
            const uint32_t total = l.segStart[nseg];
            // a last segment without end, so that the walk below stops there without a
            // bounds test (entries past the end are masked)
            if (lane == 0) {
                l.segStart[nseg + 1] = 0xFFFFFFFFu;
                l.segBeg[nseg] = 0;
                l.segTab[nseg] = 0;
            }
            // groups of repetitions: lane g < G finds the segments of the tables before
            // the end of group g (segments are listed in table order) and their entries
            uint32_t gseg_mine = nseg, gend_mine = total;
            if (lane < p.G) {
                const uint32_t a_end = (uint32_t)(((int64_t)(lane + 1) * L) / p.G);
                uint32_t lo = 0, hi = nseg;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (l.segTab[mid] < a_end)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                gseg_mine = lo;
                gend_mine = l.segStart[lo];
            }
            // lane g < G: the stopping threshold after group g at this level and filter
            // threshold (tau changes only at the end of a level); +2 (never) elsewhere
            const float thr_mine = lane < p.G ? stopw[((i - 1) * p.G + lane) * kTauCols + (tau + 1)] : 2.0f;
            wsync();
            // each lane's entries f = base + u * 64 + lane only grow between two tests, so it
            // walks the segments of those groups once, keeping the current one's end and
            // base offset in registers
            int sg = -1;
            uint32_t segEnd = 0, ebase = 0;
            uint64_t tqc = 0; // the query's sketch for the current segment's table
            uint32_t gbeg = 0;
            bool stop = false;
            for (int32_t g = 0; g < p.G;) {
            // groups g .. h up to the next test: h is the first group whose end lies at least
            // tmin entries past gbeg, else the level's last group
            const uint64_t far = __ballot(lane >= g && lane < p.G && gend_mine - gbeg >= (uint32_t)p.tmin);
            const int32_t h = far ? (int32_t)__builtin_ctzll(far) : p.G - 1;
            const uint32_t gend = __builtin_amdgcn_readfirstlane(__shfl(gend_mine, h));
            if (g > 0) {
                sg = (int)__builtin_amdgcn_readfirstlane(__shfl(gseg_mine, g - 1)) - 1;
                segEnd = 0;
            }
            st.c_scan += gend - gbeg;
            // LATE tiles: the previous chunk's passing entries (at most UCAP) wait in upos
            // as table positions, and their point ids are read together with this chunk's
            // sketches, so that positions are read for passing entries only and no load
            // waits for another.  Other tiles read the position of every entry with its
            // sketch.
            int nu = 0;
            for (uint32_t base = gbeg; base < gend; base += WCH) {
                uint32_t ev[EPT];
                uint64_t tqv[EPT];
                uint64_t skv[EPT];
                // (entries past the group's end load entry 0 of table 0 and are masked out,
                // so that every load is unconditional)
                uint32_t uid = 0;
                if constexpr (TL::LATE) uid = read_pos<PB>(p.pos, lane < nu ? l.upos[lane] : 0u);
                int lim[EPT]; // the entry's threshold: tau, or -1 past the end
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const uint32_t f = base + u * WV + lane;
                    const bool in = f < gend;
                    if (f >= segEnd) {
                        do {
                            ++sg;
                            segEnd = l.segStart[sg + 1];
                        } while (f >= segEnd);
                        const uint32_t tjc = l.segTab[sg];
                        tqc = l.tq[tjc];
                        ebase = tjc * (uint32_t)n + l.segBeg[sg] - l.segStart[sg];
                    }
                    lim[u] = in ? tau : -1;
                    tqv[u] = tqc;
                    const uint32_t e = in ? ebase + f : 0u;
                    skv[u] = ld_u64<(TL::NT >= 1)>(p.tsk + e);
                    ev[u] = TL::LATE ? e : read_pos<PB>(p.pos, e);
                }
                if constexpr (TL::LATE) {
                    if (lane < nu) l.pending[st.pend + lane] = uid;
                    st.pend += nu;
                }
                // (every entry is tested, without a branch: an entry past the end fails
                // against -1)
                bool ps[EPT];
                uint64_t mk[EPT];
                int np = 0;
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    ps[u] = (int)__popcll(skv[u] ^ tqv[u]) <= lim[u];
                    mk[u] = __ballot(ps[u]);
                    np += __popcll(mk[u]);
                }
                if (TL::LATE && np <= TL::UCAP) {
                    wsync();
                    int at = 0;
#pragma unroll
                    for (int u = 0; u < EPT; ++u) {
                        if (ps[u]) l.upos[at + lanes_below(mk[u])] = ev[u];
                        at += __popcll(mk[u]);
                    }
                    nu = np;
                } else {
                    // (LATE: more passing entries than upos holds, as on a level where the
                    // filter passes nearly everything: their ids are read now, all loads in
                    // flight)
                    if constexpr (TL::LATE) {
#pragma unroll
                        for (int u = 0; u < EPT; ++u) ev[u] = read_pos<PB>(p.pos, ps[u] ? ev[u] : 0u);
                        nu = 0;
                    }
#pragma unroll
                    for (int u = 0; u < EPT; ++u) {
                        if (ps[u]) l.pending[st.pend + lanes_below(mk[u])] = ev[u];
                        st.pend += __popcll(mk[u]);
                    }
                }
                if (st.pend >= RB) {
                    st.c_pass += st.pend;
                    wsync();
                    wave_process<DT, TL>(p, l, st);
                }
            }
            if (TL::LATE && nu > 0) {
                wsync();
                const uint32_t uid = read_pos<PB>(p.pos, lane < nu ? l.upos[lane] : 0u);
                if (lane < nu) l.pending[st.pend + lane] = uid;
                st.pend += nu;
            }
            if (st.pend > 0) {
                st.c_pass += st.pend;
                wsync();
                wave_process<DT, TL>(p, l, st);
            }
            wave_merge(l, st);
            // the next group with entries (G if none): the groups before it add nothing, so
            // the tests after h and after each of them see the same k-th inner product and
            // one ballot takes them in order
            const uint64_t more = __ballot(lane > h && lane < p.G && gend_mine > gend);
            const int32_t nxt = more ? (int32_t)__builtin_ctzll(more) : p.G;
            if (st.top == st.k) {
                const float ipk = key_ip(l.top[st.k - 1]);
                stop = __ballot(lane >= h && lane < nxt && ipk >= thr_mine) != 0;
                if (!stop && nxt == p.G && p.filter) {
                    // largest t with ipk <= tauv[t] (-1 if none): lane t tests t, one load each
                    const uint64_t mk = __ballot(ipk <= p.tauv[lane]);
                    tau = (ipk <= p.tauv[64]) ? 64 : (mk ? 63 - __clzll((long long)mk) : -1);
                }
            }
            if (stop) break;
            gbeg = gend;
            g = nxt;
            }
            if (stop) {
                stopped = true;
                stop_level = i;
                break;
            }
        }
        if (!stopped) {
            // level 0: linear scan, every point re-ranked, in blocks of PCAP positions
            for (int64_t base = 0; base < n; base += PCAP) {
                const int rc = (int)min((int64_t)PCAP, n - base);
                for (int t = lane; t < rc; t += WV) l.pending[t] = (uint32_t)(base + t);
                wsync();
                wave_rerank<DT, TL>(p, l, l.pending, rc, st);
                wsync();
            }
            wave_merge(l, st);
            st.c_rerank += n;
            stop_level = 0;
        }
        for (int t = lane; t < p.kmax; t += WV) {
            const int64_t o = q * p.kmax + t;
            if (t < st.k) {
                const unsigned long long key = l.top[t];
                p.out_ids[o] = (int32_t)key_id(key);
                if (p.out_ips) p.out_ips[o] = key_ip(key);
            } else {
                p.out_ids[o] = -1;
                if (p.out_ips) p.out_ips[o] = -INFINITY;
            }
        }
        if (lane == 0 && p.stats) {
            pf_query_stats s;
            s.stop_level = stop_level;
            s.wave_us = (int32_t)fminf((float)(wall_clock64() - t_begin) * p.us_per_tick, 2.0e9f);
            s.c_scan = st.c_scan;
            s.c_pass = st.c_pass;
            s.c_rerank = st.c_rerank;
            s.c_exact = st.c_exact;
            s.c_upper = st.c_upper;
            s.c_q8 = st.c_q8;
            p.stats[q] = s;
        }
        wsync();
        if (p.queue)
            qi = __shfl((int64_t)(lane == 0 ? atomicAdd(p.queue, 1u) : 0u), 0);
        else
            qi += gridDim.x;
    }
}

// ---------------------------------------------------------------------- kernel table
// (the instantiations for 4-byte positions are built here; those for 3-byte positions in
// k_search_pos3.hip, which includes this file with PF_SEARCH_KERNELS_ONLY defined)

// tile shapes the library is built with (the autotuner chooses among them)
using T88 = Tile<8, 8>;
using T48 = Tile<4, 8>;
using T168 = Tile<16, 8>;
using T84 = Tile<8, 4>;
using T84o4 = Tile<8, 4, 4>; // registers capped for 4 waves per SIMD (16 per CU)
using T84o4l = Tile<8, 4, 4, true, 8>;  // ids read for passing entries only, one chunk late
using T84o4q8 = Tile<8, 4, 4, false, 8>;   // 8 summary rows in flight per group
using T84o4lN1 = Tile<8, 4, 4, true, 8, false, 1>; // the late shape, sketches non-temporal
using T84o4lN2 = Tile<8, 4, 4, true, 8, false, 2>; // ... and summary rows non-temporal too

// the same shape for summary rows without header (one scale for all rows)
template <class TL> using SharedScale = Tile<TL::EPT, TL::U, TL::WPE, TL::LATE, TL::UQ, true, TL::NT>;

template <int PB, int DT, bool SH> static const void *search_kernel_dt(int tile) {
    switch (tile) {
    case 1: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T48>, T48>, PB>;
    case 2: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T168>, T168>, PB>;
    case 3: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T84>, T84>, PB>;
    case 4: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T84o4>, T84o4>, PB>;
    case 5: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T84o4l>, T84o4l>, PB>;
    case 6: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T84o4q8>, T84o4q8>, PB>;
    case 7: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T84o4lN1>, T84o4lN1>, PB>;
    case 8: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T84o4lN2>, T84o4lN2>, PB>;
    default: return (const void *)k_search<DT, std::conditional_t<SH, SharedScale<T88>, T88>, PB>;
    }
}

// kernels for rows of at most 64, 128 or 256 floats, or any length; rows of 121 .. 128
// and 249 .. 256 floats have summaries without header (shared scale), others of at most
// 256 floats their header inline; longer rows read a separate header when they have one
template <int PB> static const void *search_kernel_of(int dt, int tile, bool shared) {
    switch (dt) {
    case 1: return search_kernel_dt<PB, 1, false>(tile);
    case 2: return shared ? search_kernel_dt<PB, 2, true>(tile) : search_kernel_dt<PB, 2, false>(tile);
    case 4: return shared ? search_kernel_dt<PB, 4, true>(tile) : search_kernel_dt<PB, 4, false>(tile);
    default: return search_kernel_dt<PB, 0, false>(tile);
    }
}


#ifndef PF_SEARCH_KERNELS_ONLY
// ====================================================================== host side
// (tile table, occupancy, launch; everything above this line is device code)

// chunks of 64 floats per row, as a kernel specialisation (0 = any length)
static int row_chunks(int32_t dpad) {
    const int t = (dpad + 63) / 64;
    return t <= 1 ? 1 : t <= 2 ? 2 : t <= 4 ? 4 : 0;
}

static constexpr int kNumTiles = 9;
static const char *kTileNames[kNumTiles] = {"ept8-u8", "ept4-u8", "ept16-u8", "ept8-u4", "ept8-u4-o4",
                                            "ept8-u4q8-o4-late", "ept8-u4q8-o4", "ept8-u4q8-o4-late-nts",
                                            "ept8-u4q8-o4-late-nt"};

template <class TL> static size_t tile_lds(const Index &ix, int32_t kmax) {
    return search_lds_offsets(ix.L, kmax, ix.dpad, TL::PCAP, TL::CW, TL::UCAP, ix.rq).total;
}
static size_t search_lds_bytes(const Index &ix, int32_t kmax, int tile) {
    switch (tile) {
    case 1: return tile_lds<T48>(ix, kmax);
    case 2: return tile_lds<T168>(ix, kmax);
    case 3: return tile_lds<T84>(ix, kmax);
    case 4: return tile_lds<T84o4>(ix, kmax);
    case 5: return tile_lds<T84o4l>(ix, kmax);
    case 6: return tile_lds<T84o4q8>(ix, kmax);
    case 7: return tile_lds<T84o4lN1>(ix, kmax);
    case 8: return tile_lds<T84o4lN2>(ix, kmax);
    default: return tile_lds<T88>(ix, kmax);
    }
}

// kernels for the index's position width (3-byte ones live in k_search_pos3.hip)
static const void *search_kernel(int dt, int tile, bool shared, int32_t posb) {
    return posb == 3 ? search_kernel_pos3(dt, tile, shared) : search_kernel_of<4>(dt, tile, shared);
}

int32_t search_tile_count() { return kNumTiles; }
// the shape used when none is given or tuned: the fastest on the 1 M-point, d = 100
// mixture at k = 10 both with static query slots and with the work queue
int32_t search_default_tile() { return 7; }
const char *search_tile_name(int32_t t) { return (t >= 0 && t < kNumTiles) ? kTileNames[t] : "?"; }

// resident query waves per CU for a tile shape (occupancy from registers and LDS)
int32_t search_waves_per_cu(const Index &ix, int32_t kmax, int32_t tile) {
    int per_cu = 0;
    const size_t lds = search_lds_bytes(ix, kmax, tile);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, search_kernel(row_chunks(ix.dpad), tile, ix.qco == 0, ix.posb), WV, lds) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    return per_cu;
}

int64_t launch_search(Index &ix, const SearchArgs &a, const uint32_t *ranges, hipStream_t s) {
    if (a.m <= 0) return 0;
    const int dt = row_chunks(ix.dpad);
    const int tile = (a.tile >= 0 && a.tile < kNumTiles) ? a.tile : search_default_tile();
    const size_t lds = search_lds_bytes(ix, a.kmax, tile);
    const void *fn = search_kernel(dt, tile, ix.qco == 0, ix.posb);
    PF_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = search_waves_per_cu(ix, a.kmax, tile);
    if (a.waves_per_cu > 0) per_cu = std::min(per_cu, a.waves_per_cu);
    const int64_t slots = std::max<int64_t>(1, std::min<int64_t>(a.m, (int64_t)ix.num_cus * per_cu));
    SearchK p;
    p.Xh = ix.Xh.as<uint16_t>();
    p.Xl = ix.Xl.as<uint16_t>();
    p.hs = ix.hs;
    p.ls = ix.ls;
    p.spare = ix.hs - ix.dpad;
    p.prefilter = a.prefilter;
    p.Xq = ix.Xq.as<uint8_t>();
    p.Xqh = ix.qco ? nullptr : ix.Xqh.as<uint8_t>();
    p.s8 = ix.s8;
    p.a8 = ix.a8;
    p.rq = ix.rq;
    p.qco = ix.qco;
    p.pos = ix.tpos.p;
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
    p.qstride = a.qstride > 0 ? a.qstride : a.m;
    p.ks = a.ks;
    p.kconst = a.kconst;
    p.kmax = a.kmax;
    p.qtab = a.qtab;
    p.tauv = a.tauv;
    p.stopw = a.stopw;
    p.G = a.groups;
    p.tmin = a.test_entries;
    p.filter = a.filter;
    p.queue = a.queue;
    p.order = a.order;
    p.out_ids = a.out_ids;
    p.out_ips = a.out_ips;
    p.stats = a.stats;
    p.us_per_tick = ix.wall_khz > 0 ? (float)(1000.0 / ix.wall_khz) : 0.0f;
    if (a.queue) launch_fill_u32(a.queue, 1, 0u, s);
    void *args[] = {&p};
    PF_HIP(hipLaunchKernel(fn, dim3((unsigned)slots), dim3(WV), args, lds, s));
    return slots;
}

#endif // PF_SEARCH_KERNELS_ONLY

} // namespace pf
