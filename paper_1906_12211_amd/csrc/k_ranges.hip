// Prefix ranges of the level-synchronous walk (Sec. 4.2 "Retrieving candidate points"):
// for every (query q, table j) and level i = P+1..K, the entries of table j whose codes
// share the query's i-bit prefix form the range [lo_i, hi_i) of the query's P-bit prefix
// bucket [B0, B1) (the P-bit prefix table answers the levels i <= P directly).  With
// lcp(c) the common prefix length of code c and the query code (at least P inside the
// bucket) and lt(c) = [c < query code]:
//   lo_i = B0 + #{lt, lcp < i},   hi_i = B0 + #{lt} + #{not lt, lcp >= i}.
// ranges[q][j][i - P - 1] = (lo_i, hi_i).  Inside the bucket every code has the query's
// leading P bits, so the kernels read only the stored low K - P bits of each code (8-, 16-
// or 32-bit suffixes) and compare them with the query's.
#include "pf_device.h"
#include "pf_internal.h"

namespace pf {

static constexpr int kLoads = 8; // code loads in flight per lane
// buckets of at most 255 W entries (so that no lane counts more than 255 in a bin): one group
// of W lanes per pair; larger ones: one binary search per bound and level
template <int W> constexpr uint32_t group_max() { return 255u * W; }

// One group of W lanes (a DPP row for W = 16, half of one for W = 8) per (q, j) pair: the
// group reads its bucket W kLoads entries at a time (W consecutive codes per load
// instruction, kLoads in flight), each lane counts its entries per (lcp - P, lt) in 8-bit
// fields of NR registers per flag (bin b in byte b & 3 of register b >> 2; at most 255
// entries per lane), the fields are widened to 16 bits and summed over the group, and lane r
// writes levels P + 1 + r, P + 1 + r + W, ...  Pairs with larger buckets are appended to the
// list for k_ranges_wave.  W = 8 suits small buckets: twice as many pairs per wave.
template <int NR, int W, class S>
__global__ __launch_bounds__(256) void k_ranges_group(const S *__restrict__ tsuf,
                                                      const uint32_t *__restrict__ off, int64_t n, int32_t L,
                                                      int32_t K, int32_t P, const uint32_t *__restrict__ qcode,
                                                      int64_t m, uint32_t *__restrict__ ranges,
                                                      uint32_t *__restrict__ big, uint32_t *__restrict__ nbig) {
    static_assert(W == 8 || W == 16, "groups of 8 or 16 lanes");
    const int g = threadIdx.x & (W - 1);
    const int64_t t = ((int64_t)blockIdx.x * 256 + threadIdx.x) / W;
    if (t >= m * L) return; // whole groups leave together
    const int64_t q = t / L;
    const int32_t j = (int32_t)(t - q * L);
    const int32_t nl = K - P;
    const uint32_t qc = qcode[(int64_t)j * m + q];
    const int64_t np1 = ((int64_t)1 << P) + 1;
    const uint32_t b = qc >> (K - P);
    const uint32_t B0 = off[(int64_t)j * np1 + b];
    const uint32_t B1 = off[(int64_t)j * np1 + b + 1];
    if (B1 - B0 > group_max<W>()) {
        if (g == 0) big[atomicAdd(nbig, 1u)] = (uint32_t)t;
        return;
    }
    const S *tc = tsuf + (int64_t)j * n;
    const uint32_t qs = qc & ((1u << nl) - 1u); // the query's low nl bits (nl <= 19)
    const int sh = 32 - nl;
    uint32_t clt[NR], cge[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) clt[r] = cge[r] = 0;
    for (uint32_t e0 = B0 + g; e0 < B1; e0 += W * kLoads) {
        uint32_t c[kLoads];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) c[u] = tc[e0 + W * u < B1 ? e0 + W * u : B0];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            if (e0 + W * u < B1) {
                const uint32_t x = (c[u] ^ qs) << sh;
                const int bin = x ? __clz(x) : nl; // common prefix length beyond the P bits
                const uint32_t inc = 1u << (8 * (bin & 3));
                const bool lt = c[u] < qs;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const uint32_t v = (bin >> 2) == r ? inc : 0u;
                    clt[r] += lt ? v : 0u;
                    cge[r] += lt ? 0u : v;
                }
            }
        }
    }
    // widen to 16-bit fields (even bytes, odd bytes) and sum over the group
    auto gsum = [](uint32_t v) { return W == 16 ? row_sum16u(v) : half_row_sum8u(v); };
    uint32_t lte[NR], lto[NR], gee[NR], geo[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        lte[r] = gsum(clt[r] & 0x00FF00FFu);
        lto[r] = gsum((clt[r] >> 8) & 0x00FF00FFu);
        gee[r] = gsum(cge[r] & 0x00FF00FFu);
        geo[r] = gsum((cge[r] >> 8) & 0x00FF00FFu);
    }
    // lane g writes levels g, g + W, ...: lo counts lt with bin <= level index, hi counts
    // not-lt with bin > level index (nl <= 19 levels)
    uint32_t *out = ranges + t * (int64_t)nl * 2;
#pragma unroll
    for (int half = 0; half < (W == 16 ? 2 : 3); ++half) {
        const int ri = g + W * half;
        if (ri < nl) {
            uint32_t lo = B0, hi = B0;
#pragma unroll
            for (int bb = 0; bb < 4 * NR; ++bb) {
                const int sft = 16 * ((bb & 3) >> 1);
                const uint32_t nlt = (((bb & 1) ? lto[bb >> 2] : lte[bb >> 2]) >> sft) & 0xFFFFu;
                const uint32_t nge = (((bb & 1) ? geo[bb >> 2] : gee[bb >> 2]) >> sft) & 0xFFFFu;
                hi += nlt;
                if (bb <= ri) lo += nlt;
                if (bb > ri) hi += nge;
            }
            out[2 * ri] = lo;
            out[2 * ri + 1] = hi;
        }
    }
}

// one wave per listed (q, j) pair (bucket above the group kernel's limit), waves striding over
// the list: lane 2r + s binary-searches bound s (0: lo, 1: hi) of level P + 1 + r
template <class S>
__global__ __launch_bounds__(256) void k_ranges_wave(const S *__restrict__ tsuf,
                                                     const uint32_t *__restrict__ off, int64_t n, int32_t L,
                                                     int32_t K, int32_t P, const uint32_t *__restrict__ qcode,
                                                     int64_t m, uint32_t *__restrict__ ranges,
                                                     const uint32_t *__restrict__ big,
                                                     const uint32_t *__restrict__ nbig) {
    const int lane = threadIdx.x & 63;
    const uint32_t count = *nbig;
    const uint32_t nw = gridDim.x * 4;
    for (uint32_t w = blockIdx.x * 4 + (threadIdx.x >> 6); w < count; w += nw) {
        const int64_t t = big[w];
        const int64_t q = t / L;
        const int32_t j = (int32_t)(t - q * L);
        const int32_t nl = K - P;
        if (lane >= 2 * nl) continue;
        const uint32_t qc = qcode[(int64_t)j * m + q];
        const int64_t np1 = ((int64_t)1 << P) + 1;
        const uint32_t b = qc >> (K - P);
        const S *tc = tsuf + (int64_t)j * n;
        const int lev = P + 1 + (lane >> 1);
        const uint64_t pre = (uint64_t)(qc >> (K - lev));
        // the bound's code, relative to the bucket's first code (b << (K - P)): in [0, 2^(K-P)]
        const uint64_t target = ((lane & 1) ? ((pre + 1) << (K - lev)) : (pre << (K - lev))) -
                                ((uint64_t)b << (K - P));
        uint32_t lo = off[(int64_t)j * np1 + b], hi = off[(int64_t)j * np1 + b + 1];
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if ((uint64_t)tc[mid] < target)
                lo = mid + 1;
            else
                hi = mid;
        }
        ranges[t * (int64_t)nl * 2 + lane] = lo;
    }
}

template <int NR, int W, class S> static const void *group_kernel() {
    return (const void *)k_ranges_group<NR, W, S>;
}

template <int W, class S> static const void *group_kernel_of(int nr) {
    return nr <= 1 ? group_kernel<1, W, S>() : nr <= 2 ? group_kernel<2, W, S>() : nr <= 3 ? group_kernel<3, W, S>()
         : nr <= 4 ? group_kernel<4, W, S>() : group_kernel<5, W, S>();
}

template <class S> static const void *group_kernel_of(int nr, int w) {
    return w == 8 ? group_kernel_of<8, S>(nr) : group_kernel_of<16, S>(nr);
}

// lanes per (query, table) pair: 8 where a P-bit bucket holds at most 64 entries on average
// (more pairs per wave: 0.14 against 0.19 ms at 1 M points, 15 entries), else 16 (3.2 against
// 3.4 ms at 10 M points, 152 entries)
static int group_lanes(const Index &ix) { return (ix.n >> ix.P) <= 64 ? 8 : 16; }

size_t ranges_list_bytes(int64_t m, int32_t L) { return (size_t)(m * L + 1) * sizeof(uint32_t); }

void launch_ranges(Index &ix, const SearchArgs &a, uint32_t *ranges, hipStream_t s) {
    if (ix.K <= ix.P || a.m <= 0) return;
    ix.rlist.ensure(ranges_list_bytes(a.m, ix.L));
    launch_ranges_into(ix, a, ranges, ix.rlist.as<uint32_t>(), s);
}

void launch_ranges_into(const Index &ix, const SearchArgs &a, uint32_t *ranges, uint32_t *rlist, hipStream_t s) {
    if (ix.K <= ix.P || a.m <= 0) return;
    const int64_t pairs = a.m * ix.L;
    PF_CHECK(pairs < ((int64_t)1 << 32), PF_EINVAL, "search: more than 2^32 (query, table) pairs in one call");
    uint32_t *nbig = rlist;
    uint32_t *big = nbig + 1;
    launch_fill_u32(nbig, 1, 0u, s);
    // registers of 8-bit bin counters per flag: bins lcp - P = 0 .. K - P
    const int nr = (ix.K - ix.P + 1 + 3) / 4;
    const int32_t w = ix.sufw;
    const int W = group_lanes(ix);
    const void *fn = w == 1 ? group_kernel_of<uint8_t>(nr, W)
                   : w == 2 ? group_kernel_of<uint16_t>(nr, W) : group_kernel_of<uint32_t>(nr, W);
    const void *tc = ix.tsuf.p;
    const uint32_t *of = ix.off.as<uint32_t>();
    int64_t n = ix.n;
    int32_t L = ix.L, K = ix.K, P = ix.P;
    const uint32_t *qc = a.qcode;
    int64_t m = a.m;
    void *args[] = {(void *)&tc, (void *)&of, (void *)&n, (void *)&L, (void *)&K, (void *)&P,
                    (void *)&qc, (void *)&m, (void *)&ranges, (void *)&big, (void *)&nbig};
    PF_HIP(hipLaunchKernel(fn, dim3((unsigned)((pairs * W + 255) / 256)), dim3(256), args, 0, s));
    // the list's length is known only on the device: a fixed grid strides over it
    const int64_t wg = std::min<int64_t>((pairs + 3) / 4, (int64_t)ix.num_cus * 8);
    if (w == 1)
        hipLaunchKernelGGL(k_ranges_wave<uint8_t>, dim3((unsigned)std::max<int64_t>(1, wg)), dim3(256), 0, s,
                           static_cast<const uint8_t *>(tc), of, n, L, K, P, qc, m, ranges, big, nbig);
    else if (w == 2)
        hipLaunchKernelGGL(k_ranges_wave<uint16_t>, dim3((unsigned)std::max<int64_t>(1, wg)), dim3(256), 0, s,
                           static_cast<const uint16_t *>(tc), of, n, L, K, P, qc, m, ranges, big, nbig);
    else
        hipLaunchKernelGGL(k_ranges_wave<uint32_t>, dim3((unsigned)std::max<int64_t>(1, wg)), dim3(256), 0, s,
                           static_cast<const uint32_t *>(tc), of, n, L, K, P, qc, m, ranges, big, nbig);
    PF_HIP(hipGetLastError());
}

} // namespace pf
