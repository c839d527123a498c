// The LSH forest as sorted arrays (Sec. 4.1; Sec. 4.2 "Retrieving candidate points"):
// repetition j is the array of (code, position) pairs sorted by code, equal codes in
// position order.  All L tables are sorted together by a stable LSD radix sort over
// 8-bit digits (three passes for K = 24): per 4096-key tile a 256-bin histogram, a
// per-table exclusive scan over (digit, tile), then a stable scatter in which each
// wave ranks its keys by ballot matching and the tile is reordered in LDS so that the
// writes of one digit go out contiguously.
// The prefix table (P-bit prefix positions, Sec. 4.2) and the table-local sketches
// (the sketch a repetition reads, Sec. 4.2 "Filtering candidate points") follow.
#include "pf_device.h"
#include "pf_internal.h"

namespace pf {

static constexpr int kTile = 4096;
static constexpr int kPer = kTile / 256;

__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                    int32_t shift, int32_t nblk,
                                                    uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    const int32_t blk = blockIdx.x, j = blockIdx.y;
    h[tid] = 0;
    __syncthreads();
    const uint32_t *kj = keys + (int64_t)j * n;
    const int64_t base = (int64_t)blk * kTile;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t e = base + r * 256 + tid;
        if (e < n) atomicAdd(&h[(kj[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[((int64_t)j * 256 + tid) * nblk + blk] = h[tid];
}

// exclusive scan, per table, of the 256 * nblk counts in (digit, tile) order
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t *__restrict__ hist, int32_t nblk) {
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t cnt = (int64_t)256 * nblk;
    uint32_t *h = hist + (int64_t)blockIdx.x * cnt;
    const int64_t per = (cnt + 255) / 256;
    const int64_t a = tid * per, b = min(cnt, a + per);
    uint32_t s = 0;
    for (int64_t e = a; e < b; ++e) s += h[e];
    // inclusive scan of the thread sums
    uint32_t v = s;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    uint32_t pre = v - s;
    for (int i = 0; i < w; ++i) pre += wsum[i];
    for (int64_t e = a; e < b; ++e) {
        const uint32_t c = h[e];
        h[e] = pre;
        pre += c;
    }
}

template <bool FIRST>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin, int64_t n,
                                                       int32_t shift, int32_t nblk,
                                                       const uint32_t *__restrict__ offs,
                                                       uint32_t *__restrict__ kout,
                                                       uint32_t *__restrict__ vout) {
    __shared__ uint32_t skey[kTile];
    __shared__ uint32_t sval[kTile];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t blk = blockIdx.x, j = blockIdx.y;
    const int64_t base = (int64_t)blk * kTile;
    const uint32_t *kj = kin + (int64_t)j * n;
    const uint32_t *vj = FIRST ? nullptr : vin + (int64_t)j * n;

    uint32_t key[kPer], val[kPer], rank[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t e = base + r * 256 + tid;
        key[r] = e < n ? kj[e] : 0u;
        val[r] = e < n ? (FIRST ? (uint32_t)e : vj[e]) : 0u;
    }
    run[tid] = 0;
    for (int i = 0; i < 4; ++i) wcnt[i][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t e = base + r * 256 + tid;
        const bool valid = e < n;
        const uint32_t dg = (key[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t rw = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rw == 0) wcnt[w][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t lr = 0;
        if (valid) {
            lr = run[dg] + rw;
            for (int i = 0; i < w; ++i) lr += wcnt[i][dg];
        }
        rank[r] = lr;
        __syncthreads();
        run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
        __syncthreads();
    }
    // exclusive scan of the tile's digit counts
    {
        const uint32_t c = run[tid];
        uint32_t v = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(v, o);
            if (lane >= o) v += t;
        }
        if (lane == 63) wsum[w] = v;
        __syncthreads();
        uint32_t pre = v - c;
        for (int i = 0; i < w; ++i) pre += wsum[i];
        dstart[tid] = pre;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t e = base + r * 256 + tid;
        if (e < n) {
            const uint32_t dg = (key[r] >> shift) & 255u;
            const uint32_t p = dstart[dg] + rank[r];
            skey[p] = key[r];
            sval[p] = val[r];
        }
    }
    __syncthreads();
    const int64_t cnt = min((int64_t)kTile, n - base);
    const uint32_t *oj = offs + (int64_t)j * 256 * nblk;
    uint32_t *ko = kout + (int64_t)j * n;
    uint32_t *vo = vout + (int64_t)j * n;
    for (int64_t p = tid; p < cnt; p += 256) {
        const uint32_t k = skey[p];
        const uint32_t dg = (k >> shift) & 255u;
        const int64_t dst = (int64_t)oj[(int64_t)dg * nblk + blk] + (p - dstart[dg]);
        if (dst < n) {
            ko[dst] = k;
            vo[dst] = sval[p];
        }
    }
}

void sort_tables(const uint32_t *codes, int64_t n, int32_t L, int32_t K, uint32_t *tcode,
                 uint32_t *tidx, DevBuf &scratch, hipStream_t s) {
    const int32_t nblk = (int32_t)((n + kTile - 1) / kTile);
    const int passes = (K + 7) / 8;
    const size_t hist_bytes = (size_t)L * 256 * nblk * sizeof(uint32_t);
    const size_t kv_bytes = (size_t)L * n * sizeof(uint32_t);
    scratch.ensure(hist_bytes + 2 * kv_bytes + 256);
    uint32_t *hist = scratch.as<uint32_t>();
    uint32_t *ka = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(scratch.p) + hist_bytes);
    uint32_t *va = ka + (size_t)L * n;
    // every slot is written by the scatter; zero them first so that no pass can ever
    // read an uninitialised position
    launch_fill_u32(ka, (int64_t)(2 * (size_t)L * n), 0u, s);
    launch_fill_u32(tcode, (int64_t)((size_t)L * n), 0u, s);
    launch_fill_u32(tidx, (int64_t)((size_t)L * n), 0u, s);
    // ping-pong so that the last pass lands in (tcode, tidx)
    const uint32_t *kin = codes;
    const uint32_t *vin = nullptr;
    for (int p = 0; p < passes; ++p) {
        const bool last = (p == passes - 1);
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        uint32_t *kout = to_out ? tcode : ka;
        uint32_t *vout = to_out ? tidx : va;
        (void)last;
        const int32_t shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk, L), dim3(256), 0, s, kin, n, shift, nblk, hist);
        PF_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_radix_scan, dim3(L), dim3(256), 0, s, hist, nblk);
        PF_HIP(hipGetLastError());
        if (p == 0)
            hipLaunchKernelGGL(k_radix_scatter<true>, dim3(nblk, L), dim3(256), 0, s, kin, vin, n,
                               shift, nblk, hist, kout, vout);
        else
            hipLaunchKernelGGL(k_radix_scatter<false>, dim3(nblk, L), dim3(256), 0, s, kin, vin, n,
                               shift, nblk, hist, kout, vout);
        PF_HIP(hipGetLastError());
        kin = kout;
        vin = vout;
    }
}

// off[j][p] = number of entries of table j whose leading P bits are < p, p = 0..2^P
__global__ __launch_bounds__(256) void k_prefix(const uint32_t *__restrict__ tcode, int64_t n,
                                                int32_t K, int32_t P, uint32_t *__restrict__ off) {
    const int64_t np1 = ((int64_t)1 << P) + 1;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t j = blockIdx.y;
    if (p >= np1) return;
    const uint32_t *tc = tcode + (int64_t)j * n;
    const uint64_t target = (uint64_t)p << (K - P);
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((uint64_t)tc[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    off[(int64_t)j * np1 + p] = (uint32_t)lo;
}

void prefix_tables(const uint32_t *tcode, int64_t n, int32_t L, int32_t K, int32_t P, uint32_t *off,
                   hipStream_t s) {
    const int64_t np1 = ((int64_t)1 << P) + 1;
    hipLaunchKernelGGL(k_prefix, dim3((unsigned)((np1 + 255) / 256), L), dim3(256), 0, s, tcode, n, K,
                       P, off);
    PF_HIP(hipGetLastError());
}

// Resident form of the sorted codes: inside a table's P-bit prefix bucket every code has
// the bucket's leading P bits, which the prefix table already holds (entry e lies in
// bucket b iff off[b] <= e < off[b + 1]), so only the low K - P bits of each code are kept,
// in 8 bits when K - P <= 8, 16 bits when K - P <= 16, else 32 (nothing when K <= P).
template <class S>
__global__ __launch_bounds__(256) void k_code_suffix(const uint32_t *__restrict__ tcode, int64_t total,
                                                     uint32_t mask, S *__restrict__ suf) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        suf[i] = (S)(tcode[i] & mask);
}

int32_t code_suffix_bytes(int32_t K, int32_t P) { return K <= P ? 0 : K - P <= 8 ? 1 : K - P <= 16 ? 2 : 4; }

int32_t prefix_bits_min(int32_t K) { return std::min(13, K); }
int32_t prefix_bits_max(int32_t K) { return std::min(24, K); }

// The prefix width with the fewest resident bytes per table: its prefix table
// (4 (2^P + 1) bytes) and the suffixes of n codes; the narrower one on a tie.
int32_t choose_prefix_bits(int64_t n, int32_t K) {
    int32_t best = prefix_bits_min(K);
    uint64_t best_b = ~0ull;
    for (int32_t P = prefix_bits_min(K); P <= prefix_bits_max(K); ++P) {
        const uint64_t b = 4ull * ((1ull << P) + 1ull) + (uint64_t)n * (uint64_t)code_suffix_bytes(K, P);
        if (b < best_b) {
            best_b = b;
            best = P;
        }
    }
    return best;
}

void code_suffixes(const uint32_t *tcode, int64_t n, int32_t L, int32_t K, int32_t P, void *suf, hipStream_t s) {
    const int32_t w = code_suffix_bytes(K, P);
    if (w == 0) return;
    const int64_t total = (int64_t)L * n;
    const uint32_t mask = K - P >= 32 ? 0xFFFFFFFFu : ((1u << (K - P)) - 1u);
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    if (w == 1)
        hipLaunchKernelGGL(k_code_suffix<uint8_t>, dim3(blocks), dim3(256), 0, s, tcode, total, mask,
                           static_cast<uint8_t *>(suf));
    else if (w == 2)
        hipLaunchKernelGGL(k_code_suffix<uint16_t>, dim3(blocks), dim3(256), 0, s, tcode, total, mask,
                           static_cast<uint16_t *>(suf));
    else
        hipLaunchKernelGGL(k_code_suffix<uint32_t>, dim3(blocks), dim3(256), 0, s, tcode, total, mask,
                           static_cast<uint32_t *>(suf));
    PF_HIP(hipGetLastError());
}

// The full sorted codes again (export): code = (bucket of e) << (K - P) | suffix.
template <class S>
__global__ __launch_bounds__(256) void k_code_join(const S *__restrict__ suf, const uint32_t *__restrict__ off,
                                                   int64_t n, int32_t K, int32_t P, uint32_t *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t j = blockIdx.y;
    if (e >= n) return;
    const int64_t np1 = ((int64_t)1 << P) + 1;
    const uint32_t *oj = off + (int64_t)j * np1;
    // the bucket: the largest b with off[b] <= e (off is non-decreasing, off[0] = 0)
    int64_t lo = 0, hi = np1 - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo + 1) >> 1);
        if ((int64_t)oj[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    const uint32_t sfx = suf ? (uint32_t)suf[(int64_t)j * n + e] : 0u;
    out[(int64_t)j * n + e] = K > P ? (((uint32_t)lo << (K - P)) | sfx) : (uint32_t)lo;
}

void join_codes(const void *suf, const uint32_t *off, int64_t n, int32_t L, int32_t K, int32_t P, uint32_t *out,
                hipStream_t s) {
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)L);
    const int32_t w = code_suffix_bytes(K, P);
    if (w == 4)
        hipLaunchKernelGGL(k_code_join<uint32_t>, grid, dim3(256), 0, s, static_cast<const uint32_t *>(suf), off, n,
                           K, P, out);
    else if (w == 1)
        hipLaunchKernelGGL(k_code_join<uint8_t>, grid, dim3(256), 0, s, static_cast<const uint8_t *>(suf), off, n,
                           K, P, out);
    else
        hipLaunchKernelGGL(k_code_join<uint16_t>, grid, dim3(256), 0, s, static_cast<const uint16_t *>(suf), off, n,
                           K, P, out);
    PF_HIP(hipGetLastError());
}

// tsk[j][e] = sketch[j mod M][tidx[j][e]]: the sketch repetition j reads, stored in the
// table's own order so that the filter streams it contiguously.
__global__ __launch_bounds__(256) void k_gather_sk(const uint32_t *__restrict__ tidx,
                                                   const uint64_t *__restrict__ sk, int64_t n,
                                                   int32_t M, uint64_t *__restrict__ tsk) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t j = blockIdx.y;
    if (e >= n) return;
    const uint64_t *sj = sk + (int64_t)(j % M) * n;
    tsk[(int64_t)j * n + e] = sj[tidx[(int64_t)j * n + e]];
}

void gather_sketches(const uint32_t *tidx, const uint64_t *sk, int64_t n, int32_t L, int32_t M,
                     uint64_t *tsk, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_sk, dim3((unsigned)((n + 255) / 256), L), dim3(256), 0, s, tidx, sk, n,
                       M, tsk);
    PF_HIP(hipGetLastError());
}

// Table positions in 3 bytes (every position below 2^24): thread t packs entries 4t .. 4t + 3
// into the 12 bytes 12t .. 12t + 11 and writes only the words that hold bytes of its
// entries, so that a partial last group stays inside 3 count + 4 bytes.
__global__ __launch_bounds__(256) void k_pack_pos3(const uint32_t *__restrict__ in, int64_t count,
                                                   uint32_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t e0 = 4 * t;
    if (e0 >= count) return;
    const int ne = (int)min((int64_t)4, count - e0);
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = u < ne ? (in[e0 + u] & 0xFFFFFFu) : 0u;
    uint32_t *o = out + 3 * t;
    o[0] = v[0] | (v[1] << 24);
    if (ne >= 2) o[1] = (v[1] >> 8) | (v[2] << 16);
    if (ne >= 3) o[2] = (v[2] >> 16) | (v[3] << 8);
}

__global__ __launch_bounds__(256) void k_unpack_pos(const uint8_t *__restrict__ in, int64_t count, int32_t posb,
                                                    uint32_t *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < count; g += stride)
        out[g] = posb == 4 ? read_pos<4>(in, (uint32_t)g) : read_pos<3>(in, (uint32_t)g);
}

int32_t pos_bytes_for(int64_t n, int32_t want) { return (want == 3 && n <= (1ll << 24)) ? 3 : 4; }

void pack_positions(const uint32_t *in, int64_t count, int32_t posb, uint8_t *out, hipStream_t s) {
    if (count <= 0) return;
    // the padding after the positions reads as zeros (two words from the one holding the
    // first padding byte; the pack below rewrites the position bytes among them)
    launch_fill_u32(reinterpret_cast<uint32_t *>(out + (count * posb) / 4 * 4), 2, 0u, s);
    if (posb == 4) {
        if (static_cast<const void *>(in) != static_cast<const void *>(out))
            PF_HIP(hipMemcpyAsync(out, in, (size_t)count * 4, hipMemcpyDeviceToDevice, s));
        return;
    }
    const int64_t groups = (count + 3) / 4;
    hipLaunchKernelGGL(k_pack_pos3, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, in, count,
                       reinterpret_cast<uint32_t *>(out));
    PF_HIP(hipGetLastError());
}

void unpack_positions(const uint8_t *in, int64_t count, int32_t posb, uint32_t *out, hipStream_t s) {
    if (count <= 0) return;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_unpack_pos, dim3((unsigned)blocks), dim3(256), 0, s, in, count, posb, out);
    PF_HIP(hipGetLastError());
}

} // namespace pf
