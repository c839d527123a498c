// Random-hyperplane hashing (Sec. 2.2: bit = 1 iff <a, x> >= 0) of many rows at once.
//
// The projection P = X . H^T is a dense contraction, so it runs on the gfx950 matrix
// cores: every FP32 operand v is split into two BF16 parts v = hi + lo + r with
// hi = bf16(v), lo = bf16(v - hi), |r| <= 2^-16 |v|, and the three products hi.hi,
// hi.lo and lo.hi are accumulated in FP32 by v_mfma_f32_32x32x16_bf16.  The dropped
// terms and the FP32 accumulation bound the error of every projection by a per-column
// beta (computed on the host, see pf_api.cpp); a bit whose |P| <= beta may have the
// wrong sign and is recomputed exactly as the FP64 sequential sum that defines it.
// Output is written word-wise: each 32-column block of the GEMM is one u32 word per
// row (a table code or half of a 64-bit sketch), packed with wave ballots.
#include "pf_internal.h"

namespace pf {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

static constexpr int kFlagBuf = 512; // per-workgroup LDS buffer of flagged (row, col)

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t *word_ptr(uint32_t *codes, uint32_t *skw, int64_t n, int32_t L,
                                              int32_t wb, int64_t row) {
    if (wb < L) return codes + (int64_t)wb * n + row;
    const int32_t s = wb - L;
    return skw + 2 * ((int64_t)(s >> 1) * n + row) + (s & 1);
}

// One workgroup: ROWS rows of X (kept in LDS as BF16 hi/lo) against the word blocks
// [blockIdx.y * wpy, ...); wave w takes every fourth word block.  MFMA operand layout
// (32x32x16 BF16): lane l supplies A[l % 32][8 (l / 32) .. +8) and B[8 (l / 32) .. +8)[l % 32];
// accumulator register r of lane l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
template <int ROWS>
__global__ __launch_bounds__(256) void k_hash_bf16x3(
    const float *__restrict__ X, int64_t n, int32_t dpad, int32_t kp, const uint16_t *__restrict__ Hhi,
    const uint16_t *__restrict__ Hlo, const float *__restrict__ beta, int32_t words, int32_t L,
    uint32_t kmask, int32_t wpy, uint32_t *__restrict__ codes, uint32_t *__restrict__ skw,
    uint32_t *__restrict__ flist, unsigned int *__restrict__ fcount, uint32_t fcap) {
    extern __shared__ __align__(16) uint16_t lds_x[];
    __shared__ uint32_t fbuf[2 * kFlagBuf];
    __shared__ unsigned int fcnt, fbase;
    uint16_t *xhi = lds_x;
    uint16_t *xlo = lds_x + ROWS * kp;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * ROWS;

    for (int idx = tid; idx < ROWS * kp; idx += 256) {
        const int r = idx / kp, c = idx - r * kp;
        const int64_t gr = row0 + r;
        float v = 0.0f;
        if (gr < n && c < dpad) v = X[gr * dpad + c];
        const uint16_t h = bf16_rne(v);
        const float hf = __uint_as_float((uint32_t)h << 16);
        xhi[idx] = h;
        xlo[idx] = bf16_rne(v - hf);
    }
    if (tid == 0) fcnt = 0;
    __syncthreads();

    const int wb0 = blockIdx.y * wpy;
    const int wb1 = min(words, wb0 + wpy);
    const int cl = lane & 31, kh = lane >> 5;
    constexpr int RT = ROWS / 32;

    for (int wb = wb0 + w; wb < wb1; wb += 4) {
        f32x16_t acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][r] = 0.0f;
        const int col = wb * 32 + cl;
        const uint16_t *bh = Hhi + (int64_t)col * kp + 8 * kh;
        const uint16_t *bl = Hlo + (int64_t)col * kp + 8 * kh;
        for (int ks = 0; ks < kp; ks += 16) {
            const bf16x8_t b_h = *(const bf16x8_t *)(bh + ks);
            const bf16x8_t b_l = *(const bf16x8_t *)(bl + ks);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int ao = (rt * 32 + cl) * kp + ks + 8 * kh;
                const bf16x8_t a_h = *(const bf16x8_t *)(xhi + ao);
                const bf16x8_t a_l = *(const bf16x8_t *)(xlo + ao);
                acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_h, acc[rt], 0, 0, 0);
                acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_l, acc[rt], 0, 0, 0);
                acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_l, b_h, acc[rt], 0, 0, 0);
            }
        }
        const float bta = beta[col];
        uint32_t wordv = 0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float P = acc[rt][r];
                const uint64_t mb = __ballot(P >= 0.0f);
                const uint64_t mf = __ballot(fabsf(P) <= bta);
                // lane l assembles the word of tile row l % 32 of row tile l / 32
                if ((lane >> 5) == rt && ((lane & 31) >> 3) == (r >> 2) && (lane & 3) == (r & 3))
                    wordv = ((lane >> 2) & 1) ? (uint32_t)(mb >> 32) : (uint32_t)mb;
                if (mf) {
                    if ((mf >> lane) & 1ull) {
                        const int64_t grow = row0 + rt * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
                        if (grow < n) {
                            const unsigned pos = atomicAdd(&fcnt, 1u);
                            if (pos < (unsigned)kFlagBuf) {
                                fbuf[2 * pos] = (uint32_t)grow;
                                fbuf[2 * pos + 1] = (uint32_t)col;
                            } else {
                                const unsigned gp = atomicAdd(fcount, 1u);
                                if (gp < fcap) {
                                    flist[2 * (int64_t)gp] = (uint32_t)grow;
                                    flist[2 * (int64_t)gp + 1] = (uint32_t)col;
                                }
                            }
                        }
                    }
                }
            }
        }
        const int64_t grow = row0 + lane;
        if (lane < ROWS && grow < n) {
            uint32_t *wp = word_ptr(codes, skw, n, L, wb, grow);
            *wp = (wb < L) ? (wordv & kmask) : wordv;
        }
    }
    __syncthreads();
    const unsigned nf = min(fcnt, (unsigned)kFlagBuf);
    if (tid == 0) fbase = nf ? atomicAdd(fcount, nf) : 0u;
    __syncthreads();
    for (unsigned t = tid; t < nf; t += 256) {
        const unsigned gp = fbase + t;
        if (gp < fcap) {
            flist[2 * (int64_t)gp] = fbuf[2 * t];
            flist[2 * (int64_t)gp + 1] = fbuf[2 * t + 1];
        }
    }
}

// Rows of at most 16 KS padded elements (kp <= 16 KS; KS = 8 or 16, the latter with two
// waves per SIMD for the registers): a workgroup takes 128 rows, 32 per
// wave, against the word blocks [blockIdx.y * wpy, ...), all four waves on the same word
// block.  Each wave keeps its rows' A fragments (BF16 hi and lo of every k step) in
// registers for the whole launch.  A word block's B fragments (32 columns x kp, hi and lo)
// are copied once per workgroup, with coalesced 16-byte loads, into LDS; the next block's
// copy is loaded into registers while the current one is multiplied.  Every load of the
// loop is unconditional (the last block loads itself again, missing chunks load chunk 0)
// and the flag bound is read before the next block's loads, so that no wait in the loop
// covers them.  The products and their order are those of k_hash_bf16x3 (per k step, k
// ascending: hi.hi, hi.lo, lo.hi), so every projection, flag and bit is the same.  A
// workgroup meets about n_cols / 1,000 flagged bits per row on unit vectors, so its LDS
// buffer holds 4,096 of them (global appends, whose wait would cover the next block's
// loads, are then rare).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
static constexpr int kArRows = 128, kArFlags = 4096;

__device__ __forceinline__ uint32_t bf16_pair(float v0, float v1, bool lo_part) {
    const uint16_t h0 = bf16_rne(v0), h1 = bf16_rne(v1);
    if (!lo_part) return (uint32_t)h0 | ((uint32_t)h1 << 16);
    const uint16_t l0 = bf16_rne(v0 - __uint_as_float((uint32_t)h0 << 16));
    const uint16_t l1 = bf16_rne(v1 - __uint_as_float((uint32_t)h1 << 16));
    return (uint32_t)l0 | ((uint32_t)l1 << 16);
}

template <int KS, int WPE>
__global__ __launch_bounds__(256, WPE) void k_hash_bf16x3_ar(
    const float *__restrict__ X, int64_t n, int32_t dpad, int32_t kp, const uint16_t *__restrict__ Hhi,
    const uint16_t *__restrict__ Hlo, const float *__restrict__ beta, int32_t words, int32_t L,
    uint32_t kmask, int32_t wpy, uint32_t *__restrict__ codes, uint32_t *__restrict__ skw,
    uint32_t *__restrict__ flist, unsigned int *__restrict__ fcount, uint32_t fcap) {
    constexpr int kArStride = KS * 16 + 8; // LDS elements per B column (16 bytes of padding)
    __shared__ __align__(16) uint16_t bsh[2][32 * kArStride];
    __shared__ uint32_t fbuf[2 * kArFlags];
    __shared__ unsigned int fcnt, fbase;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int cl = lane & 31, kh = lane >> 5;
    const int ksn = kp / 16;
    const int64_t row0 = (int64_t)blockIdx.x * kArRows + 32 * w;

    // A fragments: lane l holds row row0 + l % 32, elements 16 ks + 8 (l / 32) .. + 7
    u32x4_t a_h[KS], a_l[KS];
    {
        const int64_t gr = row0 + cl;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            float v[8];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = ks * 16 + 8 * kh + 4 * h;
                float4 f = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (ks < ksn && gr < n && c < dpad) f = *reinterpret_cast<const float4 *>(X + gr * dpad + c);
                v[4 * h] = f.x;
                v[4 * h + 1] = f.y;
                v[4 * h + 2] = f.z;
                v[4 * h + 3] = f.w;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a_h[ks][e] = bf16_pair(v[2 * e], v[2 * e + 1], false);
                a_l[ks][e] = bf16_pair(v[2 * e], v[2 * e + 1], true);
            }
        }
    }
    if (tid == 0) fcnt = 0;

    // B staging: 16-byte chunk q of a plane's word block (4 kp chunks) goes to column q / (kp / 8);
    // thread t moves chunks t, t + 256 (and t + 512, t + 768 when KS = 16) of both planes,
    // chunks past the block's end loading chunk 0 and storing nothing
    static_assert(KS == 8 || KS == 16, "k steps");
    const int nq = 4 * kp, qpc = kp / 8;
    auto chunk = [&](int i, int &q, int &d) {
        const int qq = tid + 256 * i;
        q = qq < nq ? qq : 0;
        const int c = q / qpc;
        d = qq < nq ? c * kArStride + (q - c * qpc) * 8 : -1;
    };
    int q0, q1, q2 = 0, q3 = 0, d0, d1, d2 = -1, d3 = -1;
    chunk(0, q0, d0);
    chunk(1, q1, d1);
    if constexpr (KS == 16) {
        chunk(2, q2, d2);
        chunk(3, q3, d3);
    }
    uint4 sh0, sh1, sh2, sh3, sl0, sl1, sl2, sl3;
#define PF_LOAD_B(WB)                                                                                  \
    {                                                                                                  \
        const uint4 *bh_ = reinterpret_cast<const uint4 *>(Hhi + (int64_t)(WB) * 32 * kp);                \
        const uint4 *bl_ = reinterpret_cast<const uint4 *>(Hlo + (int64_t)(WB) * 32 * kp);                \
        sh0 = bh_[q0];                                                                                 \
        sl0 = bl_[q0];                                                                                 \
        sh1 = bh_[q1];                                                                                 \
        sl1 = bl_[q1];                                                                                 \
        if constexpr (KS == 16) {                                                                      \
            sh2 = bh_[q2];                                                                             \
            sl2 = bl_[q2];                                                                             \
            sh3 = bh_[q3];                                                                             \
            sl3 = bl_[q3];                                                                             \
        }                                                                                              \
    }
#define PF_STORE_B(D, H, LO)                                                                           \
    if ((D) >= 0) {                                                                                    \
        *reinterpret_cast<uint4 *>(&bsh[0][(D)]) = (H);                                                \
        *reinterpret_cast<uint4 *>(&bsh[1][(D)]) = (LO);                                               \
    }

    const int wb0 = blockIdx.y * wpy;
    const int wb1 = min(words, wb0 + wpy);
    PF_LOAD_B(wb0);
    for (int wb = wb0; wb < wb1; ++wb) {
        __syncthreads(); // every wave is done with the previous block's B
        PF_STORE_B(d0, sh0, sl0)
        PF_STORE_B(d1, sh1, sl1)
        if constexpr (KS == 16) {
            PF_STORE_B(d2, sh2, sl2)
            PF_STORE_B(d3, sh3, sl3)
        }
        __syncthreads();
        const int col = wb * 32 + cl;
        const float bta = beta[col];
        PF_LOAD_B(min(wb + 1, wb1 - 1));
        f32x16_t acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks < ksn) {
                const int bo = cl * kArStride + 16 * ks + 8 * kh;
                const bf16x8_t b_h = *reinterpret_cast<const bf16x8_t *>(&bsh[0][bo]);
                const bf16x8_t b_l = *reinterpret_cast<const bf16x8_t *>(&bsh[1][bo]);
                const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, a_h[ks]);
                const bf16x8_t al = __builtin_bit_cast(bf16x8_t, a_l[ks]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b_h, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, b_l, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b_h, acc, 0, 0, 0);
            }
        }
        uint32_t wordv = 0, fl = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float P = acc[r];
            const uint64_t mb = __ballot(P >= 0.0f);
            // lane t < 32 assembles the word of tile row t (register 4 (t / 8) + t % 4, half (t / 4) % 2)
            if ((cl >> 3) == (r >> 2) && (lane & 3) == (r & 3))
                wordv = ((lane >> 2) & 1) ? (uint32_t)(mb >> 32) : (uint32_t)mb;
            fl |= (fabsf(P) <= bta ? 1u : 0u) << r;
        }
        if (fl) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if ((fl >> r) & 1u) {
                    const int64_t grow = row0 + 8 * (r >> 2) + 4 * kh + (r & 3);
                    if (grow < n) {
                        const unsigned pos = atomicAdd(&fcnt, 1u);
                        if (pos < (unsigned)kArFlags) {
                            fbuf[2 * pos] = (uint32_t)grow;
                            fbuf[2 * pos + 1] = (uint32_t)col;
                        } else {
                            const unsigned gp = atomicAdd(fcount, 1u);
                            if (gp < fcap) {
                                flist[2 * (int64_t)gp] = (uint32_t)grow;
                                flist[2 * (int64_t)gp + 1] = (uint32_t)col;
                            }
                        }
                    }
                }
            }
        }
        const int64_t grow = row0 + lane;
        if (lane < 32 && grow < n) {
            uint32_t *wp = word_ptr(codes, skw, n, L, wb, grow);
            *wp = (wb < L) ? (wordv & kmask) : wordv;
        }
    }
    __syncthreads();
    const unsigned nf = min(fcnt, (unsigned)kArFlags);
    if (tid == 0) fbase = nf ? atomicAdd(fcount, nf) : 0u;
    __syncthreads();
    for (unsigned t = tid; t < nf; t += 256) {
        const unsigned gp = fbase + t;
        if (gp < fcap) {
            flist[2 * (int64_t)gp] = fbuf[2 * t];
            flist[2 * (int64_t)gp + 1] = fbuf[2 * t + 1];
        }
    }
}

#undef PF_LOAD_B
#undef PF_STORE_B

__device__ __forceinline__ double dot_seq64(const float *__restrict__ a, const float *__restrict__ x,
                                            int32_t d) {
    double s = 0.0;
    if ((d & 3) == 0) {
        // the same sequence of additions, the operands read four at a time (rows of a
        // multiple of 4 floats start 16-byte aligned)
        const float4 *a4 = reinterpret_cast<const float4 *>(a), *x4 = reinterpret_cast<const float4 *>(x);
        for (int32_t c = 0; c < d / 4; ++c) {
            const float4 u = a4[c], v = x4[c];
            s = s + (double)u.x * (double)v.x;
            s = s + (double)u.y * (double)v.y;
            s = s + (double)u.z * (double)v.z;
            s = s + (double)u.w * (double)v.w;
        }
        return s;
    }
    for (int32_t c = 0; c < d; ++c) s = s + (double)a[c] * (double)x[c];
    return s;
}

// Fix the flagged bits with the FP64 sequential projection.  If more bits were flagged
// than the list holds, every word is recomputed in FP64 instead.
__global__ __launch_bounds__(256) void k_hash_fix(const float *__restrict__ X, int64_t n, int32_t dpad,
                                                  int32_t d, const float *__restrict__ hp,
                                                  const int32_t *__restrict__ colrow, int32_t words,
                                                  int32_t L, uint32_t kmask, uint32_t *codes,
                                                  uint32_t *skw, const uint32_t *__restrict__ flist,
                                                  const unsigned int *__restrict__ fcount,
                                                  uint32_t fcap) {
    const unsigned cnt = *fcount;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cnt <= fcap) {
        for (int64_t t = t0; t < (int64_t)cnt; t += stride) {
            const int64_t row = flist[2 * t];
            const int32_t col = (int32_t)flist[2 * t + 1];
            const int32_t hr = colrow[col];
            const double s = dot_seq64(hp + (int64_t)hr * d, X + row * dpad, d);
            const uint32_t bit = 1u << (col & 31);
            uint32_t *wp = word_ptr(codes, skw, n, L, col >> 5, row);
            if (s >= 0.0)
                atomicOr(wp, bit);
            else
                atomicAnd(wp, ~bit);
        }
    } else {
        for (int64_t t = t0; t < n * (int64_t)words; t += stride) {
            const int64_t row = t / words;
            const int32_t wb = (int32_t)(t - row * words);
            uint32_t wv = 0;
            for (int b = 0; b < 32; ++b) {
                const int32_t hr = colrow[wb * 32 + b];
                if (hr < 0) continue;
                if (dot_seq64(hp + (int64_t)hr * d, X + row * dpad, d) >= 0.0) wv |= 1u << b;
            }
            *word_ptr(codes, skw, n, L, wb, row) = (wb < L) ? (wv & kmask) : wv;
        }
    }
}

// Reference arithmetic: every projection as the FP64 sequential sum.  One wave per
// (row, pair of words); lane l owns column 64 p + l.
__global__ __launch_bounds__(256) void k_hash_fp64(const float *__restrict__ X, int64_t n, int32_t dpad,
                                                   int32_t d, const float *__restrict__ hp,
                                                   const int32_t *__restrict__ colrow, int32_t words,
                                                   int32_t L, uint32_t kmask, uint32_t *codes,
                                                   uint32_t *skw) {
    const int lane = threadIdx.x & 63;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int32_t pairs = (words + 1) / 2;
    if (task >= n * (int64_t)pairs) return;
    const int64_t row = task / pairs;
    const int32_t pw = (int32_t)(task - row * pairs);
    const int32_t col = pw * 64 + lane;
    bool bit = false;
    if (col < words * 32) {
        const int32_t hr = colrow[col];
        if (hr >= 0) bit = dot_seq64(hp + (int64_t)hr * d, X + row * dpad, d) >= 0.0;
    }
    const uint64_t mb = __ballot(bit);
    if (lane < 2) {
        const int32_t wb = 2 * pw + lane;
        if (wb < words) {
            const uint32_t wv = lane ? (uint32_t)(mb >> 32) : (uint32_t)mb;
            *word_ptr(codes, skw, n, L, wb, row) = (wb < L) ? (wv & kmask) : wv;
        }
    }
}

// Pooling (Sec. 3.2): table j's code from the pool bits, h_{t+1,j} = pool function
// sel[j K + t] as bit K-1-t.  One thread per (point, table); pool bits word-major.
__global__ __launch_bounds__(256) void k_pool_codes(const uint32_t *__restrict__ pbits, int64_t n,
                                                    const int32_t *__restrict__ sel, int32_t L, int32_t K,
                                                    uint32_t *__restrict__ codes) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t j = blockIdx.y;
    if (i >= n || j >= L) return;
    uint32_t code = 0;
    for (int32_t t = 0; t < K; ++t) {
        const int32_t f = sel[(int64_t)j * K + t];
        code |= ((pbits[(int64_t)(f >> 5) * n + i] >> (f & 31)) & 1u) << (K - 1 - t);
    }
    codes[(int64_t)j * n + i] = code;
}

static void hash_gemm(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint32_t *skw, uint32_t kmask,
                      const int32_t *colrow, char *scratch, uint32_t fcap, hipStream_t s);
static void hash_gemm_wide(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint32_t *skw,
                           uint32_t kmask, const uint16_t *Hhi, const uint16_t *Hlo, uint32_t *flist,
                           unsigned int *fcount, uint32_t fcap, hipStream_t s);

// Cross-polytope codes with three Hadamard rotations (Sec. 2.2, Sec. 4.3): one wave per
// point (four per workgroup), the point zero padded to d' in the wave's LDS as FP64.  For
// each function: flip the coordinates whose sign bit is set, apply the Walsh-Hadamard
// butterflies h = 1, 2, 4, ... ((y[j], y[j+h]) -> (a + b, a - b) for bit h of j clear,
// the same operations in the same precision as the definition), three rounds; then the
// largest |y_i| (smallest i on ties) by a wave reduction, value = [y_i < 0] d' + i.  The
// code is the first K bits of the table's c values concatenated.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_cp_hash(const float *__restrict__ X, int64_t n, int32_t dpad, int32_t d,
                                                 int32_t dp, int32_t ell, int32_t c, int32_t L, int32_t K,
                                                 const uint32_t *__restrict__ sign, uint32_t *__restrict__ codes) {
    extern __shared__ double cp_lds[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    if (i >= n) return; // the whole wave leaves; only wave-local LDS is used below
    double *y = cp_lds + (int64_t)w * dp;
    const float *xr = X + i * (int64_t)dpad;
    const int32_t sw = (dp + 31) / 32;
    for (int32_t j = 0; j < L; ++j) {
        uint64_t cat = 0;
        for (int32_t f = 0; f < c; ++f) {
            const int64_t fn = (int64_t)j * c + f;
            for (int e = lane; e < dp; e += 64) y[e] = e < d ? (double)xr[e] : 0.0;
            for (int k = 0; k < 3; ++k) {
                const uint32_t *sg = sign + (fn * 3 + k) * sw;
                wave_lds_sync();
                for (int e = lane; e < dp; e += 64)
                    if ((sg[e >> 5] >> (e & 31)) & 1u) y[e] = -y[e];
                for (int h = 1; h < dp; h <<= 1) {
                    wave_lds_sync();
                    for (int q = lane; q < dp / 2; q += 64) {
                        const int jj = (q / h) * 2 * h + (q % h);
                        const double a = y[jj], b = y[jj + h];
                        y[jj] = a + b;
                        y[jj + h] = a - b;
                    }
                }
            }
            wave_lds_sync();
            double best = -1.0;
            int bi = 0;
            for (int e = lane; e < dp; e += 64) {
                const double v = fabs(y[e]);
                if (v > best) {
                    best = v;
                    bi = e;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o);
                const int oi = __shfl_xor(bi, o);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            const uint32_t v = (y[bi] < 0.0 ? (uint32_t)dp : 0u) + (uint32_t)bi;
            cat = (cat << ell) | v;
            wave_lds_sync();
        }
        if (lane == 0) codes[(int64_t)j * n + i] = (uint32_t)(cat >> (c * ell - K));
    }
}

// The same codes with the point in registers, for d' <= 256: lane l holds elements
// l + 64 t (t < E = max(1, d'/64)); butterflies of stride h < 64 pair lanes l and l^h
// (exchanged across lanes), larger strides pair registers of one lane.  The lane whose
// element has bit h clear computes a + b, its partner a - b, with a, b the same operands as
// in the definition.  A table's sign words are loaded once, before its first function.
// value of lane l ^ H for a 64-bit value: DPP for H <= 8 (quad_perm; row_shl:H hands lane
// l the value of lane l + H, row_shr:H that of l - H, within rows of 16), ds_swizzle for
// H = 16 (xor within 32 lanes), a lane permute for H = 32.  Called with every lane of the
// wave active.
template <int CTRL> __device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int H> __device__ __forceinline__ uint32_t xor_lane32(uint32_t v, int lane) {
    if constexpr (H == 1) return dpp32<0xB1>(v);
    else if constexpr (H == 2) return dpp32<0x4E>(v);
    else if constexpr (H == 4 || H == 8) {
        // both moves on every lane (a DPP read of a lane outside the active mask is not
        // defined), then a select
        const uint32_t up = dpp32<0x100 + H>(v), down = dpp32<0x110 + H>(v);
        return (lane & H) ? down : up;
    }
    else if constexpr (H == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
    else return (uint32_t)__shfl_xor((int)v, 32);
}
template <int H> __device__ __forceinline__ double xor_lane(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = xor_lane32<H>((uint32_t)u, lane), hi = xor_lane32<H>((uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <int H> __device__ __forceinline__ void fht_stage(double *y, int E, int lane) {
    const bool upper = (lane & H) != 0;
    for (int t = 0; t < E; ++t) {
        const double o = xor_lane<H>(y[t], lane);
        y[t] = upper ? (o - y[t]) : (y[t] + o);
    }
}
template <int H> __device__ __forceinline__ void argmax_step(double &best, double &bv, int &bi, int lane) {
    const double ob = xor_lane<H>(best, lane), ov = xor_lane<H>(bv, lane);
    const int oi = (int)xor_lane32<H>((uint32_t)bi, lane);
    if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bv = ov;
        bi = oi;
    }
}

template <int E>
__global__ __launch_bounds__(256) void k_cp_hash_reg(const float *__restrict__ X, int64_t n, int32_t dpad, int32_t d,
                                                     int32_t dp, int32_t ell, int32_t c, int32_t L, int32_t K,
                                                     const uint32_t *__restrict__ sign,
                                                     uint32_t *__restrict__ codes) {
    constexpr int CMAX = 32; // functions per table (c = ceil(K / ell) <= 32)
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const float *xr = X + i * (int64_t)dpad;
    const bool live = lane < dp; // d' < 64 leaves lanes idle
    double x0[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int e = lane + 64 * t;
        x0[t] = (live && e < d) ? (double)xr[e] : 0.0;
    }
    const int32_t sw = (dp + 31) / 32;
    for (int32_t j = 0; j < L; ++j) {
        // this lane's sign bits of the table's functions: bit (f, k, t)
        uint32_t sbits[CMAX];
#pragma unroll
        for (int f = 0; f < CMAX; ++f) sbits[f] = 0;
        for (int f = 0; f < c; ++f) {
            uint32_t b = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int t = 0; t < E; ++t) {
                    const int e = lane + 64 * t;
                    const uint32_t wv = live ? sign[((int64_t)j * c + f) * 3 * sw + k * sw + (e >> 5)] : 0u;
                    b |= ((wv >> (e & 31)) & 1u) << (k * E + t);
                }
            sbits[f] = b;
        }
        uint64_t cat = 0;
        for (int f = 0; f < c; ++f) {
            double y[E];
#pragma unroll
            for (int t = 0; t < E; ++t) y[t] = x0[t];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
#pragma unroll
                for (int t = 0; t < E; ++t)
                    if ((sbits[f] >> (k * E + t)) & 1u) y[t] = -y[t];
                // strides below 64 pair lanes (d' < 64: only strides below d', whose partners
                // stay among the live lanes)
                if (dp > 1) fht_stage<1>(y, E, lane);
                if (dp > 2) fht_stage<2>(y, E, lane);
                if (dp > 4) fht_stage<4>(y, E, lane);
                if (dp > 8) fht_stage<8>(y, E, lane);
                if (dp > 16) fht_stage<16>(y, E, lane);
                if (dp > 32) fht_stage<32>(y, E, lane);
#pragma unroll
                for (int hb = 1; hb < E; hb <<= 1)
#pragma unroll
                    for (int t = 0; t < E; ++t)
                        if (!(t & hb)) {
                            const double a = y[t], b = y[t + hb];
                            y[t] = a + b;
                            y[t + hb] = a - b;
                        }
            }
            double best = -1.0, bv = 0.0;
            int bi = 0;
#pragma unroll
            for (int t = 0; t < E; ++t)
                if (live && fabs(y[t]) > best) {
                    best = fabs(y[t]);
                    bv = y[t];
                    bi = lane + 64 * t;
                }
            argmax_step<32>(best, bv, bi, lane);
            argmax_step<16>(best, bv, bi, lane);
            argmax_step<8>(best, bv, bi, lane);
            argmax_step<4>(best, bv, bi, lane);
            argmax_step<2>(best, bv, bi, lane);
            argmax_step<1>(best, bv, bi, lane);
            cat = (cat << ell) | ((bv < 0.0 ? (uint32_t)dp : 0u) + (uint32_t)bi);
        }
        if (lane == 0) codes[(int64_t)j * n + i] = (uint32_t)(cat >> (c * ell - K));
    }
}

void cp_codes(const Index &ix, const float *X, int64_t n, uint32_t *codes, hipStream_t s) {
    if (n <= 0) return;
    if (ix.cp_dp <= 256 && ix.cp_c <= 32) {
        const dim3 grid((unsigned)((n + 3) / 4));
        if (ix.cp_dp <= 64)
            hipLaunchKernelGGL(k_cp_hash_reg<1>, grid, dim3(256), 0, s, X, n, ix.dpad, ix.d, ix.cp_dp, ix.cp_ell,
                               ix.cp_c, ix.L, ix.K, ix.cpsign.as<uint32_t>(), codes);
        else if (ix.cp_dp <= 128)
            hipLaunchKernelGGL(k_cp_hash_reg<2>, grid, dim3(256), 0, s, X, n, ix.dpad, ix.d, ix.cp_dp, ix.cp_ell,
                               ix.cp_c, ix.L, ix.K, ix.cpsign.as<uint32_t>(), codes);
        else
            hipLaunchKernelGGL(k_cp_hash_reg<4>, grid, dim3(256), 0, s, X, n, ix.dpad, ix.d, ix.cp_dp, ix.cp_ell,
                               ix.cp_c, ix.L, ix.K, ix.cpsign.as<uint32_t>(), codes);
        PF_HIP(hipGetLastError());
        return;
    }
    const size_t lds = (size_t)4 * ix.cp_dp * sizeof(double);
    PF_HIP(hipFuncSetAttribute((const void *)k_cp_hash, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_cp_hash, dim3((unsigned)((n + 3) / 4)), dim3(256), lds, s, X, n, ix.dpad, ix.d, ix.cp_dp,
                       ix.cp_ell, ix.cp_c, ix.L, ix.K, ix.cpsign.as<uint32_t>(), codes);
    PF_HIP(hipGetLastError());
}


// scratch of hash_rows_into for n rows: the pool bits (with a pool), then the GEMM's
// flagged-bit count and list of at most fcap (row, column) pairs
static void hash_scratch_parts(const Index &ix, int64_t n, size_t *pool_bytes, uint32_t *fcap) {
    const HashPlan &hp = ix.plan;
    *pool_bytes = hp.pool ? ((size_t)n * hp.cw * sizeof(uint32_t) + 255) / 256 * 256 : 0;
    const uint64_t want = (uint64_t)n * (uint64_t)hp.ncols / 64u + 65536u;
    *fcap = (uint32_t)std::min<uint64_t>(want, 1ull << 30);
}

size_t hash_scratch_bytes(const Index &ix, int64_t n) {
    size_t pool_bytes;
    uint32_t fcap;
    hash_scratch_parts(ix, n, &pool_bytes, &fcap);
    return pool_bytes + 256 + (size_t)fcap * 8;
}

void hash_rows(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint64_t *sketches,
               DevBuf &scratch, hipStream_t s) {
    if (n <= 0) return;
    // the scratch is the caller's and outlives the queued kernels
    scratch.ensure(hash_scratch_bytes(ix, n));
    hash_rows_into(ix, X, n, codes, sketches, scratch.as<char>(), s);
}

void hash_rows_into(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint64_t *sketches,
                    char *scratch, hipStream_t s) {
    if (n <= 0) return;
    const HashPlan &hp = ix.plan;
    size_t pool_bytes;
    uint32_t fcap;
    hash_scratch_parts(ix, n, &pool_bytes, &fcap);
    uint32_t *table_codes = codes;
    if (hp.pool) codes = reinterpret_cast<uint32_t *>(scratch); // the GEMM writes the pool bits; codes are gathered at the end
    launch_fill_u32(codes, n * (int64_t)hp.cw, 0u, s);
    launch_fill_u32(reinterpret_cast<uint32_t *>(sketches), 2 * n * (int64_t)hp.M, 0u, s);
    const uint32_t kmask = (hp.pool || hp.K >= 32) ? 0xFFFFFFFFu : ((1u << hp.K) - 1u);
    uint32_t *skw = reinterpret_cast<uint32_t *>(sketches);
    const int32_t *colrow = ix.hcolrow.as<int32_t>();
    if (ix.hash_mode == PF_HASH_FP64 || hp.kp > 512) {
        const int64_t tasks = n * (int64_t)((hp.words + 1) / 2);
        hipLaunchKernelGGL(k_hash_fp64, dim3((unsigned)((tasks + 3) / 4)), dim3(256), 0, s, X, n,
                           ix.dpad, hp.d, ix.hp.as<float>(), colrow, hp.words, hp.cw, kmask, codes, skw);
        PF_HIP(hipGetLastError());
    } else {
        hash_gemm(ix, X, n, codes, skw, kmask, colrow, scratch + pool_bytes, fcap, s);
    }
    if (ix.family == PF_FAMILY_FHTCP) cp_codes(ix, X, n, table_codes, s);
    if (hp.pool) {
        hipLaunchKernelGGL(k_pool_codes, dim3((unsigned)((n + 255) / 256), (unsigned)hp.L), dim3(256), 0, s,
                           (const uint32_t *)codes, n, ix.psel.as<int32_t>(), hp.L, hp.K, table_codes);
        PF_HIP(hipGetLastError());
    }
}

// split-BF16 GEMM of the rows against the plan's columns, then the FP64 fix of the
// flagged bits
static void hash_gemm(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint32_t *skw, uint32_t kmask,
                      const int32_t *colrow, char *scratch, uint32_t fcap, hipStream_t s) {
    const HashPlan &hp = ix.plan;
    // scratch: the flagged-bit count, then room for fcap flagged (row, column) pairs
    unsigned int *fcount = reinterpret_cast<unsigned int *>(scratch);
    uint32_t *flist = reinterpret_cast<uint32_t *>(scratch + 256);
    launch_fill_u32(reinterpret_cast<uint32_t *>(fcount), 1, 0u, s);

    const uint16_t *Hhi = ix.hbf.as<uint16_t>();
    const uint16_t *Hlo = Hhi + (size_t)hp.ncols * hp.kp;
    if (hp.kp <= 256) {
        const int64_t bx = (n + kArRows - 1) / kArRows;
        int32_t gy = 1;
        if (bx < 4096) gy = (int32_t)std::min<int64_t>((hp.words + 3) / 4, (4096 + bx - 1) / bx);
        const int32_t wpy = (hp.words + gy - 1) / gy;
        gy = (hp.words + wpy - 1) / wpy;
        if (hp.kp <= 128)
            hipLaunchKernelGGL((k_hash_bf16x3_ar<8, 3>), dim3((unsigned)bx, (unsigned)gy), dim3(256), 0, s, X, n,
                               ix.dpad, hp.kp, Hhi, Hlo, ix.hbeta.as<float>(), hp.words, hp.cw, kmask, wpy, codes,
                               skw, flist, fcount, fcap);
        else
            hipLaunchKernelGGL((k_hash_bf16x3_ar<16, 2>), dim3((unsigned)bx, (unsigned)gy), dim3(256), 0, s, X, n,
                               ix.dpad, hp.kp, Hhi, Hlo, ix.hbeta.as<float>(), hp.words, hp.cw, kmask, wpy, codes,
                               skw, flist, fcount, fcap);
        PF_HIP(hipGetLastError());
    } else {
        hash_gemm_wide(ix, X, n, codes, skw, kmask, Hhi, Hlo, flist, fcount, fcap, s);
    }
    hipLaunchKernelGGL(k_hash_fix, dim3(1024), dim3(256), 0, s, X, n, ix.dpad, hp.d, ix.hp.as<float>(),
                       colrow, hp.words, hp.cw, kmask, codes, skw, flist, fcount, fcap);
    PF_HIP(hipGetLastError());
}

// rows of more than 256 padded elements: the row tile in LDS, B fragments from global memory
static void hash_gemm_wide(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint32_t *skw,
                           uint32_t kmask, const uint16_t *Hhi, const uint16_t *Hlo, uint32_t *flist,
                           unsigned int *fcount, uint32_t fcap, hipStream_t s) {
    const HashPlan &hp = ix.plan;
    const bool big = hp.kp > 256;
    const int rows = big ? 32 : 64;
    const int64_t bx = (n + rows - 1) / rows;
    int32_t gy = 1;
    if (bx < 4096) gy = (int32_t)std::min<int64_t>((hp.words + 3) / 4, (4096 + bx - 1) / bx);
    const int32_t wpy = (hp.words + gy - 1) / gy;
    gy = (hp.words + wpy - 1) / wpy;
    const size_t lds = (size_t)2 * rows * hp.kp * sizeof(uint16_t);
    if (big) {
        PF_HIP(hipFuncSetAttribute((const void *)k_hash_bf16x3<32>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_hash_bf16x3<32>, dim3((unsigned)bx, (unsigned)gy), dim3(256), lds, s, X, n,
                           ix.dpad, hp.kp, Hhi, Hlo, ix.hbeta.as<float>(), hp.words, hp.cw, kmask, wpy,
                           codes, skw, flist, fcount, fcap);
    } else {
        PF_HIP(hipFuncSetAttribute((const void *)k_hash_bf16x3<64>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_hash_bf16x3<64>, dim3((unsigned)bx, (unsigned)gy), dim3(256), lds, s, X, n,
                           ix.dpad, hp.kp, Hhi, Hlo, ix.hbeta.as<float>(), hp.words, hp.cw, kmask, wpy,
                           codes, skw, flist, fcount, fcap);
    }
    PF_HIP(hipGetLastError());
}

} // namespace pf
