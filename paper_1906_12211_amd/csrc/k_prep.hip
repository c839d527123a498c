// Vector storage (Sec. 4.2 "Vector storage"): every data and query vector is stored at
// unit length.  The squared norm is an FP64 sum in index order, the square root and the
// quotient are FP64 (IEEE, correctly rounded on gfx950), and each quotient is rounded
// once to FP32.  Rows are written with a padded stride (a multiple of 4 floats, zero
// filled) so that the re-rank kernel can use 16-byte loads.
#include "pf_internal.h"

namespace pf {

// A workgroup normalises a tile of rows: the tile is read into LDS with coalesced loads,
// eight in flight per thread, one thread per row sums its squares sequentially from LDS
// (row stride d + 1 against bank conflicts), and the quotients are written back coalesced.
// Tile positions fit 32 bits (rows_per_block * (d + 1) elements of LDS).
__global__ __launch_bounds__(256) void k_normalize(const float *__restrict__ x, int64_t n, int32_t d,
                                                   int32_t ld_in, float *__restrict__ out,
                                                   int32_t dpad, int32_t rows_per_block,
                                                   unsigned long long *bad) {
    extern __shared__ float tile[];
    double *nrm = reinterpret_cast<double *>(tile + (((size_t)rows_per_block * (d + 1) + 1) & ~(size_t)1));
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int rows = (int)min((int64_t)rows_per_block, n - r0);
    const int ld = d + 1;
    const float *xb = x + r0 * (int64_t)ld_in;
    const int total = rows * d;
    for (int t0 = tid; t0 < total; t0 += 8 * 256) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + 256 * u;
            if (t < total) {
                const int r = t / d, c = t - r * d;
                v[u] = xb[(int64_t)r * ld_in + c];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + 256 * u;
            if (t < total) {
                const int r = t / d, c = t - r * d;
                tile[r * ld + c] = v[u];
            }
        }
    }
    __syncthreads();
    for (int r = tid; r < rows; r += blockDim.x) {
        double s = 0.0;
        for (int32_t c = 0; c < d; ++c) {
            const double v = (double)tile[r * ld + c];
            s = s + v * v;
        }
        const double q = sqrt(s);
        const bool ok = q > 0.0 && isfinite(q);
        if (!ok) atomicMin(bad, (unsigned long long)(r0 + r));
        nrm[r] = ok ? q : 0.0;
    }
    __syncthreads();
    // x and out may alias (same stride): every element was read into LDS above
    float *ob = out + r0 * (int64_t)dpad;
    for (int t = tid; t < rows * dpad; t += 256) {
        const int r = t / dpad, c = t - r * dpad;
        const double q = nrm[r];
        ob[t] = (c < d && q > 0.0) ? (float)((double)tile[r * ld + c] / q) : 0.0f;
    }
}

void launch_normalize(const float *x, int64_t n, int32_t d, int32_t ld_in, float *out, int32_t dpad,
                      unsigned long long *bad, hipStream_t s) {
    if (n <= 0) return;
    // about 64 KB of LDS per workgroup: at most 256 rows, at least one
    const int32_t rpb = (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, 16000 / (d + 1)));
    const size_t lds = (((size_t)rpb * (d + 1) + 1) & ~(size_t)1) * sizeof(float) + (size_t)rpb * sizeof(double);
    PF_HIP(hipFuncSetAttribute((const void *)k_normalize, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int64_t blocks = (n + rpb - 1) / rpb;
    hipLaunchKernelGGL(k_normalize, dim3((unsigned)blocks), dim3(256), lds, s, x, n, d, ld_in, out, dpad, rpb,
                       bad);
    PF_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t count, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) p[t] = v;
}

void launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t s) {
    if (count <= 0) return;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
    PF_HIP(hipGetLastError());
}

// Vector storage as two 16-bit planes.  Element c of row r (c < dpad) has its upper
// half (the value truncated to bfloat16) at hi[r * hs + c] and its lower half at
// hi[r * hs + dpad + c] when c < spare = hs - dpad (the padding of the upper row), else
// at lo[r * ls + c - spare]; ls = dpad - spare.  ((upper << 16) | lower) is the FP32
// value exactly, and the two planes hold 4 dpad bytes per row, as the FP32 array did.
__global__ __launch_bounds__(256) void k_split_planes(const uint32_t *__restrict__ X, int64_t n, int32_t dpad,
                                                      int32_t hs, int32_t ls, uint16_t *__restrict__ hi,
                                                      uint16_t *__restrict__ lo) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t spare = hs - dpad;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * dpad; t += stride) {
        const int64_t r = t / dpad;
        const int32_t c = (int32_t)(t - r * dpad);
        const uint32_t v = X[t];
        hi[r * hs + c] = (uint16_t)(v >> 16);
        if (c < spare)
            hi[r * hs + dpad + c] = (uint16_t)(v & 0xFFFFu);
        else
            lo[r * ls + c - spare] = (uint16_t)(v & 0xFFFFu);
    }
}

__global__ __launch_bounds__(256) void k_join_planes(const uint16_t *__restrict__ hi, const uint16_t *__restrict__ lo,
                                                     int64_t n, int32_t dpad, int32_t hs, int32_t ls,
                                                     uint32_t *__restrict__ X) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t spare = hs - dpad;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * dpad; t += stride) {
        const int64_t r = t / dpad;
        const int32_t c = (int32_t)(t - r * dpad);
        const uint32_t w = c < spare ? hi[r * hs + dpad + c] : lo[r * ls + c - spare];
        X[t] = ((uint32_t)hi[r * hs + c] << 16) | w;
    }
}

void plane_strides(int32_t dpad, int32_t *hs, int32_t *ls) {
    // upper rows padded to whole 128-byte lines when the padding can hold lower halves
    // (at most dpad of them), so that a row is read as whole lines; else unpadded
    const int32_t h = (dpad + 63) / 64 * 64;
    *hs = h <= 2 * dpad ? h : dpad;
    *ls = dpad - (*hs - dpad);
}

void launch_split_planes(const float *X, int64_t n, int32_t dpad, uint16_t *hi, uint16_t *lo, hipStream_t s) {
    if (n <= 0) return;
    int32_t hs, ls;
    plane_strides(dpad, &hs, &ls);
    const int64_t blocks = std::min<int64_t>((n * dpad + 255) / 256, 65536);
    hipLaunchKernelGGL(k_split_planes, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const uint32_t *>(X), n, dpad, hs, ls, hi, lo);
    PF_HIP(hipGetLastError());
}

void launch_join_planes(const uint16_t *hi, const uint16_t *lo, int64_t n, int32_t dpad, float *X, hipStream_t s) {
    if (n <= 0) return;
    int32_t hs, ls;
    plane_strides(dpad, &hs, &ls);
    const int64_t blocks = std::min<int64_t>((n * dpad + 255) / 256, 65536);
    hipLaunchKernelGGL(k_join_planes, dim3((unsigned)blocks), dim3(256), 0, s, hi, lo, n, dpad, hs, ls,
                       reinterpret_cast<uint32_t *>(X));
    PF_HIP(hipGetLastError());
}

// Largest |x_i| over every row, into *gmax as FP32 bits (which order like the values for
// x >= 0; *gmax starts at 0): one atomic per wave.
__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ X, int64_t total, uint32_t *gmax) {
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        m = fmaxf(m, fabsf(X[i]));
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(gmax, __float_as_uint(m));
}

// 8-bit row summaries for the re-rank's first bound: an FP32 scale s, the int32 A =
// sum_i |c_i| (the 8-byte header) and the int8 c_i = rint(x_i / s), i < dpad.  Row r of
// out (rq bytes, a multiple of 128) holds the codes from byte co on, zero padded.  When
// the header fits in front of the codes without another 128-byte line (co = 8) it is the
// row's first 8 bytes and s = max_i |x_i| / 127 of the row; otherwise (co = 0) every row
// takes the same s = G / 127, G the largest |x_i| of all rows (gmax[0]), gmax[1] receives
// the largest A of any row, so that a bound needs no per-row header read, and the headers
// go to row r of hdr for the export only.  With the FP32 divisions correctly rounded,
// |x_i / s| <= 127 (1 + 2^-24), so |c_i| <= 127 and |x_i - s c_i| <= s (1/2 + 2^-16).
// One 64-lane wave per row, the waves striding over the rows; a wave folds its rows' sums
// into one register and makes one atomic update of gmax[1] at its end.
__global__ __launch_bounds__(256) void k_rows8(const float *__restrict__ X, int64_t n, int32_t dpad, int32_t rq,
                                               int32_t co, uint32_t *__restrict__ gmax,
                                               uint8_t *__restrict__ out, uint8_t *__restrict__ hdr) {
    const int lane = threadIdx.x & 63;
    const float gsc = co ? 0.0f : __uint_as_float(*gmax) / 127.0f;
    int32_t amax = 0;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4) {
        const float *x = X + r * dpad;
        float sc = gsc;
        if (co) {
            float mx = 0.0f;
            for (int c = lane; c < dpad; c += 64) mx = fmaxf(mx, fabsf(x[c]));
            for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
            sc = mx / 127.0f;
        }
        uint8_t *row = out + r * (int64_t)rq;
        int32_t asum = 0;
        for (int c = lane; c < rq - co; c += 64) {
            int32_t q = 0;
            if (c < dpad && sc > 0.0f) {
                const float v = rintf(x[c] / sc);
                q = (int32_t)fminf(127.0f, fmaxf(-127.0f, v));
            }
            row[co + c] = (uint8_t)(int8_t)q;
            asum += q < 0 ? -q : q;
        }
        for (int o = 32; o >= 1; o >>= 1) asum += __shfl_xor(asum, o);
        if (lane == 0) {
            uint8_t *h = co ? row : hdr + r * 8;
            *reinterpret_cast<float *>(h) = sc;
            *reinterpret_cast<int32_t *>(h + 4) = asum;
        }
        amax = max(amax, asum);
    }
    if (!co && lane == 0) atomicMax(gmax + 1, (uint32_t)amax);
}

void rows8_layout(int32_t dpad, int32_t *rq, int32_t *co) {
    const int32_t lines = (dpad + 127) / 128 * 128;
    *co = 8 + dpad <= lines ? 8 : 0;
    *rq = (*co + dpad + 127) / 128 * 128;
}

void launch_rows8(const float *X, int64_t n, int32_t dpad, uint8_t *out, uint8_t *hdr, uint32_t *gmax,
                  hipStream_t s) {
    if (n <= 0) return;
    int32_t rq, co;
    rows8_layout(dpad, &rq, &co);
    if (co == 0) {
        launch_fill_u32(gmax, 2, 0u, s);
        const int64_t total = n * (int64_t)dpad;
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, s, X, total, gmax);
        PF_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_rows8, dim3((unsigned)std::min<int64_t>((n + 3) / 4, 16384)), dim3(256), 0, s, X, n, dpad, rq, co,
                       gmax, out, hdr);
    PF_HIP(hipGetLastError());
}

// Read-only streaming kernel (a measurement aid, not part of the method): every lane reads
// 16-byte words, four in flight, grid-stride over the buffer, and folds them into one
// word that is stored only if it equals a constant, so the loads cannot be removed.  NT:
// non-temporal loads (streamed past the caches).  Its rate is the read bandwidth a plain
// streaming access pattern reaches on the device.
template <bool NT>
__global__ __launch_bounds__(256) void k_read_stream(const uint4 *__restrict__ p, int64_t n16,
                                                     uint32_t *__restrict__ sink) {
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const v4u *q = reinterpret_cast<const v4u *>(p);
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        v4u v[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) v[f] = NT ? __builtin_nontemporal_load(q + i + f * stride) : q[i + f * stride];
#pragma unroll
        for (int f = 0; f < 4; ++f) acc ^= v[f].x ^ v[f].y ^ v[f].z ^ v[f].w;
    }
    for (; i < n16; i += stride) {
        const v4u v = q[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9E3779B9u) sink[threadIdx.x] = acc;
}

double read_bandwidth_gbs(uint64_t bytes, int32_t reps, int32_t num_cus, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    DevBuf buf, sink;
    buf.alloc((size_t)n16 * 16);
    sink.alloc(256 * sizeof(uint32_t));
    launch_fill_u32(buf.as<uint32_t>(), n16 * 4, 0x01020304u, s);
    hipEvent_t e0, e1;
    PF_HIP(hipEventCreate(&e0));
    PF_HIP(hipEventCreate(&e1));
    float best = 0.0f;
    // the best of plain and non-temporal loads at 2, 8 and 32 workgroups per CU
    for (int nt = 0; nt < 2; ++nt)
        for (int per_cu : {2, 8, 32}) {
            const unsigned blocks = (unsigned)std::max(1, num_cus) * (unsigned)per_cu;
            for (int32_t r = 0; r <= reps; ++r) { // launch 0 warms up
                PF_HIP(hipEventRecord(e0, s));
                if (nt)
                    hipLaunchKernelGGL(k_read_stream<true>, dim3(blocks), dim3(256), 0, s, buf.as<const uint4>(), n16,
                                       sink.as<uint32_t>());
                else
                    hipLaunchKernelGGL(k_read_stream<false>, dim3(blocks), dim3(256), 0, s, buf.as<const uint4>(),
                                       n16, sink.as<uint32_t>());
                PF_HIP(hipGetLastError());
                PF_HIP(hipEventRecord(e1, s));
                PF_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                PF_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (r > 0 && (best == 0.0f || ms < best)) best = ms;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)n16 * 16.0 / ((double)best * 1e-3) / 1e9;
}

// Random-read kernel (a measurement aid, not part of the method): every lane issues R
// 4-byte loads, eight in flight, at word indices drawn from SplitMix64 of (seed, lane,
// load) and masked to the buffer's power-of-two word count, so every load is in bounds
// and hits a line no neighbouring lane reads.  NT: non-temporal loads.  Its rate, against
// the streaming read rate, gives the memory traffic one scattered 4-byte read costs.
__device__ __forceinline__ uint64_t probe_mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
template <bool NT>
__global__ __launch_bounds__(256) void k_read_random(const uint32_t *__restrict__ p, uint64_t mask, int32_t R,
                                                     uint64_t seed, uint32_t *__restrict__ sink) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t acc = 0;
    for (int32_t r = 0; r < R; r += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint64_t i = probe_mix(seed ^ ((t << 20) + (uint64_t)(r + u))) & mask;
            v[u] = NT ? __builtin_nontemporal_load(p + i) : p[i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    if (acc == 0x9E3779B9u) sink[threadIdx.x] = acc;
}

double random_read_rate(uint64_t bytes, int32_t reps, int32_t num_cus, hipStream_t s) {
    uint64_t words = 1;
    while (words * 2 <= bytes / 4) words *= 2;
    constexpr int32_t R = 64;
    const unsigned blocks = (unsigned)std::max(1, num_cus) * 64u;
    DevBuf buf, sink;
    buf.alloc((size_t)words * 4);
    sink.alloc(256 * sizeof(uint32_t));
    launch_fill_u32(buf.as<uint32_t>(), (int64_t)words, 0x01020304u, s);
    hipEvent_t e0, e1;
    PF_HIP(hipEventCreate(&e0));
    PF_HIP(hipEventCreate(&e1));
    float best = 0.0f;
    for (int nt = 0; nt < 2; ++nt)
        for (int32_t r = 0; r <= reps; ++r) { // launch 0 warms up
            PF_HIP(hipEventRecord(e0, s));
            if (nt)
                hipLaunchKernelGGL(k_read_random<true>, dim3(blocks), dim3(256), 0, s, buf.as<const uint32_t>(),
                                   words - 1, R, (uint64_t)(2 * r + nt), sink.as<uint32_t>());
            else
                hipLaunchKernelGGL(k_read_random<false>, dim3(blocks), dim3(256), 0, s, buf.as<const uint32_t>(),
                                   words - 1, R, (uint64_t)(2 * r + nt), sink.as<uint32_t>());
            PF_HIP(hipGetLastError());
            PF_HIP(hipEventRecord(e1, s));
            PF_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            PF_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0 && (best == 0.0f || ms < best)) best = ms;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)blocks * 256.0 * R / ((double)best * 1e-3);
}


} // namespace pf
