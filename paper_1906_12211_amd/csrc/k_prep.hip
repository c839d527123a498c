// Vector storage (Sec. 4.2 "Vector storage"): every data and query vector is stored at
// unit length.  The squared norm is an FP64 sum in index order, the square root and the
// quotient are FP64 (IEEE, correctly rounded on gfx950), and each quotient is rounded
// once to FP32.  Rows are written with a padded stride (a multiple of 4 floats, zero
// filled) so that the re-rank kernel can use 16-byte loads.
#include "pf_internal.h"

namespace pf {

__global__ __launch_bounds__(256) void k_normalize(const float *__restrict__ x, int64_t n, int32_t d,
                                                   int32_t ld_in, float *__restrict__ out,
                                                   int32_t dpad, unsigned long long *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *row = x + i * (int64_t)ld_in;
    double s = 0.0;
    for (int32_t c = 0; c < d; ++c) {
        const double v = (double)row[c];
        s = s + v * v;
    }
    const double nrm = sqrt(s);
    float *o = out + i * (int64_t)dpad;
    if (!(nrm > 0.0) || !isfinite(nrm)) {
        atomicMin(bad, (unsigned long long)i);
        for (int32_t c = 0; c < dpad; ++c) o[c] = 0.0f;
        return;
    }
    // x and out may alias (same stride): read the element before writing it
    for (int32_t c = 0; c < d; ++c) o[c] = (float)((double)row[c] / nrm);
    for (int32_t c = d; c < dpad; ++c) o[c] = 0.0f;
}

void launch_normalize(const float *x, int64_t n, int32_t d, int32_t ld_in, float *out, int32_t dpad,
                      unsigned long long *bad, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_normalize, dim3((unsigned)blocks), dim3(256), 0, s, x, n, d, ld_in, out,
                       dpad, bad);
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

} // namespace pf
