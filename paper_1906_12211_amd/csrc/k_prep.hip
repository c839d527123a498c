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

// Vector storage as two 16-bit planes: hi[i] = upper half of the FP32 bit pattern of
// X[i] (X[i] truncated to bfloat16), lo[i] = lower half; (hi << 16) | lo is X[i] exactly.
__global__ __launch_bounds__(256) void k_split_planes(const uint32_t *__restrict__ X, int64_t count,
                                                      uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) {
        const uint32_t v = X[t];
        hi[t] = (uint16_t)(v >> 16);
        lo[t] = (uint16_t)(v & 0xFFFFu);
    }
}

__global__ __launch_bounds__(256) void k_join_planes(const uint16_t *__restrict__ hi, const uint16_t *__restrict__ lo,
                                                     int64_t count, uint32_t *__restrict__ X) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride)
        X[t] = ((uint32_t)hi[t] << 16) | (uint32_t)lo[t];
}

void launch_split_planes(const float *X, int64_t count, uint16_t *hi, uint16_t *lo, hipStream_t s) {
    if (count <= 0) return;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_split_planes, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const uint32_t *>(X), count, hi, lo);
    PF_HIP(hipGetLastError());
}

void launch_join_planes(const uint16_t *hi, const uint16_t *lo, int64_t count, float *X, hipStream_t s) {
    if (count <= 0) return;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_join_planes, dim3((unsigned)blocks), dim3(256), 0, s, hi, lo, count,
                       reinterpret_cast<uint32_t *>(X));
    PF_HIP(hipGetLastError());
}

} // namespace pf
