// Kernels of the learned scheduler: per-query features and a 98-128-128-2 FP32 MLP
// (forward, mean-squared-error gradient, backward, Adam).  The network only orders the
// batched search's work queue; the stopping rule alone decides when a query ends.
#include "pf_device.h"
#include "pf_internal.h"

namespace pf {

// Features of query q (98 FP32): the 64 bits of its sketch 0 as +1 / -1, then
// log2(1 + size of the query's F-bit prefix bucket, F = min(13, K)) in tables 0..31 (0
// when L < 32; read from the P-bit prefix table, P >= F),
// then the query's log2 k and log2(1/delta) (qparam, computed on the host).
__global__ __launch_bounds__(256) void k_features(const uint32_t *__restrict__ qcode,
                                                  const uint64_t *__restrict__ qsk,
                                                  const uint32_t *__restrict__ off, int64_t m, int32_t L,
                                                  int32_t K, int32_t P, const float *__restrict__ qparam,
                                                  float *__restrict__ feat) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * kSchedIn) return;
    const int64_t q = t / kSchedIn;
    const int f = (int)(t - q * kSchedIn);
    float v = 0.0f;
    if (f < 64) {
        v = ((qsk[q] >> f) & 1ull) ? 1.0f : -1.0f; // sketch 0 is the first M x m row block
    } else if (f >= 96) {
        v = qparam[2 * q + (f - 96)];
    } else {
        const int j = f - 64;
        if (j < L) {
            const int64_t np1 = ((int64_t)1 << P) + 1;
            const int32_t F = min(13, K);
            const uint32_t b = qcode[(int64_t)j * m + q] >> (K - F);
            const uint32_t *oj = off + (int64_t)j * np1;
            const uint32_t sz = oj[(int64_t)(b + 1) << (P - F)] - oj[(int64_t)b << (P - F)];
            v = log2f(1.0f + (float)sz);
        }
    }
    feat[t] = v;
}

// dy = d(loss)/dy for loss = mean over the B x 2 outputs of (y - target)^2; loss summed
// into *acc (FP64) in one fixed order by a single wave
__global__ __launch_bounds__(64) void k_mse(const float *__restrict__ y, const float *__restrict__ tgt,
                                            const int32_t *__restrict__ rows, int64_t B, float *__restrict__ dy,
                                            double *acc) {
    const int lane = threadIdx.x;
    const double inv = 1.0 / (double)(B * kSchedOut);
    double part = 0.0;
    for (int64_t t = lane; t < B * kSchedOut; t += 64) {
        const int64_t r = t / kSchedOut;
        const int c = (int)(t - r * kSchedOut);
        const float e = y[t] - tgt[(rows ? (int64_t)rows[r] : r) * kSchedOut + c];
        dy[t] = (float)(2.0 * inv) * e;
        part += (double)e * (double)e;
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) *acc += part * inv;
}

// din[r][i] = (sum_o dout[r][o] W[i][o]) * [h[r][i] > 0]   (h: the layer input, post-ReLU)
__global__ __launch_bounds__(256) void k_dense_bwd_in(const float *__restrict__ dout, const float *__restrict__ W,
                                                      const float *__restrict__ h, int32_t nin, int32_t nout,
                                                      int64_t B, float *__restrict__ din) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * nin) return;
    const int64_t r = t / nin;
    const int i = (int)(t - r * nin);
    float s = 0.0f;
    const float *g = dout + r * nout;
    const float *w = W + (int64_t)i * nout;
    for (int o = 0; o < nout; ++o) s = s + g[o] * w[o];
    din[t] = h[t] > 0.0f ? s : 0.0f;
}

// Weight gradient of a dense layer, dW[i][o] = sum_r in[row(r)][i] dout[r][o] and db[o] =
// sum_r dout[r][o], in two deterministic stages.  Workgroup (x, y, c) takes the 32 x 32 tile
// i0 = 32x, o0 = 32y over the rows of chunk c (rows c cr .. min(B, (c + 1) cr) - 1), staging 64
// rows of both operands at a time in LDS and adding them in row order (lane t: input i0 + t / 8,
// outputs o0 + 4 (t % 8) .. + 3; the y = 0 workgroups also sum the bias columns); the chunks'
// partial sums are then added in chunk order.
constexpr int kWgTile = 32, kWgRows = 64;
__global__ __launch_bounds__(256) void k_dense_wgrad_part(const float *__restrict__ in,
                                                          const int32_t *__restrict__ rows,
                                                          const float *__restrict__ dout, int32_t nin, int32_t nout,
                                                          int64_t B, int64_t cr, float *__restrict__ part,
                                                          float *__restrict__ partb) {
    __shared__ float s_in[kWgRows][kWgTile + 1];
    __shared__ float s_out[kWgRows][kWgTile + 1];
    const int t = threadIdx.x;
    const int i0 = (int)blockIdx.x * kWgTile, o0 = (int)blockIdx.y * kWgTile;
    const int64_t c = blockIdx.z, r0 = c * cr, r1 = min(B, r0 + cr);
    const int ii = t >> 3, oq = (t & 7) * 4;
    const bool bias = blockIdx.x == 0 && t < kWgTile;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (int64_t rb = r0; rb < r1; rb += kWgRows) {
        const int rn = (int)min((int64_t)kWgRows, r1 - rb);
        for (int e = t; e < kWgRows * kWgTile; e += 256) {
            const int r = e / kWgTile, cc = e % kWgTile;
            float a = 0.0f, b = 0.0f;
            if (r < rn) {
                const int64_t src = rows ? (int64_t)rows[rb + r] : rb + r;
                if (i0 + cc < nin) a = in[src * nin + i0 + cc];
                if (o0 + cc < nout) b = dout[(rb + r) * nout + o0 + cc];
            }
            s_in[r][cc] = a;
            s_out[r][cc] = b;
        }
        __syncthreads();
        for (int r = 0; r < rn; ++r) {
            const float a = s_in[r][ii];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = acc[u] + a * s_out[r][oq + u];
        }
        if (bias)
            for (int r = 0; r < rn; ++r) bsum = bsum + s_out[r][t];
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + ii, o = o0 + oq + u;
        if (i < nin && o < nout) part[(c * nin + i) * nout + o] = acc[u];
    }
    if (bias && o0 + t < nout) partb[c * nout + o0 + t] = bsum;
}

__global__ __launch_bounds__(256) void k_dense_wgrad_sum(const float *__restrict__ part,
                                                         const float *__restrict__ partb, int32_t nin, int32_t nout,
                                                         int32_t nc, float *__restrict__ dW, float *__restrict__ db) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nw = (int64_t)nin * nout;
    if (t < nw) {
        float s = 0.0f;
        for (int32_t c = 0; c < nc; ++c) s = s + part[c * nw + t];
        dW[t] = s;
    } else if (t < nw + nout) {
        const int64_t o = t - nw;
        float s = 0.0f;
        for (int32_t c = 0; c < nc; ++c) s = s + partb[c * nout + o];
        db[o] = s;
    }
}

static void dense_wgrad(const float *in, const int32_t *rows, const float *dout, int32_t nin, int32_t nout,
                        int64_t B, float *dW, float *db, float *scratch, hipStream_t s) {
    const int64_t nc = std::min<int64_t>(kWgradChunks, (B + 127) / 128);
    const int64_t cr = (B + nc - 1) / nc;
    float *part = scratch, *partb = scratch + nc * nin * nout;
    const dim3 grid((unsigned)((nin + kWgTile - 1) / kWgTile), (unsigned)((nout + kWgTile - 1) / kWgTile),
                    (unsigned)nc);
    hipLaunchKernelGGL(k_dense_wgrad_part, grid, dim3(256), 0, s, in, rows, dout, nin, nout, B, cr, part, partb);
    const int64_t n = (int64_t)nin * nout + nout;
    hipLaunchKernelGGL(k_dense_wgrad_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float *)part,
                       (const float *)partb, nin, nout, (int32_t)nc, dW, db);
}

// Adam (Kingma, Ba 2015) with bias correction, step t >= 1
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m1, float *__restrict__ m2, int64_t count,
                                              float lr, float b1, float b2, float eps, int32_t t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float ah = a / (1.0f - powf(b1, (float)t));
    const float vh = v / (1.0f - powf(b2, (float)t));
    p[i] = p[i] - lr * ah / (sqrtf(vh) + eps);
}

static unsigned grid_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// The whole forward pass for kFwdRows rows per workgroup: the rows, h1 and h2 stay in LDS
// and every output out[r][o] = act(sum_i in[r][i] W[i][o] + b[o]) is summed in one fixed
// order (i ascending, FP32, then the bias).  Thread t owns column t % 128 of rows t / 128,
// t / 128 + 2, ...
constexpr int kFwdRows = 32;
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ x, const int32_t *__restrict__ rows,
                                                     const float *__restrict__ params, int64_t B,
                                                     float *__restrict__ h1, float *__restrict__ h2,
                                                     float *__restrict__ y) {
    __shared__ float sx[kFwdRows * kSchedIn];
    __shared__ float sh1[kFwdRows * kSchedHidden];
    __shared__ float sh2[kFwdRows * kSchedHidden];
    const float *W1 = params + kOffW1, *b1 = params + kOffB1, *W2 = params + kOffW2, *b2 = params + kOffB2,
                *W3 = params + kOffW3, *b3 = params + kOffB3;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kFwdRows;
    const int nr = (int)min((int64_t)kFwdRows, B - r0);
    for (int t = tid; t < nr * kSchedIn; t += 256) {
        const int r = t / kSchedIn, i = t - r * kSchedIn;
        sx[t] = x[(rows ? (int64_t)rows[r0 + r] : r0 + r) * kSchedIn + i];
    }
    __syncthreads();
    constexpr int kPer = kFwdRows * kSchedHidden / 256; // rows per thread
    const int o = tid % kSchedHidden, rb = tid / kSchedHidden;
    float acc[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) acc[j] = 0.0f;
    for (int i = 0; i < kSchedIn; ++i) {
        const float w = W1[i * kSchedHidden + o];
#pragma unroll
        for (int j = 0; j < kPer; ++j) acc[j] = acc[j] + sx[(rb + 2 * j) * kSchedIn + i] * w;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int r = rb + 2 * j;
        float v = acc[j] + b1[o];
        v = v < 0.0f ? 0.0f : v;
        sh1[r * kSchedHidden + o] = v;
        if (r < nr) h1[(r0 + r) * kSchedHidden + o] = v;
        acc[j] = 0.0f;
    }
    __syncthreads();
    for (int i = 0; i < kSchedHidden; ++i) {
        const float w = W2[i * kSchedHidden + o];
#pragma unroll
        for (int j = 0; j < kPer; ++j) acc[j] = acc[j] + sh1[(rb + 2 * j) * kSchedHidden + i] * w;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int r = rb + 2 * j;
        float v = acc[j] + b2[o];
        v = v < 0.0f ? 0.0f : v;
        sh2[r * kSchedHidden + o] = v;
        if (r < nr) h2[(r0 + r) * kSchedHidden + o] = v;
    }
    __syncthreads();
    if (tid < nr * kSchedOut) {
        const int r = tid / kSchedOut, oo = tid - r * kSchedOut;
        float v = 0.0f;
        for (int i = 0; i < kSchedHidden; ++i) v = v + sh2[r * kSchedHidden + i] * W3[i * kSchedOut + oo];
        y[(r0 + r) * kSchedOut + oo] = v + b3[oo];
    }
}

void launch_features(const Index &ix, const uint32_t *qcode, const uint64_t *qsk, int64_t m,
                     const float *qparam, float *feat, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_features, dim3(grid_for(m * kSchedIn)), dim3(256), 0, s, qcode, qsk, ix.off.as<uint32_t>(),
                       m, ix.L, ix.K, ix.P, qparam, feat);
    PF_HIP(hipGetLastError());
}

void mlp_forward(const float *params, const float *x, const int32_t *rows, int64_t B, float *h1, float *h2,
                 float *y, hipStream_t s) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((B + kFwdRows - 1) / kFwdRows)), dim3(256), 0, s, x, rows,
                       params, B, h1, h2, y);
    PF_HIP(hipGetLastError());
}

void mlp_backward(const float *params, const float *x, const int32_t *rows, const float *tgt, int64_t B,
                  const float *h1, const float *h2, const float *y, float *dy, float *dh2, float *dh1, float *grad,
                  double *loss_acc, float *wscratch, hipStream_t s) {
    const float *W2 = params + kOffW2, *W3 = params + kOffW3;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(64), 0, s, y, tgt, rows, B, dy, loss_acc);
    dense_wgrad(h2, nullptr, dy, kSchedHidden, kSchedOut, B, grad + kOffW3, grad + kOffB3, wscratch, s);
    hipLaunchKernelGGL(k_dense_bwd_in, dim3(grid_for(B * kSchedHidden)), dim3(256), 0, s, (const float *)dy, W3, h2,
                       kSchedHidden, kSchedOut, B, dh2);
    dense_wgrad(h1, nullptr, dh2, kSchedHidden, kSchedHidden, B, grad + kOffW2, grad + kOffB2, wscratch, s);
    hipLaunchKernelGGL(k_dense_bwd_in, dim3(grid_for(B * kSchedHidden)), dim3(256), 0, s, (const float *)dh2, W2,
                       h1, kSchedHidden, kSchedHidden, B, dh1);
    dense_wgrad(x, rows, dh1, kSchedIn, kSchedHidden, B, grad + kOffW1, grad + kOffB1, wscratch, s);
    PF_HIP(hipGetLastError());
}

// Sort keys of the longest-predicted-first order: ascending unsigned keys = descending
// predicted cost (column 1 of y, B x 2); the map is monotone on the FP32 total order, and
// a NaN prediction sorts last.
__global__ __launch_bounds__(256) void k_lpt_keys(const float *__restrict__ y, int64_t B,
                                                  uint32_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float v = y[i * 2 + 1];
    keys[i] = isnan(v) ? 0xFFFFFFFFu : ~ord_of(v);
}

void launch_lpt_keys(const float *y, int64_t B, uint32_t *keys, hipStream_t s) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_lpt_keys, dim3(grid_for(B)), dim3(256), 0, s, y, B, keys);
    PF_HIP(hipGetLastError());
}

void mlp_adam(float *params, const float *grad, float *m1, float *m2, float lr, int32_t t, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(kSchedParams)), dim3(256), 0, s, params, grad, m1, m2,
                       (int64_t)kSchedParams, lr, 0.9f, 0.999f, 1e-8f, t);
    PF_HIP(hipGetLastError());
}

} // namespace pf
