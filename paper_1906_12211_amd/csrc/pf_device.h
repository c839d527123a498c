// Device helpers shared by the search kernel and the decision-table kernel (HIP sources
// only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pf {

// columns of a decision-table row: filter threshold T = -1..64
constexpr int kTauCols = 66;

// FP32 values as unsigned keys in the same total order (and back)
__device__ __forceinline__ uint32_t ord_of(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_of(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

} // namespace pf
