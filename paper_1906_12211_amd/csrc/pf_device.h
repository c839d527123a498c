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

// integer sum over the 16 lanes of a DPP row, in every lane of the row (every lane of
// the row must be active)
template <int CTRL> __device__ __forceinline__ uint32_t dpp_u(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t row_sum16u(uint32_t s) {
    s += dpp_u<0x128>(s); // row_ror:8
    s += dpp_u<0x124>(s); // row_ror:4
    s += dpp_u<0x122>(s); // row_ror:2
    s += dpp_u<0x121>(s); // row_ror:1
    return s;
}

// sum over the 8 lanes of each half of a DPP row (every lane of the half gets it)
__device__ __forceinline__ uint32_t half_row_sum8u(uint32_t s) {
    s += dpp_u<0xB1>(s);  // quad_perm [1, 0, 3, 2]
    s += dpp_u<0x4E>(s);  // quad_perm [2, 3, 0, 1]
    s += dpp_u<0x141>(s); // row_half_mirror
    return s;
}

// table position g of a positions array stored in PB bytes each (4, or 3 little endian;
// a 3-byte array carries 8 bytes of padding so that the word after any entry's last byte
// can be read)
template <int PB> __device__ __forceinline__ uint32_t read_pos(const void *__restrict__ pos, uint32_t g) {
    if constexpr (PB == 4) {
        return static_cast<const uint32_t *>(pos)[g];
    } else {
        static_assert(PB == 3, "positions are stored in 3 or 4 bytes");
        const uint64_t b = 3ull * g;
        const uint32_t *w = static_cast<const uint32_t *>(pos) + (b >> 2);
        const uint64_t two = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        return (uint32_t)(two >> (8 * (b & 3))) & 0xFFFFFFu;
    }
}

} // namespace pf
