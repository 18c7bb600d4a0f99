// Cross-lane moves inside a 64-lane wavefront that stay in the vector ALU
// (DPP and the gfx950 permlane swaps), for code that would otherwise send
// every permutation through the LDS crossbar (ds_bpermute / ds_swizzle).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jabba {

__device__ __forceinline__ uint32_t lane_index() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// value of lane (lane ^ M), M a power of two below 64
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "M: a power of two below 64");
    const int x = (int)v;
    if constexpr (M == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else if constexpr (M == 4) {
        const int up = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xF, 0xF, false);  // row_shl:4, lane + 4
        const int dn = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4, lane - 4
        return (uint32_t)((lane_index() & 4u) ? dn : up);
    } else if constexpr (M == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (M == 16) {
        // odd rows of the first operand swap with even rows of the second:
        // [0] holds rows (0, 0, 2, 2), [1] rows (1, 1, 3, 3)
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane_index() & 16u) ? r[0] : r[1];
    } else {
        // upper half of the first operand swaps with the lower half of the
        // second: [0] holds halves (0, 0), [1] halves (1, 1)
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane_index() & 32u) ? r[0] : r[1];
    }
}

template <int M>
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v) {
    const uint32_t lo = xor_lane<M>((uint32_t)v);
    const uint32_t hi = xor_lane<M>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <int M>
__device__ __forceinline__ double xor_lane_f64(double v) {
    return __longlong_as_double((long long)xor_lane_u64<M>((uint64_t)__double_as_longlong(v)));
}

// value of lane + 1; the last lane receives `last`
__device__ __forceinline__ uint32_t next_lane(uint32_t v, uint32_t last) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)last, (int)v, 0x130, 0xF, 0xF, false);  // wave_shl:1
}

// value of a lane selected by a DPP control within the rows in RowMask;
// lanes without a source (outside the row, or in a masked row) keep `old`
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_keep(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, Ctrl, RowMask, 0xF, false);
}

}  // namespace jabba
