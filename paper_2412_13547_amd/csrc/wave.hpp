// Wave64 cross-lane primitives for gfx950 built on DPP (data-parallel
// primitives: the cross-lane move is a modifier of an ordinary VALU
// instruction, no LDS round trip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tgs {

// DPP control codes (GCN / CDNA encoding)
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowRor8 = 0x128;   // rotate by 8 within each row of 16 lanes
constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2, 3, 0, 1]

// Inclusive prefix sum over the 64 lanes: Hillis-Steele within each row of
// 16 lanes (shifts 1, 2, 4, 8; lanes shifted in from outside the row add 0),
// then lane 15 of rows 0 and 2 is added to rows 1 and 3, and lane 31 to
// rows 2 and 3.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kDppRowShr1, 0xF, 0xF, false));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kDppRowShr2, 0xF, 0xF, false));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kDppRowShr4, 0xF, 0xF, false));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kDppRowShr8, 0xF, 0xF, false));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kDppRowBcast15, 0xA, 0xF, false));
    x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kDppRowBcast31, 0xC, 0xF, false));
    return x;
}

// Exclusive prefix sum; `total` receives the sum over all 64 lanes.
__device__ __forceinline__ uint32_t wave_exclusive_sum(uint32_t x, uint32_t& total) {
    const uint32_t incl = wave_inclusive_sum(x);
    total = uint32_t(__builtin_amdgcn_readlane(int(incl), 63));
    return incl - x;
}

__device__ __forceinline__ uint32_t wave_total(uint32_t x) {
    return uint32_t(__builtin_amdgcn_readlane(int(wave_inclusive_sum(x)), 63));
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << __lane_id()) - 1;
}

}  // namespace tgs
