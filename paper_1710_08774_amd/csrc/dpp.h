// Whole-wave lane shifts by one lane through DPP (wave_shr:1 / wave_shl:1):
// the inner rotation of a window along the lane axis without LDS.  Every
// lane of the wave must be active; the lane shifted in at the wave edge
// receives 0.
#pragma once
#include <hip/hip_runtime.h>

namespace hfav {

__device__ __forceinline__ int dpp_from_left(int v) {      // value of lane l - 1
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_from_right(int v) {     // value of lane l + 1
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
}
template <bool LEFT>
__device__ __forceinline__ double lane_shift(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    const int rlo = LEFT ? dpp_from_left(lo) : dpp_from_right(lo);
    const int rhi = LEFT ? dpp_from_left(hi) : dpp_from_right(hi);
    return __longlong_as_double(((long long)rhi << 32) | (unsigned int)rlo);
}
template <bool LEFT>
__device__ __forceinline__ float lane_shift(float v) {
    const int b = __float_as_int(v);
    return __int_as_float(LEFT ? dpp_from_left(b) : dpp_from_right(b));
}

}  // namespace hfav
