// Output stores of the bandwidth-bound kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace hfav {

// Store of a value written exactly once and not read again by this launch:
// NT selects the non-temporal (streaming) form.
template <bool NT, class T>
__device__ __forceinline__ void store_out(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

}  // namespace hfav
