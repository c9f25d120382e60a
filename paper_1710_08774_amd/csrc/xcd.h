// XCD-aware workgroup order.  An MI355X dispatches consecutive workgroup ids
// round-robin over its 8 XCDs, each with its own L2.  Remapping the id so
// that every XCD receives a contiguous range of logical tiles puts tiles
// that share halo cache lines on the same L2 at about the same time.
#pragma once
#include <hip/hip_runtime.h>

namespace hfav {

constexpr int kNumXcd = 8;

// Bijection of [0, n): workgroup w (on XCD w % 8) -> logical tile id.
//   g == 0: identity (hardware order);
//   g > 0 : each group of 8g workgroups gives every XCD g consecutive tiles
//           (a tail shorter than 8g keeps the identity);
//   g < 0 : every XCD gets one contiguous range of about n/8 tiles.
__device__ __forceinline__ int xcd_tile(int w, int n, int g) {
    if (g == 0) return w;
    const int k = w % kNumXcd;
    if (g < 0) {
        const int q = n / kNumXcd, r = n % kNumXcd, idx = w / kNumXcd;
        return k * q + (k < r ? k : r) + idx;
    }
    const int span = kNumXcd * g;
    if (w >= (n / span) * span) return w;
    const int base = w - w % span, idx = (w % span) / kNumXcd;
    return base + k * g + idx;
}

}  // namespace hfav
