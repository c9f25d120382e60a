// Streaming-bandwidth probes: plain device copies moving the bytes of a
// fused chain, flat or in the tile-and-segment order of the streaming
// stencil kernels, timed beside the chains as the practical ceiling.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/hfav.h"
#include "../../include/hfav_probe.h"
#include "internal.h"

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void copy_flat_kernel(const u32x4 *src, u32x4 *dst, int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

struct SegArgs {
    const char *src;
    char *dst;
    int64_t slab, row, slabs;
    int band, tile_rows, seg;
    int nv;          // accesses per band
    int tiles_x;     // tiles across a row
    int ntiles;      // tiles per slab
};

// One workgroup: one tile through `seg` slabs.  Each lane takes the tile's
// accesses t = lane, lane + 256, ... and moves 4 slabs of each at a time.
template <class V>
__global__ __launch_bounds__(256) void copy_seg_kernel(SegArgs a) {
    const int tile = blockIdx.x % a.ntiles, sg = blockIdx.x / a.ntiles;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int64_t base = (int64_t)tx * a.band + (int64_t)ty * a.tile_rows * a.row;
    const int per = a.tile_rows * a.nv;
    const int64_t s0 = (int64_t)sg * a.seg;
    const int64_t s1 = s0 + a.seg < a.slabs ? s0 + a.seg : a.slabs;
    int64_t s = s0;
    for (; s + 4 <= s1; s += 4) {
        for (int t = threadIdx.x; t < per; t += 256) {
            const int r = t / a.nv, c = t - r * a.nv;
            const int64_t off = s * a.slab + base + (int64_t)r * a.row + (int64_t)c * (int64_t)sizeof(V);
            const V v0 = *(const V *)(a.src + off);
            const V v1 = *(const V *)(a.src + off + a.slab);
            const V v2 = *(const V *)(a.src + off + 2 * a.slab);
            const V v3 = *(const V *)(a.src + off + 3 * a.slab);
            *(V *)(a.dst + off) = v0;
            *(V *)(a.dst + off + a.slab) = v1;
            *(V *)(a.dst + off + 2 * a.slab) = v2;
            *(V *)(a.dst + off + 3 * a.slab) = v3;
        }
    }
    for (; s < s1; ++s)
        for (int t = threadIdx.x; t < per; t += 256) {
            const int r = t / a.nv, c = t - r * a.nv;
            const int64_t off = s * a.slab + base + (int64_t)r * a.row + (int64_t)c * (int64_t)sizeof(V);
            *(V *)(a.dst + off) = *(const V *)(a.src + off);
        }
}

}  // namespace

extern "C" int hfav_copy_probe(const hfav_copy_desc *d, const void *src, void *dst, void *stream) {
    if (!d || !src || !dst) return hfav_fail(HFAV_EINVAL, "hfav_copy_probe: null argument");
    hipStream_t s = (hipStream_t)stream;
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return hfav_fail(HFAV_EINVAL, "hfav_copy_probe: unaligned buffer");
    if (d->pattern == HFAV_COPY_FLAT) {
        if (d->bytes <= 0 || d->bytes % 16) return hfav_fail(HFAV_EINVAL, "hfav_copy_probe: bytes");
        const int64_t n16 = d->bytes / 16, nb = (n16 + 255) / 256;
        if (nb > INT32_MAX) return hfav_fail(HFAV_EINVAL, "hfav_copy_probe: too large");
        hipLaunchKernelGGL(copy_flat_kernel, dim3((unsigned)nb), dim3(256), 0, s, (const u32x4 *)src, (u32x4 *)dst,
                           n16);
    } else if (d->pattern == HFAV_COPY_SEGMENTS) {
        const int ab = d->access_bytes;
        if ((ab != 4 && ab != 8 && ab != 16) || d->band_bytes <= 0 || d->band_bytes % ab || d->row_bytes <= 0 ||
            d->row_bytes % d->band_bytes || d->slab_bytes <= 0 || d->slab_bytes % d->row_bytes || d->tile_rows <= 0 ||
            (d->slab_bytes / d->row_bytes) % d->tile_rows || d->slabs <= 0 || d->seg <= 0)
            return hfav_fail(HFAV_EINVAL, "hfav_copy_probe: inconsistent segment geometry");
        SegArgs a;
        a.src = (const char *)src;
        a.dst = (char *)dst;
        a.slab = d->slab_bytes;
        a.row = d->row_bytes;
        a.slabs = d->slabs;
        a.band = d->band_bytes;
        a.tile_rows = d->tile_rows;
        a.seg = d->seg;
        a.nv = d->band_bytes / ab;
        const int64_t tiles_x = d->row_bytes / d->band_bytes;
        const int64_t tiles = tiles_x * (d->slab_bytes / d->row_bytes / d->tile_rows);
        const int64_t nb = tiles * ((d->slabs + d->seg - 1) / d->seg);
        if (nb > INT32_MAX || tiles > INT32_MAX) return hfav_fail(HFAV_EINVAL, "hfav_copy_probe: too many tiles");
        a.tiles_x = (int)tiles_x;
        a.ntiles = (int)tiles;
        if (ab == 4) hipLaunchKernelGGL(copy_seg_kernel<unsigned int>, dim3((unsigned)nb), dim3(256), 0, s, a);
        else if (ab == 8) hipLaunchKernelGGL(copy_seg_kernel<u32x2>, dim3((unsigned)nb), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(copy_seg_kernel<u32x4>, dim3((unsigned)nb), dim3(256), 0, s, a);
    } else {
        return hfav_fail(HFAV_EINVAL, "hfav_copy_probe: unknown pattern");
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hfav_fail(HFAV_EDEVICE, std::string("hfav_copy_probe: ") + hipGetErrorString(e));
    return HFAV_OK;
}
