// Fused horizontal-diffusion chain for gfx950 (Performance, "COSMO
// Micro-Kernels": ulapstage, flux_x, flux_y and ustage merged into one
// iteration nest; rolling windows of 3 rows for the Laplacian and 2 for the
// y flux, 2 elements for the x flux; Design, "Contraction").
//
// Mapping: a workgroup owns B consecutive columns of one k plane and streams
// down a segment of rows.  Each new input row is read from HBM once,
// coalesced, into a 4-row LDS ring with a 2-column halo (the "outer"
// rotation of rows); the Laplacian window (rows j and j+1, columns i-1..i+1)
// and the y-flux window (rows j-1 and j) live in registers, and the x flux at
// i-1 is recomputed by the lane from the same registers instead of being
// exchanged.  One barrier per row.
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "ops.h"

namespace hfav {

template <class T>
struct HArgs {
    const T *in;
    T *out;
    int ni, nj, nk, seg;
    T coeff;
};

__device__ __forceinline__ int pwrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <class T, int B>
__global__ __launch_bounds__(B) void hdiff_kernel(HArgs<T> a) {
    constexpr int W = B + 4;              // row slot: columns i0-2 .. i0+B+1
    __shared__ T ring[4][W];
    const int t = threadIdx.x;
    const int i0 = blockIdx.x * B;
    const int j0 = blockIdx.y * a.seg;
    const int j1 = min(j0 + a.seg, a.nj);
    const int k = blockIdx.z;
    const int ni = a.ni, nj = a.nj;
    const T *plane = a.in + (size_t)k * nj * ni;
    T *oplane = a.out + (size_t)k * nj * ni;
    // lane t keeps its own column (slot t+2); lanes 0..3 also fetch the
    // four halo columns (slots 0, 1, B+2, B+3)
    const int col = pwrap(i0 + t, ni);
    const int hs = t < 2 ? t : t + B;     // halo slot for lanes 0..3
    const int hcol = pwrap(i0 - 2 + hs, ni);

    auto load_row = [&](int j) {
        const T *r = plane + (size_t)pwrap(j, nj) * ni;
        T *s = ring[j & 3];
        s[t + 2] = r[col];
        if (t < 4) s[hs] = r[hcol];
    };
    auto L = [&](int j, int d) { return ring[j & 3][t + 2 + d]; };
    auto lap_at = [&](int j, int d) {
        return hdiff_lap(L(j, d), L(j, d + 1), L(j, d - 1), L(j + 1, d), L(j - 1, d));
    };

    // prologue: rows j0-2 .. j0+1, the Laplacian of rows j0-1 (centre) and
    // j0 (three columns), and the y flux of row j0-1
    load_row(j0 - 2);
    load_row(j0 - 1);
    load_row(j0);
    load_row(j0 + 1);
    __syncthreads();
    T lm1 = lap_at(j0 - 1, 0);
    T la = lap_at(j0, -1), lb = lap_at(j0, 0), lc = lap_at(j0, 1);
    T fym = hdiff_flux(lm1, lb, L(j0 - 1, 0), L(j0, 0));
    __syncthreads();

    for (int j = j0; j < j1; ++j) {
        load_row(j + 2);                    // overwrites row j-2's slot
        __syncthreads();
        // Laplacian of row j+1 at columns i-1, i, i+1
        const T na = lap_at(j + 1, -1), nb = lap_at(j + 1, 0), nc = lap_at(j + 1, 1);
        const T u = L(j, 0);
        const T fx0 = hdiff_flux(lb, lc, u, L(j, 1));
        const T fxm = hdiff_flux(la, lb, L(j, -1), u);
        const T fy0 = hdiff_flux(lb, nb, u, L(j + 1, 0));
        if (i0 + t < ni) oplane[(size_t)j * ni + i0 + t] = hdiff_out(u, fx0, fxm, fy0, fym, a.coeff);
        fym = fy0;
        la = na; lb = nb; lc = nc;
        // no second barrier: the next write goes to row j-1's slot, which no
        // lane still in this step reads, and a lane cannot run two rows ahead
        // of the post-load barrier
    }
}

template <class T>
static hipError_t hdiff_dispatch(const HdiffLaunch &L, hipStream_t s) {
    HArgs<T> a;
    a.in = (const T *)L.in;
    a.out = (T *)L.out;
    a.ni = L.ni; a.nj = L.nj; a.nk = L.nk;
    a.seg = L.cfg.seg > 0 ? L.cfg.seg : 32;
    a.coeff = (T)L.coeff;
    int B = L.cfg.block;
    if (B != 64 && B != 128 && B != 256 && B != 512) B = 256;
    dim3 grid((L.ni + B - 1) / B, (L.nj + a.seg - 1) / a.seg, L.nk);
    switch (B) {
    case 64: hipLaunchKernelGGL((hdiff_kernel<T, 64>), grid, dim3(64), 0, s, a); break;
    case 128: hipLaunchKernelGGL((hdiff_kernel<T, 128>), grid, dim3(128), 0, s, a); break;
    case 512: hipLaunchKernelGGL((hdiff_kernel<T, 512>), grid, dim3(512), 0, s, a); break;
    default: hipLaunchKernelGGL((hdiff_kernel<T, 256>), grid, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_hdiff(const HdiffLaunch &L, hipStream_t s) {
    return L.dtype == HFAV_F64 ? hdiff_dispatch<double>(L, s) : hdiff_dispatch<float>(L, s);
}

}  // namespace hfav
