// Fused 7-point Laplacian chain (lap1 = L7(u), lap2 = L7(lap1),
// out = u + alpha*lap2) for gfx950: the biharmonic update used for the
// precision study.  The 7-point Laplacian is the paper's example of a kernel
// that fuses without special handling (Design, "Reductions & broadcasts &
// splits").
//
// 2.5-D streaming: a workgroup owns a TX x TY tile of the x-y plane and walks
// a segment of z planes.  Each u plane (tile plus a 2-cell halo) is read from
// HBM once into a 4-plane LDS ring; the intermediate lap1 is contracted to a
// 2-plane LDS ring over the tile plus a 1-cell halo (the planes k and k+1 its
// consumer needs), and its centre value at plane k-1 stays in a register.
// Two barriers per plane.
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "ops.h"

namespace hfav {

template <class T>
struct BArgs {
    const T *in;
    T *out;
    int nx, ny, nz, seg;
    T alpha;
};

__device__ __forceinline__ int w3(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <class T, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void lap7_chain_kernel(BArgs<T> a) {
    constexpr int NT = TX * TY;
    constexpr int UX = TX + 4, UY = TY + 4;     // u tile with halo 2
    constexpr int LX = TX + 2, LY = TY + 2;     // lap1 tile with halo 1
    __shared__ T su[4][UY][UX];
    __shared__ T sl[2][LY][LX];
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int k0 = blockIdx.z * a.seg;
    const int k1 = min(k0 + a.seg, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t plane = (size_t)nx * ny;

    auto load_plane = [&](int k) {
        const T *p = a.in + (size_t)w3(k, nz) * plane;
        T(*s)[UX] = su[k & 3];
        for (int q = tid; q < UX * UY; q += NT) {
            const int qx = q % UX, qy = q / UX;
            s[qy][qx] = p[(size_t)w3(y0 - 2 + qy, ny) * nx + w3(x0 - 2 + qx, nx)];
        }
    };
    // lap1 at plane k for point (hx, hy) of the halo-1 frame
    auto lap1_at = [&](int k, int hx, int hy) {
        T(*c)[UX] = su[k & 3];
        const int ux = hx + 1, uy = hy + 1;
        return lap7(c[uy][ux], c[uy][ux + 1], c[uy][ux - 1], c[uy + 1][ux], c[uy - 1][ux],
                    su[(k + 1) & 3][uy][ux], su[(k - 1) & 3][uy][ux]);
    };
    auto lap1_plane = [&](int k) {
        T(*d)[LX] = sl[k & 1];
        for (int q = tid; q < LX * LY; q += NT) {
            const int hx = q % LX, hy = q / LX;
            d[hy][hx] = lap1_at(k, hx, hy);
        }
    };

    // prologue: u planes k0-2 .. k0+1; lap1 at k0-1 (own centre) and k0 (tile)
    load_plane(k0 - 2);
    load_plane(k0 - 1);
    load_plane(k0);
    load_plane(k0 + 1);
    __syncthreads();
    T lm = lap1_at(k0 - 1, tx + 1, ty + 1);
    lap1_plane(k0);
    __syncthreads();

    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < nx && gy < ny;
    for (int k = k0; k < k1; ++k) {
        load_plane(k + 2);                 // replaces plane k-2
        __syncthreads();
        lap1_plane(k + 1);                 // replaces lap1 plane k-1
        __syncthreads();
        T(*l0)[LX] = sl[k & 1];
        const int hx = tx + 1, hy = ty + 1;
        const T lc = l0[hy][hx];
        const T lap2 = lap7(lc, l0[hy][hx + 1], l0[hy][hx - 1], l0[hy + 1][hx], l0[hy - 1][hx],
                            sl[(k + 1) & 1][hy][hx], lm);
        if (own) a.out[(size_t)k * plane + (size_t)gy * nx + gx] = axpy(su[k & 3][ty + 2][tx + 2], lap2, a.alpha);
        lm = lc;
    }
}

template <class T>
static hipError_t lap7_dispatch(const Lap7ChainLaunch &L, hipStream_t s) {
    BArgs<T> a;
    a.in = (const T *)L.in;
    a.out = (T *)L.out;
    a.nx = L.nx; a.ny = L.ny; a.nz = L.nz;
    a.seg = L.cfg.seg > 0 ? L.cfg.seg : 32;
    a.alpha = (T)L.alpha;
    int tx = 64, ty = 4;
    switch (L.cfg.variant) {
    case 1: tx = 32; ty = 8; break;
    case 2: tx = 64; ty = 8; break;
    case 3: tx = 128; ty = 2; break;
    case 4: tx = 32; ty = 4; break;
    default: break;
    }
    dim3 grid((L.nx + tx - 1) / tx, (L.ny + ty - 1) / ty, (L.nz + a.seg - 1) / a.seg);
    switch (L.cfg.variant) {
    case 1: hipLaunchKernelGGL((lap7_chain_kernel<T, 32, 8>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((lap7_chain_kernel<T, 64, 8>), grid, dim3(512), 0, s, a); break;
    case 3: hipLaunchKernelGGL((lap7_chain_kernel<T, 128, 2>), grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((lap7_chain_kernel<T, 32, 4>), grid, dim3(128), 0, s, a); break;
    default: hipLaunchKernelGGL((lap7_chain_kernel<T, 64, 4>), grid, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_lap7_chain(const Lap7ChainLaunch &L, hipStream_t s) {
    return L.dtype == HFAV_F64 ? lap7_dispatch<double>(L, s) : lap7_dispatch<float>(L, s);
}

}  // namespace hfav
