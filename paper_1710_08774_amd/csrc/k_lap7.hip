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
// Two barriers per plane; plane loads are software-pipelined P planes ahead
// through registers.
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "ops.h"
#include "xcd.h"

namespace hfav {

template <class T>
struct BArgs {
    const T *in;
    T *out;
    int nx, ny, nz, seg, xcd;
    T alpha;
};

__device__ __forceinline__ int w3(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <class T, int TX, int TY, int P>
__global__ __launch_bounds__(TX * TY) void lap7_chain_kernel(BArgs<T> a) {
    constexpr int NT = TX * TY;
    constexpr int UX = TX + 4, UY = TY + 4;     // u tile with halo 2
    constexpr int LX = TX + 2, LY = TY + 2;     // lap1 tile with halo 1
    constexpr int M = (UX * UY + NT - 1) / NT;  // u points loaded per lane per plane
    __shared__ T su[4][UY][UX];
    __shared__ T sl[2][LY][LX];
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    // logical tile: x tile fastest, then y tile, then z segment
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, nsg = (nz + a.seg - 1) / a.seg;
    const int tile = xcd_tile(blockIdx.x, ntx * nty * nsg, a.xcd);
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY;
    const int k0 = (tile / (ntx * nty)) * a.seg;
    const int k1 = min(k0 + a.seg, a.nz);
    const size_t plane = (size_t)nx * ny;
    // per-lane offsets of its u points inside a plane (wrapped), fixed for
    // the whole segment
    int goff[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int q = tid + m * NT;
        const int qx = q % UX, qy = q / UX;
        goff[m] = q < UX * UY ? w3(y0 - 2 + qy, ny) * nx + w3(x0 - 2 + qx, nx) : 0;
    }
    auto fetch = [&](int k, T *v) {
        const T *p = a.in + (size_t)w3(k, nz) * plane;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (tid + m * NT < UX * UY) v[m] = p[goff[m]];
    };
    auto commit = [&](int k, const T *v) {
        T *s = &su[k & 3][0][0];
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (tid + m * NT < UX * UY) s[tid + m * NT] = v[m];
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

    // software pipeline: planes k+2 .. k+1+P in flight in registers
    T pv[P][M];
#pragma unroll
    for (int q = 0; q < P; ++q) {
#pragma unroll
        for (int m = 0; m < M; ++m) pv[q][m] = T(0);
        if (k0 + 2 + q <= k1 + 1) fetch(k0 + 2 + q, pv[q]);
    }
    // prologue: u planes k0-2 .. k0+1; lap1 at k0-1 (own centre) and k0 (tile)
    for (int r = -2; r <= 1; ++r) {
        T v[M];
        fetch(k0 + r, v);
        commit(k0 + r, v);
    }
    __syncthreads();
    T lm = lap1_at(k0 - 1, tx + 1, ty + 1);
    lap1_plane(k0);
    __syncthreads();

    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < nx && gy < ny;
    for (int kb = k0; kb < k1; kb += P) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = kb + q;
            if (k >= k1) break;
            commit(k + 2, pv[q]);              // replaces plane k-2
            if (k + 2 + P <= k1 + 1) fetch(k + 2 + P, pv[q]);
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
}

template <class T>
static hipError_t lap7_dispatch(const Lap7ChainLaunch &L, hipStream_t s) {
    BArgs<T> a;
    a.in = (const T *)L.in;
    a.out = (T *)L.out;
    a.nx = L.nx; a.ny = L.ny; a.nz = L.nz;
    a.seg = L.cfg.seg > 0 ? L.cfg.seg : 32;
    a.alpha = (T)L.alpha;
    a.xcd = L.cfg.xcd;
    int tx = 64, ty = 4;
    switch (L.cfg.variant) {
    case 1: tx = 32; ty = 8; break;
    case 2: tx = 64; ty = 8; break;
    case 3: tx = 128; ty = 2; break;
    case 4: tx = 32; ty = 4; break;
    case 5: tx = 64; ty = 16; break;
    default: break;
    }
    // tile_y selects the prefetch depth (planes in flight): 1, 2 or 4
    const int P = L.cfg.tile_y == 1 ? 1 : L.cfg.tile_y == 4 ? 4 : 2;
    dim3 grid(((L.nx + tx - 1) / tx) * ((L.ny + ty - 1) / ty) * ((L.nz + a.seg - 1) / a.seg));
#define B7(TX_, TY_, PP) hipLaunchKernelGGL((lap7_chain_kernel<T, TX_, TY_, PP>), grid, dim3(TX_ * TY_), 0, s, a)
#define B7P(TX_, TY_)                 \
    switch (P) {                      \
    case 1: B7(TX_, TY_, 1); break;   \
    case 4: B7(TX_, TY_, 4); break;   \
    default: B7(TX_, TY_, 2); break;  \
    }
    switch (L.cfg.variant) {
    case 1: B7P(32, 8); break;
    case 2: B7P(64, 8); break;
    case 3: B7P(128, 2); break;
    case 4: B7P(32, 4); break;
    case 5: B7P(64, 16); break;
    default: B7P(64, 4); break;
    }
#undef B7P
#undef B7
    return hipGetLastError();
}

hipError_t launch_lap7_chain(const Lap7ChainLaunch &L, hipStream_t s) {
    return L.dtype == HFAV_F64 ? lap7_dispatch<double>(L, s) : lap7_dispatch<float>(L, s);
}

}  // namespace hfav
