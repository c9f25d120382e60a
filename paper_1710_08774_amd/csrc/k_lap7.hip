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
// through registers.  A workgroup of NT lanes may own a tile of R = TX*TY/NT
// output points per lane (lane t owns points t, t + NT, ...): larger tiles
// re-read less of their 2-cell halo from HBM.
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "ops.h"
#include "store.h"
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

template <class T, int TX, int TY, int P, bool NTS, int NT = TX * TY>
__global__ __launch_bounds__(NT) void lap7_chain_kernel(BArgs<T> a) {
    constexpr int R = TX * TY / NT;             // output points per lane
    static_assert(R * NT == TX * TY, "the tile must be a multiple of the workgroup");
    constexpr int UX = TX + 4, UY = TY + 4;     // u tile with halo 2
    constexpr int LX = TX + 2, LY = TY + 2;     // lap1 tile with halo 1
    constexpr int M = (UX * UY + NT - 1) / NT;  // u points loaded per lane per plane
    __shared__ T su[4][UY][UX];
    __shared__ T sl[2][LY][LX];
    const int tid = threadIdx.x;
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
    // owned output points: tile coordinates, and lap1 at plane k-1 (the
    // point's own centre, kept in a register)
    int tx[R], ty[R];
    bool own[R];
    T lm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        tx[r] = (tid + r * NT) % TX;
        ty[r] = (tid + r * NT) / TX;
        own[r] = x0 + tx[r] < nx && y0 + ty[r] < ny;
        lm[r] = lap1_at(k0 - 1, tx[r] + 1, ty[r] + 1);
    }
    lap1_plane(k0);
    __syncthreads();

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
            T *out = a.out + (size_t)k * plane;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int hx = tx[r] + 1, hy = ty[r] + 1;
                const T lc = l0[hy][hx];
                const T lap2 = lap7(lc, l0[hy][hx + 1], l0[hy][hx - 1], l0[hy + 1][hx], l0[hy - 1][hx],
                                    sl[(k + 1) & 1][hy][hx], lm[r]);
                if (own[r])
                    store_out<NTS>(out + (size_t)(y0 + ty[r]) * nx + (x0 + tx[r]),
                                   axpy(su[k & 3][ty[r] + 2][tx[r] + 2], lap2, a.alpha));
                lm[r] = lc;
            }
        }
    }
}

// Variant with the z windows in registers.  Every lane owns up to two points
// of the (TX+4) x (TY+4) u tile for the whole segment and keeps, per point,
// u at planes k..k+2 and lap1 at planes k-1..k in registers; only the x-y
// neighbours go through LDS, one plane of u and one of lap1 at a time (each
// double-buffered), so a plane costs 4 + 4 LDS reads per point instead of
// 7 + 7 and needs no per-point index arithmetic.  Two barriers per plane.
// Lane t owns point t; the points past NT are dealt out to the waves in
// equal contiguous runs, so every wave carries the same load between
// barriers and its accesses stay coalesced.
template <class T, int TX, int TY, int P, bool NTS>
__global__ __launch_bounds__(TX * TY) void lap7_reg_kernel(BArgs<T> a) {
    constexpr int NT = TX * TY;
    constexpr int UX = TX + 4, UY = TY + 4, NU = UX * UY;
    constexpr int M = 2;
    constexpr int NW = NT / 64;
    constexpr int EW = (NU - NT + NW - 1) / NW;     // extra points per wave
    static_assert(NT % 64 == 0 && NU > NT && EW <= 64, "tile must need at most two points per lane");
    __shared__ T su[2][NU];
    __shared__ T sl[2][NU];
    const int tid = threadIdx.x;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, nsg = (nz + a.seg - 1) / a.seg;
    const int tile = xcd_tile(blockIdx.x, ntx * nty * nsg, a.xcd);
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY;
    const int k0 = (tile / (ntx * nty)) * a.seg;
    const int k1 = min(k0 + a.seg, nz);
    const size_t plane = (size_t)nx * ny;
    // owned points (index q in the u tile, row-major with row UX)
    int qi[M], goff[M], obase[M];
    bool ou[M], ol[M], oo[M];
    qi[0] = tid;
    qi[1] = (tid % 64) < EW ? NT + EW * (tid / 64) + tid % 64 : NU;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int q = qi[m];
        const int px = q % UX, py = q / UX;
        ou[m] = q < NU;
        ol[m] = ou[m] && px >= 1 && px < UX - 1 && py >= 1 && py < UY - 1;
        const int gx = x0 + px - 2, gy = y0 + py - 2;
        oo[m] = ou[m] && px >= 2 && px < UX - 2 && py >= 2 && py < UY - 2 && gx < nx && gy < ny;
        goff[m] = ou[m] ? w3(gy, ny) * nx + w3(gx, nx) : 0;
        obase[m] = oo[m] ? gy * nx + gx : 0;
    }
    auto fetch = [&](int k, T *v) {
        const T *p = a.in + (size_t)w3(k, nz) * plane;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (ou[m]) v[m] = p[goff[m]];
    };
    // 7-point Laplacian of a plane held in LDS at owned point m, with the
    // z neighbours t (plane above) and b (plane below) from registers
    auto lap_at = [&](const T *pl, int m, T c, T t, T b) {
        const int q = qi[m];
        return lap7(c, pl[q + 1], pl[q - 1], pl[q + UX], pl[q - UX], t, b);
    };

    T ua[M], ub[M], uc[M], la[M], lb[M];
    T pv[P][M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        ua[m] = ub[m] = uc[m] = la[m] = lb[m] = T(0);
#pragma unroll
        for (int q = 0; q < P; ++q) pv[q][m] = T(0);
    }
    // prologue: u(k0-2) .. u(k0+2); lap1(k0-1) to registers, lap1(k0) to
    // registers and LDS
    {
        T t0[M], t1[M];
        fetch(k0 - 2, t0);
        fetch(k0 - 1, t1);
        fetch(k0, ua);
        fetch(k0 + 1, ub);
        fetch(k0 + 2, uc);
#pragma unroll
        for (int q = 0; q < P; ++q)
            if (k0 + 3 + q <= k1 + 1) fetch(k0 + 3 + q, pv[q]);
        T *s1 = su[(k0 - 1) & 1];
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (ou[m]) s1[qi[m]] = t1[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (ol[m]) la[m] = lap_at(s1, m, t1[m], ua[m], t0[m]);
        T *s0 = su[k0 & 1];
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (ou[m]) s0[qi[m]] = ua[m];
        __syncthreads();
        T *l0 = sl[k0 & 1];
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (ol[m]) {
                lb[m] = lap_at(s0, m, ua[m], ub[m], t1[m]);
                l0[qi[m]] = lb[m];
            }
    }
    for (int kb = k0; kb < k1; kb += P) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = kb + q;
            if (k >= k1) break;
            T *sup = su[(k + 1) & 1];
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (ou[m]) sup[qi[m]] = ub[m];
            __syncthreads();
            // lap1 at plane k+1
            T lc[M];
            T *slp = sl[(k + 1) & 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                lc[m] = T(0);
                if (ol[m]) {
                    lc[m] = lap_at(sup, m, ub[m], uc[m], ua[m]);
                    slp[qi[m]] = lc[m];
                }
            }
            __syncthreads();
            // lap2 and the update at plane k
            const T *slk = sl[k & 1];
            T *out = a.out + (size_t)k * plane;
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (oo[m]) store_out<NTS>(out + obase[m], axpy(ua[m], lap_at(slk, m, lb[m], lc[m], la[m]), a.alpha));
            // rotate the z windows; the prefetched plane k+3 enters
#pragma unroll
            for (int m = 0; m < M; ++m) {
                ua[m] = ub[m]; ub[m] = uc[m]; uc[m] = pv[q][m];
                la[m] = lb[m]; lb[m] = lc[m];
            }
            if (k + 3 + P <= k1 + 1) fetch(k + 3 + P, pv[q]);
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
    // variant: tile shape and kernel in the low 5 bits; bit 5 makes the
    // output stores non-temporal
    const int var = L.cfg.variant & 31;
    const bool nt = (L.cfg.variant & 32) != 0;
    switch (var) {
    case 1: tx = 32; ty = 8; break;
    case 2: tx = 64; ty = 8; break;
    case 3: tx = 128; ty = 2; break;
    case 4: tx = 32; ty = 4; break;
    case 5: case 10: tx = 64; ty = 16; break;
    case 6: tx = 64; ty = 32; break;
    case 7: tx = 128; ty = 16; break;
    // the 4-point tiles need more LDS than a workgroup has in FP64: there
    // they run as 64 x 32
    case 8: tx = sizeof(T) == 4 ? 128 : 64; ty = 32; break;
    case 9: tx = sizeof(T) == 4 ? 256 : 64; ty = sizeof(T) == 4 ? 16 : 32; break;
    case 11: tx = 64; ty = 8; break;
    case 12: tx = 32; ty = 8; break;
    case 13: tx = 128; ty = 8; break;
    case 14: tx = 32; ty = 16; break;
    default: break;
    }
    // tile_y selects the prefetch depth (planes in flight): 1, 2 or 4
    const int P = L.cfg.tile_y == 1 ? 1 : L.cfg.tile_y == 4 ? 4 : 2;
    dim3 grid(((L.nx + tx - 1) / tx) * ((L.ny + ty - 1) / ty) * ((L.nz + a.seg - 1) / a.seg));
#define B7N(TX_, TY_, PP, NN)                                                                                      \
    do {                                                                                                           \
        if (nt) hipLaunchKernelGGL((lap7_chain_kernel<T, TX_, TY_, PP, true, NN>), grid, dim3(NN), 0, s, a);       \
        else hipLaunchKernelGGL((lap7_chain_kernel<T, TX_, TY_, PP, false, NN>), grid, dim3(NN), 0, s, a);         \
    } while (0)
#define B7(TX_, TY_, PP) B7N(TX_, TY_, PP, TX_ * TY_)
#define B7P(TX_, TY_)                 \
    switch (P) {                      \
    case 1: B7(TX_, TY_, 1); break;   \
    case 4: B7(TX_, TY_, 4); break;   \
    default: B7(TX_, TY_, 2); break;  \
    }
    // tiles larger than a workgroup: 1024 lanes, 2 or 4 points per lane
#define B7L(TX_, TY_)                          \
    switch (P) {                               \
    case 1: B7N(TX_, TY_, 1, 1024); break;     \
    case 4: B7N(TX_, TY_, 4, 1024); break;     \
    default: B7N(TX_, TY_, 2, 1024); break;    \
    }
#define R7(TX_, TY_, PP)                                                                                   \
    do {                                                                                                   \
        if (nt) hipLaunchKernelGGL((lap7_reg_kernel<T, TX_, TY_, PP, true>), grid, dim3(TX_ * TY_), 0, s, a);   \
        else hipLaunchKernelGGL((lap7_reg_kernel<T, TX_, TY_, PP, false>), grid, dim3(TX_ * TY_), 0, s, a);     \
    } while (0)
#define R7P(TX_, TY_)                 \
    switch (P) {                      \
    case 1: R7(TX_, TY_, 1); break;   \
    case 4: R7(TX_, TY_, 4); break;   \
    default: R7(TX_, TY_, 2); break;  \
    }
    switch (var) {
    case 1: B7P(32, 8); break;
    case 2: B7P(64, 8); break;
    case 3: B7P(128, 2); break;
    case 4: B7P(32, 4); break;
    case 5: B7P(64, 16); break;
    case 6: B7L(64, 32); break;
    case 7: B7L(128, 16); break;
    case 8:
        if constexpr (sizeof(T) == 4) { B7L(128, 32); } else { B7L(64, 32); }
        break;
    case 9:
        if constexpr (sizeof(T) == 4) { B7L(256, 16); } else { B7L(64, 32); }
        break;
    case 10: R7P(64, 16); break;
    case 11: R7P(64, 8); break;
    case 12: R7P(32, 8); break;
    case 13: R7P(128, 8); break;
    case 14: R7P(32, 16); break;
    default: B7P(64, 4); break;
    }
#undef R7P
#undef R7
#undef B7L
#undef B7P
#undef B7
#undef B7N
    return hipGetLastError();
}

hipError_t launch_lap7_chain(const Lap7ChainLaunch &L, hipStream_t s) {
    return L.dtype == HFAV_F64 ? lap7_dispatch<double>(L, s) : lap7_dispatch<float>(L, s);
}

}  // namespace hfav
