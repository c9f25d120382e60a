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
// exchanged.  One barrier per row.  Row loads are software-pipelined P rows
// ahead through registers so that enough bytes are in flight per CU to cover
// HBM latency.
#include <algorithm>
#include <hip/hip_runtime.h>
#include "dpp.h"
#include "kernels.h"
#include "ops.h"
#include "store.h"
#include "xcd.h"

namespace hfav {

template <class T>
struct HArgs {
    const T *in;
    T *out;
    int ni, nj, nk, seg, xcd;
    T coeff;
    // in-place: original values of the columns i0-2 .. i0+1 at every x-tile
    // boundary i0 (xb[((k*nj + j)*ntx + tile)*4 + c]) and of the rows
    // j0-2 .. j0+1 at every row-segment start j0 (yb[((k*nsg + s)*4 + r)*ni + i])
    const T *xb, *yb;
};

__device__ __forceinline__ int pwrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// In/out chaining (Design, "In/out chaining"): out may alias in.  Within a
// tile every input row is fetched before the tile writes it and rows j-2 ..
// j+1 stay in the LDS ring (the rolling input buffer), so only values that
// another tile reads are at risk: the 2-wide halo columns at each x-tile
// boundary and the 2 halo rows at each segment boundary.  A copy kernel
// saves them before the fused kernel runs; with IP the fused kernel reads
// every value outside its own tile from those copies.
template <class T>
__global__ __launch_bounds__(256) void hdiff_halo_copy_kernel(HArgs<T> a, int B) {
    const int ni = a.ni, nj = a.nj, nk = a.nk;
    const int ntx = (ni + B - 1) / B, nsg = (nj + a.seg - 1) / a.seg;
    T *xb = const_cast<T *>(a.xb), *yb = const_cast<T *>(a.yb);
    const size_t nx = (size_t)nk * nj * ntx * 4, ny = (size_t)nk * nsg * 4 * ni;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < nx + ny; q += (size_t)gridDim.x * 256) {
        if (q < nx) {
            const int c = (int)(q & 3), t = (int)((q >> 2) % ntx);
            const size_t kj = (q >> 2) / ntx;                         // k*nj + j
            xb[q] = a.in[kj * ni + pwrap(t * B - 2 + c, ni)];
        } else {
            const size_t r = q - nx;
            const int i = (int)(r % ni), row = (int)((r / ni) & 3);
            const size_t ks = (r / ni) >> 2;                          // k*nsg + s
            const int k = (int)(ks / nsg), sg = (int)(ks % nsg);
            yb[r] = a.in[((size_t)k * nj + pwrap(sg * a.seg - 2 + row, nj)) * ni + i];
        }
    }
}

template <class T, int B, int P, bool NT, bool IP = false>
__global__ __launch_bounds__(B) void hdiff_kernel(HArgs<T> a) {
    constexpr int W = B + 4;              // row slot: columns i0-2 .. i0+B+1
    __shared__ T ring[4][W];
    const int t = threadIdx.x;
    const int ni = a.ni, nj = a.nj;
    // logical tile: x tile fastest, then row segment, then plane
    const int ntx = (ni + B - 1) / B, nsg = (nj + a.seg - 1) / a.seg;
    const int tile = xcd_tile(blockIdx.x, ntx * nsg * a.nk, a.xcd);
    const int i0 = (tile % ntx) * B;
    const int j0 = ((tile / ntx) % nsg) * a.seg;
    const int j1 = min(j0 + a.seg, a.nj);
    const int k = tile / (ntx * nsg);
    const T *plane = a.in + (size_t)k * nj * ni;
    T *oplane = a.out + (size_t)k * nj * ni;
    // lane t keeps its own column (slot t+2); lanes 0..3 also fetch the
    // four halo columns (slots 0, 1, B+2, B+3)
    const int col = pwrap(i0 + t, ni);
    const int hs = t < 2 ? t : t + B;     // halo slot for lanes 0..3
    const int hcol = pwrap(i0 - 2 + hs, ni);
    const bool halo = t < 4;

    auto fetch = [&](int j, T &v, T &h) {
        if constexpr (IP) {
            if (j < j0 || j >= j1) {        // another segment's row: its saved copy
                const int sg = j < j0 ? tile / ntx % nsg : (tile / ntx % nsg + 1) % nsg;
                const int row = j < j0 ? j - j0 + 2 : j - j1 + 2;
                const T *r = a.yb + ((size_t)k * nsg + sg) * 4 * ni + (size_t)row * ni;
                v = r[col];
                if (halo) h = r[hcol];
                return;
            }
            // own row: own columns from the field, the rest from the saved
            // boundary columns (left halo: this tile's boundary; right halo
            // and lanes past the row end: the next boundary, wrapped)
            const int tx = tile % ntx;
            const T *xr = a.xb + ((size_t)k * nj + j) * ntx * 4;
            const T *xl = xr + (size_t)tx * 4, *xn = xr + (size_t)((tx + 1) % ntx) * 4;
            const int w = i0 + t - ni;      // >= 0: past the row end, wrapped to column w
            v = w < 0 ? plane[(size_t)j * ni + i0 + t] : xn[2 + (w < 2 ? w : 1)];
            if (halo) h = t < 2 ? xl[t] : xn[2 + (t - 2)];
            return;
        }
        const T *r = plane + (size_t)pwrap(j, nj) * ni;
        v = r[col];
        if (halo) h = r[hcol];
    };
    auto commit = [&](int j, T v, T h) {
        T *s = ring[j & 3];
        s[t + 2] = v;
        if (halo) s[hs] = h;
    };
    auto L = [&](int j, int d) { return ring[j & 3][t + 2 + d]; };
    auto lap_at = [&](int j, int d) {
        return hdiff_lap(L(j, d), L(j, d + 1), L(j, d - 1), L(j + 1, d), L(j - 1, d));
    };

    // software pipeline: rows j+2 .. j+1+P are in flight in registers while
    // row j is computed, so each workgroup keeps P row loads outstanding
    T pv[P], ph[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        ph[q] = T(0);
        if (j0 + 2 + q <= j1 + 1) fetch(j0 + 2 + q, pv[q], ph[q]);
    }
    // prologue: rows j0-2 .. j0+1, the Laplacian of rows j0-1 (centre) and
    // j0 (three columns), and the y flux of row j0-1
    for (int r = -2; r <= 1; ++r) {
        T v, h = T(0);
        fetch(j0 + r, v, h);
        commit(j0 + r, v, h);
    }
    __syncthreads();
    T lm1 = lap_at(j0 - 1, 0);
    T la = lap_at(j0, -1), lb = lap_at(j0, 0), lc = lap_at(j0, 1);
    T fym = hdiff_flux(lm1, lb, L(j0 - 1, 0), L(j0, 0));
    __syncthreads();

    for (int jb = j0; jb < j1; jb += P) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int j = jb + q;
            if (j >= j1) break;
            commit(j + 2, pv[q], ph[q]);        // overwrites row j-2's slot
            if (j + 2 + P <= j1 + 1) fetch(j + 2 + P, pv[q], ph[q]);
            __syncthreads();
            // Laplacian of row j+1 at columns i-1, i, i+1
            const T na = lap_at(j + 1, -1), nb = lap_at(j + 1, 0), nc = lap_at(j + 1, 1);
            const T u = L(j, 0);
            const T fx0 = hdiff_flux(lb, lc, u, L(j, 1));
            const T fxm = hdiff_flux(la, lb, L(j, -1), u);
            const T fy0 = hdiff_flux(lb, nb, u, L(j + 1, 0));
            if (i0 + t < ni) store_out<NT>(oplane + (size_t)j * ni + i0 + t, hdiff_out(u, fx0, fxm, fy0, fym, a.coeff));
            fym = fy0;
            la = na; lb = nb; lc = nc;
            // no second barrier: the next write goes to row j-1's slot, which
            // no lane still in this step reads, and a lane cannot run two rows
            // ahead of the post-commit barrier
        }
    }
}

// ------------------------------------------------------------------ DPP variant
// Neighbour exchange along the lane axis through DPP lane shifts instead of
// LDS ("inner rotation" in registers): lane l takes lane l-1's value with
// wave_shr:1 and lane l+1's with wave_shl:1, a VALU move.  Each lane then
// computes one Laplacian per row instead of three; only the two lanes at
// the edges of each wave read their missing neighbour from the LDS row ring
// (filled as in the kernel above).  The column's rows j .. j+2 stay in
// registers.  Arithmetic is unchanged, so results are bit-identical.
template <class T, int B, int P, bool NT, bool IP = false>
__global__ __launch_bounds__(B) void hdiff_dpp_kernel(HArgs<T> a) {
    constexpr int W = B + 4;
    __shared__ T ring[4][W];
    const int t = threadIdx.x, lane = t & 63;
    const int ni = a.ni, nj = a.nj;
    const int ntx = (ni + B - 1) / B, nsg = (nj + a.seg - 1) / a.seg;
    const int tile = xcd_tile(blockIdx.x, ntx * nsg * a.nk, a.xcd);
    const int i0 = (tile % ntx) * B;
    const int j0 = ((tile / ntx) % nsg) * a.seg;
    const int j1 = min(j0 + a.seg, a.nj);
    const int k = tile / (ntx * nsg);
    const T *plane = a.in + (size_t)k * nj * ni;
    T *oplane = a.out + (size_t)k * nj * ni;
    const int col = pwrap(i0 + t, ni);
    const int hs = t < 2 ? t : t + B;
    const int hcol = pwrap(i0 - 2 + hs, ni);
    const bool halo = t < 4;
    auto fetch = [&](int j, T &v, T &h) {
        if constexpr (IP) {
            if (j < j0 || j >= j1) {        // another segment's row: its saved copy
                const int sg = j < j0 ? tile / ntx % nsg : (tile / ntx % nsg + 1) % nsg;
                const int row = j < j0 ? j - j0 + 2 : j - j1 + 2;
                const T *r = a.yb + ((size_t)k * nsg + sg) * 4 * ni + (size_t)row * ni;
                v = r[col];
                if (halo) h = r[hcol];
                return;
            }
            // own row: own columns from the field, the rest from the saved
            // boundary columns (left halo: this tile's boundary; right halo
            // and lanes past the row end: the next boundary, wrapped)
            const int tx = tile % ntx;
            const T *xr = a.xb + ((size_t)k * nj + j) * ntx * 4;
            const T *xl = xr + (size_t)tx * 4, *xn = xr + (size_t)((tx + 1) % ntx) * 4;
            const int w = i0 + t - ni;      // >= 0: past the row end, wrapped to column w
            v = w < 0 ? plane[(size_t)j * ni + i0 + t] : xn[2 + (w < 2 ? w : 1)];
            if (halo) h = t < 2 ? xl[t] : xn[2 + (t - 2)];
            return;
        }
        const T *r = plane + (size_t)pwrap(j, nj) * ni;
        v = r[col];
        if (halo) h = r[hcol];
    };
    auto commit = [&](int j, T v, T h) {
        T *s = ring[j & 3];
        s[t + 2] = v;
        if (halo) s[hs] = h;
    };
    auto L = [&](int j, int d) { return ring[j & 3][t + 2 + d]; };
    auto lap_at = [&](int j, int d) {
        return hdiff_lap(L(j, d), L(j, d + 1), L(j, d - 1), L(j + 1, d), L(j - 1, d));
    };

    T pv[P], ph[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        ph[q] = T(0);
        pv[q] = T(0);
        if (j0 + 2 + q <= j1 + 1) fetch(j0 + 2 + q, pv[q], ph[q]);
    }
    T u0 = T(0), u1 = T(0);
    for (int r = -2; r <= 1; ++r) {
        T v, h = T(0);
        fetch(j0 + r, v, h);
        commit(j0 + r, v, h);
        if (r == 0) u0 = v;
        if (r == 1) u1 = v;
    }
    __syncthreads();
    T uw0 = L(j0, -1), ue0 = L(j0, 1);
    T la = lap_at(j0, -1), lb = lap_at(j0, 0), lc = lap_at(j0, 1);
    T fym = hdiff_flux(lap_at(j0 - 1, 0), lb, L(j0 - 1, 0), u0);
    __syncthreads();

    for (int jb = j0; jb < j1; jb += P) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int j = jb + q;
            if (j >= j1) break;
            const T u2 = pv[q];
            commit(j + 2, pv[q], ph[q]);
            if (j + 2 + P <= j1 + 1) fetch(j + 2 + P, pv[q], ph[q]);
            __syncthreads();
            // row j+1: neighbours by lane shifts, wave edges from the ring
            T uw1 = lane_shift<true>(u1), ue1 = lane_shift<false>(u1);
            if (lane == 0) uw1 = L(j + 1, -1);
            if (lane == 63) ue1 = L(j + 1, 1);
            const T nb = hdiff_lap(u1, ue1, uw1, u2, u0);
            T na = lane_shift<true>(nb), nc = lane_shift<false>(nb);
            if (lane == 0) na = lap_at(j + 1, -1);
            if (lane == 63) nc = lap_at(j + 1, 1);
            const T fx0 = hdiff_flux(lb, lc, u0, ue0);
            const T fxm = hdiff_flux(la, lb, uw0, u0);
            const T fy0 = hdiff_flux(lb, nb, u0, u1);
            if (i0 + t < ni) store_out<NT>(oplane + (size_t)j * ni + i0 + t, hdiff_out(u0, fx0, fxm, fy0, fym, a.coeff));
            fym = fy0;
            la = na; lb = nb; lc = nc;
            uw0 = uw1; ue0 = ue1;
            u0 = u1; u1 = u2;
        }
    }
}

static int hdiff_block(const hfav_config &c) {
    return (c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512) ? c.block : 256;
}

size_t hdiff_inplace_bytes(int ni, int nj, int nk, int dtype, const hfav_config &cfg) {
    const int B = hdiff_block(cfg), seg = cfg.seg > 0 ? cfg.seg : 32;
    const size_t ntx = (ni + B - 1) / B, nsg = (nj + seg - 1) / seg;
    const size_t es = dtype == HFAV_F64 ? 8 : 4;
    const size_t xbytes = ((size_t)nk * nj * ntx * 4 * es + 255) / 256 * 256;
    return xbytes + (size_t)nk * nsg * 4 * ni * es;
}

template <class T>
static hipError_t hdiff_dispatch(const HdiffLaunch &L, hipStream_t s) {
    HArgs<T> a;
    a.in = (const T *)L.in;
    a.out = (T *)L.out;
    a.ni = L.ni; a.nj = L.nj; a.nk = L.nk;
    a.seg = L.cfg.seg > 0 ? L.cfg.seg : 32;
    a.coeff = (T)L.coeff;
    a.xcd = L.cfg.xcd;
    a.xb = a.yb = nullptr;
    const int B = hdiff_block(L.cfg);
    if (L.halo) {
        // in place: save the at-risk halo columns and rows, then run the
        // fused kernel reading them from the copies (the plain LDS-ring
        // kernel; the DPP variant and the store hint are not used here)
        const int ntx = (L.ni + B - 1) / B;
        a.xb = (const T *)L.halo;
        const size_t xbytes = ((size_t)L.nk * L.nj * ntx * 4 * sizeof(T) + 255) / 256 * 256;
        a.yb = (const T *)((const char *)L.halo + xbytes);
        const int nsg = (L.nj + a.seg - 1) / a.seg;
        const size_t n = (size_t)L.nk * L.nj * ntx * 4 + (size_t)L.nk * nsg * 4 * L.ni;
        const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
        hipLaunchKernelGGL((hdiff_halo_copy_kernel<T>), dim3(nb), dim3(256), 0, s, a, B);
        const int pv = L.cfg.variant & 7;
        const int P = pv == 1 ? 1 : pv == 2 ? 2 : pv == 4 ? 8 : 4;
        dim3 grid(((L.ni + B - 1) / B) * nsg * L.nk);
#define HI_LAUNCH(BB, PP) hipLaunchKernelGGL((hdiff_kernel<T, BB, PP, false, true>), grid, dim3(BB), 0, s, a)
#define HI_P(BB)                               \
    switch (P) {                               \
    case 1: HI_LAUNCH(BB, 1); break;           \
    case 2: HI_LAUNCH(BB, 2); break;           \
    case 8: HI_LAUNCH(BB, 8); break;           \
    default: HI_LAUNCH(BB, 4); break;          \
    }
        switch (B) {
        case 64: HI_P(64); break;
        case 128: HI_P(128); break;
        case 512: HI_P(512); break;
        default: HI_P(256); break;
        }
#undef HI_P
#undef HI_LAUNCH
        return hipGetLastError();
    }
    // variant: bit 4 makes the output stores non-temporal, bit 3 selects
    // the DPP kernel; the low bits give the prefetch depth (rows in flight
    // per workgroup) 1 -> 1, 2 -> 2, 4 -> 8, else 4
    const bool dpp = (L.cfg.variant & 8) != 0;
    const bool nt = (L.cfg.variant & 16) != 0;
    const int pv = L.cfg.variant & 7;
    const int P = pv == 1 ? 1 : pv == 2 ? 2 : pv == 4 ? 8 : 4;
    dim3 grid(((L.ni + B - 1) / B) * ((L.nj + a.seg - 1) / a.seg) * L.nk);
#define HD_LAUNCH(BB, PP)                                                                             \
    do {                                                                                              \
        if (dpp && nt) hipLaunchKernelGGL((hdiff_dpp_kernel<T, BB, PP, true>), grid, dim3(BB), 0, s, a); \
        else if (dpp) hipLaunchKernelGGL((hdiff_dpp_kernel<T, BB, PP, false>), grid, dim3(BB), 0, s, a); \
        else if (nt) hipLaunchKernelGGL((hdiff_kernel<T, BB, PP, true>), grid, dim3(BB), 0, s, a);       \
        else hipLaunchKernelGGL((hdiff_kernel<T, BB, PP, false>), grid, dim3(BB), 0, s, a);              \
    } while (0)
#define HD_P(BB)                               \
    switch (P) {                               \
    case 1: HD_LAUNCH(BB, 1); break;           \
    case 2: HD_LAUNCH(BB, 2); break;           \
    case 8: HD_LAUNCH(BB, 8); break;           \
    default: HD_LAUNCH(BB, 4); break;          \
    }
    switch (B) {
    case 64: HD_P(64); break;
    case 128: HD_P(128); break;
    case 512: HD_P(512); break;
    default: HD_P(256); break;
    }
#undef HD_P
#undef HD_LAUNCH
    return hipGetLastError();
}

hipError_t launch_hdiff(const HdiffLaunch &L, hipStream_t s) {
    return L.dtype == HFAV_F64 ? hdiff_dispatch<double>(L, s) : hdiff_dispatch<float>(L, s);
}

}  // namespace hfav
