// Both directional Godunov sweeps of a time step in one kernel (Design,
// "Fusing iteration nests": the x sweep and the y sweep are nests of equal
// rank, so they fuse; their dataflow through the x-swept state U^x is along
// j only).  The y sweep of row j reads U^x at rows j-2 .. j+1, which the
// kernel produces row by row and keeps in registers and a 3-row LDS window
// per lane: U^x never goes to HBM, and each step reads U and writes the new
// state once (64 B per cell-step in FP64 instead of 128).
//
// One wave per tile of W = 60 output columns x a segment of rows.  Lane l
// holds column c0 - 2 + l; the x neighbours (primitive state, minus face,
// flux) come from the adjacent lanes through DPP wave shifts, so lanes 2 ..
// 61 hold valid x-swept values and lanes 0, 1, 62, 63 are the halo.  Every
// row of the segment plus four halo rows is x-swept by the wave, then fed
// to the y sweep's register windows, exactly as the separate y sweep
// streams it.  The formulas per cell are those of the two separate sweeps
// (the same device rule bodies; the compiler may contract multiply-adds
// differently in this kernel, so results agree to rounding).
//
// Price: the x sweep runs on 64 lanes for 60 columns and on 4 extra rows per
// segment, about 1.07 x 1.25 (16-row segments) of its work.  The sweeps are
// FP64-ALU bound, not HBM bound, so this kernel trades bytes that were not
// the bottleneck for arithmetic that is.
#include <hip/hip_runtime.h>
#include "dpp.h"
#include "euler_common.h"
#include "kernels.h"
#include "ops.h"
#include "xcd.h"

namespace hfav {
namespace {

constexpr int XY_W = 60;      // output columns per wave

// neighbour's value, or the lane's own at the wave edge (keeps the halo
// lanes' arithmetic on physical states)
template <bool PREV, class T>
__device__ __forceinline__ T nb(T v, bool edge) {
    const T s = lane_shift<PREV>(v);
    return edge ? v : s;
}
template <bool PREV, class T>
__device__ __forceinline__ Prim<T> nb(const Prim<T> &w, bool edge) {
    return Prim<T>{nb<PREV>(w.r, edge), nb<PREV>(w.un, edge), nb<PREV>(w.ut, edge), nb<PREV>(w.p, edge),
                   nb<PREV>(w.c, edge)};
}

template <class T, class A, bool G14>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void euler_xy_kernel(EArgs<T> a) {
    __shared__ T s_u[3][4][64];            // U^x of the lane's last three rows (y frame)
    const int nx = a.nx, ny = a.ny, l = threadIdx.x;
    const int ns = (nx + XY_W - 1) / XY_W, nsg = (ny + a.seg - 1) / a.seg;
    const int tile = xcd_tile(blockIdx.x, ns * nsg, a.xcd);
    const int c0 = (tile % ns) * XY_W;
    const int j0 = (tile / ns) * a.seg, j1 = min(j0 + a.seg, ny);
    const int col = c0 - 2 + l;
    const int cw = bwrap(col, nx, a.bc);
    const bool out_lane = l >= 2 && l < 2 + XY_W && col < nx;
    const T g = G14 ? T(1.4) : (T)a.g;
    const double dt = read_dt(a.dt_src, a.dt_mode, a.cfl);
    const T nu = (T)dt;
    const A nuA = (A)dt;

    // x sweep of row r at this lane's column (valid on lanes 2 .. 61); all
    // 64 lanes take part, the DPP shifts need the whole wave
    auto xrow = [&](int r, T *ux) {
        const size_t o = (size_t)bwrap(r, ny, a.bcy) * nx + cw;
        const T u0 = a.rho[o], u1 = a.mn[o], u2 = a.mt[o], u3 = a.E[o];
        const Prim<T> w = euler_prim(u0, u1, u2, u3, g);
        T plus[4], minus[4], mr[4], G[4], F[4];
        slope_trace(nb<true>(w, l == 0), w, nb<false>(w, l == 63), nu, plus, minus);
#pragma unroll
        for (int q = 0; q < 4; ++q) mr[q] = nb<false>(minus[q], l == 63);
        riemann_T<T, G14>(plus, mr, g, a.niter, G, a.newton_all);      // face col + 1/2
        euler_flux(G, g, F);
        T Fm[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) Fm[q] = nb<true>(F[q], l == 0);   // face col - 1/2
        ux[0] = euler_update(u0, F[0], Fm[0], nuA);
        ux[1] = euler_update(u1, F[1], Fm[1], nuA);
        ux[2] = euler_update(u2, F[2], Fm[2], nuA);
        ux[3] = euler_update(u3, F[3], Fm[3], nuA);
    };
    // x-swept row r in the y frame (rho, my, mx, E): its primitive state,
    // and the conserved state kept in LDS slot `slot` (>= 0) for the update
    auto P = [&](int r, int slot) {
        T ux[4];
        xrow(r, ux);
        if (slot >= 0) {
            s_u[slot][0][l] = ux[0]; s_u[slot][1][l] = ux[2]; s_u[slot][2][l] = ux[1]; s_u[slot][3][l] = ux[3];
        }
        return euler_prim(ux[0], ux[2], ux[1], ux[3], g);
    };

    // the y sweep over rows j0 .. j1-1, streaming as the separate y sweep:
    // row r enters the window (wa, wb, wc) = rows (r-2, r-1, r); one call
    // site for the x sweep keeps the code compact
    double smax = 0.0;
    Prim<T> wa{}, wb{}, wc{};
    T fp[4], Fm[4];
    for (int r = j0 - 2; r <= j1 + 1; ++r) {
        const Prim<T> wn = P(r, r >= j0 ? (r - j0) % 3 : -1);
        wa = wb;
        wb = wc;
        wc = wn;
        if (r < j0) continue;
        if (r == j0) {                               // plus face of row j0-1
            T minus[4];
            slope_trace(wa, wb, wc, nu, fp, minus);
            continue;
        }
        const int j = r - 1;                         // rows j-1, j, j+1 in the window
        T plus[4], minus[4], G[4], F[4];
        slope_trace(wa, wb, wc, nu, plus, minus);
        riemann_T<T, G14>(fp, minus, g, a.niter, G, a.newton_all);
        euler_flux(G, g, F);                         // flux at j-1/2
        if (j > j0 && out_lane) {
            const int su = (j - 1 - j0) % 3;         // slot of row j-1
            const size_t o = (size_t)(j - 1) * nx + col;
            const T rr = euler_update(s_u[su][0][l], F[0], Fm[0], nuA);
            const T my = euler_update(s_u[su][1][l], F[1], Fm[1], nuA);
            const T mx = euler_update(s_u[su][2][l], F[2], Fm[2], nuA);
            const T e = euler_update(s_u[su][3][l], F[3], Fm[3], nuA);
            a.orho[o] = rr; a.omn[o] = mx; a.omt[o] = my; a.oE[o] = e;
            if (a.smax_out) smax = fmax(smax, (double)euler_speed(rr, mx, my, e, g));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) { Fm[q] = F[q]; fp[q] = plus[q]; }
    }
    if (a.smax_out) block_max_to<64>(smax, a.smax_out);
}

template <class T, class A>
hipError_t launch_xy_t(const EulerLaunch &L, hipStream_t s) {
    EArgs<T> a;
    a.rho = (const T *)L.in[0]; a.mn = (const T *)L.in[1]; a.mt = (const T *)L.in[2]; a.E = (const T *)L.in[3];
    a.orho = (T *)L.out[0]; a.omn = (T *)L.out[1]; a.omt = (T *)L.out[2]; a.oE = (T *)L.out[3];
    a.nx = L.nx; a.ny = L.ny; a.bc = L.bc; a.bcy = L.bcy;
    a.g = L.gamma; a.niter = L.niter;
    a.dt_src = L.dt_src; a.dt_mode = L.dt_mode; a.cfl = L.cfl;
    a.smax_out = L.smax_out;
    a.seg = L.cfg.seg > 0 ? L.cfg.seg : 16;
    a.xcd = L.cfg.xcd;
    a.newton_all = (L.cfg.variant & EULER_NEWTON_ALL) != 0;
    a.halo = nullptr;
    a.nsg = 0;
    const int ns = (L.nx + XY_W - 1) / XY_W, nsg = (L.ny + a.seg - 1) / a.seg;
    const dim3 grid((unsigned)(ns * nsg));
    if (L.gamma == 1.4) hipLaunchKernelGGL((euler_xy_kernel<T, A, true>), grid, dim3(64), 0, s, a);
    else hipLaunchKernelGGL((euler_xy_kernel<T, A, false>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_euler_xy(const EulerLaunch &L, hipStream_t s) {
    if (L.nx < 1 || L.ny < 1) return hipErrorInvalidValue;
    if (L.dtype == HFAV_F64) return launch_xy_t<double, double>(L, s);
    if (L.precision == HFAV_PREC_F32_F64ACC) return launch_xy_t<float, double>(L, s);
    return launch_xy_t<float, float>(L, s);
}

}  // namespace hfav
