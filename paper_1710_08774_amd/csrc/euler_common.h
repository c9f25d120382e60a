// Shared by the Godunov sweep kernels: kernel arguments, boundary index
// arithmetic, the time step, slopes + trace of one cell, and the workgroup
// maximum of the CFL reduction.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "ops.h"

namespace hfav {

template <class T>
struct EArgs {
    const T *rho, *mn, *mt, *E;
    T *orho, *omn, *omt, *oE;
    int nx, ny, bc;
    double g;
    int niter;
    const double *dt_src;
    int dt_mode;
    double cfl;
    double *smax_out;
    int seg;
    int xcd;
    int bcy;           // boundary along y of the two-sweep kernel
    int newton_all;    // take every Newton step (no stop at a repeated iterate)
    // in place (goal q written over axiom q): the state of the cells around
    // every segment boundary b of every line (cells b-2 .. b+1, boundary
    // b = s * seg for s < nsg), saved before the sweep; null otherwise.
    // Layout [field][s][cell][line].
    const T *halo;
    int nsg;
};

// configuration variant bit of the Euler families: every Newton step taken
constexpr int EULER_NEWTON_ALL = 64;

__device__ __forceinline__ int bwrap(int i, int n, int bc) {
    if (bc == HFAV_BC_PERIODIC) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ double read_dt(const double *src, int mode, double cfl) {
    double v = *src;
    return mode == DT_VALUE ? v : cfl / v;
}

// Slopes and trace for one cell from its primitive window (m-1, m, m+1).
template <class T>
__device__ __forceinline__ void slope_trace(const Prim<T> &wm, const Prim<T> &w0, const Prim<T> &wp,
                                            T nu, T *plus, T *minus) {
    T dr = vanleer(wm.r, w0.r, wp.r);
    T du = vanleer(wm.un, w0.un, wp.un);
    T dv = vanleer(wm.ut, w0.ut, wp.ut);
    T dp = vanleer(wm.p, w0.p, wp.p);
    euler_trace(w0, dr, du, dv, dp, nu, plus, minus);
}

template <int B>
__device__ __forceinline__ void block_max_to(double v, double *out) {
    __shared__ double red[B / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();            // red[] may still be read by a previous call
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
#pragma unroll
        for (int q = 1; q < B / 64; ++q) m = fmax(m, red[q]);
        atomic_max_nonneg(out, m);
    }
}

}  // namespace hfav
