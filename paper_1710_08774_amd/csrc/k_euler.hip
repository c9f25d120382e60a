// Fused directionally split Godunov sweeps for gfx950 (Performance,
// "Hydro2D": constoprim + equation_of_state, slope, trace, qleftright,
// riemann, cmpflx and update_cons_vars fused into one iteration nest per
// pass, all intermediates contracted to rolling windows; Design,
// "Contraction").
//
// x pass (dependencies along the contiguous axis): one workgroup walks a row
// in chunks of B cells, one lane per cell.  The contracted windows along i
// (primitive state 3 cells, plus-face state 2 cells, flux 2 interfaces) are
// LDS rings of B+4 entries, so every value is produced once and read by its
// neighbour lanes: no halo recomputation except two cells per row.  Each
// lane solves exactly one Riemann problem per chunk.
//
// y pass (dependencies along the strided axis): one lane per column, lanes
// along i give coalesced row loads, and each lane streams down a segment of
// rows keeping the windows in registers (the "outer" rotation).  A segment
// recomputes two halo cells and one interface at its top.  The CFL
// reduction of the updated state is fused into this pass (wave reduction,
// then one atomic max per workgroup).
//
// Strip pass (either direction, the default for both): the LDS rings of the
// x pass laid along the sweep for W adjacent lines and C cells of each per
// chunk, over segments of a line, so that short work items (one wave per x
// segment, 4-row strips for y) fill the chip evenly.  The batched sweeps run
// the same strip body on (grid, line, segment) items.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "euler_common.h"
#include "ops.h"
#include "xcd.h"

namespace hfav {

// One grid (or one grid of a batch) as seen by a sweep body.
template <class T>
struct EView {
    const T *rho, *mn, *mt, *E;
    T *orho, *omn, *omt, *oE;
    int nx, ny;
};

template <class T>
__device__ __forceinline__ EView<T> full_view(const EArgs<T> &a) {
    return EView<T>{a.rho, a.mn, a.mt, a.E, a.orho, a.omn, a.omt, a.oE, a.nx, a.ny};
}

// ------------------------------------------------------------------ x pass
// LDS of the x pass.  Rings of R = B + 4 slots indexed by cell modulo R: a
// chunk touches cells c0-2 .. c0+B, and a barrier separates every write of a
// slot from the last read of the cell it held before.
template <class T, int B>
struct XLds {
    static constexpr int R = B + 4;
    T w[5][R];      // primitive window (r, un, ut, p, c)
    T f[4][R];      // plus-face state
    T F[4][R];      // interface flux: slot of cell p holds F(p-1/2)
    T F0[4];        // F(-1/2) for the periodic wrap
    T Fn[4];        // F(nx-1/2) for a transmissive right end
};

// Sweep one row (row index j of view v) with the whole workgroup.
template <class T, class A, bool G14, int B>
__device__ __forceinline__ void x_row(const EArgs<T> &a, const EView<T> &v, int j, double dt, XLds<T, B> &S) {
    constexpr int R = XLds<T, B>::R;
    const int nx = v.nx;
    const int t = threadIdx.x;
    const size_t row = (size_t)j * nx;
    const T g = G14 ? T(1.4) : (T)a.g;     // gamma 7/5: constants fold
    const T nu = (T)dt;
    const A nuA = (A)dt;
    int ob = 0;                 // slot of cell c0 (c0 mod R)
    // slot of cell c0 + d for d in [-2, B + 1]
    auto slot = [&](int d) {
        int sl = ob + d;
        sl += sl < 0 ? R : 0;
        return sl >= R ? sl - R : sl;
    };
    auto load_cell = [&](int cell, T *u) {
        const size_t o = row + bwrap(cell, nx, a.bc);
        u[0] = v.rho[o]; u[1] = v.mn[o]; u[2] = v.mt[o]; u[3] = v.E[o];
    };
    auto put = [&](int sl, const T *u) {
        Prim<T> w = euler_prim(u[0], u[1], u[2], u[3], g);
        S.w[0][sl] = w.r; S.w[1][sl] = w.un; S.w[2][sl] = w.ut; S.w[3][sl] = w.p; S.w[4][sl] = w.c;
    };
    auto get_prim = [&](int sl) {
        Prim<T> w;
        w.r = S.w[0][sl]; w.un = S.w[1][sl]; w.ut = S.w[2][sl]; w.p = S.w[3][sl]; w.c = S.w[4][sl];
        return w;
    };

    __syncthreads();            // the previous row of a persistent loop is done with the rings
    // prologue: cells -2, -1, 0 and the plus face of cell -1
    if (t < 3) {
        T u[4];
        load_cell(t - 2, u);
        put(slot(t - 2), u);
    }
    __syncthreads();
    if (t == 0) {
        T plus[4], minus[4];
        slope_trace(get_prim(slot(-2)), get_prim(slot(-1)), get_prim(slot(0)), nu, plus, minus);
        const int sl = slot(-1);
#pragma unroll
        for (int q = 0; q < 4; ++q) S.f[q][sl] = plus[q];
    }

    for (int c0 = 0; c0 < nx; c0 += B) {
        ob = c0 % R;
        const int p = c0 + t;
        const bool act = p < nx;
        const int sm = slot(t - 1), s0 = slot(t), sp = slot(t + 1);
        // stage 1: conserved state of the cell entering the window.  The
        // previous chunk read these primitive slots in its stage 2 (stage 3
        // for the right end), and two barriers have passed since
        T unew[4];
        if (act) load_cell(p + 1, unew);
        if (act) put(sp, unew);
        __syncthreads();
        // stage 2: slopes + trace of cell p; the plus face goes to its right
        // neighbour through LDS, the minus face stays in registers
        T minus[4];
        if (act) {
            T plus[4];
            slope_trace(get_prim(sm), get_prim(s0), get_prim(sp), nu, plus, minus);
#pragma unroll
            for (int q = 0; q < 4; ++q) S.f[q][s0] = plus[q];
        }
        __syncthreads();
        // stage 3: Riemann problem and flux at interface p-1/2
        if (act) {
            T L[4], G[4], F[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) L[q] = S.f[q][sm];
            riemann_T<T, G14>(L, minus, g, a.niter, G, a.newton_all);
            euler_flux(G, g, F);
#pragma unroll
            for (int q = 0; q < 4; ++q) S.F[q][s0] = F[q];
            if (p == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) S.F0[q] = F[q];
            }
            if (a.bc != HFAV_BC_PERIODIC && p == nx - 1) {
                // right ghost cell copies cell nx-1 and has zero slopes, so
                // its minus face is the primitive state of cell nx-1
                T Lr[4], Rr[4], Gr[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) Lr[q] = S.f[q][s0];
                Rr[0] = S.w[0][s0]; Rr[1] = S.w[1][s0]; Rr[2] = S.w[2][s0]; Rr[3] = S.w[3][s0];
                riemann_T<T, G14>(Lr, Rr, g, a.niter, Gr, a.newton_all);
                euler_flux(Gr, g, S.Fn);
            }
        }
        __syncthreads();
        // stage 4: conservative update of cell p-1 (and of cell nx-1 at the end)
        if (act && p >= 1) {
            const size_t o = row + (p - 1);
            // the conserved state of cell p-1 comes back from the cache (the
            // lane two to the left loaded it two stages ago)
            v.orho[o] = euler_update(v.rho[o], S.F[0][s0], S.F[0][sm], nuA);
            v.omn[o] = euler_update(v.mn[o], S.F[1][s0], S.F[1][sm], nuA);
            v.omt[o] = euler_update(v.mt[o], S.F[2][s0], S.F[2][sm], nuA);
            v.oE[o] = euler_update(v.E[o], S.F[3][s0], S.F[3][sm], nuA);
        }
        if (act && p == nx - 1) {
            const size_t o = row + p;
            const T *Fp = a.bc == HFAV_BC_PERIODIC ? S.F0 : S.Fn;
            v.orho[o] = euler_update(v.rho[o], Fp[0], S.F[0][s0], nuA);
            v.omn[o] = euler_update(v.mn[o], Fp[1], S.F[1][s0], nuA);
            v.omt[o] = euler_update(v.mt[o], Fp[2], S.F[2][s0], nuA);
            v.oE[o] = euler_update(v.E[o], Fp[3], S.F[3][s0], nuA);
        }
    }
}

template <class T, class A, bool G14, int B, int WPE>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(WPE))) void euler_x_kernel(EArgs<T> a) {
    __shared__ XLds<T, B> S;
    x_row<T, A, G14, B>(a, full_view(a), blockIdx.x, read_dt(a.dt_src, a.dt_mode, a.cfl), S);
}

// ------------------------------------------------------------------ y pass
// Sweep one tile (columns i0 .. i0+B-1, rows j0 .. j1-1) along y.  Each lane
// keeps the conserved state of its last three cells in its own LDS slots
// (read back two rows later by the update).  Returns the lane's largest
// signal speed of the updated cells (0 when want_smax is false).
template <class T, class A, bool G14, int B>
__device__ __forceinline__ double y_tile(const EArgs<T> &a, const EView<T> &v, int i0, int j0, int j1, double dt,
                                         bool want_smax, T (*s_u)[4][B]) {
    const int nx = v.nx, ny = v.ny;
    const int t = threadIdx.x;
    const int i = i0 + t;
    const T g = G14 ? T(1.4) : (T)a.g;     // gamma 7/5: constants fold
    const T nu = (T)dt;
    const A nuA = (A)dt;
    double smax = 0.0;
    if (i < nx) {
        auto P = [&](int jj, int slot) {
            const size_t o = (size_t)bwrap(jj, ny, a.bc) * nx + i;
            const T r = v.rho[o], mn = v.mn[o], mt = v.mt[o], e = v.E[o];
            if (slot >= 0) {
                s_u[slot][0][t] = r; s_u[slot][1][t] = mn; s_u[slot][2][t] = mt; s_u[slot][3][t] = e;
            }
            return euler_prim(r, mn, mt, e, g);
        };
        Prim<T> w0 = P(j0 - 2, -1), w1 = P(j0 - 1, -1), w2 = P(j0, 0);
        T fp[4], Fm[4];
        {
            T minus[4];
            slope_trace(w0, w1, w2, nu, fp, minus);     // plus face of cell j0-1
        }
        // window: w1 = cell j-1, w2 = cell j; cell j0 + m sits in slot m % 3
        int snew = 1;                                   // slot of cell j+1
        for (int j = j0; j <= j1; ++j) {
            const Prim<T> w3 = P(j + 1, snew);
            T plus[4], minus[4], G[4], F[4];
            slope_trace(w1, w2, w3, nu, plus, minus);
            riemann_T<T, G14>(fp, minus, g, a.niter, G, a.newton_all);
            euler_flux(G, g, F);                         // flux at j-1/2
            if (j > j0) {
                const int su = snew == 2 ? 0 : snew + 1; // slot of cell j-1
                const size_t o = (size_t)(j - 1) * nx + i;
                const T r = euler_update(s_u[su][0][t], F[0], Fm[0], nuA);
                const T mn = euler_update(s_u[su][1][t], F[1], Fm[1], nuA);
                const T mt = euler_update(s_u[su][2][t], F[2], Fm[2], nuA);
                const T e = euler_update(s_u[su][3][t], F[3], Fm[3], nuA);
                v.orho[o] = r; v.omn[o] = mn; v.omt[o] = mt; v.oE[o] = e;
                if (want_smax) smax = fmax(smax, (double)euler_speed(r, mt, mn, e, g));
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) { Fm[q] = F[q]; fp[q] = plus[q]; }
            w1 = w2;
            w2 = w3;
            snew = snew == 2 ? 0 : snew + 1;
        }
    }
    return smax;
}

template <class T, class A, bool G14, int B, int WPE>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(WPE))) void euler_y_kernel(EArgs<T> a) {
    __shared__ T s_u[3][4][B];
    const int nx = a.nx, ny = a.ny;
    // logical tile: column tile fastest, then row segment
    const int ntx = (nx + B - 1) / B, nsg = (ny + a.seg - 1) / a.seg;
    const int tile = xcd_tile(blockIdx.x, ntx * nsg, a.xcd);
    const int i0 = (tile % ntx) * B;
    const int j0 = (tile / ntx) * a.seg;
    const int j1 = min(j0 + a.seg, ny);
    const double smax = y_tile<T, A, G14, B>(a, full_view(a), i0, j0, j1, read_dt(a.dt_src, a.dt_mode, a.cfl),
                                             a.smax_out != nullptr, s_u);
    if (a.smax_out) block_max_to<B>(smax, a.smax_out);
}

// ------------------------------------------------------------------ strip pass
// Either direction: a workgroup of W x C lanes sweeps W adjacent lines (rows
// for x, columns for y; lane w of a chunk row handles line line0 + w) over
// the cells j0 .. j1-1 of each line, C cells of every line per chunk.
// Neighbours along the sweep are other lanes, so the contracted windows are
// LDS rings (primitive state 3 cells, plus-face state 2 cells, flux 2
// interfaces), each value produced once; the segment recomputes two halo
// cells and one interface at its start.  With W = 64 along x for the y pass,
// every global access of a wave is one coalesced 512-byte row piece.
template <class T, int W, int C>
struct SLds {
    static constexpr int RW = C + 2;    // cells c0-1 .. c0+C
    static constexpr int RF = C + 2;    // cells c0-2 .. c0+C-1
    T w[5][RW][W];      // primitive state
    // plus-face state of cell p, replaced (once its reader has it) by the
    // flux F(p+1/2): one ring serves both windows
    T fF[4][RF][W];
    // conserved state as loaded, for the update two cells behind (another
    // lane's load: through LDS instead of a second read through the caches)
    T u[4][RW][W];
};

// index along the sweep with the boundary applied (division only off the grid)
__device__ __forceinline__ int wrap_cell(int i, int n, int bc) {
    return (unsigned)i < (unsigned)n ? i : bwrap(i, n, bc);
}

// In place (IP), a segment [j0, j1) of a line writes only its own cells but
// reads cells j0-2 .. j1+1: the two cells before it and the two after it
// belong to the neighbouring segments (with a periodic wrap, the first and
// the last segment are neighbours; a single segment wraps onto itself), which
// may already have written them.  Those reads come from the copy saved
// before the sweep (a.halo).  A read that a transmissive end clamps onto a
// cell of the segment itself stays direct (it comes before the segment
// writes that cell); so do the reads of the segment's own cells, each made
// before the cell is written (the update of cell p-1 reads it in the same
// statement).
template <class T, class A, bool G14, int W, int C, bool IP = false>
__device__ __forceinline__ double strip(const EArgs<T> &a, const EView<T> &v, bool xdir, int line0, int j0, int j1,
                                        double dt, bool want_smax, SLds<T, W, C> &S) {
    using L = SLds<T, W, C>;
    static_assert(L::RW == L::RF, "one slot index serves both rings");
    // with W = 64 a wave sweeps one cell of each of 64 lines: q is uniform
    // over the wave, and the slot arithmetic below stays scalar
    const int t = threadIdx.x, wl = t % W;
    const int q = W == 64 ? __builtin_amdgcn_readfirstlane(t / W) : t / W;
    const int n = xdir ? v.nx : v.ny;
    const int nlines = xdir ? v.ny : v.nx;
    const bool lact = line0 + wl < nlines;
    const size_t sa = xdir ? (size_t)1 : (size_t)v.nx;          // stride along the sweep
    const size_t lb = (size_t)(line0 + wl) * (xdir ? (size_t)v.nx : (size_t)1);
    const T g = G14 ? T(1.4) : (T)a.g;     // gamma 7/5: constants fold
    const T nu = (T)dt;
    const A nuA = (A)dt;
    double smax = 0.0;
    auto addr = [&](int cell) { return lb + (size_t)wrap_cell(cell, n, a.bc) * sa; };
    // conserved state of a cell (unwrapped index along the sweep)
    auto load_u = [&](int cell, T *u) {
        const int wc = wrap_cell(cell, n, a.bc);
        if (IP && (cell < j0 || cell >= j1) && (a.bc == HFAV_BC_PERIODIC || wc < j0 || wc >= j1)) {
            const int s0 = j0 / a.seg;
            const int sb = cell < j0 ? s0 : (s0 + 1 == a.nsg ? 0 : s0 + 1);     // boundary
            const int c = cell < j0 ? cell - (j0 - 2) : 2 + (cell - j1);        // cell slot 0..3
            const size_t fs = (size_t)a.nsg * 4 * nlines;                        // field stride
            const size_t h = ((size_t)sb * 4 + c) * nlines + (line0 + wl);
            u[0] = a.halo[h]; u[1] = a.halo[fs + h]; u[2] = a.halo[2 * fs + h]; u[3] = a.halo[3 * fs + h];
            return;
        }
        const size_t o = lb + (size_t)wc * sa;
        u[0] = v.rho[o]; u[1] = v.mn[o]; u[2] = v.mt[o]; u[3] = v.E[o];
    };
    // ring slot of a cell (both rings: cell - j0 + 2 modulo C + 2)
    auto fs = [&](int cell) { return (cell - j0 + 2) % L::RF; };
    auto put = [&](int sl, const Prim<T> &w) {
        S.w[0][sl][wl] = w.r; S.w[1][sl][wl] = w.un; S.w[2][sl][wl] = w.ut; S.w[3][sl][wl] = w.p;
        S.w[4][sl][wl] = w.c;
    };
    auto get = [&](int sl) {
        Prim<T> w;
        w.r = S.w[0][sl][wl]; w.un = S.w[1][sl][wl]; w.ut = S.w[2][sl][wl]; w.p = S.w[3][sl][wl];
        w.c = S.w[4][sl][wl];
        return w;
    };

    __syncthreads();            // a previous segment of a persistent loop is done with the rings
    // prologue: cells j0-2, j0-1, j0 (C may be below 3) and the plus face of
    // cell j0-1
    for (int k = q; lact && k < 3; k += C) {
        T u0[4];
        load_u(j0 - 2 + k, u0);
        put(fs(j0 - 2 + k), euler_prim(u0[0], u0[1], u0[2], u0[3], g));
        if (k == 2) {
#pragma unroll
            for (int f = 0; f < 4; ++f) S.u[f][fs(j0)][wl] = u0[f];
        }
    }
    __syncthreads();
    if (lact && q == 0) {
        T plus[4], minus[4];
        slope_trace(get(fs(j0 - 2)), get(fs(j0 - 1)), get(fs(j0)), nu, plus, minus);
        const int sl = fs(j0 - 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) S.fF[k][sl][wl] = plus[k];
    }
    // the ring holds C + 2 cells: the first chunk's cell j0 + C takes the
    // slot of cell j0 - 2, which the reads just above must be done with
    __syncthreads();
    for (int c0 = j0; c0 <= j1; c0 += C) {
        const int p = c0 + q;
        const bool act = lact && p <= j1;
        // slot of cell p + d for d in [-2, 1], from the chunk's base slot
        // (wave-uniform) with one wrap each way instead of a division
        const int wb = (c0 - j0 + 2) % L::RW;
        auto sl = [&](int d) {
            int s = wb + q + d;
            s -= s >= L::RW ? L::RW : 0;
            return s < 0 ? s + L::RW : s;
        };
        // stage 1: the cell entering the window.  The previous chunk read
        // these primitive slots in its stage 2, and two barriers have
        // passed since (the prologue's reads: the barrier before the loop)
        T un[4];
        if (act) load_u(p + 1, un);
        if (act) {
            const int s1 = sl(1);
            put(s1, euler_prim(un[0], un[1], un[2], un[3], g));
#pragma unroll
            for (int f = 0; f < 4; ++f) S.u[f][s1][wl] = un[f];
        }
        __syncthreads();
        // stage 2: slopes and trace of cell p; the plus face goes to the
        // lane of cell p+1 through LDS, the minus face stays in registers
        T minus[4];
        if (act) {
            T plus[4];
            slope_trace(get(sl(-1)), get(sl(0)), get(sl(1)), nu, plus, minus);
            const int s0 = sl(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) S.fF[k][s0][wl] = plus[k];
        }
        __syncthreads();
        // stage 3: Riemann problem and flux at interface p-1/2; the flux
        // takes the slot of the plus face of cell p-1, whose only reader is
        // this lane (just above), so no barrier separates the two
        T Lf[4];
        if (act) {
            const int sm = sl(-1);
#pragma unroll
            for (int k = 0; k < 4; ++k) Lf[k] = S.fF[k][sm][wl];
        }
        if (act) {
            T G[4], F[4];
            riemann_T<T, G14>(Lf, minus, g, a.niter, G, a.newton_all);
            euler_flux(G, g, F);
            const int sm = sl(-1);
#pragma unroll
            for (int k = 0; k < 4; ++k) S.fF[k][sm][wl] = F[k];
        }
        __syncthreads();
        // stage 4: conservative update of cell p-1 (inside the grid: no wrap)
        // from F(p-1/2) (slot of p-1) and F(p-3/2) (slot of p-2); the state
        // of p-1 from its slot of the conserved-state ring, which the next
        // chunk's stage 1 of this same lane is the first to overwrite
        if (act && p > j0) {
            const size_t o = lb + (size_t)(p - 1) * sa;
            const int s1 = sl(-1), s2 = sl(-2);
            const T r = euler_update(S.u[0][s1][wl], S.fF[0][s1][wl], S.fF[0][s2][wl], nuA);
            const T mn = euler_update(S.u[1][s1][wl], S.fF[1][s1][wl], S.fF[1][s2][wl], nuA);
            const T mt = euler_update(S.u[2][s1][wl], S.fF[2][s1][wl], S.fF[2][s2][wl], nuA);
            const T e = euler_update(S.u[3][s1][wl], S.fF[3][s1][wl], S.fF[3][s2][wl], nuA);
            v.orho[o] = r; v.omn[o] = mn; v.omt[o] = mt; v.oE[o] = e;
            if (want_smax) smax = fmax(smax, (double)euler_speed(r, mt, mn, e, g));
        }
    }
    return smax;
}

// x pass as strips: one workgroup per segment of a.seg cells of W adjacent
// rows (C = block / W lanes along each row); a segment recomputes two halo
// cells and one interface at its start, like a y segment.  W = 2 with one
// wave (32 cells of 2 rows per chunk) gives each wave a more compact patch
// of interfaces than W = 1.
template <class T, class A, bool G14, int W, int C, bool IP = false>
__global__ __launch_bounds__(W * C) __attribute__((amdgpu_waves_per_eu(4))) void euler_x_strip_kernel(EArgs<T> a) {
    __shared__ SLds<T, W, C> S;
    const int nsg = (a.nx + a.seg - 1) / a.seg, nb = (a.ny + W - 1) / W;
    const int tile = xcd_tile(blockIdx.x, nb * nsg, a.xcd);
    const int j = (tile / nsg) * W, i0 = (tile % nsg) * a.seg;
    strip<T, A, G14, W, C, IP>(a, full_view(a), true, j, i0, min(i0 + a.seg, a.nx),
                               read_dt(a.dt_src, a.dt_mode, a.cfl), false, S);
}

// y pass as strips: W columns x C rows per chunk (W * C lanes), segments of
// a.seg rows.  A wave holds 64 / W rows of W columns: narrower tiles make
// each wave's cells a more compact patch and a chunk cover more rows (fewer
// barriers per cell); every row piece a wave reads stays W * 8 >= 128 bytes
// for FP64.
template <class T, class A, bool G14, int W, int C, bool IP = false>
__global__ __launch_bounds__(W * C) __attribute__((amdgpu_waves_per_eu(4))) void euler_y_strip_kernel(EArgs<T> a) {
    __shared__ SLds<T, W, C> S;
    const int ntx = (a.nx + W - 1) / W, nsg = (a.ny + a.seg - 1) / a.seg;
    const int tile = xcd_tile(blockIdx.x, ntx * nsg, a.xcd);
    const int i0 = (tile % ntx) * W;
    const int j0 = (tile / ntx) * a.seg;
    const int j1 = min(j0 + a.seg, a.ny);
    const double smax = strip<T, A, G14, W, C, IP>(a, full_view(a), false, i0, j0, j1,
                                                   read_dt(a.dt_src, a.dt_mode, a.cfl), a.smax_out != nullptr, S);
    if (a.smax_out) block_max_to<W * C>(smax, a.smax_out);
}

// Saves the state of the cells b-2 .. b+1 around every segment boundary
// b = s * seg (s < nsg) of every line, boundary applied, for an in-place
// sweep (layout [field][s][cell][line]: consecutive threads take
// consecutive lines, contiguous in memory for the y sweep).
template <class T>
__global__ __launch_bounds__(256) void euler_halo_save_kernel(EArgs<T> a, int xdir, T *halo) {
    const int n = xdir ? a.nx : a.ny, nlines = xdir ? a.ny : a.nx;
    const size_t per_field = (size_t)a.nsg * 4 * nlines;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < 4 * per_field; q += (size_t)gridDim.x * 256) {
        const int f = (int)(q / per_field);
        const size_t r = q - (size_t)f * per_field;
        const int line = (int)(r % nlines);
        const int sc = (int)(r / nlines), c = sc & 3, sg = sc >> 2;
        const int cell = bwrap(sg * a.seg - 2 + c, n, a.bc);
        const size_t o = xdir ? (size_t)line * a.nx + cell : (size_t)cell * a.nx + line;
        const T *src = f == 0 ? a.rho : f == 1 ? a.mn : f == 2 ? a.mt : a.E;
        halo[q] = src[o];
    }
}

// ------------------------------------------------------------------ batches
// Many independent grids in packed buffers: grid g's plane q starts at
// base + off_g with off_g the sum of nx*ny over the grids before it.  A
// persistent pool of workgroups walks the work items of all grids in
// grid-stride order; items of one grid are contiguous, so each workgroup
// finds the grid of its next item by advancing a monotone cursor over the
// per-grid sizes held in the kernel arguments (no device table).  Every grid
// has its own dt (from its own smax slot) and its own CFL reduction slot.
struct BatchDims {
    int n;
    unsigned short nx[HFAV_MAX_BATCH], ny[HFAV_MAX_BATCH];
    unsigned char seg[HFAV_MAX_BATCH];   // y-pass segment length per grid
};

struct Cursor {
    int g;          // current grid
    long long base; // first item of grid g
    long long off;  // element offset of grid g in the packed buffers
};

template <class F>
__device__ __forceinline__ void advance(Cursor &c, long long item, const BatchDims &d, F count) {
    while (c.g < d.n && item >= c.base + count(c.g)) {
        c.base += count(c.g);
        c.off += (long long)d.nx[c.g] * d.ny[c.g];
        ++c.g;
    }
}

template <class T>
__device__ __forceinline__ EView<T> grid_view(const EArgs<T> &a, const BatchDims &d, const Cursor &c) {
    return EView<T>{a.rho + c.off, a.mn + c.off, a.mt + c.off, a.E + c.off,
                    a.orho + c.off, a.omn + c.off, a.omt + c.off, a.oE + c.off, d.nx[c.g], d.ny[c.g]};
}

// x items: segments of BATCH_XSEG cells of two rows, one wave each (the
// strip body with W = 2, C = 32, as the single-grid x sweep's default: each
// wave on a compact patch of 32 cells x 2 rows)
constexpr int BATCH_XSEG = 191, BATCH_XROWS = 2, BATCH_YCOLS = 16;

__device__ __forceinline__ long long pool_x_items(const BatchDims &d, int g) {
    return (long long)((d.ny[g] + BATCH_XROWS - 1) / BATCH_XROWS) * ((d.nx[g] + BATCH_XSEG - 1) / BATCH_XSEG);
}

__device__ __forceinline__ long long pool_y_items(const BatchDims &d, int g) {
    return (long long)((d.nx[g] + BATCH_YCOLS - 1) / BATCH_YCOLS) * ((d.ny[g] + d.seg[g] - 1) / d.seg[g]);
}

template <class T, class A, bool G14>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void euler_x_batch_kernel(EArgs<T> a, BatchDims d, long long items) {
    __shared__ SLds<T, BATCH_XROWS, 64 / BATCH_XROWS> S;
    Cursor c{0, 0, 0};
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        advance(c, it, d, [&](int g) { return pool_x_items(d, g); });
        const EView<T> v = grid_view(a, d, c);
        const int nsg = (v.nx + BATCH_XSEG - 1) / BATCH_XSEG;
        const int local = (int)(it - c.base);
        const int j = (local / nsg) * BATCH_XROWS, i0 = (local % nsg) * BATCH_XSEG;
        const double dt = read_dt(a.dt_src + c.g, a.dt_mode, a.cfl);
        strip<T, A, G14, BATCH_XROWS, 64 / BATCH_XROWS>(a, v, true, j, i0, min(i0 + BATCH_XSEG, v.nx), dt, false, S);
    }
}

// y items: tiles of 16 columns x seg[g] rows in chunks of 16 rows (the
// single-grid y sweep's default shape)
template <class T, class A, bool G14>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void euler_y_batch_kernel(EArgs<T> a, BatchDims d, long long items) {
    __shared__ SLds<T, BATCH_YCOLS, 256 / BATCH_YCOLS> S;
    Cursor c{0, 0, 0};
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        advance(c, it, d, [&](int g) { return pool_y_items(d, g); });
        const EView<T> v = grid_view(a, d, c);
        const int ntx = (v.nx + BATCH_YCOLS - 1) / BATCH_YCOLS;
        const int tile = (int)(it - c.base);
        const int i0 = (tile % ntx) * BATCH_YCOLS, j0 = (tile / ntx) * d.seg[c.g];
        const int j1 = min(j0 + (int)d.seg[c.g], v.ny);
        const double dt = read_dt(a.dt_src + c.g, a.dt_mode, a.cfl);
        const double smax = strip<T, A, G14, BATCH_YCOLS, 256 / BATCH_YCOLS>(a, v, false, i0, j0, j1, dt,
                                                                              a.smax_out != nullptr, S);
        if (a.smax_out) block_max_to<256>(smax, a.smax_out + c.g);
    }
}

// ------------------------------------------------------------------ batch step
// Both sweeps of a time step for every grid of a batch in ONE persistent
// launch.  x items: 4 rows x a 191-cell segment (lanes take 4 adjacent rows
// of 64-cell chunks); y items: 64 columns x seg[g] rows, as in the y pool.
// x items write the x-swept state to a workspace copy; a y item of grid g
// reads it once every x item of g has finished.
//
// Every item of a grid runs on ONE XCD, so the x-swept state passes through
// that XCD's L2 only: the 8 L2 caches are not coherent with each other
// within a launch, and making every x item's stores visible to all of them
// (an L2 write-back per x item) tripled the step time.  Before the step the
// grids are dealt to the XCDs in snake order over their sizes, largest
// first (cells balance to within about one small grid), and each XCD has its
// own cursor: a workgroup reads its XCD from the hardware register and draws
// that XCD's items, the x items of its grids before any y item.
//
// Ordering within an XCD: after an x item each wave waits until its stores
// have reached the L2 (vmcnt 0, the release of an agent with one L2), then a
// barrier and one counter increment for the grid; a y item polls its grid's
// counter until it holds the grid's x item count, then every thread acquires
// at device scope (L1 invalidated) before reading.
//
// Progress: an item is only handed to a running workgroup, and the x items a
// y item waits for were handed out before it on the same XCD, so running
// workgroups hold them and finish them without waiting.  The wait is still
// bounded (spin_limit polls): a y item that gives up skips its work, sets
// status bit 0 and writes NaN into its grid's CFL slot.  A workgroup whose
// XCD index is not below the XCD count takes no item (its XCD has no list);
// the last workgroup to finish sets status bit 1 if an XCD's items were not
// all taken (an XCD without workgroups).
struct StepBatch {
    void *w;                        // x-swept state: 4 planes (rho, mx, my, E) of w_stride elements
    long long w_stride;
    unsigned char *ctl;             // control block, zeroed and dealt by the init kernel
    int nxcd;                       // XCDs of the device (1..8)
    int spin_limit;
    unsigned wait_extra;            // added to the awaited count (0; 1 only to test the give-up path)
};

// control block (bytes): status, exit count, per-XCD cursors and x / y item
// totals, per-grid counters (STEP_BATCH_CNT_OFFSET), per-grid XCD
constexpr int SB_STATUS = 0, SB_EXIT = 4, SB_CURSOR = 64, SB_XTOT = 128, SB_YTOT = 192;
constexpr int SB_XCD = (int)STEP_BATCH_CNT_OFFSET + 4 * HFAV_MAX_BATCH;
constexpr int SB_MAX_XCD = 8;
static_assert(SB_XCD + HFAV_MAX_BATCH <= (int)STEP_BATCH_CTL_BYTES, "step control block");

constexpr int STEP_XROWS = 4;

__device__ __forceinline__ long long step_x_items(const BatchDims &d, int g) {
    return (long long)((d.ny[g] + STEP_XROWS - 1) / STEP_XROWS) * ((d.nx[g] + BATCH_XSEG - 1) / BATCH_XSEG);
}

__device__ __forceinline__ long long step_y_items(const BatchDims &d, int g) {
    return (long long)((d.nx[g] + 63) / 64) * ((d.ny[g] + d.seg[g] - 1) / d.seg[g]);
}

// advance a cursor over the grids dealt to XCD k
template <class F>
__device__ __forceinline__ void advance_on(Cursor &c, long long item, const BatchDims &d, const unsigned char *xcd,
                                           int k, F count) {
    while (c.g < d.n && (xcd[c.g] != k || item >= c.base + count(c.g))) {
        if (xcd[c.g] == k) c.base += count(c.g);
        c.off += (long long)d.nx[c.g] * d.ny[c.g];
        ++c.g;
    }
}

template <class T, class A, bool G14>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void euler_step_batch_kernel(
    EArgs<T> a, BatchDims d, StepBatch sb) {
    using LX = SLds<T, STEP_XROWS, 64>;
    using LY = SLds<T, 64, 4>;
    __shared__ __align__(16) unsigned char lds[sizeof(LX) > sizeof(LY) ? sizeof(LX) : sizeof(LY)];
    __shared__ long long s_item;
    __shared__ int s_go;
    LX &SX = *reinterpret_cast<LX *>(lds);
    LY &SY = *reinterpret_cast<LY *>(lds);
    unsigned *status = (unsigned *)(sb.ctl + SB_STATUS);
    unsigned long long *cursor = (unsigned long long *)(sb.ctl + SB_CURSOR);
    const long long *xtot = (const long long *)(sb.ctl + SB_XTOT), *ytot = (const long long *)(sb.ctl + SB_YTOT);
    unsigned *cnt = (unsigned *)(sb.ctl + STEP_BATCH_CNT_OFFSET);
    const unsigned char *xcd = sb.ctl + SB_XCD;
    // XCC_ID hardware register, bits 3:0
    const int k = (int)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
    if (k < sb.nxcd) {
        EArgs<T> ay = a;
        ay.bc = a.bcy;
        T *w = (T *)sb.w;
        const long long ws = sb.w_stride;
        const long long nxi = xtot[k], total = nxi + ytot[k];
        Cursor cx{0, 0, 0}, cy{0, 0, 0};    // the items a workgroup draws increase
        for (;;) {
            __syncthreads();                // everyone has read s_item / s_go of the previous item
            if (threadIdx.x == 0) s_item = (long long)atomicAdd(cursor + k, 1ull);
            __syncthreads();
            const long long it = s_item;
            if (it >= total) break;
            if (it < nxi) {
                advance_on(cx, it, d, xcd, k, [&](int g) { return step_x_items(d, g); });
                const int g = cx.g;
                const long long o = cx.off;
                const EView<T> v{a.rho + o, a.mn + o, a.mt + o, a.E + o,
                                 w + o, w + ws + o, w + 2 * ws + o, w + 3 * ws + o, d.nx[g], d.ny[g]};
                const int nsg = (v.nx + BATCH_XSEG - 1) / BATCH_XSEG;
                const int local = (int)(it - cx.base);
                const int j = (local / nsg) * STEP_XROWS, i0 = (local % nsg) * BATCH_XSEG;
                const double dt = read_dt(a.dt_src + g, a.dt_mode, a.cfl);
                strip<T, A, G14, STEP_XROWS, 64>(a, v, true, j, i0, min(i0 + BATCH_XSEG, v.nx), dt, false, SX);
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt + g, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                advance_on(cy, it - nxi, d, xcd, k, [&](int g) { return step_y_items(d, g); });
                const int g = cy.g;
                if (threadIdx.x == 0) {
                    const unsigned need = (unsigned)step_x_items(d, g) + sb.wait_extra;
                    int polls = 0;
                    bool ok = __hip_atomic_load(cnt + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
                    while (!ok && polls < sb.spin_limit) {
                        __builtin_amdgcn_s_sleep(2);
                        ++polls;
                        ok = __hip_atomic_load(cnt + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
                    }
                    s_go = ok;
                    if (!ok) {
                        atomicOr(status, 1u);
                        if (a.smax_out) atomic_max_nonneg(a.smax_out + g, __longlong_as_double(0x7ff8000000000000ll));
                    }
                }
                __syncthreads();
                if (!s_go) continue;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const long long o = cy.off;
                // y frame: normal momentum my, tangential mx
                const EView<T> v{w + o, w + 2 * ws + o, w + ws + o, w + 3 * ws + o,
                                 a.orho + o, a.omt + o, a.omn + o, a.oE + o, d.nx[g], d.ny[g]};
                const int ntx = (v.nx + 63) / 64;
                const int tile = (int)(it - nxi - cy.base);
                const int i0 = (tile % ntx) * 64, j0 = (tile / ntx) * d.seg[g];
                const int j1 = min(j0 + (int)d.seg[g], v.ny);
                const double dt = read_dt(a.dt_src + g, a.dt_mode, a.cfl);
                const double smax = strip<T, A, G14, 64, 4>(ay, v, false, i0, j0, j1, dt, a.smax_out != nullptr, SY);
                if (a.smax_out) block_max_to<256>(smax, a.smax_out + g);
            }
        }
    }
    // the last workgroup to finish: were all items of every XCD taken?
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add((unsigned *)(sb.ctl + SB_EXIT), 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
            gridDim.x - 1) {
        for (int q = 0; q < sb.nxcd; ++q)
            if (__hip_atomic_load(cursor + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                (unsigned long long)(xtot[q] + ytot[q]))
                atomicOr(status, 2u);
    }
}

// Before each step: zero the status, exit count, cursors, per-grid counters
// and CFL slots, and deal the grids to the XCDs (rank by cells, largest
// first, ties by index; snake order over the ranks) with each XCD's item
// totals.
__global__ __launch_bounds__(256) void step_batch_init_kernel(BatchDims d, unsigned char *ctl, int nxcd, double *smax) {
    __shared__ unsigned long long s_x[SB_MAX_XCD], s_y[SB_MAX_XCD];
    __shared__ long long s_cells[HFAV_MAX_BATCH];
    const int n = d.n, t = threadIdx.x;
    unsigned *w32 = (unsigned *)ctl;
    for (int q = t; q < SB_XTOT / 4; q += 256) w32[q] = 0u;                 // status, exit, cursors
    for (int q = t; q < n; q += 256) w32[STEP_BATCH_CNT_OFFSET / 4 + q] = 0u;
    if (smax)
        for (int q = t; q < n; q += 256) smax[q] = 0.0;
    if (t < SB_MAX_XCD) s_x[t] = s_y[t] = 0ull;
    // the cells of every grid in LDS: the rank loop below reads them all
    for (int g = t; g < n; g += 256) s_cells[g] = (long long)d.nx[g] * d.ny[g];
    __syncthreads();
    for (int g = t; g < n; g += 256) {
        const long long cg = s_cells[g];
        int r = 0;
#pragma unroll 8
        for (int h = 0; h < n; ++h) {
            const long long ch = s_cells[h];
            r += ch > cg || (ch == cg && h < g);
        }
        const int p = r % (2 * nxcd), k = p < nxcd ? p : 2 * nxcd - 1 - p;
        ctl[SB_XCD + g] = (unsigned char)k;
        atomicAdd(&s_x[k], (unsigned long long)step_x_items(d, g));
        atomicAdd(&s_y[k], (unsigned long long)step_y_items(d, g));
    }
    __syncthreads();
    if (t < SB_MAX_XCD) {
        ((long long *)(ctl + SB_XTOT))[t] = (long long)s_x[t];
        ((long long *)(ctl + SB_YTOT))[t] = (long long)s_y[t];
    }
}

template <class T, int B>
__global__ __launch_bounds__(B) void euler_smax_batch_kernel(const T *rho, const T *mx, const T *my, const T *E,
                                                             BatchDims d, double g, double *out) {
    // one workgroup per grid
    long long off = 0;
    for (int h = 0; h < (int)blockIdx.x; ++h) off += (long long)d.nx[h] * d.ny[h];
    const long long n = (long long)d.nx[blockIdx.x] * d.ny[blockIdx.x];
    double m = 0.0;
    for (long long q = threadIdx.x; q < n; q += B)
        m = fmax(m, (double)euler_speed(rho[off + q], mx[off + q], my[off + q], E[off + q], (T)g));
    block_max_to<B>(m, out + blockIdx.x);
}

__global__ void fill_batch_kernel(double *p, int n, double v) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = v;
}

// ------------------------------------------------------------------ smax
template <class T, int B>
__global__ __launch_bounds__(B) void euler_smax_kernel(const T *rho, const T *mx, const T *my,
                                                       const T *E, int n, double g, double *out) {
    double m = 0.0;
    for (int q = blockIdx.x * B + threadIdx.x; q < n; q += gridDim.x * B)
        m = fmax(m, (double)euler_speed(rho[q], mx[q], my[q], E[q], (T)g));
    block_max_to<B>(m, out);
}

__global__ void fill_scalar_kernel(double *p, double v) { *p = v; }
__global__ void dt_from_smax_kernel(const double *smax, double cfl, double *out) { *out = cfl / *smax; }

// ------------------------------------------------------------------ launchers
template <class T>
static EArgs<T> make_args(const EulerLaunch &L) {
    EArgs<T> a;
    a.rho = (const T *)L.in[0]; a.mn = (const T *)L.in[1]; a.mt = (const T *)L.in[2]; a.E = (const T *)L.in[3];
    a.orho = (T *)L.out[0]; a.omn = (T *)L.out[1]; a.omt = (T *)L.out[2]; a.oE = (T *)L.out[3];
    a.nx = L.nx; a.ny = L.ny; a.bc = L.bc;
    a.g = L.gamma; a.niter = L.niter;
    a.dt_src = L.dt_src; a.dt_mode = L.dt_mode; a.cfl = L.cfl;
    a.smax_out = L.smax_out;
    a.seg = L.cfg.seg > 0 ? L.cfg.seg : 16;
    a.xcd = L.cfg.xcd;
    a.newton_all = (L.cfg.variant & EULER_NEWTON_ALL) != 0;
    a.halo = (const T *)L.halo;
    a.nsg = 0;
    return a;
}

int euler_x_strip_rows(const hfav_config &cfg) { return cfg.tile_y > 1 ? cfg.tile_y : 1; }

bool euler_x_strip_ok(const hfav_config &cfg) {
    const int w = euler_x_strip_rows(cfg);
    if (w == 1) return cfg.block == 64 || cfg.block == 128 || cfg.block == 256;
    return w == 2 && cfg.block == 64;
}

int euler_y_strip_cols(const hfav_config &cfg) { return cfg.tile_y > 1 ? cfg.tile_y : 64; }

bool euler_y_strip_ok(const hfav_config &cfg) {
    const int w = euler_y_strip_cols(cfg);
    if (w == 64) return cfg.block == 128 || cfg.block == 256 || cfg.block == 512;
    return (w == 32 || w == 16 || w == 8) && cfg.block == 256;
}

int euler_strip_seg(int n, int dir, const hfav_config &cfg) {
    if (dir == 0) return cfg.seg > 0 && cfg.seg < n ? cfg.seg : n;
    return cfg.seg > 0 ? cfg.seg : 16;
}

size_t euler_inplace_bytes(int nx, int ny, int dir, int dtype, const hfav_config &cfg) {
    const int n = dir == 0 ? nx : ny, nlines = dir == 0 ? ny : nx;
    const size_t nsg = (n + euler_strip_seg(n, dir, cfg) - 1) / euler_strip_seg(n, dir, cfg);
    return 4 * nsg * 4 * (size_t)nlines * (dtype == HFAV_F64 ? 8 : 4);
}

// in place: save the segment-boundary cells, then run the in-place strip
template <class T>
static hipError_t save_halos(EArgs<T> &a, bool xdir, hipStream_t s) {
    const int n = xdir ? a.nx : a.ny, nlines = xdir ? a.ny : a.nx;
    a.nsg = (n + a.seg - 1) / a.seg;
    const size_t total = 4 * (size_t)a.nsg * 4 * nlines;
    const unsigned nb = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL((euler_halo_save_kernel<T>), dim3(nb), dim3(256), 0, s, a, xdir ? 1 : 0,
                       const_cast<T *>(a.halo));
    return hipGetLastError();
}

// The variant sets the occupancy the compiler must reach: 0 leaves the
// register budget free, 1 asks for at least 4 waves per SIMD (at most 128
// VGPRs), 2 for 5 waves (96 VGPRs; the Riemann solver's state partly spills
// to scratch).
#define E_LAUNCH(KER, BB)                                                                     \
    switch (L.cfg.variant & ~EULER_NEWTON_ALL) {                                              \
    case 1: hipLaunchKernelGGL((KER<T, A, G14, BB, 4>), grid, dim3(BB), 0, s, a); break;      \
    case 2: hipLaunchKernelGGL((KER<T, A, G14, BB, 5>), grid, dim3(BB), 0, s, a); break;      \
    default: hipLaunchKernelGGL((KER<T, A, G14, BB, 1>), grid, dim3(BB), 0, s, a); break;     \
    }

template <class T, class A, bool G14>
static hipError_t euler_x_dispatch(const EulerLaunch &L, hipStream_t s) {
    EArgs<T> a = make_args<T>(L);
    dim3 grid(L.ny);
    if ((L.cfg.variant & ~EULER_NEWTON_ALL) == 3) {
        // segments of cfg.seg cells (0: whole rows) of W = tile_y rows (1
        // when tile_y <= 1), block / W lanes along each row
        if (!euler_x_strip_ok(L.cfg)) return hipErrorInvalidValue;
        const int W = euler_x_strip_rows(L.cfg);
        a.seg = euler_strip_seg(L.nx, 0, L.cfg);
        grid = dim3((unsigned)(((L.ny + W - 1) / W) * ((L.nx + a.seg - 1) / a.seg)));
        if (L.halo) {
            if (L.cfg.block != 64) return hipErrorInvalidValue;
            const hipError_t e = save_halos(a, true, s);
            if (e != hipSuccess) return e;
            if (W == 2) hipLaunchKernelGGL((euler_x_strip_kernel<T, A, G14, 2, 32, true>), grid, dim3(64), 0, s, a);
            else hipLaunchKernelGGL((euler_x_strip_kernel<T, A, G14, 1, 64, true>), grid, dim3(64), 0, s, a);
            return hipGetLastError();
        }
        switch (W * 1024 + L.cfg.block) {
        case 2 * 1024 + 64: hipLaunchKernelGGL((euler_x_strip_kernel<T, A, G14, 2, 32>), grid, dim3(64), 0, s, a); break;
        case 1 * 1024 + 128: hipLaunchKernelGGL((euler_x_strip_kernel<T, A, G14, 1, 128>), grid, dim3(128), 0, s, a); break;
        case 1 * 1024 + 256: hipLaunchKernelGGL((euler_x_strip_kernel<T, A, G14, 1, 256>), grid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((euler_x_strip_kernel<T, A, G14, 1, 64>), grid, dim3(64), 0, s, a); break;
        }
        return hipGetLastError();
    }
    if (L.halo) return hipErrorInvalidValue;      // in place: strip kernels only
    switch (L.cfg.block) {
    case 64: E_LAUNCH(euler_x_kernel, 64); break;
    case 128: E_LAUNCH(euler_x_kernel, 128); break;
    default: E_LAUNCH(euler_x_kernel, 256); break;
    }
    return hipGetLastError();
}

template <class T, class A, bool G14>
static hipError_t euler_y_dispatch(const EulerLaunch &L, hipStream_t s) {
    EArgs<T> a = make_args<T>(L);
    if ((L.cfg.variant & ~EULER_NEWTON_ALL) == 3) {
        // W = tile_y columns per workgroup (64 when tile_y <= 1), block / W
        // rows per chunk
        const int W = euler_y_strip_cols(L.cfg);
        if (!euler_y_strip_ok(L.cfg)) return hipErrorInvalidValue;
        dim3 grid(((L.nx + W - 1) / W) * ((L.ny + a.seg - 1) / a.seg));
        if (L.halo) {
            if (L.cfg.block != 256) return hipErrorInvalidValue;
            const hipError_t e = save_halos(a, false, s);
            if (e != hipSuccess) return e;
            if (W == 16) hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 16, 16, true>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 64, 4, true>), grid, dim3(256), 0, s, a);
            return hipGetLastError();
        }
        switch (W * 1024 + L.cfg.block) {
        case 64 * 1024 + 128: hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 64, 2>), grid, dim3(128), 0, s, a); break;
        case 64 * 1024 + 512: hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 64, 8>), grid, dim3(512), 0, s, a); break;
        case 32 * 1024 + 256: hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 32, 8>), grid, dim3(256), 0, s, a); break;
        case 16 * 1024 + 256: hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 16, 16>), grid, dim3(256), 0, s, a); break;
        case 8 * 1024 + 256: hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 8, 32>), grid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((euler_y_strip_kernel<T, A, G14, 64, 4>), grid, dim3(256), 0, s, a); break;
        }
        return hipGetLastError();
    }
    if (L.halo) return hipErrorInvalidValue;      // in place: strip kernels only
    const int B = (L.cfg.block == 64 || L.cfg.block == 128 || L.cfg.block == 256) ? L.cfg.block : 64;
    dim3 grid(((L.nx + B - 1) / B) * ((L.ny + a.seg - 1) / a.seg));
    switch (B) {
    case 128: E_LAUNCH(euler_y_kernel, 128); break;
    case 256: E_LAUNCH(euler_y_kernel, 256); break;
    default: E_LAUNCH(euler_y_kernel, 64); break;
    }
    return hipGetLastError();
}
#undef E_LAUNCH

template <bool X>
static hipError_t euler_dispatch(const EulerLaunch &L, hipStream_t s) {
    const bool g14 = L.gamma == 1.4;
    if (L.dtype == HFAV_F64) {
        if (g14) return X ? euler_x_dispatch<double, double, true>(L, s) : euler_y_dispatch<double, double, true>(L, s);
        return X ? euler_x_dispatch<double, double, false>(L, s) : euler_y_dispatch<double, double, false>(L, s);
    }
    if (L.precision == HFAV_PREC_F32_F64ACC) {
        if (g14) return X ? euler_x_dispatch<float, double, true>(L, s) : euler_y_dispatch<float, double, true>(L, s);
        return X ? euler_x_dispatch<float, double, false>(L, s) : euler_y_dispatch<float, double, false>(L, s);
    }
    if (g14) return X ? euler_x_dispatch<float, float, true>(L, s) : euler_y_dispatch<float, float, true>(L, s);
    return X ? euler_x_dispatch<float, float, false>(L, s) : euler_y_dispatch<float, float, false>(L, s);
}

hipError_t launch_euler_x(const EulerLaunch &L, hipStream_t s) { return euler_dispatch<true>(L, s); }
hipError_t launch_euler_y(const EulerLaunch &L, hipStream_t s) { return euler_dispatch<false>(L, s); }

hipError_t launch_euler_smax(const void *const *U, int n, double gamma, double *out, int dtype,
                             hipStream_t s) {
    const int B = 256;
    int nb = (n + B - 1) / B;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    if (dtype == HFAV_F64)
        hipLaunchKernelGGL((euler_smax_kernel<double, B>), dim3(nb), dim3(B), 0, s,
                           (const double *)U[0], (const double *)U[1], (const double *)U[2],
                           (const double *)U[3], n, gamma, out);
    else
        hipLaunchKernelGGL((euler_smax_kernel<float, B>), dim3(nb), dim3(B), 0, s,
                           (const float *)U[0], (const float *)U[1], (const float *)U[2],
                           (const float *)U[3], n, gamma, out);
    return hipGetLastError();
}

hipError_t launch_fill_scalar(double *p, double v, hipStream_t s) {
    hipLaunchKernelGGL(fill_scalar_kernel, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_dt_from_smax(const double *smax, double cfl, double *out, hipStream_t s) {
    hipLaunchKernelGGL(dt_from_smax_kernel, dim3(1), dim3(1), 0, s, smax, cfl, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batch launchers
static BatchDims make_dims(const EulerBatch &Bt) {
    BatchDims d;
    d.n = Bt.n;
    for (int g = 0; g < Bt.n; ++g) {
        d.nx[g] = (unsigned short)Bt.nx[g];
        d.ny[g] = (unsigned short)Bt.ny[g];
        d.seg[g] = (unsigned char)Bt.seg[g];
    }
    return d;
}

template <class T, class A, bool G14>
static hipError_t batch_dispatch(const EulerLaunch &L, const EulerBatch &Bt, bool x, hipStream_t s) {
    EArgs<T> a = make_args<T>(L);
    const BatchDims d = make_dims(Bt);
    long long items = 0;
    for (int g = 0; g < Bt.n; ++g) {
        if (Bt.seg[g] < 1) return hipErrorInvalidValue;
        items += x ? (long long)((Bt.ny[g] + BATCH_XROWS - 1) / BATCH_XROWS) * ((Bt.nx[g] + BATCH_XSEG - 1) / BATCH_XSEG)
                   : (long long)((Bt.nx[g] + BATCH_YCOLS - 1) / BATCH_YCOLS) * ((Bt.ny[g] + Bt.seg[g] - 1) / Bt.seg[g]);
    }
    // resident pool: 4 waves per SIMD on 256 CUs (the register budget at
    // which the sweep bodies run without spilling: at 5 waves the unrolled
    // Newton loop spilled 72-84 bytes per lane and a step took 17.1-17.3 ms
    // against 15.6), as one-wave x workgroups or four-wave y workgroups
    const long long cap = (long long)(Bt.workgroups > 0 ? Bt.workgroups : (x ? 256 * 16 : 256 * 4));
    const unsigned nwg = (unsigned)(items < cap ? items : cap);
    if (nwg == 0) return hipSuccess;
    if (x) hipLaunchKernelGGL((euler_x_batch_kernel<T, A, G14>), dim3(nwg), dim3(64), 0, s, a, d, items);
    else hipLaunchKernelGGL((euler_y_batch_kernel<T, A, G14>), dim3(nwg), dim3(256), 0, s, a, d, items);
    return hipGetLastError();
}

hipError_t launch_euler_batch(const EulerLaunch &L, const EulerBatch &Bt, bool x, hipStream_t s) {
    if (Bt.n < 1 || Bt.n > HFAV_MAX_BATCH) return hipErrorInvalidValue;
    const bool g14 = L.gamma == 1.4;
    if (L.dtype == HFAV_F64)
        return g14 ? batch_dispatch<double, double, true>(L, Bt, x, s) : batch_dispatch<double, double, false>(L, Bt, x, s);
    if (L.precision == HFAV_PREC_F32_F64ACC)
        return g14 ? batch_dispatch<float, double, true>(L, Bt, x, s) : batch_dispatch<float, double, false>(L, Bt, x, s);
    return g14 ? batch_dispatch<float, float, true>(L, Bt, x, s) : batch_dispatch<float, float, false>(L, Bt, x, s);
}

// workspace of the one-launch batch step: the control block, then the
// x-swept state as 4 planes, each padded to 256 bytes
static size_t step_batch_plane(long long cells, int dtype) {
    const size_t es = dtype == HFAV_F64 ? 8 : 4;
    return ((size_t)cells * es + 255) / 256 * 256;
}

size_t step_batch_ws_bytes(long long cells, int dtype) {
    return STEP_BATCH_CTL_BYTES + 4 * step_batch_plane(cells, dtype);
}

// XCDs of the current device: 32 compute units each on gfx950 (1 to 8)
static int device_xcds() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int x = cus / 32;
    return x < 1 ? 1 : (x > SB_MAX_XCD ? SB_MAX_XCD : x);
}

template <class T, class A, bool G14>
static hipError_t step_batch_dispatch(const EulerLaunch &L, const EulerBatch &Bt, void *ws, int spin_limit,
                                      unsigned wait_extra, hipStream_t s) {
    EArgs<T> a = make_args<T>(L);
    a.bcy = L.bcy;
    const BatchDims d = make_dims(Bt);
    StepBatch sb;
    long long cells = 0;
    for (int g = 0; g < Bt.n; ++g) {
        if (Bt.seg[g] < 1) return hipErrorInvalidValue;
        cells += (long long)Bt.nx[g] * Bt.ny[g];
    }
    sb.nxcd = device_xcds();
    if (sb.nxcd < 1) return hipErrorInvalidDevice;
    sb.ctl = (unsigned char *)ws;
    sb.w = (char *)ws + STEP_BATCH_CTL_BYTES;
    sb.w_stride = (long long)(step_batch_plane(cells, L.dtype) / sizeof(T));
    sb.spin_limit = spin_limit;
    sb.wait_extra = wait_extra;
    hipLaunchKernelGGL(step_batch_init_kernel, dim3(1), dim3(256), 0, s, d, sb.ctl, sb.nxcd, L.smax_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // resident pool: 4 four-wave workgroups per CU (4 waves per SIMD),
    // dealt round robin to the XCDs by the hardware (a workgroup without an
    // item left on its XCD exits at once); progress does not depend on it
    const unsigned nwg = (unsigned)(Bt.workgroups > 0 ? Bt.workgroups : 256 * 4);
    hipLaunchKernelGGL((euler_step_batch_kernel<T, A, G14>), dim3(nwg), dim3(256), 0, s, a, d, sb);
    return hipGetLastError();
}

hipError_t launch_euler_step_batch(const EulerLaunch &L, const EulerBatch &Bt, void *ws, int spin_limit,
                                   unsigned wait_extra, hipStream_t s) {
    if (Bt.n < 1 || Bt.n > HFAV_MAX_BATCH || !ws || spin_limit < 0) return hipErrorInvalidValue;
    const bool g14 = L.gamma == 1.4;
    if (L.dtype == HFAV_F64)
        return g14 ? step_batch_dispatch<double, double, true>(L, Bt, ws, spin_limit, wait_extra, s)
                   : step_batch_dispatch<double, double, false>(L, Bt, ws, spin_limit, wait_extra, s);
    if (L.precision == HFAV_PREC_F32_F64ACC)
        return g14 ? step_batch_dispatch<float, double, true>(L, Bt, ws, spin_limit, wait_extra, s)
                   : step_batch_dispatch<float, double, false>(L, Bt, ws, spin_limit, wait_extra, s);
    return g14 ? step_batch_dispatch<float, float, true>(L, Bt, ws, spin_limit, wait_extra, s)
               : step_batch_dispatch<float, float, false>(L, Bt, ws, spin_limit, wait_extra, s);
}

hipError_t launch_euler_smax_batch(const void *const *U, const EulerBatch &Bt, double gamma, double *out, int dtype,
                                   hipStream_t s) {
    if (Bt.n < 1 || Bt.n > HFAV_MAX_BATCH) return hipErrorInvalidValue;
    const BatchDims d = make_dims(Bt);
    if (dtype == HFAV_F64)
        hipLaunchKernelGGL((euler_smax_batch_kernel<double, 256>), dim3(Bt.n), dim3(256), 0, s,
                           (const double *)U[0], (const double *)U[1], (const double *)U[2], (const double *)U[3],
                           d, gamma, out);
    else
        hipLaunchKernelGGL((euler_smax_batch_kernel<float, 256>), dim3(Bt.n), dim3(256), 0, s,
                           (const float *)U[0], (const float *)U[1], (const float *)U[2], (const float *)U[3],
                           d, gamma, out);
    return hipGetLastError();
}

hipError_t launch_fill_batch(double *p, int n, double v, hipStream_t s) {
    hipLaunchKernelGGL(fill_batch_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace hfav
