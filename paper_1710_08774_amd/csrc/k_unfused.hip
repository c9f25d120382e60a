// Unfused execution: one kernel per rule over the full iteration space,
// every intermediate a full array in HBM (the starting point the paper
// transforms: Design, "Dataflow"; the "autovec" baselines of the Performance
// section).  Each kernel evaluates the same device rule body as the fused
// families, one lane per cell, reading every input reference at its offset
// with the boundary applied as index arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "ops.h"
#include "xcd.h"

namespace hfav {

// rows (cells along i at one j) of one plane k that a workgroup of the
// rule kernels walks
constexpr int UF_ROWS = 8;

struct UArgs {
    const void *in[UF_MAX_IN];
    int off[UF_MAX_IN][3];
    long long shift[UF_MAX_IN];       // elements from a cell to reference r when no wrap applies:
                                      // (dk * ny + dj) * nx (the i offset is added per lane)
    void *out[UF_MAX_OUT];
    double param[UF_MAX_PARAM];
    int nx, ny, nz;
    int bc[3];
    int n_in;
    int brow;                         // in[1] is a row term (broadcast along i)
    int ntx;                          // 256-cell pieces per row
    int nrb;                          // row blocks per plane: ceil(ny / UF_ROWS)
    int nblk;                         // workgroups: ntx * nrb * nz
    int wide;                         // bit a: some |offset| along axis a reaches a whole axis
    int djmin, djmax, dkmin, dkmax;   // offset ranges along j and k over the references
};

// general wrap (any offset)
__device__ __forceinline__ int uwrap(int i, int n, int bc) {
    if (bc == HFAV_BC_PERIODIC) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
// wrap for -n <= i < 2n: one compare and select per side
__device__ __forceinline__ int xwrap(int i, int n, int bc) {
    if (bc == HFAV_BC_PERIODIC) {
        i = i < 0 ? i + n : i;
        return i >= n ? i - n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
__device__ __forceinline__ int awrap(int i, int n, int bc, bool wide) {
    return wide ? uwrap(i, n, bc) : xwrap(i, n, bc);
}

// The cells of a lane: workgroup w covers 256 cells along i of UF_ROWS
// consecutive rows of one plane; workgroups are ordered so that every XCD
// walks one contiguous range of row blocks (neighbouring rows share its L2).
// A block whose rows and plane reach no boundary through any reference
// ("interior": all but the first and last blocks of a plane for the usual
// stencils, and no offset along i as long as a row) reads reference r at the
// fixed element shift[r] plus the lane's wrapped i; the others wrap j and k
// per reference and row.
struct UCell {
    int i, j, k;
    int row;                          // k * ny + j
};
__device__ __forceinline__ UCell ucell0(const UArgs &a, int &j1, bool &interior) {
    const int w = xcd_tile((int)blockIdx.x, a.nblk, -1);
    const int t = w / a.ntx;                  // row block over (k, block of j)
    UCell c;
    c.i = (w - t * a.ntx) * 256 + (int)threadIdx.x;
    c.k = t / a.nrb;
    c.j = (t - c.k * a.nrb) * UF_ROWS;
    c.row = c.k * a.ny + c.j;
    j1 = min(c.j + UF_ROWS, a.ny);
    interior = c.j + a.djmin >= 0 && j1 - 1 + a.djmax < a.ny && c.k + a.dkmin >= 0 && c.k + a.dkmax < a.nz &&
               !(a.wide & 1);
    return c;
}

template <class T, bool FAST>
__device__ __forceinline__ T ld(const UArgs &a, int r, const UCell &c) {
    if (FAST) return ((const T *)a.in[r])[(long long)c.row * a.nx + a.shift[r] + xwrap(c.i + a.off[r][0], a.nx, a.bc[0])];
    const int ii = awrap(c.i + a.off[r][0], a.nx, a.bc[0], a.wide & 1);
    const int jj = awrap(c.j + a.off[r][1], a.ny, a.bc[1], a.wide & 2);
    const int kk = awrap(c.k + a.off[r][2], a.nz, a.bc[2], a.wide & 4);
    return ((const T *)a.in[r] + ((size_t)kk * a.ny + jj) * a.nx)[ii];
}
__device__ __forceinline__ double lds0(const UArgs &a, int r) { return *(const double *)a.in[r]; }

template <class T>
__device__ __forceinline__ void st(const UArgs &a, int o, const UCell &c, T v) {
    ((T *)a.out[o] + (size_t)c.row * a.nx)[c.i] = v;
}

// outputs of a rule body (it fills v[0 .. rule_nout - 1])
template <int OP>
constexpr int rule_nout() {
    return OP == HFAV_OP_EULER_PRIM ? 5
         : OP == HFAV_OP_EULER_TRACE ? 8
         : (OP == HFAV_OP_EULER_SLOPE || OP == HFAV_OP_EULER_RIEMANN || OP == HFAV_OP_EULER_FLUX ||
            OP == HFAV_OP_EULER_UPDATE) ? 4
         : 1;
}

template <int OP, class T, class A, bool G14, bool FAST>
__device__ __forceinline__ void rule_cell(const UArgs &a, const UCell &cell, T *v);

// the hydro rules compute far more per byte than they stream
template <int OP>
constexpr bool euler_rule() {
    return OP == HFAV_OP_EULER_PRIM || OP == HFAV_OP_EULER_SLOPE || OP == HFAV_OP_EULER_TRACE ||
           OP == HFAV_OP_EULER_RIEMANN || OP == HFAV_OP_EULER_FLUX || OP == HFAV_OP_EULER_UPDATE;
}

// The rows of a block two at a time: both rows' outputs are computed into
// registers before either is stored, so the loads of the second row do not
// wait behind the first row's stores (an output may alias no input, but the
// compiler cannot know that) and twice the bytes are in flight per wave.
// The hydro rules take one row at a time: paired, the Riemann rule needs
// 129 registers (3 waves per SIMD) for no streaming gain.
template <int OP, class T, class A, bool G14, bool FAST>
__device__ __forceinline__ void rule_rows(const UArgs &a, UCell c, int j1) {
    constexpr int NO = rule_nout<OP>();
    for (; !euler_rule<OP>() && c.j + 1 < j1; c.j += 2, c.row += 2) {
        UCell d = c;
        ++d.j;
        ++d.row;
        T v0[NO], v1[NO];
        rule_cell<OP, T, A, G14, FAST>(a, c, v0);
        rule_cell<OP, T, A, G14, FAST>(a, d, v1);
#pragma unroll
        for (int q = 0; q < NO; ++q) st<T>(a, q, c, v0[q]);
#pragma unroll
        for (int q = 0; q < NO; ++q) st<T>(a, q, d, v1[q]);
    }
    for (; c.j < j1; ++c.j, ++c.row) {
        T v0[NO];
        rule_cell<OP, T, A, G14, FAST>(a, c, v0);
#pragma unroll
        for (int q = 0; q < NO; ++q) st<T>(a, q, c, v0[q]);
    }
}

template <int OP, class T, class A, bool G14>
__global__ __launch_bounds__(256) void rule_kernel(UArgs a) {
    int j1;
    bool interior;
    const UCell cell = ucell0(a, j1, interior);
    if (cell.i >= a.nx) return;
    if (interior) rule_rows<OP, T, A, G14, true>(a, cell, j1);
    else rule_rows<OP, T, A, G14, false>(a, cell, j1);
}

template <int OP, class T, class A, bool G14, bool FAST>
__device__ __forceinline__ void rule_cell(const UArgs &a, const UCell &cell, T *v) {
#define IN(r) ld<T, FAST>(a, r, cell)
#define OUT(o, x) (v[o] = (x))
    if constexpr (OP == HFAV_OP_HDIFF_LAP) {
        OUT(0, hdiff_lap(IN(0), IN(1), IN(2), IN(3), IN(4)));
    } else if constexpr (OP == HFAV_OP_HDIFF_FLX || OP == HFAV_OP_HDIFF_FLY) {
        OUT(0, hdiff_flux(IN(0), IN(1), IN(2), IN(3)));
    } else if constexpr (OP == HFAV_OP_HDIFF_OUT) {
        OUT(0, hdiff_out(IN(0), IN(1), IN(2), IN(3), IN(4), (T)a.param[0]));
    } else if constexpr (OP == HFAV_OP_EULER_PRIM) {
        Prim<T> w = euler_prim(IN(0), IN(1), IN(2), IN(3), (T)a.param[0]);
        OUT(0, w.r); OUT(1, w.un); OUT(2, w.ut);
        OUT(3, w.p); OUT(4, w.c);
    } else if constexpr (OP == HFAV_OP_EULER_SLOPE) {
#pragma unroll
        for (int q = 0; q < 4; ++q) OUT(q, vanleer(IN(3 * q), IN(3 * q + 1), IN(3 * q + 2)));
    } else if constexpr (OP == HFAV_OP_EULER_TRACE) {
        Prim<T> w;
        w.r = IN(0); w.un = IN(1); w.ut = IN(2); w.p = IN(3); w.c = IN(4);
        T plus[4], minus[4];
        euler_trace(w, IN(5), IN(6), IN(7), IN(8), (T)lds0(a, 9), plus, minus);
#pragma unroll
        for (int q = 0; q < 4; ++q) { OUT(q, plus[q]); OUT(4 + q, minus[q]); }
    } else if constexpr (OP == HFAV_OP_EULER_RIEMANN) {
        T L[4] = {IN(0), IN(1), IN(2), IN(3)};
        T R[4] = {IN(4), IN(5), IN(6), IN(7)};
        T G[4];
        riemann_T<T, G14>(L, R, (T)a.param[0], (int)a.param[1], G);
#pragma unroll
        for (int q = 0; q < 4; ++q) OUT(q, G[q]);
    } else if constexpr (OP == HFAV_OP_EULER_FLUX) {
        T G[4] = {IN(0), IN(1), IN(2), IN(3)};
        T F[4];
        euler_flux(G, (T)a.param[0], F);
#pragma unroll
        for (int q = 0; q < 4; ++q) OUT(q, F[q]);
    } else if constexpr (OP == HFAV_OP_EULER_UPDATE) {
        const A nu = (A)lds0(a, 12);
#pragma unroll
        for (int q = 0; q < 4; ++q) OUT(q, euler_update(IN(q), IN(4 + q), IN(8 + q), nu));
    } else if constexpr (OP == HFAV_OP_LAP7) {
        OUT(0, lap7(IN(0), IN(1), IN(2), IN(3), IN(4), IN(5), IN(6)));
    } else if constexpr (OP == HFAV_OP_AXPY) {
        OUT(0, axpy(IN(0), IN(1), (T)a.param[0]));
    } else if constexpr (OP == HFAV_OP_SUMSQ) {
        T acc = T(0);
        for (int r = 0; r < a.n_in; ++r) {
            const T v = IN(r);
            acc = fma(v, v, acc);
        }
        OUT(0, acc);
    } else if constexpr (OP == HFAV_OP_DIV0) {
        const T b = a.brow ? ((const T *)a.in[1])[cell.row] : IN(1);
        OUT(0, b != T(0) ? IN(0) / b : T(0));
    }
#undef IN
#undef OUT
}

// ------------------------------------------------------------------ streaming rules, two cells per lane
// The rules that only stream (the diffusion, Laplacian, AXPY and DIV0
// bodies) run with SV = 2 consecutive cells per lane: every reference is
// one load of both cells per lane (unaligned when its i offset is odd,
// which global memory accepts), the body is evaluated per cell, and the two
// outputs are one store.  Lanes whose cells reach a row end, or a
// reference that wraps along i, load per cell as the scalar kernel does.
// Same arithmetic per cell as rule_cell.  FP64 only: in FP32 the per-cell
// kernel measured faster (the 7-point Laplacian at 512^3: 0.34 ms, against
// 0.51 with four cells per lane).
template <int OP>
constexpr int stream_nref() {
    return OP == HFAV_OP_HDIFF_LAP || OP == HFAV_OP_HDIFF_OUT ? 5
         : OP == HFAV_OP_HDIFF_FLX || OP == HFAV_OP_HDIFF_FLY ? 4
         : OP == HFAV_OP_LAP7 ? 7
         : 2;                                            // AXPY, DIV0
}
template <int OP>
constexpr bool is_stream_rule() {
    return OP == HFAV_OP_HDIFF_LAP || OP == HFAV_OP_HDIFF_FLX || OP == HFAV_OP_HDIFF_FLY ||
           OP == HFAV_OP_HDIFF_OUT || OP == HFAV_OP_LAP7 || OP == HFAV_OP_AXPY || OP == HFAV_OP_DIV0;
}

template <int OP, class T>
__device__ __forceinline__ T stream_body(const UArgs &a, const T *x) {
    if constexpr (OP == HFAV_OP_HDIFF_LAP) return hdiff_lap(x[0], x[1], x[2], x[3], x[4]);
    else if constexpr (OP == HFAV_OP_HDIFF_FLX || OP == HFAV_OP_HDIFF_FLY) return hdiff_flux(x[0], x[1], x[2], x[3]);
    else if constexpr (OP == HFAV_OP_HDIFF_OUT) return hdiff_out(x[0], x[1], x[2], x[3], x[4], (T)a.param[0]);
    else if constexpr (OP == HFAV_OP_LAP7) return lap7(x[0], x[1], x[2], x[3], x[4], x[5], x[6]);
    else if constexpr (OP == HFAV_OP_AXPY) return axpy(x[0], x[1], (T)a.param[0]);
    else return x[1] != T(0) ? x[0] / x[1] : T(0);      // DIV0
}

// two cells per lane: a 256-lane piece covers 512 cells of a row (rows of
// 512 cells fill every lane); 16-byte accesses in FP64, 8-byte in FP32
constexpr int SV = 2;
template <class T> struct VecOf { typedef T type __attribute__((ext_vector_type(SV))); };

template <int OP, class T, bool FAST>
__device__ __forceinline__ void stream_row(const UArgs &a, const UCell &c, T (&o)[SV]) {
    constexpr int V = SV, NR = stream_nref<OP>();
    using VT = typename VecOf<T>::type;
    const bool full = c.i + V <= a.nx;
    T x[NR][V];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (OP == HFAV_OP_DIV0 && r == 1 && a.brow) {     // row term: one value for the row
            const T b = ((const T *)a.in[1])[c.row];
#pragma unroll
            for (int e = 0; e < V; ++e) x[r][e] = b;
            continue;
        }
        const int i0 = c.i + a.off[r][0];
        if (FAST && full && i0 >= 0 && i0 + V <= a.nx) {
            VT w;
            __builtin_memcpy(&w, (const T *)a.in[r] + ((long long)c.row * a.nx + a.shift[r] + i0), sizeof(VT));
#pragma unroll
            for (int e = 0; e < V; ++e) x[r][e] = w[e];
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                UCell ce = c;
                ce.i = c.i + e;
                x[r][e] = ce.i < a.nx ? ld<T, FAST>(a, r, ce) : T(0);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
        T xe[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) xe[r] = x[r][e];
        o[e] = stream_body<OP, T>(a, xe);
    }
}

template <class T>
__device__ __forceinline__ void stream_store(const UArgs &a, const UCell &c, const T (&o)[SV]) {
    constexpr int V = SV;
    using VT = typename VecOf<T>::type;
    T *p = (T *)a.out[0] + (size_t)c.row * a.nx + c.i;
    if (c.i + V <= a.nx) {
        VT w;
#pragma unroll
        for (int e = 0; e < V; ++e) w[e] = o[e];
        __builtin_memcpy(p, &w, sizeof(VT));
    } else {
        for (int e = 0; e < V && c.i + e < a.nx; ++e) p[e] = o[e];
    }
}

// the rows of a block two at a time (both computed before either is stored)
template <int OP, class T, bool FAST>
__device__ __forceinline__ void stream_rows(const UArgs &a, UCell c, int j1) {
    constexpr int V = SV;
    for (; c.j + 1 < j1; c.j += 2, c.row += 2) {
        UCell d = c;
        ++d.j;
        ++d.row;
        T o0[V], o1[V];
        stream_row<OP, T, FAST>(a, c, o0);
        stream_row<OP, T, FAST>(a, d, o1);
        stream_store<T>(a, c, o0);
        stream_store<T>(a, d, o1);
    }
    if (c.j < j1) {
        T o0[V];
        stream_row<OP, T, FAST>(a, c, o0);
        stream_store<T>(a, c, o0);
    }
}

// a.ntx counts pieces of 256 * V cells; lane t owns cells t * V .. t * V + V - 1 of its piece
template <int OP, class T>
__global__ __launch_bounds__(256) void stream_rule_kernel(UArgs a) {
    constexpr int V = SV;
    int j1;
    bool interior;
    UCell cell = ucell0(a, j1, interior);
    // ucell0 numbers lanes one cell apart: spread them V cells apart
    const int piece = (cell.i - (int)threadIdx.x) / 256;
    cell.i = piece * 256 * V + (int)threadIdx.x * V;
    if (cell.i >= a.nx) return;
    if (interior) stream_rows<OP, T, true>(a, cell, j1);
    else stream_rows<OP, T, false>(a, cell, j1);
}

// SQRT over n elements (a grid or a row term)
template <class T>
__global__ __launch_bounds__(256) void rule_sqrt_kernel(UArgs a, size_t n) {
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx < n) ((T *)a.out[0])[idx] = sqrt(((const T *)a.in[0])[idx]);
}

// SUM_I: one workgroup per row of i, the row's sum into the row term
template <class T>
__global__ __launch_bounds__(256) void rule_sum_i_kernel(UArgs a) {
    __shared__ T part[4];
    const T *x = (const T *)a.in[0] + (size_t)blockIdx.x * a.nx;
    T s = T(0);
    for (int i = threadIdx.x; i < a.nx; i += 256) s += x[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) ((T *)a.out[0])[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

// reduction rule: accumulate max(|u|+c, |v|+c) into a 0-D term
template <class T>
__global__ __launch_bounds__(256) void rule_smax_kernel(UArgs a) {
    __shared__ double red[4];
    const size_t n = (size_t)a.nx * a.ny * a.nz;
    double m = 0.0;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256)
        m = fmax(m, (double)euler_speed(((const T *)a.in[0])[q], ((const T *)a.in[1])[q],
                                        ((const T *)a.in[2])[q], ((const T *)a.in[3])[q],
                                        (T)a.param[0]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomic_max_nonneg((double *)a.out[0], fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

__global__ void rule_dt_kernel(UArgs a) {
    *(double *)a.out[0] = a.param[0] / *(const double *)a.in[0];
}

template <int OP, class T, class A, bool G14>
static void launch_op(const UArgs &a, size_t n, hipStream_t s) {
    (void)n;
    if constexpr (is_stream_rule<OP>() && sizeof(T) == 8) {
        // pieces of 256 * SV cells per row
        constexpr int V = SV;
        UArgs b = a;
        b.ntx = (a.nx + 256 * V - 1) / (256 * V);
        b.nblk = b.ntx * a.nrb * a.nz;
        hipLaunchKernelGGL((stream_rule_kernel<OP, T>), dim3((unsigned)b.nblk), dim3(256), 0, s, b);
    } else {
        hipLaunchKernelGGL((rule_kernel<OP, T, A, G14>), dim3((unsigned)a.nblk), dim3(256), 0, s, a);
    }
}

template <class T, class A, bool G14>
static hipError_t dispatch_rule(const UnfusedRule &R, const UArgs &a, hipStream_t s) {
    const size_t n = (size_t)R.nx * R.ny * R.nz;
    switch (R.op) {
    case HFAV_OP_HDIFF_LAP: launch_op<HFAV_OP_HDIFF_LAP, T, A, G14>(a, n, s); break;
    case HFAV_OP_HDIFF_FLX: launch_op<HFAV_OP_HDIFF_FLX, T, A, G14>(a, n, s); break;
    case HFAV_OP_HDIFF_FLY: launch_op<HFAV_OP_HDIFF_FLY, T, A, G14>(a, n, s); break;
    case HFAV_OP_HDIFF_OUT: launch_op<HFAV_OP_HDIFF_OUT, T, A, G14>(a, n, s); break;
    case HFAV_OP_EULER_PRIM: launch_op<HFAV_OP_EULER_PRIM, T, A, G14>(a, n, s); break;
    case HFAV_OP_EULER_SLOPE: launch_op<HFAV_OP_EULER_SLOPE, T, A, G14>(a, n, s); break;
    case HFAV_OP_EULER_TRACE: launch_op<HFAV_OP_EULER_TRACE, T, A, G14>(a, n, s); break;
    case HFAV_OP_EULER_RIEMANN: launch_op<HFAV_OP_EULER_RIEMANN, T, A, G14>(a, n, s); break;
    case HFAV_OP_EULER_FLUX: launch_op<HFAV_OP_EULER_FLUX, T, A, G14>(a, n, s); break;
    case HFAV_OP_EULER_UPDATE: launch_op<HFAV_OP_EULER_UPDATE, T, A, G14>(a, n, s); break;
    case HFAV_OP_LAP7: launch_op<HFAV_OP_LAP7, T, A, G14>(a, n, s); break;
    case HFAV_OP_AXPY: launch_op<HFAV_OP_AXPY, T, A, G14>(a, n, s); break;
    case HFAV_OP_SUMSQ: launch_op<HFAV_OP_SUMSQ, T, A, G14>(a, n, s); break;
    case HFAV_OP_DIV0: launch_op<HFAV_OP_DIV0, T, A, G14>(a, n, s); break;
    case HFAV_OP_SQRT: {
        const size_t m = R.out_rank == R.ndim ? n : (size_t)R.ny * R.nz;
        hipLaunchKernelGGL((rule_sqrt_kernel<T>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, m);
        break;
    }
    case HFAV_OP_SUM_I:
        hipLaunchKernelGGL((rule_sum_i_kernel<T>), dim3((unsigned)((size_t)R.ny * R.nz)), dim3(256), 0, s, a);
        break;
    case HFAV_OP_EULER_SMAX: {
        unsigned nb = (unsigned)((n + 255) / 256);
        if (nb > 4096) nb = 4096;
        hipLaunchKernelGGL((rule_smax_kernel<T>), dim3(nb), dim3(256), 0, s, a);
        break;
    }
    case HFAV_OP_EULER_DT:
        hipLaunchKernelGGL(rule_dt_kernel, dim3(1), dim3(1), 0, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// bit a set when some offset along axis a reaches a whole axis length (the
// wrap then takes a modulo instead of one compare per side)
template <class OFF>
static int wide_bits(int n_in, const OFF &off, int nx, int ny, int nz) {
    const int n[3] = {nx, ny, nz};
    int w = 0;
    for (int r = 0; r < n_in; ++r)
        for (int d = 0; d < 3; ++d)
            if (off[r][d] >= n[d] || -off[r][d] >= n[d]) w |= 1 << d;
    return w;
}

hipError_t launch_unfused_rule(const UnfusedRule &R, hipStream_t s) {
    UArgs a;
    for (int r = 0; r < UF_MAX_IN; ++r) {
        a.in[r] = r < R.n_in ? R.in[r] : nullptr;
        for (int d = 0; d < 3; ++d) a.off[r][d] = r < R.n_in ? R.off[r][d] : 0;
    }
    for (int o = 0; o < UF_MAX_OUT; ++o) a.out[o] = o < R.n_out ? R.out[o] : nullptr;
    for (int q = 0; q < UF_MAX_PARAM; ++q) a.param[q] = R.param[q];
    a.nx = R.nx; a.ny = R.ny; a.nz = R.nz;
    for (int d = 0; d < 3; ++d) a.bc[d] = R.bc[d];
    a.n_in = R.n_in;
    a.brow = R.n_in > 1 && R.in_rank[1] == R.ndim - 1;
    a.ntx = (R.nx + 255) / 256;
    a.nrb = (R.ny + UF_ROWS - 1) / UF_ROWS;
    const int64_t nblk = (int64_t)a.ntx * a.nrb * R.nz;
    if (nblk > INT32_MAX || (int64_t)R.ny * R.nz > INT32_MAX) return hipErrorInvalidValue;
    a.nblk = (int)nblk;
    a.wide = wide_bits(R.n_in, R.off, R.nx, R.ny, R.nz);
    a.djmin = a.djmax = a.dkmin = a.dkmax = 0;
    for (int r = 0; r < UF_MAX_IN; ++r) {
        a.shift[r] = r < R.n_in ? ((long long)R.off[r][2] * R.ny + R.off[r][1]) * R.nx : 0;
        if (r >= R.n_in) continue;
        a.djmin = std::min(a.djmin, R.off[r][1]); a.djmax = std::max(a.djmax, R.off[r][1]);
        a.dkmin = std::min(a.dkmin, R.off[r][2]); a.dkmax = std::max(a.dkmax, R.off[r][2]);
    }
    double g = R.param[0];
    const bool g14 = (R.op == HFAV_OP_EULER_RIEMANN) && g == 1.4;
    if (R.dtype == HFAV_F64)
        return g14 ? dispatch_rule<double, double, true>(R, a, s) : dispatch_rule<double, double, false>(R, a, s);
    if (R.precision == HFAV_PREC_F32_F64ACC)
        return g14 ? dispatch_rule<float, double, true>(R, a, s) : dispatch_rule<float, double, false>(R, a, s);
    return g14 ? dispatch_rule<float, float, true>(R, a, s) : dispatch_rule<float, float, false>(R, a, s);
}

// ------------------------------------------------------------------ STAR
enum { STAR_MAX = 96 };
struct SArgs {
    const void *in[STAR_MAX];
    int off[STAR_MAX][3];
    double coeff[STAR_MAX];
    int n_in;
    void *out;
    int nx, ny, nz;
    int bc[3];
    int ntx, nrb, nblk, wide;                 // as in UArgs
    int djmin, djmax, dkmin, dkmax;
};

template <class T>
__global__ __launch_bounds__(256) void star_rule_kernel(SArgs a) {
    // reference order, every product and sum rounded (no contraction)
#pragma clang fp contract(off)
    const int w = xcd_tile((int)blockIdx.x, a.nblk, -1);
    const int t = w / a.ntx;
    const int i = (w - t * a.ntx) * 256 + (int)threadIdx.x;
    if (i >= a.nx) return;
    const int k = t / a.nrb;
    const int j0 = (t - k * a.nrb) * UF_ROWS, j1 = min(j0 + UF_ROWS, a.ny);
    const bool interior =
        j0 + a.djmin >= 0 && j1 - 1 + a.djmax < a.ny && k + a.dkmin >= 0 && k + a.dkmax < a.nz && !(a.wide & 1);
    for (int j = j0; j < j1; ++j) {
        const long long row = (long long)k * a.ny + j;
        T acc = T(0);
        for (int r = 0; r < a.n_in; ++r) {
            long long o;
            if (interior) {
                o = (row + (long long)a.off[r][2] * a.ny + a.off[r][1]) * a.nx + xwrap(i + a.off[r][0], a.nx, a.bc[0]);
            } else {
                const int ii = awrap(i + a.off[r][0], a.nx, a.bc[0], a.wide & 1);
                const int jj = awrap(j + a.off[r][1], a.ny, a.bc[1], a.wide & 2);
                const int kk = awrap(k + a.off[r][2], a.nz, a.bc[2], a.wide & 4);
                o = ((long long)kk * a.ny + jj) * a.nx + ii;
            }
            acc += (T)a.coeff[r] * ((const T *)a.in[r])[o];
        }
        ((T *)a.out + row * a.nx)[i] = acc;
    }
}

hipError_t launch_star_rule(const StarRule &R, hipStream_t s) {
    if (R.n_in < 1 || R.n_in > STAR_MAX) return hipErrorInvalidValue;
    SArgs a;
    a.n_in = R.n_in;
    int off[STAR_MAX][3];
    a.djmin = a.djmax = a.dkmin = a.dkmax = 0;
    for (int r = 0; r < STAR_MAX; ++r) {
        a.in[r] = r < R.n_in ? R.in[r] : nullptr;
        for (int d = 0; d < 3; ++d) off[r][d] = a.off[r][d] = r < R.n_in ? R.off[3 * r + d] : 0;
        a.coeff[r] = r < R.n_in ? R.coeff[r] : 0.0;
        a.djmin = std::min(a.djmin, off[r][1]); a.djmax = std::max(a.djmax, off[r][1]);
        a.dkmin = std::min(a.dkmin, off[r][2]); a.dkmax = std::max(a.dkmax, off[r][2]);
    }
    a.out = R.out;
    a.nx = R.nx; a.ny = R.ny; a.nz = R.nz;
    for (int d = 0; d < 3; ++d) a.bc[d] = R.bc[d];
    a.ntx = (R.nx + 255) / 256;
    a.nrb = (R.ny + UF_ROWS - 1) / UF_ROWS;
    const int64_t nblk = (int64_t)a.ntx * a.nrb * R.nz;
    if (nblk > INT32_MAX || (int64_t)R.ny * R.nz > INT32_MAX) return hipErrorInvalidValue;
    a.nblk = (int)nblk;
    a.wide = wide_bits(R.n_in, off, R.nx, R.ny, R.nz);
    const unsigned nb = (unsigned)a.nblk;
    if (R.dtype == HFAV_F64) hipLaunchKernelGGL((star_rule_kernel<double>), dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((star_rule_kernel<float>), dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hfav
