// Fused normalisation chain (Design, "Reductions & broadcasts & splits";
// Performance, "Normalization Example").  Per field q of nq:
//   flux      f_q = c0_q u_q(i) + cp_q u_q(i+1)       (STAR along i)
//   square    e   = sum_q f_q^2                       (SUMSQ)
//   reduce    s   = sum over the row of e             (SUM_I: init 0 in the
//                                                      prologue, accumulate in
//                                                      the steady state)
//   root      n   = sqrt(s)                           (SQRT: the epilogue)
//   divide    d_q = f_q / n, 0 where n = 0            (DIV0: broadcast of n)
//   update    out_q = u_q + alpha_q d_q               (AXPY)
// The reduction feeding the broadcast splits the inner (i) loop into two
// sweeps, but not the loops outside it: one workgroup owns one row (the
// outer iteration) and runs both sweeps, so f never leaves the chip.
//
// Variant 0 keeps the row's u in registers, cells i = t + m*B for m < M: HBM
// sees each u once and each out once.  u(i+1) comes from the next lane
// through a DPP wave shift; the last lane of a wave takes it from an LDS
// copy of every wave's first lane; the row end wraps (periodic) or repeats
// the last cell (transmissive).  f is recomputed in the second sweep from
// the same registers, so both sweeps see the same f bit for bit.
// Variant 1 streams rows of any length twice (u is read twice).  Variants
// 2 and 3 are variant 0 with non-temporal stores (2) or non-temporal loads
// and stores (3).
//
// The division runs as a multiply by 1/n, one reciprocal per row: at most
// one rounding more than the quotient.
#include <hip/hip_runtime.h>
#include "dpp.h"
#include "kernels.h"
#include "ops.h"

namespace hfav {
namespace {

template <class T>
struct NArgs {
    const T *u[NORM_MAX_Q];
    T *out[NORM_MAX_Q];
    T *norm;                          // row goal, or null
    T c0[NORM_MAX_Q], cp[NORM_MAX_Q], alpha[NORM_MAX_Q];
    int ni;
    int periodic;
};

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block-wide sum of one value per thread, the same result in every thread
template <class T>
__device__ __forceinline__ T block_sum(T v, T *part) {
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[w] = v;
    __syncthreads();
    T s = T(0);
    for (int k = 0; k < nw; ++k) s += part[k];
    return s;
}

// Row element at a 32-bit byte offset from a uniform row pointer (rows hold
// fewer than 2^28 cells): the load takes the scalar-base + vector-offset form
// instead of a 64-bit address per lane.
// NT: non-temporal (streaming) access, for data touched exactly once.
template <bool NT, class T>
__device__ __forceinline__ T row_ld(const T *row, unsigned i) {
    const T *p = (const T *)((const char *)row + i * (unsigned)sizeof(T));
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void row_st(T *row, unsigned i, T v) {
    T *p = (T *)((char *)row + i * (unsigned)sizeof(T));
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <class T>
__device__ __forceinline__ T flux(const NArgs<T> &a, int q, T u0, T u1) {
    return fma(a.cp[q], u1, a.c0[q] * u0);
}

template <class T, int NQ, int M, int NT>
__global__ __launch_bounds__(1024) void norm_reg_kernel(NArgs<T> a) {
    __shared__ T first[NQ][M][16];    // lane-0 value of every wave, per field and slot
    __shared__ T part[16];
    const int B = blockDim.x, t = threadIdx.x, lane = t & 63, w = t >> 6, nw = B >> 6;
    const int ni = a.ni;
    const size_t base = (size_t)blockIdx.x * ni;
    // row pointers are uniform (scalar registers); cells index them with
    // 32-bit offsets
    const T *ur[NQ];
    T *orow[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { ur[q] = a.u[q] + base; orow[q] = a.out[q] + base; }
    // every lane loads, the index clamped into the row: no branches around
    // the loads.  Slots past the row end hold a copy of the last cell; they
    // are nobody's neighbour and stay out of the sum.
    T u[NQ][M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = t + m * B;
        const unsigned ic = (unsigned)(i < ni ? i : ni - 1);
#pragma unroll
        for (int q = 0; q < NQ; ++q) u[q][m] = row_ld<(NT & 1) != 0>(ur[q], ic);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int m = 0; m < M; ++m) first[q][m][w] = u[q][m];
    }
    __syncthreads();
    // u(i+1) of cell i = t + m*B.  Lane 63's neighbour is lane 0 of the next
    // wave, or of wave 0 one slot on; the row's last cell wraps or repeats.
    // Selects only, no branches: the LDS addresses are uniform per wave.
    const int wn = w + 1 < nw ? w + 1 : 0, mo = w + 1 < nw ? 0 : 1;
    auto next = [&](int q, int m) -> T {
        const int mm = m + mo < M ? m + mo : M - 1;
        T e = first[q][mm][wn];
        T w0 = first[q][0][0];
        // read unconditionally: otherwise the compiler moves each LDS read
        // into a branch of its own, which splits the sweep into blocks and
        // keeps every slot's neighbour live at once
        asm volatile("" : "+v"(e), "+v"(w0));
        const T v = lane_shift<false>(u[q][m]);
        const T wrapv = a.periodic ? w0 : u[q][m];
        const int i = t + m * B;
        return i == ni - 1 ? wrapv : (lane == 63 ? e : v);
    };
    // sweep 1: flux, square, accumulate
    T s = T(0);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        T e = T(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T f = flux(a, q, u[q][m], next(q, m));
            e = q == 0 ? f * f : fma(f, f, e);
        }
        s += t + m * B < ni ? e : T(0);
        // keep the scheduler from hoisting every slot's LDS and DPP reads
        // at once (their results would all be live together)
        __builtin_amdgcn_sched_barrier(0);
    }
    // finalise: row norm and its reciprocal
    const T S = block_sum(s, part);
    const T nrm = sqrt(S);
    const T rn = nrm != T(0) ? T(1) / nrm : T(0);
    if (a.norm && t == 0) a.norm[blockIdx.x] = nrm;
    // Only u stays live across the reduction: the empty asm makes the
    // compiler treat u as rewritten, so the second sweep recomputes f
    // instead of holding NQ*M more values in registers.
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int m = 0; m < M; ++m) asm volatile("" : "+v"(u[q][m]));
    // sweep 2: divide (broadcast of the norm) and update
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const unsigned i = (unsigned)(t + m * B);
        if (i < (unsigned)ni) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const T f = flux(a, q, u[q][m], next(q, m));
                row_st<(NT & 2) != 0>(orow[q], i, axpy(u[q][m], f * rn, a.alpha[q]));
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <class T, int NQ>
__global__ __launch_bounds__(256) void norm_stream_kernel(NArgs<T> a) {
    __shared__ T part[16];
    const int B = blockDim.x, t = threadIdx.x, ni = a.ni;
    const size_t base = (size_t)blockIdx.x * ni;
    auto nb = [&](int i) { return i + 1 < ni ? i + 1 : (a.periodic ? 0 : ni - 1); };
    T s = T(0);
    for (int i = t; i < ni; i += B) {
        const int ip = nb(i);
        T e = T(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T f = flux(a, q, a.u[q][base + i], a.u[q][base + ip]);
            e = q == 0 ? f * f : fma(f, f, e);
        }
        s += e;
    }
    const T S = block_sum(s, part);
    const T nrm = sqrt(S);
    const T rn = nrm != T(0) ? T(1) / nrm : T(0);
    if (a.norm && t == 0) a.norm[blockIdx.x] = nrm;
    for (int i = t; i < ni; i += B) {
        const int ip = nb(i);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T u0 = a.u[q][base + i];
            const T f = flux(a, q, u0, a.u[q][base + ip]);
            a.out[q][base + i] = axpy(u0, f * rn, a.alpha[q]);
        }
    }
}

template <class T, int NQ, int NT>
hipError_t launch_reg(const NArgs<T> &a, const NormLaunch &L, hipStream_t s) {
    const dim3 grid((unsigned)L.nrows), blk((unsigned)L.cfg.block);
    switch (L.cfg.seg) {
    case 1: hipLaunchKernelGGL((norm_reg_kernel<T, NQ, 1, NT>), grid, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL((norm_reg_kernel<T, NQ, 2, NT>), grid, blk, 0, s, a); break;
    case 4: hipLaunchKernelGGL((norm_reg_kernel<T, NQ, 4, NT>), grid, blk, 0, s, a); break;
    case 8:
        if constexpr (NQ * 8 <= NORM_REG_BUDGET) {
            hipLaunchKernelGGL((norm_reg_kernel<T, NQ, 8, NT>), grid, blk, 0, s, a);
            break;
        }
        return hipErrorInvalidValue;
    case 16:
        if constexpr (NQ * 16 <= NORM_REG_BUDGET) {
            hipLaunchKernelGGL((norm_reg_kernel<T, NQ, 16, NT>), grid, blk, 0, s, a);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class T, int NQ>
hipError_t launch_q(const NArgs<T> &a, const NormLaunch &L, hipStream_t s) {
    switch (L.cfg.variant) {
    case 1:
        hipLaunchKernelGGL((norm_stream_kernel<T, NQ>), dim3((unsigned)L.nrows), dim3((unsigned)L.cfg.block), 0,
                           s, a);
        return hipGetLastError();
    case 2: return launch_reg<T, NQ, 2>(a, L, s);
    case 3: return launch_reg<T, NQ, 3>(a, L, s);
    default: return launch_reg<T, NQ, 0>(a, L, s);
    }
}

template <class T>
hipError_t launch_t(const NormLaunch &L, hipStream_t s) {
    NArgs<T> a;
    for (int q = 0; q < NORM_MAX_Q; ++q) {
        const bool on = q < L.nq;
        a.u[q] = on ? (const T *)L.u[q] : nullptr;
        a.out[q] = on ? (T *)L.out[q] : nullptr;
        a.c0[q] = on ? (T)L.c0[q] : T(0);
        a.cp[q] = on ? (T)L.cp[q] : T(0);
        a.alpha[q] = on ? (T)L.alpha[q] : T(0);
    }
    a.norm = (T *)L.norm;
    a.ni = L.ni;
    a.periodic = L.bc == HFAV_BC_PERIODIC;
    switch (L.nq) {
    case 1: return launch_q<T, 1>(a, L, s);
    case 2: return launch_q<T, 2>(a, L, s);
    case 3: return launch_q<T, 3>(a, L, s);
    case 4: return launch_q<T, 4>(a, L, s);
    case 5: return launch_q<T, 5>(a, L, s);
    case 6: return launch_q<T, 6>(a, L, s);
    case 7: return launch_q<T, 7>(a, L, s);
    case 8: return launch_q<T, 8>(a, L, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool norm_config_ok(int nq, int ni, const hfav_config &c) {
    if (nq < 1 || nq > NORM_MAX_Q || ni < 1) return false;
    if (c.variant == 1) return c.block == 64 || c.block == 128 || c.block == 256;
    if (c.variant != 0 && c.variant != 2 && c.variant != 3) return false;
    if (c.block < 64 || c.block > 1024 || (c.block & 63)) return false;
    if (c.seg != 1 && c.seg != 2 && c.seg != 4 && c.seg != 8 && c.seg != 16) return false;
    if (nq * c.seg > NORM_REG_BUDGET) return false;
    return (int64_t)c.block * c.seg >= ni;
}

hfav_config norm_default_config(int nq, int ni, int dtype) {
    // measured on MI355X (4 fields, rows of 1024 and 4096 cells): rows of
    // about 256 lanes of up to 8 cells, non-temporal loads and stores in
    // FP64, non-temporal stores in FP32
    hfav_config c{256, 1, 0, 1, 0};
    int mmax = 1;
    while (mmax < 16 && nq * mmax * 2 <= NORM_REG_BUDGET) mmax *= 2;
    int m = 1;
    while (m < mmax && (ni + m - 1) / m > 256) m *= 2;
    int b = 64;
    while (b < 1024 && (int64_t)b * m < ni) b *= 2;
    if ((int64_t)b * m >= ni) {
        c.block = b;
        c.seg = m;
        c.variant = dtype == HFAV_F64 ? 3 : 2;
    }
    return c;
}

hipError_t launch_norm(const NormLaunch &L, hipStream_t s) {
    if (!norm_config_ok(L.nq, L.ni, L.cfg) || L.nrows < 1) return hipErrorInvalidValue;
    return L.dtype == HFAV_F64 ? launch_t<double>(L, s) : launch_t<float>(L, s);
}

}  // namespace hfav
