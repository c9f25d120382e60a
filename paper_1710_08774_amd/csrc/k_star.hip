// Fused groups of linear star-stencil stages (random chains for the tuning
// study).  A group of G consecutive stages runs as one kernel: a workgroup
// owns a TX (x TY) tile across the lanes and streams along the outermost
// axis (y for 2-D chains, z for 3-D).  The output of stage s is contracted
// to a ring of 2 r_{s+1} + 1 planes in LDS (the reuse span of its consumer,
// Design "Contraction"), computed over the tile plus the halo the remaining
// stages need (the Minkowski sum of their radii, Design "Variables and
// storage").  The input planes enter the first ring once, from HBM.
// Each output is accumulated from zero in the offset order below with every
// product and sum rounded separately.
//
// Coefficients of stage s are laid out (f_out, f_in, 1 + 2 r nd) in the
// star-offset order: centre, then for each axis x, y(, z) the pairs -d, +d
// for d = 1..r.  They are read with wave-uniform addresses.
#include <hip/hip_runtime.h>
#include "kernels.h"

namespace hfav {

struct SGStage {
    int r, fin, fout;
    int coff;          // first coefficient of the stage in the table
    int lds;           // element offset of the stage's input ring in LDS
    int planes;        // ring depth of the stage's input: 2r+1
    int hx, hy;        // halo of the stage's input plane along x and y
    int px, py;        // input plane extent: TX + 2hx, TY + 2hy
};

struct SGArgs {
    const void *in[SG_MAX_F];
    void *out[SG_MAX_F];
    const double *coeff;
    int nstage, nd;
    int nx, ny, nz;
    int seg;
    SGStage st[SG_MAX_STAGES];
};

__device__ __forceinline__ int sgwrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}
__device__ __forceinline__ int sgmod(int q, int m) {
    q %= m;
    return q < 0 ? q + m : q;
}

template <class T, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void star_group_kernel(SGArgs a) {
    extern __shared__ unsigned char smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    constexpr int NT = TX * TY;
    const int tid = threadIdx.x;
    const bool three = a.nd == 3;
    // streamed axis: y in 2-D, z in 3-D; tile axes x (and y in 3-D)
    const int nstream = three ? a.nz : a.ny;
    const int ntx = (a.nx + TX - 1) / TX;
    const int nty = three ? (a.ny + TY - 1) / TY : 1;
    const int nsg = (nstream + a.seg - 1) / a.seg;
    int b = blockIdx.x;
    const int x0 = (b % ntx) * TX;
    b /= ntx;
    const int y0 = three ? (b % nty) * TY : 0;
    b /= nty;
    const int p0 = (b % nsg) * a.seg;
    const int p1 = min(p0 + a.seg, nstream);
    const int G = a.nstage;
    // lead of each stage's output plane over the group's output plane
    int lead[SG_MAX_STAGES + 1];
    lead[G] = 0;
    for (int s = G - 1; s >= 0; --s) lead[s] = lead[s + 1] + a.st[s].r;
    const size_t plane = three ? (size_t)a.nx * a.ny : (size_t)a.nx;
    const size_t fstride = (size_t)a.nx * a.ny * a.nz;

    // value of input ring of stage s: field f, plane q, in-plane (ix, iy)
    auto ring = [&](int s, int f, int q, int ix, int iy) -> T & {
        const SGStage &S = a.st[s];
        const int slot = sgmod(q, S.planes);
        return smem[S.lds + ((size_t)(f * S.planes + slot) * S.py + iy) * S.px + ix];
    };
    // one star stage: output field o at in-plane point (ix, iy) of the
    // stage's own output frame, plane q
    auto eval = [&](int s, int o, int q, int ix, int iy) -> T {
        // products and sums rounded one by one, in the offset order (no
        // multiply-add contraction): the same rounding as evaluating the
        // stage term by term
#pragma clang fp contract(off)
        const SGStage &S = a.st[s];
        const int n_off = 1 + 2 * S.r * a.nd;
        const double *c = a.coeff + S.coff + (size_t)o * S.fin * n_off;
        // output frame -> input frame: shift by the stage radius
        const int jx = ix + S.r, jy = three ? iy + S.r : 0;
        T acc = T(0);
        for (int f = 0; f < S.fin; ++f, c += n_off) {
            acc += (T)c[0] * ring(s, f, q, jx, jy);
            int k = 1;
            for (int d = 1; d <= S.r; ++d, k += 2) {
                acc += (T)c[k] * ring(s, f, q, jx - d, jy);
                acc += (T)c[k + 1] * ring(s, f, q, jx + d, jy);
            }
            if (three) {
                for (int d = 1; d <= S.r; ++d, k += 2) {
                    acc += (T)c[k] * ring(s, f, q, jx, jy - d);
                    acc += (T)c[k + 1] * ring(s, f, q, jx, jy + d);
                }
            }
            for (int d = 1; d <= S.r; ++d, k += 2) {
                acc += (T)c[k] * ring(s, f, q - d, jx, jy);
                acc += (T)c[k + 1] * ring(s, f, q + d, jx, jy);
            }
        }
        return acc;
    };

    // warm-up: stage s output is valid 2*(r_1+..+r_s) iterations after start
    const int pstart = p0 - 2 * lead[0];
    for (int p = pstart; p < p1; ++p) {
        __syncthreads();
        // stage-0 ring: input plane p + lead[0] over the tile and its halo
        {
            const SGStage &S = a.st[0];
            const int q = p + lead[0];
            const size_t pbase = (size_t)sgwrap(q, nstream) * plane;
            const int npt = S.px * S.py;
            for (int f = 0; f < S.fin; ++f) {
                const T *src = (const T *)a.in[f];
                for (int t = tid; t < npt; t += NT) {
                    const int ix = t % S.px, iy = t / S.px;
                    const int gx = sgwrap(x0 - S.hx + ix, a.nx);
                    const size_t off = three ? (size_t)sgwrap(y0 - S.hy + iy, a.ny) * a.nx + gx : (size_t)gx;
                    ring(0, f, q, ix, iy) = src[pbase + off];
                }
            }
        }
        __syncthreads();
        // inner stages: output plane p + lead[s] into the next ring
        for (int s = 0; s + 1 < G; ++s) {
            const SGStage &N = a.st[s + 1];     // ring receiving stage s's output
            const int q = p + lead[s + 1];
            const int npt = N.px * N.py;
            for (int o = 0; o < N.fin; ++o)
                for (int t = tid; t < npt; t += NT) {
                    const int ix = t % N.px, iy = t / N.px;
                    ring(s + 1, o, q, ix, iy) = eval(s, o, q, ix, iy);
                }
            __syncthreads();
        }
        // last stage: the group's output plane p, tile only
        if (p >= p0) {
            const int s = G - 1;
            const SGStage &S = a.st[s];
            const int tx = tid % TX, ty = tid / TX;
            const int gx = x0 + tx, gy = y0 + ty;
            if (gx < a.nx && (!three || gy < a.ny)) {
                const size_t dst = (size_t)p * plane + (three ? (size_t)gy * a.nx : 0) + gx;
                for (int o = 0; o < S.fout; ++o) ((T *)a.out[o])[dst] = eval(s, o, p, tx, ty);
            }
        }
    }
    (void)fstride;
}

// LDS bytes of a group; also fills the ring layout of every stage.
size_t star_group_lds(StarGroupLaunch &L, int tx, int ty, size_t elem) {
    const bool three = L.nd == 3;
    int h = 0;
    for (int s = 0; s < L.nstage; ++s) h += L.st[s].r;
    size_t off = 0;
    for (int s = 0; s < L.nstage; ++s) {
        StarGroupLaunch::Stage &S = L.st[s];
        // input of stage s is needed with the halo of stages s..G-1
        int hs = 0;
        for (int t = s; t < L.nstage; ++t) hs += L.st[t].r;
        S.hx = hs;
        S.hy = three ? hs : 0;
        S.px = tx + 2 * S.hx;
        S.py = three ? ty + 2 * S.hy : 1;
        S.planes = 2 * S.r + 1;
        S.lds = (int)off;
        off += (size_t)S.fin * S.planes * S.px * S.py;
    }
    (void)h;
    return off * elem;
}

template <class T, int TX, int TY>
static hipError_t star_launch(StarGroupLaunch &L, hipStream_t s) {
    const size_t lds = star_group_lds(L, TX, TY, sizeof(T));
    if (lds > SG_MAX_LDS) return hipErrorInvalidValue;
    SGArgs a;
    for (int f = 0; f < SG_MAX_F; ++f) {
        a.in[f] = f < L.st[0].fin ? L.in[f] : nullptr;
        a.out[f] = f < L.st[L.nstage - 1].fout ? L.out[f] : nullptr;
    }
    a.coeff = L.coeff;
    a.nstage = L.nstage;
    a.nd = L.nd;
    a.nx = L.nx; a.ny = L.ny; a.nz = L.nz;
    a.seg = L.seg > 0 ? L.seg : 32;
    for (int q = 0; q < L.nstage; ++q) {
        const StarGroupLaunch::Stage &S = L.st[q];
        a.st[q] = SGStage{S.r, S.fin, S.fout, S.coff, S.lds, S.planes, S.hx, S.hy, S.px, S.py};
    }
    const bool three = L.nd == 3;
    const int nstream = three ? L.nz : L.ny;
    const long long nblk = (long long)((L.nx + TX - 1) / TX) * (three ? (L.ny + TY - 1) / TY : 1) *
                           ((nstream + a.seg - 1) / a.seg);
    hipLaunchKernelGGL((star_group_kernel<T, TX, TY>), dim3((unsigned)nblk), dim3(TX * TY), lds, s, a);
    return hipGetLastError();
}

// tile shapes (variant): 2-D chains use TY = 1
template <class T>
static hipError_t star_dispatch(StarGroupLaunch &L, hipStream_t s) {
    if (L.nd == 2) {
        switch (L.tile) {
        case 0: return star_launch<T, 64, 1>(L, s);
        case 1: return star_launch<T, 128, 1>(L, s);
        case 2: return star_launch<T, 256, 1>(L, s);
        default: return star_launch<T, 512, 1>(L, s);
        }
    }
    switch (L.tile) {
    case 0: return star_launch<T, 16, 4>(L, s);
    case 1: return star_launch<T, 32, 4>(L, s);
    case 2: return star_launch<T, 16, 16>(L, s);
    default: return star_launch<T, 32, 8>(L, s);
    }
}

hipError_t launch_star_group(StarGroupLaunch &L, hipStream_t s) {
    if (L.nstage < 1 || L.nstage > SG_MAX_STAGES) return hipErrorInvalidValue;
    return L.dtype == HFAV_F64 ? star_dispatch<double>(L, s) : star_dispatch<float>(L, s);
}

size_t star_group_lds_bytes(const StarGroupLaunch &L0) {
    StarGroupLaunch L = L0;
    int tx, ty;
    if (L.nd == 2) { tx = L.tile == 0 ? 64 : L.tile == 1 ? 128 : L.tile == 2 ? 256 : 512; ty = 1; }
    else {
        static const int txs[4] = {16, 32, 16, 32}, tys[4] = {4, 4, 16, 8};
        const int v = L.tile < 0 || L.tile > 3 ? 3 : L.tile;
        tx = txs[v]; ty = tys[v];
    }
    return star_group_lds(L, tx, ty, L.dtype == HFAV_F64 ? 8 : 4);
}

}  // namespace hfav
