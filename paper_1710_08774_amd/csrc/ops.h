// Device-side rule bodies ("user kernels" in the paper's sense, Design
// "Fundamentals": homogeneous, side-effect free, order agnostic).  The fused
// kernel families and the unfused one-kernel-per-rule path call the same
// functions, so the two paths evaluate identical arithmetic per cell.
//
// Quotients and square-root reciprocals of the Euler rules use the hardware
// estimates refined to about one unit in the last place (frcp, frsq) rather
// than correctly rounded division: the results differ from the oracle's by
// rounding only, at a fraction of the instruction count.
//
// Template parameter T is the storage/arithmetic type (double or float).
// In the F32_F64ACC precision the Riemann pressure iteration and the
// conservative-update accumulation run in double whatever T is.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace hfav {

// ------------------------------------------------------------------ hdiff
// COSMO horizontal diffusion (Performance, "COSMO Micro-Kernels").
// These bandwidth-bound rules are evaluated without FMA contraction, in the
// operation order written, so that a limiter decision never depends on
// whether a multiply-add was fused.
template <class T>
__device__ __forceinline__ T hdiff_lap(T c, T e, T w, T n, T s) {
#pragma clang fp contract(off)
    return (e + w) + (n + s) - T(4) * c;
}
// forward difference of lap, zeroed when it points up the gradient of u
template <class T>
__device__ __forceinline__ T hdiff_flux(T l0, T l1, T u0, T u1) {
#pragma clang fp contract(off)
    T f = l1 - l0;
    return (f * (u1 - u0) > T(0)) ? T(0) : f;
}
template <class T>
__device__ __forceinline__ T hdiff_out(T u, T fx0, T fxm, T fy0, T fym, T coeff) {
#pragma clang fp contract(off)
    return u - coeff * ((fx0 - fxm) + (fy0 - fym));
}

// ------------------------------------------------------------------ lap7
template <class T>
__device__ __forceinline__ T lap7(T c, T e, T w, T n, T s, T t, T b) {
#pragma clang fp contract(off)
    return ((e + w) + (n + s)) + (t + b) - T(6) * c;
}
template <class T>
__device__ __forceinline__ T axpy(T a, T b, T alpha) {
#pragma clang fp contract(off)
    return a + alpha * b;
}

// ------------------------------------------------------------------ euler
// Reciprocal from the hardware estimate refined by one Newton step
// (relative error about one unit in the last place); float keeps division.
__device__ __forceinline__ double frcp(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
}
__device__ __forceinline__ float frcp(float d) { return 1.0f / d; }

// 1/sqrt(x) for positive finite x: hardware estimate and one third-order
// correction (relative error about one unit in the last place)
__device__ __forceinline__ double frsq(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// sqrt(x) for positive finite x: x times the refined reciprocal square
// root (about one unit in the last place); float keeps the library sqrt.
__device__ __forceinline__ double fsqrt(double x) { return x * frsq(x); }
__device__ __forceinline__ float fsqrt(float x) { return sqrtf(x); }

// Primitive state of one cell: constoprim + equation_of_state.
template <class T>
struct Prim { T r, un, ut, p, c; };

template <class T>
__device__ __forceinline__ Prim<T> euler_prim(T rho, T mn, T mt, T E, T g) {
    Prim<T> w;
    w.r = rho;
    const T ir = frcp(rho);
    w.un = mn * ir;
    w.ut = mt * ir;
    w.p = (g - T(1)) * (E - T(0.5) * rho * (w.un * w.un + w.ut * w.ut));
    w.c = fsqrt(g * w.p * ir);
    return w;
}

// van Leer limited slope from the three cell values around m
template <class T>
__device__ __forceinline__ T vanleer(T wm, T w0, T wp) {
    T a = w0 - wm, b = wp - w0;
    return (a * b > T(0)) ? T(2) * a * b * frcp(a + b) : T(0);
}

// Characteristic half-step trace to both faces.  A wave of speed >= 0
// contributes to the plus face (m+1/2), a wave of speed <= 0 to the minus
// face (m-1/2).  Outputs (rho, un, ut, p) for each face.
template <class T>
__device__ __forceinline__ void euler_trace(const Prim<T>& w, T dr, T du, T dv, T dp, T nu,
                                            T* plus, T* minus) {
    const T r = w.r, un = w.un, c = w.c;
    const T ic = frcp(c), ic2 = ic * ic;
    const T lam0 = un - c, lam1 = un, lam3 = un + c;
    const T rduc = r * du * ic;
    const T a0 = T(0.5) * (dp * ic2 - rduc);
    const T a1 = dr - dp * ic2;
    const T a2 = dv;
    const T a3 = T(0.5) * (dp * ic2 + rduc);
    const T h = T(0.5);
    T cp0 = lam0 >= T(0) ? h * (T(1) - nu * lam0) * a0 : T(0);
    T cp1 = lam1 >= T(0) ? h * (T(1) - nu * lam1) * a1 : T(0);
    T cp2 = lam1 >= T(0) ? h * (T(1) - nu * lam1) * a2 : T(0);
    T cp3 = lam3 >= T(0) ? h * (T(1) - nu * lam3) * a3 : T(0);
    T cm0 = lam0 <= T(0) ? h * (T(1) + nu * lam0) * a0 : T(0);
    T cm1 = lam1 <= T(0) ? h * (T(1) + nu * lam1) * a1 : T(0);
    T cm2 = lam1 <= T(0) ? h * (T(1) + nu * lam1) * a2 : T(0);
    T cm3 = lam3 <= T(0) ? h * (T(1) + nu * lam3) * a3 : T(0);
    const T cr = c * frcp(r), cc = c * c;
    plus[0] = r + (cp0 + cp1 + cp3);
    plus[1] = un + cr * (cp3 - cp0);
    plus[2] = w.ut + cp2;
    plus[3] = w.p + cc * (cp0 + cp3);
    minus[0] = r - (cm0 + cm1 + cm3);
    minus[1] = un - cr * (cm3 - cm0);
    minus[2] = w.ut - cm2;
    minus[3] = w.p - cc * (cm0 + cm3);
}

// x^(-6/7) for x > 0 (the rarefaction branch needs no other power: x^(1/7)
// = x * x^(-6/7)).  A single-precision hardware log2/exp2 estimate w of
// x^(-1/7) (relative error e0 ~ 1e-7) is corrected once: with
// e = 1 - x w^7, the exact factor is (1 - e)^(-1/7) = 1 + t,
// t = e/7 + 4e^2/49 + O(e^3), so x^(-6/7) = w^6 (1 + 6t + 15t^2 + O(t^3)),
// an error O(e0^3) far below double rounding.
__device__ __forceinline__ double rpow67_core(double x) {
    const float l = __builtin_amdgcn_logf((float)x);            // log2
    const double w = (double)__builtin_amdgcn_exp2f(l * (-1.0f / 7.0f));
    const double w2 = w * w, w4 = w2 * w2, w6 = w4 * w2, w7 = w6 * w;
    const double e = fma(-x, w7, 1.0);
    const double t = e * fma(e, 4.0 / 49.0, 1.0 / 7.0);
    return fma(w6, t * fma(t, 15.0, 6.0), w6);
}
// Arguments outside the single-precision normal range (rare) are first
// scaled exactly by 2^(-7k), with k from the binary exponent, and the power
// by 2^(-6k) afterwards.
__device__ __forceinline__ double rpow67(double x) {
    if (x > 1e-30 && x < 1e30) return rpow67_core(x);
    int k = __builtin_amdgcn_frexp_exp(x);                      // x = m 2^e, m in [1/2, 1)
    k = (k >= 0 ? k : k - 6) / 7;                               // floor(e / 7)
    return __builtin_amdgcn_ldexp(rpow67_core(__builtin_amdgcn_ldexp(x, -7 * k)), -6 * k);
}

// Pressure-function data of one side of the Riemann problem (Toro ch. 4).
struct Side {
    double r, u, p, c;
    double ip;      // 1/p
    double irc;     // 1/(rho c)
    double sA;      // sqrt(A), A = 2/((g+1) rho)
    double B;       // (g-1)/(g+1) p
    double k2;      // 2c/(g-1)
};

template <bool G14>
__device__ __forceinline__ Side make_side(double r, double u, double p, double g) {
    if (G14) g = 1.4;     // the gamma constants below fold at compile time
    Side s;
    s.r = r; s.u = u; s.p = p;
    const double t = frsq(g * p * r);         // 1/(rho c), since rho c = sqrt(g p rho)
    s.irc = t;
    s.c = g * p * t;                          // c = sqrt(g p / rho)
    s.ip = frcp(p);
    s.sA = sqrt(2.0 / (g + 1.0)) * frsq(r);   // sqrt(2/((g+1) rho))
    s.B = (g - 1.0) / (g + 1.0) * p;
    s.k2 = 2.0 / (g - 1.0) * s.c;
    return s;
}

// f_K(p) and f_K'(p): shock branch for p > p_K, rarefaction otherwise.
// For gamma = 7/5 the rarefaction exponents are 1/7 and -6/7, computed from
// one reciprocal seventh root.
template <bool G14>
__device__ __forceinline__ void pres_fun(const Side& s, double p, double g, double& f, double& fd) {
    if (p > s.p) {
        double rs = frsq(p + s.B);            // 1/sqrt(p+B)
        double q = s.sA * rs;
        double dp = p - s.p;
        f = dp * q;
        fd = q * (1.0 - 0.5 * dp * (rs * rs));
    } else {
        double x = p * s.ip;
        if (G14) {
            const double w6 = rpow67(x);     // x^(-6/7)
            f = s.k2 * fma(x, w6, -1.0);     // k2 (x^(1/7) - 1)
            fd = s.irc * w6;
        } else {
            f = s.k2 * (pow(x, (g - 1.0) / (2.0 * g)) - 1.0);
            fd = s.irc * pow(x, -(g + 1.0) / (2.0 * g));
        }
    }
}

// x^((g-1)/(2g)) and x^(1/g) for the sampling step.
template <bool G14>
__device__ __forceinline__ void pow_g1_ig(double x, double g, double& z, double& zig) {
    if (G14) {
        z = x * rpow67(x);             // x^(1/7)
        double z2 = z * z;
        zig = z2 * z2 * z;             // x^(5/7)
    } else {
        z = pow(x, (g - 1.0) / (2.0 * g));
        zig = pow(x, 1.0 / g);
    }
}
template <bool G14>
__device__ __forceinline__ void pow_fan(double c, double g, double& c5, double& c7) {
    if (G14) {
        double c2 = c * c;
        c5 = c2 * c2 * c;              // c^(2/(g-1))
        c7 = c5 * c2;                  // c^(2g/(g-1))
    } else {
        c5 = pow(c, 2.0 / (g - 1.0));
        c7 = pow(c, 2.0 * g / (g - 1.0));
    }
}

// One Newton step of the pressure iteration, p kept above 1e-10.  The step
// f/f' only needs a relative accuracy far below the iteration's own
// convergence, so a refined reciprocal suffices.
template <bool G14>
__device__ __forceinline__ double newton_step(const Side& lo, const Side& hi, double du, double p, double g) {
    double flo, fdlo, fhi, fdhi;
    pres_fun<G14>(lo, p, g, flo, fdlo);
    pres_fun<G14>(hi, p, g, fhi, fdhi);
    return fmax(p - (flo + fhi + du) * frcp(fdlo + fdhi), 1e-10);
}

// Earlier iterates each new Newton iterate is compared with, and the first
// step after which the comparison is made.
constexpr int NEWTON_HIST = 6;
constexpr int NEWTON_TEST_FROM = 5;

// The iterate after NI Newton steps from p0 (NI known at compile time: the
// loop is unrolled and every iterate stays in its own register).
//
// A step maps p to a value that depends on p alone (the side constants are
// fixed), so if p_K == p_{K-m} the iterates repeat with period m from
// p_{K-m} on, and p_NI = p_{K-m+((NI-K) mod m)}.  Near the root the rounding
// of f/f' leaves the iterates jittering among a few neighbouring values,
// which such a repeat soon reveals.  After each step K from NEWTON_TEST_FROM
// on, the wave stops when every active lane's p_K equals one of its last
// NEWTON_HIST iterates, and each lane takes p_NI from its own cycle: bit
// for bit the iterate after all NI steps (every iterate is at least 1e-10,
// so equal values are equal bit patterns).  Lanes never leave the loop on
// their own, so the test is a few compares and one wave vote per step.
// all_steps = true takes every step.
template <bool G14, int NI>
__device__ __forceinline__ double newton_fixed(const Side& lo, const Side& hi, double du, double p0, double g,
                                               bool all_steps) {
    double h[NI + 1];
    h[0] = p0;
#pragma unroll
    for (int k = 1; k <= NI; ++k) {
        h[k] = newton_step<G14>(lo, hi, du, h[k - 1], g);
        if (k >= NEWTON_TEST_FROM && k < NI && !all_steps) {
            bool rep = false;
#pragma unroll
            for (int m = 1; m <= NEWTON_HIST && m <= k; ++m) rep = rep || h[k] == h[k - m];
            if (__all(rep)) {
                // any m with p_K == p_{K-m} gives p_NI
                double r = h[k];
#pragma unroll
                for (int m = NEWTON_HIST; m >= 1; --m)
                    if (m <= k && h[k] == h[k - m]) r = h[k - m + (NI - k) % m];
                return r;
            }
        }
    }
    return h[NI];
}

// Exact Riemann solver sampled at x/t = 0: fixed `niter` Newton steps from
// the PVRS guess, p kept above 1e-10.  Inputs/outputs (rho, un, ut, p) in
// double.  For the usual niter = 10 the steps run unrolled with the exact
// early stop of newton_fixed (all_steps = true takes every step); any other
// count runs as a plain loop of every step.
//
// The two sides are handled as the lower- and the higher-pressure side
// (lo, hi): an iterate between the two pressures, the usual case in smooth
// flow, is a shock for lo and a rarefaction for hi in every lane, so the
// lanes of a wave take the same branch of each pressure function where
// left/right order would split them.  Every sum below is symmetric in the
// sides or takes its sign from the swap, so the results are those of the
// left/right evaluation bit for bit.
template <bool G14>
__device__ __forceinline__ void riemann0(const double* L, const double* R, double g, int niter,
                                         double* W, bool all_steps = false) {
    if (G14) g = 1.4;     // the gamma constants below fold at compile time
    const bool sw = L[3] > R[3];             // the left side has the higher pressure
    const Side lo = make_side<G14>(sw ? R[0] : L[0], sw ? R[1] : L[1], sw ? R[3] : L[3], g);
    const Side hi = make_side<G14>(sw ? L[0] : R[0], sw ? L[1] : R[1], sw ? L[3] : R[3], g);
    const double du = sw ? lo.u - hi.u : hi.u - lo.u;      // u_R - u_L
    double p = 0.5 * (lo.p + hi.p) - 0.125 * du * (lo.r + hi.r) * (lo.c + hi.c);
    p = fmax(p, 1e-10);
    if (niter == 10) {
        p = newton_fixed<G14, 10>(lo, hi, du, p, g, all_steps);
    } else {
        for (int it = 0; it < niter; ++it) p = newton_step<G14>(lo, hi, du, p, g);
    }
    double flo, fdlo, fhi, fdhi;
    pres_fun<G14>(lo, p, g, flo, fdlo);
    pres_fun<G14>(hi, p, g, fhi, fdhi);
    const double us = 0.5 * (lo.u + hi.u) + 0.5 * (sw ? flo - fhi : fhi - flo);
    const double g1 = (g - 1.0) / (2.0 * g), g2 = (g + 1.0) / (2.0 * g);
    const double g5 = 2.0 / (g + 1.0), g6 = (g - 1.0) / (g + 1.0), g7 = 0.5 * (g - 1.0);
    // sample: left of the contact when 0 <= u*
    const bool left = 0.0 <= us;
    const Side& s = left != sw ? lo : hi;
    const double sg = left ? 1.0 : -1.0;     // mirror the right side onto the left case
    const double uk = sg * s.u;              // velocity in the mirrored frame
    const double ustar = sg * us;
    W[2] = left ? L[2] : R[2];
    double rr, uu, pp;
    if (p > s.p) {                           // shock
        double pm = p * s.ip;
        double sk = uk - s.c * fsqrt(g2 * pm + g1);
        if (0.0 <= sk) { rr = s.r; uu = uk; pp = s.p; }
        else { rr = s.r * (pm + g6) * frcp(pm * g6 + 1.0); uu = ustar; pp = p; }
    } else {                                 // rarefaction
        double sh = uk - s.c;
        if (0.0 <= sh) { rr = s.r; uu = uk; pp = s.p; }
        else {
            double z, zig;
            pow_g1_ig<G14>(p * s.ip, g, z, zig);
            double st = ustar - s.c * z;
            if (0.0 > st) { rr = s.r * zig; uu = ustar; pp = p; }
            else {
                double cf = g5 + g6 * frcp(s.c) * uk;
                double c5, c7;
                pow_fan<G14>(cf, g, c5, c7);
                rr = s.r * c5;
                uu = g5 * (s.c + g7 * uk);
                pp = s.p * c7;
            }
        }
    }
    W[0] = rr;
    W[1] = sg * uu;
    W[3] = pp;
}

// Godunov flux from the sampled state (cmpflx); (rho, mn, mt, E) order.
template <class T>
__device__ __forceinline__ void euler_flux(const T* G, T g, T* F) {
    const T r = G[0], un = G[1], ut = G[2], p = G[3];
    const T et = p * frcp(g - T(1)) + T(0.5) * r * (un * un + ut * ut);
    F[0] = r * un;
    F[1] = r * un * un + p;
    F[2] = r * un * ut;
    F[3] = un * (et + p);
}

// Conservative update U - nu (F(+1/2) - F(-1/2)); accumulation type A.
template <class T, class A>
__device__ __forceinline__ T euler_update(T u, T fp, T fm, A nu) {
    return (T)((A)u - nu * ((A)fp - (A)fm));
}

// Largest signal speed of one cell, max(|u|+c, |v|+c).
template <class T>
__device__ __forceinline__ T euler_speed(T rho, T mx, T my, T E, T g) {
    const T ir = frcp(rho);
    T u = mx * ir, v = my * ir;
    T p = (g - T(1)) * (E - T(0.5) * rho * (u * u + v * v));
    T c = fsqrt(g * p * ir);
    return fmax(fabs(u) + c, fabs(v) + c);
}

// Riemann problem on T-typed face states: promotes to double for the
// pressure iteration and sampling; the result is rounded back to T.
template <class T, bool G14>
__device__ __forceinline__ void riemann_T(const T* L, const T* R, T g, int niter, T* G, bool all_steps = false) {
    double l[4] = {(double)L[0], (double)L[1], (double)L[2], (double)L[3]};
    double r[4] = {(double)R[0], (double)R[1], (double)R[2], (double)R[3]};
    double w[4];
    riemann0<G14>(l, r, (double)g, niter, w, all_steps);
    G[0] = (T)w[0]; G[1] = (T)w[1]; G[2] = (T)w[2]; G[3] = (T)w[3];
}

// atomic max of a non-negative double through its bit pattern (the order of
// non-negative IEEE doubles equals the order of their bit patterns)
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(addr),
              (unsigned long long)__double_as_longlong(v));
}

}  // namespace hfav
