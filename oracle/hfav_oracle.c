/*
 * FP64 CPU oracle for the fused stencil-chain library.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP path: no headers, no helpers, no tables.
 *
 * Every chain is evaluated rule by rule, as its own loop nest over FULL
 * intermediate arrays with explicit ghost layers filled by a separate
 * boundary step (the unfused form the paper starts from: Design, "Dataflow";
 * Hydro2D's make_boundary kernel, Performance section "Hydro2D").  Nothing is
 * fused, contracted or reordered.  OpenMP parallelises the outermost loop of
 * each nest; every cell is independent and the only reduction is an exact
 * max, so results equal a serial run bit for bit.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 *
 * Chains (the paper names the kernels but gives no formulas; the readings
 * used here are listed in the design notes of the repository):
 *   hdiff   : COSMO horizontal diffusion, Performance "COSMO Micro-Kernels"
 *   euler   : directionally split Godunov step, Performance "Hydro2D"
 *             (constoprim+eos, slope, trace, qleftright, riemann, cmpflx,
 *             update_cons_vars; exact Riemann solver after Toro, ch. 4)
 *   lap7 / biharm : 7-point Laplacian chain, Design "Reductions & broadcasts
 *             & splits" names the 7-point Laplacian as a typical kernel
 *   linear chain : generic star-stencil chain interpreter
 *   mlp     : forward/backward of the tuning cost model (3 hidden layers)
 *
 * Return codes: 0 ok, 1 bad argument, 2 allocation failure,
 *               3 non-physical state (rho<=0 or p<=0), 4 Newton clamp hit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORA_OK 0
#define ORA_EARG 1
#define ORA_ENOMEM 2
#define ORA_EPHYS 3
#define ORA_ECLAMP 4

static inline int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }
static inline int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* ======================================================================
 * Horizontal diffusion (COSMO micro-kernels: ulapstage, flux_x, flux_y,
 * ustage).  Grid in[k][j][i], periodic in i and j; planes in k are
 * independent.
 *   lap[j][i] = (in[i+1]+in[i-1]) + (in[j+1]+in[j-1]) - 4 in
 *   flx[j][i] = lap[i+1]-lap[i], set to 0 when flx*(in[i+1]-in[i]) > 0
 *   fly[j][i] = lap[j+1]-lap[j], set to 0 when fly*(in[j+1]-in[j]) > 0
 *   out       = in - coeff*((flx[i]-flx[i-1]) + (fly[j]-fly[j-1]))
 * Each stage is a separate loop over a full array with the halo it needs:
 * in with halo 2, lap with halo 1, flx on i in [-1, ni), fly on j in [-1, nj).
 * The optional stage outputs receive lap, flx, fly on the interior (nk,nj,ni).
 * ====================================================================== */
int oracle_hdiff(const double *in, double *out, int nk, int nj, int ni,
                 double coeff, int limiter,
                 double *lap_o, double *flx_o, double *fly_o)
{
    if (!in || !out || nk <= 0 || nj <= 0 || ni <= 0) return ORA_EARG;
    const int pi = ni + 4, pj = nj + 4;           /* padded in: halo 2 */
    const int li = ni + 2, lj = nj + 2;           /* lap: halo 1 */
    const size_t np = (size_t)pi * pj, nl = (size_t)li * lj;
    double *pad = malloc(sizeof(double) * np * nk);
    double *lap = malloc(sizeof(double) * nl * nk);
    double *flx = malloc(sizeof(double) * (size_t)nj * (ni + 1) * nk);
    double *fly = malloc(sizeof(double) * (size_t)(nj + 1) * ni * nk);
    if (!pad || !lap || !flx || !fly) { free(pad); free(lap); free(flx); free(fly); return ORA_ENOMEM; }

    /* make_boundary: periodic fill of the halo-2 padded copy */
    #pragma omp parallel for collapse(2)
    for (int k = 0; k < nk; ++k)
        for (int j = -2; j < nj + 2; ++j)
            for (int i = -2; i < ni + 2; ++i)
                pad[k * np + (size_t)(j + 2) * pi + (i + 2)] =
                    in[((size_t)k * nj + wrap(j, nj)) * ni + wrap(i, ni)];
#define PAD(k, j, i) pad[(k) * np + (size_t)((j) + 2) * pi + ((i) + 2)]
#define LAP(k, j, i) lap[(k) * nl + (size_t)((j) + 1) * li + ((i) + 1)]
#define FLX(k, j, i) flx[((size_t)(k) * nj + (j)) * (ni + 1) + ((i) + 1)]
#define FLY(k, j, i) fly[((size_t)(k) * (nj + 1) + ((j) + 1)) * ni + (i)]

    /* ulapstage over the halo-1 region */
    #pragma omp parallel for collapse(2)
    for (int k = 0; k < nk; ++k)
        for (int j = -1; j < nj + 1; ++j)
            for (int i = -1; i < ni + 1; ++i)
                LAP(k, j, i) = (PAD(k, j, i + 1) + PAD(k, j, i - 1)) +
                               (PAD(k, j + 1, i) + PAD(k, j - 1, i)) - 4.0 * PAD(k, j, i);

    /* flux_x on i in [-1, ni) */
    #pragma omp parallel for collapse(2)
    for (int k = 0; k < nk; ++k)
        for (int j = 0; j < nj; ++j)
            for (int i = -1; i < ni; ++i) {
                double f = LAP(k, j, i + 1) - LAP(k, j, i);
                if (limiter && f * (PAD(k, j, i + 1) - PAD(k, j, i)) > 0.0) f = 0.0;
                FLX(k, j, i) = f;
            }

    /* flux_y on j in [-1, nj) */
    #pragma omp parallel for collapse(2)
    for (int k = 0; k < nk; ++k)
        for (int j = -1; j < nj; ++j)
            for (int i = 0; i < ni; ++i) {
                double f = LAP(k, j + 1, i) - LAP(k, j, i);
                if (limiter && f * (PAD(k, j + 1, i) - PAD(k, j, i)) > 0.0) f = 0.0;
                FLY(k, j, i) = f;
            }

    /* ustage */
    #pragma omp parallel for collapse(2)
    for (int k = 0; k < nk; ++k)
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i) {
                size_t o = ((size_t)k * nj + j) * ni + i;
                out[o] = PAD(k, j, i) - coeff * ((FLX(k, j, i) - FLX(k, j, i - 1)) +
                                                 (FLY(k, j, i) - FLY(k, j - 1, i)));
                if (lap_o) lap_o[o] = LAP(k, j, i);
                if (flx_o) flx_o[o] = FLX(k, j, i);
                if (fly_o) fly_o[o] = FLY(k, j, i);
            }
#undef PAD
#undef LAP
#undef FLX
#undef FLY
    free(pad); free(lap); free(flx); free(fly);
    return ORA_OK;
}

/* ======================================================================
 * Exact Riemann solver for the ideal-gas Euler equations (Toro, "Riemann
 * Solvers and Numerical Methods for Fluid Dynamics", ch. 4): pressure
 * function, Newton iteration for the star pressure from the PVRS guess,
 * star velocity, and sampling of the self-similar solution at x/t = 0.
 * The Newton iteration runs a FIXED number of steps with no early exit and
 * keeps p above eps_p.
 * ====================================================================== */
#define EPS_P 1e-10

static void pres_fun(double p, double rk, double pk, double ck, double g,
                     double *f, double *fd)
{
    if (p > pk) {                         /* shock branch */
        double A = 2.0 / ((g + 1.0) * rk);
        double B = (g - 1.0) / (g + 1.0) * pk;
        double q = sqrt(A / (p + B));
        *f = (p - pk) * q;
        *fd = q * (1.0 - (p - pk) / (2.0 * (B + p)));
    } else {                              /* rarefaction branch */
        double pr = p / pk;
        *f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
        *fd = 1.0 / (rk * ck) * pow(pr, -(g + 1.0) / (2.0 * g));
    }
}

/* Solve for (p*, u*); returns ORA_ECLAMP if the eps_p clamp was active. */
static int star_state(const double *L, const double *R, double g, int niter,
                      double *ps, double *us)
{
    double rl = L[0], ul = L[1], pl = L[3];
    double rr = R[0], ur = R[1], pr = R[3];
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    int clamp = 0;
    double p = 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr);
    if (p < EPS_P) { p = EPS_P; clamp = 1; }
    for (int it = 0; it < niter; ++it) {
        double fl, fdl, fr, fdr;
        pres_fun(p, rl, pl, cl, g, &fl, &fdl);
        pres_fun(p, rr, pr, cr, g, &fr, &fdr);
        double f = fl + fr + (ur - ul);
        double fd = fdl + fdr;
        p = p - f / fd;
        if (p < EPS_P) { p = EPS_P; clamp = 1; }
    }
    double fl, fdl, fr, fdr;
    pres_fun(p, rl, pl, cl, g, &fl, &fdl);
    pres_fun(p, rr, pr, cr, g, &fr, &fdr);
    *ps = p;
    *us = 0.5 * (ul + ur) + 0.5 * (fr - fl);
    return clamp ? ORA_ECLAMP : ORA_OK;
}

/* Sample the solution at x/t = 0.  States are (rho, un, ut, p). */
static void sample0(const double *L, const double *R, double g, double ps, double us,
                    double *W)
{
    const double g1 = (g - 1.0) / (2.0 * g), g2 = (g + 1.0) / (2.0 * g);
    const double g3 = 2.0 * g / (g - 1.0), g4 = 2.0 / (g - 1.0);
    const double g5 = 2.0 / (g + 1.0), g6 = (g - 1.0) / (g + 1.0);
    const double g7 = (g - 1.0) / 2.0;
    if (0.0 <= us) {                                   /* left of contact */
        double rl = L[0], ul = L[1], pl = L[3], cl = sqrt(g * pl / rl);
        W[2] = L[2];
        if (ps > pl) {                                 /* left shock */
            double pml = ps / pl;
            double sl = ul - cl * sqrt(g2 * pml + g1);
            if (0.0 <= sl) { W[0] = rl; W[1] = ul; W[3] = pl; }
            else { W[0] = rl * (pml + g6) / (pml * g6 + 1.0); W[1] = us; W[3] = ps; }
        } else {                                       /* left rarefaction */
            double shl = ul - cl;
            if (0.0 <= shl) { W[0] = rl; W[1] = ul; W[3] = pl; }
            else {
                double cml = cl * pow(ps / pl, g1);
                double stl = us - cml;
                if (0.0 > stl) { W[0] = rl * pow(ps / pl, 1.0 / g); W[1] = us; W[3] = ps; }
                else {
                    double c = g5 + g6 / cl * ul;
                    W[0] = rl * pow(c, g4);
                    W[1] = g5 * (cl + g7 * ul);
                    W[3] = pl * pow(c, g3);
                }
            }
        }
    } else {                                           /* right of contact */
        double rr = R[0], ur = R[1], pr = R[3], cr = sqrt(g * pr / rr);
        W[2] = R[2];
        if (ps > pr) {                                 /* right shock */
            double pmr = ps / pr;
            double sr = ur + cr * sqrt(g2 * pmr + g1);
            if (0.0 >= sr) { W[0] = rr; W[1] = ur; W[3] = pr; }
            else { W[0] = rr * (pmr + g6) / (pmr * g6 + 1.0); W[1] = us; W[3] = ps; }
        } else {                                       /* right rarefaction */
            double shr = ur + cr;
            if (0.0 >= shr) { W[0] = rr; W[1] = ur; W[3] = pr; }
            else {
                double cmr = cr * pow(ps / pr, g1);
                double str = us + cmr;
                if (0.0 < str) { W[0] = rr * pow(ps / pr, 1.0 / g); W[1] = us; W[3] = ps; }
                else {
                    double c = g5 - g6 / cr * ur;
                    W[0] = rr * pow(c, g4);
                    W[1] = g5 * (-cr + g7 * ur);
                    W[3] = pr * pow(c, g3);
                }
            }
        }
    }
}

/* Batch interface to the Riemann solver: n problems, states (n,4) each as
 * (rho, un, ut, p).  W (n,4) receives the sampled state, pstar/ustar (n)
 * the star pressure and velocity (nullable).  Returns the number of problems
 * in which the Newton clamp was active (0 normally). */
int oracle_riemann(int n, const double *L, const double *R, double g, int niter,
                   double *W, double *pstar, double *ustar)
{
    int nclamp = 0;
    #pragma omp parallel for reduction(+:nclamp)
    for (int m = 0; m < n; ++m) {
        double ps, us;
        if (star_state(L + 4 * m, R + 4 * m, g, niter, &ps, &us) != ORA_OK) ++nclamp;
        if (pstar) pstar[m] = ps;
        if (ustar) ustar[m] = us;
        if (W) sample0(L + 4 * m, R + 4 * m, g, ps, us, W + 4 * m);
    }
    return nclamp;
}

/* Evaluate the pressure function f(p) = fL(p) + fR(p) + (uR - uL). */
void oracle_riemann_f(int n, const double *L, const double *R, double g,
                      const double *p, double *f)
{
    for (int m = 0; m < n; ++m) {
        const double *a = L + 4 * m, *b = R + 4 * m;
        double fl, fdl, fr, fdr;
        pres_fun(p[m], a[0], a[3], sqrt(g * a[3] / a[0]), g, &fl, &fdl);
        pres_fun(p[m], b[0], b[3], sqrt(g * b[3] / b[0]), g, &fr, &fdr);
        f[m] = fl + fr + (b[1] - a[1]);
    }
}

/* ======================================================================
 * One directional Godunov sweep (Hydro2D pass) over U = (rho, rho u, rho v, E)
 * stored as 4 planes of (ny, nx).  dir 0 sweeps along x (normal momentum is
 * plane 1), dir 1 along y (normal momentum is plane 2).  bc 0 periodic,
 * 1 transmissive.  Every stage is a full-array loop over all lines:
 *   make_boundary -> constoprim + equation_of_state -> slope (van Leer) ->
 *   trace (characteristic, half step) -> qleftright + riemann -> cmpflx ->
 *   update_cons_vars.
 * nu = dt/dx with dx = 1.  flux_o (nullable) receives the interface fluxes
 * as (4, nlines, n+1), interface m-1/2 at index m.
 * ====================================================================== */
typedef struct { int nlines, n; double *a; } line_arr;     /* (nlines, n+4) */

int oracle_euler_sweep(double *U, int nx, int ny, int dir, double dt, double g,
                       int bc, int niter, double *flux_o)
{
    if (!U || nx <= 0 || ny <= 0 || (dir != 0 && dir != 1)) return ORA_EARG;
    const int n = dir == 0 ? nx : ny;        /* cells along the sweep */
    const int nl = dir == 0 ? ny : nx;       /* independent lines */
    const int W4 = n + 4;                    /* line storage with halo 2 */
    const size_t S = (size_t)nl * W4;
    const size_t plane = (size_t)nx * ny;
    const int fn = dir == 0 ? 1 : 2, ft = dir == 0 ? 2 : 1;
    const double nu = dt;
    /* full intermediate arrays, all with the halo-2 line layout */
    double *buf = malloc(sizeof(double) * S * (4 + 5 + 4 + 4 + 4 + 4 + 4));
    if (!buf) return ORA_ENOMEM;
    double *Ug = buf;                /* 4: conserved with ghosts */
    double *Wp = Ug + 4 * S;         /* 5: rho, un, ut, p, c */
    double *dW = Wp + 5 * S;         /* 4: slopes */
    double *Wm = dW + 4 * S;         /* 4: face state at m+1/2 (plus side) */
    double *Wn = Wm + 4 * S;         /* 4: face state at m-1/2 (minus side) */
    double *Gs = Wn + 4 * S;         /* 4: Godunov state at m+1/2 */
    double *Fx = Gs + 4 * S;         /* 4: flux at m+1/2 */
#define LA(arr, f, l, m) (arr)[(size_t)(f) * S + (size_t)(l) * W4 + ((m) + 2)]
#define UIDX(l, m) (dir == 0 ? ((size_t)(l) * nx + (m)) : ((size_t)(m) * nx + (l)))
    int bad = 0;

    /* make_boundary: the 4 conserved planes with 2 ghost cells per side;
     * the fields are reordered to (rho, m_normal, m_transverse, E) */
    #pragma omp parallel for
    for (int l = 0; l < nl; ++l)
        for (int m = -2; m < n + 2; ++m) {
            int mm = bc == 0 ? wrap(m, n) : clampi(m, n);
            size_t s = UIDX(l, mm);
            LA(Ug, 0, l, m) = U[0 * plane + s];
            LA(Ug, 1, l, m) = U[fn * plane + s];
            LA(Ug, 2, l, m) = U[ft * plane + s];
            LA(Ug, 3, l, m) = U[3 * plane + s];
        }

    /* constoprim + equation_of_state */
    #pragma omp parallel for reduction(|:bad)
    for (int l = 0; l < nl; ++l)
        for (int m = -2; m < n + 2; ++m) {
            double r = LA(Ug, 0, l, m);
            double un = LA(Ug, 1, l, m) / r;
            double ut = LA(Ug, 2, l, m) / r;
            double e = LA(Ug, 3, l, m);
            double p = (g - 1.0) * (e - 0.5 * r * (un * un + ut * ut));
            if (!(r > 0.0) || !(p > 0.0)) bad = 1;
            LA(Wp, 0, l, m) = r;
            LA(Wp, 1, l, m) = un;
            LA(Wp, 2, l, m) = ut;
            LA(Wp, 3, l, m) = p;
            LA(Wp, 4, l, m) = sqrt(g * p / r);
        }
    if (bad) { free(buf); return ORA_EPHYS; }

    /* slope: van Leer limiter on each primitive, cells m in [-1, n] */
    #pragma omp parallel for
    for (int l = 0; l < nl; ++l)
        for (int m = -1; m < n + 1; ++m)
            for (int q = 0; q < 4; ++q) {
                double a = LA(Wp, q, l, m) - LA(Wp, q, l, m - 1);
                double b = LA(Wp, q, l, m + 1) - LA(Wp, q, l, m);
                LA(dW, q, l, m) = (a * b > 0.0) ? 2.0 * a * b / (a + b) : 0.0;
            }

    /* trace: characteristic half-step extrapolation to both faces.  A wave
     * contributes to the plus face when its speed is >= 0 and to the minus
     * face when it is <= 0 (a speed of exactly zero goes to both). */
    #pragma omp parallel for
    for (int l = 0; l < nl; ++l)
        for (int m = -1; m < n + 1; ++m) {
            double r = LA(Wp, 0, l, m), un = LA(Wp, 1, l, m), ut = LA(Wp, 2, l, m);
            double p = LA(Wp, 3, l, m), c = LA(Wp, 4, l, m);
            double dr = LA(dW, 0, l, m), du = LA(dW, 1, l, m);
            double dv = LA(dW, 2, l, m), dp = LA(dW, 3, l, m);
            double lam[4] = {un - c, un, un, un + c};    /* -, entropy, shear, + */
            double alp[4] = {0.5 * (dp / (c * c) - r * du / c),
                             dr - dp / (c * c),
                             dv,
                             0.5 * (dp / (c * c) + r * du / c)};
            double cp[4], cm[4];
            for (int w = 0; w < 4; ++w) {
                cp[w] = lam[w] >= 0.0 ? 0.5 * (1.0 - nu * lam[w]) * alp[w] : 0.0;
                cm[w] = lam[w] <= 0.0 ? 0.5 * (1.0 + nu * lam[w]) * alp[w] : 0.0;
            }
            /* right eigenvectors in (rho, un, ut, p):
             * r- = (1, -c/rho, 0, c^2), r0 = (1,0,0,0), rt = (0,0,1,0),
             * r+ = (1, c/rho, 0, c^2) */
            LA(Wm, 0, l, m) = r + (cp[0] + cp[1] + cp[3]);
            LA(Wm, 1, l, m) = un + (c / r) * (cp[3] - cp[0]);
            LA(Wm, 2, l, m) = ut + cp[2];
            LA(Wm, 3, l, m) = p + c * c * (cp[0] + cp[3]);
            LA(Wn, 0, l, m) = r - (cm[0] + cm[1] + cm[3]);
            LA(Wn, 1, l, m) = un - (c / r) * (cm[3] - cm[0]);
            LA(Wn, 2, l, m) = ut - cm[2];
            LA(Wn, 3, l, m) = p - c * c * (cm[0] + cm[3]);
        }

    /* qleftright + riemann at interfaces m+1/2, m in [-1, n) */
    int nclamp = 0;
    #pragma omp parallel for reduction(+:nclamp) reduction(|:bad)
    for (int l = 0; l < nl; ++l)
        for (int m = -1; m < n; ++m) {
            double L[4], R[4], W[4], ps, us;
            for (int q = 0; q < 4; ++q) { L[q] = LA(Wm, q, l, m); R[q] = LA(Wn, q, l, m + 1); }
            if (!(L[0] > 0.0) || !(L[3] > 0.0) || !(R[0] > 0.0) || !(R[3] > 0.0)) { bad = 1; continue; }
            if (star_state(L, R, g, niter, &ps, &us) != ORA_OK) ++nclamp;
            sample0(L, R, g, ps, us, W);
            for (int q = 0; q < 4; ++q) LA(Gs, q, l, m) = W[q];
        }
    if (bad) { free(buf); return ORA_EPHYS; }

    /* cmpflx */
    #pragma omp parallel for
    for (int l = 0; l < nl; ++l)
        for (int m = -1; m < n; ++m) {
            double r = LA(Gs, 0, l, m), un = LA(Gs, 1, l, m);
            double ut = LA(Gs, 2, l, m), p = LA(Gs, 3, l, m);
            double et = p / (g - 1.0) + 0.5 * r * (un * un + ut * ut);
            LA(Fx, 0, l, m) = r * un;
            LA(Fx, 1, l, m) = r * un * un + p;
            LA(Fx, 2, l, m) = r * un * ut;
            LA(Fx, 3, l, m) = un * (et + p);
        }

    /* update_cons_vars */
    #pragma omp parallel for
    for (int l = 0; l < nl; ++l)
        for (int m = 0; m < n; ++m) {
            size_t s = UIDX(l, m);
            U[0 * plane + s] = LA(Ug, 0, l, m) - nu * (LA(Fx, 0, l, m) - LA(Fx, 0, l, m - 1));
            U[fn * plane + s] = LA(Ug, 1, l, m) - nu * (LA(Fx, 1, l, m) - LA(Fx, 1, l, m - 1));
            U[ft * plane + s] = LA(Ug, 2, l, m) - nu * (LA(Fx, 2, l, m) - LA(Fx, 2, l, m - 1));
            U[3 * plane + s] = LA(Ug, 3, l, m) - nu * (LA(Fx, 3, l, m) - LA(Fx, 3, l, m - 1));
        }
    if (flux_o) {
        /* fluxes mapped back to (rho, rho u, rho v, E) order */
        #pragma omp parallel for
        for (int l = 0; l < nl; ++l)
            for (int m = -1; m < n; ++m) {
                size_t o = (size_t)l * (n + 1) + (m + 1);
                size_t st = (size_t)nl * (n + 1);
                flux_o[0 * st + o] = LA(Fx, 0, l, m);
                flux_o[fn * st + o] = LA(Fx, 1, l, m);
                flux_o[ft * st + o] = LA(Fx, 2, l, m);
                flux_o[3 * st + o] = LA(Fx, 3, l, m);
            }
    }
#undef LA
#undef UIDX
    free(buf);
    return nclamp ? ORA_ECLAMP : ORA_OK;
}

/* Largest signal speed max(|u|+c, |v|+c) over all cells (the CFL reduction:
 * an associative max, Design "Reductions & broadcasts & splits"). */
double oracle_euler_smax(const double *U, int nx, int ny, double g)
{
    const size_t plane = (size_t)nx * ny;
    double smax = 0.0;
    #pragma omp parallel for reduction(max:smax)
    for (size_t s = 0; s < plane; ++s) {
        double r = U[s], u = U[plane + s] / r, v = U[2 * plane + s] / r;
        double p = (g - 1.0) * (U[3 * plane + s] - 0.5 * r * (u * u + v * v));
        double c = sqrt(g * p / r);
        double a = fabs(u) + c, b = fabs(v) + c;
        double m = a > b ? a : b;
        if (m > smax) smax = m;
    }
    return smax;
}

/* nsteps of the split scheme: dt = cfl/smax on the state at the start of
 * each step, then the x sweep and the y sweep with that dt.  dts (nullable)
 * receives the dt of every step. */
int oracle_euler_run(double *U, int nx, int ny, int nsteps, double g, double cfl,
                     int bc, int niter, double *dts)
{
    int rc = ORA_OK;
    for (int s = 0; s < nsteps; ++s) {
        double smax = oracle_euler_smax(U, nx, ny, g);
        double dt = cfl / smax;
        if (dts) dts[s] = dt;
        int r1 = oracle_euler_sweep(U, nx, ny, 0, dt, g, bc, niter, NULL);
        if (r1 != ORA_OK && r1 != ORA_ECLAMP) return r1;
        int r2 = oracle_euler_sweep(U, nx, ny, 1, dt, g, bc, niter, NULL);
        if (r2 != ORA_OK && r2 != ORA_ECLAMP) return r2;
        if (r1 || r2) rc = ORA_ECLAMP;
    }
    return rc;
}

/* ======================================================================
 * 7-point Laplacian chain on a periodic (nz, ny, nx) box:
 *   lap = ((u[i+1]+u[i-1]) + (u[j+1]+u[j-1])) + (u[k+1]+u[k-1]) - 6u
 * biharm: lap1 = L7(u), lap2 = L7(lap1), out = u - nu*lap2, each a full
 * array pass with its own periodic boundary fill.
 * ====================================================================== */
static void lap7_full(const double *u, double *o, int nz, int ny, int nx)
{
    #pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
#define U3(kk, jj, ii) u[((size_t)wrap(kk, nz) * ny + wrap(jj, ny)) * nx + wrap(ii, nx)]
                o[((size_t)k * ny + j) * nx + i] =
                    ((U3(k, j, i + 1) + U3(k, j, i - 1)) + (U3(k, j + 1, i) + U3(k, j - 1, i))) +
                    (U3(k + 1, j, i) + U3(k - 1, j, i)) - 6.0 * U3(k, j, i);
#undef U3
            }
}

int oracle_lap7(const double *u, double *o, int nz, int ny, int nx)
{
    if (!u || !o || nz <= 0 || ny <= 0 || nx <= 0) return ORA_EARG;
    lap7_full(u, o, nz, ny, nx);
    return ORA_OK;
}

int oracle_biharm(const double *u, double *out, int nz, int ny, int nx, double nu,
                  int nsteps, double *lap1_o, double *lap2_o)
{
    if (!u || !out || nz <= 0 || ny <= 0 || nx <= 0 || nsteps < 1) return ORA_EARG;
    const size_t N = (size_t)nz * ny * nx;
    double *l1 = malloc(sizeof(double) * N), *l2 = malloc(sizeof(double) * N);
    double *cur = malloc(sizeof(double) * N);
    if (!l1 || !l2 || !cur) { free(l1); free(l2); free(cur); return ORA_ENOMEM; }
    memcpy(cur, u, sizeof(double) * N);
    for (int s = 0; s < nsteps; ++s) {
        lap7_full(cur, l1, nz, ny, nx);
        lap7_full(l1, l2, nz, ny, nx);
        #pragma omp parallel for
        for (size_t q = 0; q < N; ++q) out[q] = cur[q] - nu * l2[q];
        if (s + 1 < nsteps) memcpy(cur, out, sizeof(double) * N);
    }
    if (lap1_o) memcpy(lap1_o, l1, sizeof(double) * N);
    if (lap2_o) memcpy(lap2_o, l2, sizeof(double) * N);
    free(l1); free(l2); free(cur);
    return ORA_OK;
}

/* ======================================================================
 * Normalisation example (Design, "Reductions & broadcasts & splits";
 * Performance, "Normalization Example"): one-dimensional flux differences
 * of a system of nq fields u[q][j][i], each row's flux vectors normalised
 * by the row's norm.  Along i the row end wraps (periodic != 0) or repeats
 * the last cell (transmissive: the last flux is 0).  Five kernels visit the
 * (j, i) space, one kernel works on rows only:
 *   flux      f[q][j][i] = u[q][j][i+1] - u[q][j][i]
 *   square    e[j][i]    = sum_q f[q][j][i]^2                (q order)
 *   accumulate s[j]      = sum_i e[j][i]  (init 0, i order; rank 2 -> 1)
 *   root      n[j]       = sqrt(s[j])                        (rank 1)
 *   divide    d[q][j][i] = f[q][j][i] / n[j]   (0 when n[j] = 0; broadcast)
 *   update    out[q][j][i] = u[q][j][i] - c d[q][j][i]
 * Each kernel is a full-array pass.  n_o (nullable) receives n (nj).
 * ====================================================================== */
int oracle_normalize(const double *u, double *out, int nq, int nj, int ni, double c, int periodic,
                     double *n_o)
{
    if (!u || !out || nq <= 0 || nj <= 0 || ni <= 0) return ORA_EARG;
    const size_t P = (size_t)nj * ni;
    double *f = malloc(sizeof(double) * P * nq), *e = malloc(sizeof(double) * P);
    double *d = malloc(sizeof(double) * P * nq), *sn = malloc(sizeof(double) * nj);
    double *nn = malloc(sizeof(double) * nj);
    if (!f || !e || !d || !sn || !nn) { free(f); free(e); free(d); free(sn); free(nn); return ORA_ENOMEM; }
    #pragma omp parallel for collapse(2)
    for (int q = 0; q < nq; ++q)
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i)
                f[q * P + (size_t)j * ni + i] =
                    u[q * P + (size_t)j * ni + (periodic ? wrap(i + 1, ni) : clampi(i + 1, ni))] -
                    u[q * P + (size_t)j * ni + i];
    #pragma omp parallel for
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            double acc = 0.0;
            for (int q = 0; q < nq; ++q) {
                double v = f[q * P + (size_t)j * ni + i];
                acc += v * v;
            }
            e[(size_t)j * ni + i] = acc;
        }
    #pragma omp parallel for
    for (int j = 0; j < nj; ++j) {
        double acc = 0.0;
        for (int i = 0; i < ni; ++i) acc += e[(size_t)j * ni + i];
        sn[j] = acc;
    }
    for (int j = 0; j < nj; ++j) nn[j] = sqrt(sn[j]);
    #pragma omp parallel for collapse(2)
    for (int q = 0; q < nq; ++q)
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i)
                d[q * P + (size_t)j * ni + i] = nn[j] > 0.0 ? f[q * P + (size_t)j * ni + i] / nn[j] : 0.0;
    #pragma omp parallel for collapse(2)
    for (int q = 0; q < nq; ++q)
        for (int j = 0; j < nj; ++j)
            for (int i = 0; i < ni; ++i) {
                size_t o = q * P + (size_t)j * ni + i;
                out[o] = u[o] - c * d[o];
            }
    if (n_o) memcpy(n_o, nn, sizeof(double) * nj);
    free(f); free(e); free(d); free(sn); free(nn);
    return ORA_OK;
}

/* ======================================================================
 * Generic linear star-stencil chain interpreter.  Stage s maps f_in fields
 * to f_out fields:  out[o](x) = sum_f sum_q c[o][f][q] * in[f](x + off[q]),
 * accumulated from 0 in (f, q) order, periodic on every axis.  Offsets of
 * all stages are packed as int triples (di, dj, dk); coefficients packed per
 * stage as (f_out, f_in, n_off).  Each stage is a full-array pass.
 * ====================================================================== */
int oracle_linear_chain(int nstage, const int *f_io /* nstage+1 */, const int *n_off,
                        const int *offs, const double *coeff,
                        const double *in, double *out, int nz, int ny, int nx)
{
    if (nstage < 1 || !f_io || !n_off || !offs || !coeff || !in || !out) return ORA_EARG;
    const size_t N = (size_t)nz * ny * nx;
    int fmax = 0;
    for (int s = 0; s <= nstage; ++s) fmax = f_io[s] > fmax ? f_io[s] : fmax;
    double *a = malloc(sizeof(double) * N * fmax), *b = malloc(sizeof(double) * N * fmax);
    if (!a || !b) { free(a); free(b); return ORA_ENOMEM; }
    memcpy(a, in, sizeof(double) * N * f_io[0]);
    const int *op = offs;
    const double *cp = coeff;
    for (int s = 0; s < nstage; ++s) {
        int fi = f_io[s], fo = f_io[s + 1], no = n_off[s];
        #pragma omp parallel for collapse(2)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    for (int o = 0; o < fo; ++o) {
                        double acc = 0.0;
                        for (int f = 0; f < fi; ++f)
                            for (int q = 0; q < no; ++q) {
                                int ii = wrap(i + op[3 * q], nx), jj = wrap(j + op[3 * q + 1], ny);
                                int kk = wrap(k + op[3 * q + 2], nz);
                                acc += cp[((size_t)o * fi + f) * no + q] *
                                       a[(size_t)f * N + ((size_t)kk * ny + jj) * nx + ii];
                            }
                        b[(size_t)o * N + ((size_t)k * ny + j) * nx + i] = acc;
                    }
        double *t = a; a = b; b = t;
        op += 3 * no;
        cp += (size_t)fo * fi * no;
    }
    memcpy(out, a, sizeof(double) * N * f_io[nstage]);
    free(a); free(b);
    return ORA_OK;
}

/* ======================================================================
 * Tuning cost model: a multilayer perceptron with 3 hidden ReLU layers of
 * width H and one linear output, trained on mean squared error.
 * Parameter layout (flat, row-major weights W[out][in]):
 *   W1 (H,d) b1 (H) W2 (H,H) b2 (H) W3 (H,H) b3 (H) W4 (1,H) b4 (1)
 * ====================================================================== */
size_t oracle_mlp_nparams(int d, int H) { return (size_t)H * d + H + 2 * ((size_t)H * H + H) + H + 1; }

static void dense(const double *W, const double *b, const double *x, double *y,
                  int nout, int nin, int relu)
{
    for (int o = 0; o < nout; ++o) {
        double acc = b[o];
        for (int i = 0; i < nin; ++i) acc += W[(size_t)o * nin + i] * x[i];
        y[o] = relu ? (acc > 0.0 ? acc : 0.0) : acc;
    }
}

int oracle_mlp_forward(int n, int d, int H, const double *x, const double *P, double *y)
{
    if (H < 1 || H > 512) return ORA_EARG;   /* hidden activations live on the stack */
    const double *W1 = P, *b1 = W1 + (size_t)H * d, *W2 = b1 + H, *b2 = W2 + (size_t)H * H;
    const double *W3 = b2 + H, *b3 = W3 + (size_t)H * H, *W4 = b3 + H, *b4 = W4 + H;
    #pragma omp parallel for
    for (int s = 0; s < n; ++s) {
        double h1[512], h2[512], h3[512];
        dense(W1, b1, x + (size_t)s * d, h1, H, d, 1);
        dense(W2, b2, h1, h2, H, H, 1);
        dense(W3, b3, h2, h3, H, H, 1);
        dense(W4, b4, h3, y + s, 1, H, 0);
    }
    return 0;
}

/* Loss L = mean_s (y_s - t_s)^2 and its gradient with respect to every
 * parameter (same layout as P), by reverse-mode chain rule, serial. */
double oracle_mlp_loss_grad(int n, int d, int H, const double *x, const double *t,
                            const double *P, double *G)
{
    if (H > 512) return NAN;
    const size_t np = oracle_mlp_nparams(d, H);
    const double *W1 = P, *b1 = W1 + (size_t)H * d, *W2 = b1 + H, *b2 = W2 + (size_t)H * H;
    const double *W3 = b2 + H, *b3 = W3 + (size_t)H * H, *W4 = b3 + H, *b4 = W4 + H;
    double *gW1 = G, *gb1 = gW1 + (size_t)H * d, *gW2 = gb1 + H, *gb2 = gW2 + (size_t)H * H;
    double *gW3 = gb2 + H, *gb3 = gW3 + (size_t)H * H, *gW4 = gb3 + H, *gb4 = gW4 + H;
    memset(G, 0, sizeof(double) * np);
    double loss = 0.0;
    for (int s = 0; s < n; ++s) {
        const double *xs = x + (size_t)s * d;
        double h1[512], h2[512], h3[512], y;
        dense(W1, b1, xs, h1, H, d, 1);
        dense(W2, b2, h1, h2, H, H, 1);
        dense(W3, b3, h2, h3, H, H, 1);
        dense(W4, b4, h3, &y, 1, H, 0);
        double r = y - t[s];
        loss += r * r;
        double dy = 2.0 * r / n;
        double d3[512], d2[512], d1[512];
        gb4[0] += dy;
        for (int i = 0; i < H; ++i) {
            gW4[i] += dy * h3[i];
            d3[i] = h3[i] > 0.0 ? dy * W4[i] : 0.0;
        }
        for (int o = 0; o < H; ++o) {
            gb3[o] += d3[o];
            for (int i = 0; i < H; ++i) gW3[(size_t)o * H + i] += d3[o] * h2[i];
        }
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) acc += W3[(size_t)o * H + i] * d3[o];
            d2[i] = h2[i] > 0.0 ? acc : 0.0;
        }
        for (int o = 0; o < H; ++o) {
            gb2[o] += d2[o];
            for (int i = 0; i < H; ++i) gW2[(size_t)o * H + i] += d2[o] * h1[i];
        }
        for (int i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) acc += W2[(size_t)o * H + i] * d2[o];
            d1[i] = h1[i] > 0.0 ? acc : 0.0;
        }
        for (int o = 0; o < H; ++o) {
            gb1[o] += d1[o];
            for (int i = 0; i < d; ++i) gW1[(size_t)o * d + i] += d1[o] * xs[i];
        }
    }
    return loss / n;
}

/* One Adam step (Kingma & Ba, 2015) with bias correction at step t >= 1. */
void oracle_adam_step(size_t np, double *P, const double *G, double *m, double *v,
                      double lr, double b1, double b2, double eps, int t)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (size_t q = 0; q < np; ++q) {
        m[q] = b1 * m[q] + (1.0 - b1) * G[q];
        v[q] = b2 * v[q] + (1.0 - b2) * G[q] * G[q];
        double mh = m[q] / c1, vh = v[q] / c2;
        P[q] -= lr * mh / (sqrt(vh) + eps);
    }
}
