"""Brute-force evaluators for tiny grids (test infrastructure).

Each goal cell is computed by direct recursion through the rules with the
boundary applied as index arithmetic at every access: no ghost arrays, no
intermediate arrays, no loop nests.  This is the independent check of the
oracle's offsets, halos and rule wiring.  Pure Python; use only on grids of
a few hundred cells.
"""
from __future__ import annotations

import functools
import math


def _w(i, n):
    return i % n


# ----------------------------------------------------------------- hdiff
def hdiff_cell(a, k, j, i, coeff=0.025, limiter=True):
    nk, nj, ni = a.shape

    def u(jj, ii):
        return float(a[k, _w(jj, nj), _w(ii, ni)])

    def lap(jj, ii):
        return (u(jj, ii + 1) + u(jj, ii - 1)) + (u(jj + 1, ii) + u(jj - 1, ii)) - 4.0 * u(jj, ii)

    def flx(jj, ii):
        f = lap(jj, ii + 1) - lap(jj, ii)
        if limiter and f * (u(jj, ii + 1) - u(jj, ii)) > 0.0:
            f = 0.0
        return f

    def fly(jj, ii):
        f = lap(jj + 1, ii) - lap(jj, ii)
        if limiter and f * (u(jj + 1, ii) - u(jj, ii)) > 0.0:
            f = 0.0
        return f

    return u(j, i) - coeff * ((flx(j, i) - flx(j, i - 1)) + (fly(j, i) - fly(j - 1, i)))


# ----------------------------------------------------------------- lap7 chains
def lap7_cell(f, k, j, i, shape):
    nz, ny, nx = shape
    g = lambda kk, jj, ii: f(_w(kk, nz), _w(jj, ny), _w(ii, nx))
    return ((g(k, j, i + 1) + g(k, j, i - 1)) + (g(k, j + 1, i) + g(k, j - 1, i))) + \
        (g(k + 1, j, i) + g(k - 1, j, i)) - 6.0 * g(k, j, i)


def biharm_cell(a, k, j, i, nu):
    shape = a.shape
    u = lambda kk, jj, ii: float(a[kk, jj, ii])
    l1 = lambda kk, jj, ii: lap7_cell(u, kk, jj, ii, shape)
    return u(k, j, i) - nu * lap7_cell(l1, k, j, i, shape)


def linear_chain_cell(chain, inp, offsets_fn, o, k, j, i):
    """Output field o at (k, j, i) of a linear star chain, by recursion."""
    _, nz, ny, nx = inp.shape
    stages = chain["stages"]
    offs = [offsets_fn(chain["ndim"], s["r"]) for s in stages]

    # memoised recursion: each (stage, field, cell) value is computed once
    @functools.lru_cache(maxsize=None)
    def val(s, f, kk, jj, ii):
        kk, jj, ii = _w(kk, nz), _w(jj, ny), _w(ii, nx)
        if s == 0:
            return float(inp[f, kk, jj, ii])
        st = stages[s - 1]
        acc = 0.0
        for ff in range(st["f_in"]):
            for q, (di, dj, dk) in enumerate(offs[s - 1]):
                acc += float(st["coeff"][f, ff, q]) * val(s - 1, ff, kk + dk, jj + dj, ii + di)
        return acc

    return val(len(stages), o, k, j, i)


# ----------------------------------------------------------------- euler
def _pf(p, rk, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rk)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - (p - pk) / (2.0 * (B + p)))
    pr = p / pk
    return (2.0 * ck / (g - 1.0) * (math.pow(pr, (g - 1.0) / (2.0 * g)) - 1.0),
            1.0 / (rk * ck) * math.pow(pr, -(g + 1.0) / (2.0 * g)))


def riemann0(L, R, g, niter=10):
    """Exact Riemann solution at x/t = 0 (Toro ch. 4); states (rho, un, ut, p)."""
    rl, ul, vl, pl = L
    rr, ur, vr, pr = R
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr)
    p = max(p, 1e-10)
    for _ in range(niter):
        fl, dl = _pf(p, rl, pl, cl, g)
        fr, dr = _pf(p, rr, pr, cr, g)
        p = max(p - (fl + fr + (ur - ul)) / (dl + dr), 1e-10)
    fl, _ = _pf(p, rl, pl, cl, g)
    fr, _ = _pf(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    g1 = (g - 1.0) / (2.0 * g)
    g2 = (g + 1.0) / (2.0 * g)
    g6 = (g - 1.0) / (g + 1.0)
    if 0.0 <= u:
        if p > pl:
            if 0.0 <= ul - cl * math.sqrt(g2 * p / pl + g1):
                return (rl, ul, vl, pl)
            return (rl * (p / pl + g6) / (p / pl * g6 + 1.0), u, vl, p)
        if 0.0 <= ul - cl:
            return (rl, ul, vl, pl)
        if 0.0 > u - cl * math.pow(p / pl, g1):
            return (rl * math.pow(p / pl, 1.0 / g), u, vl, p)
        c = 2.0 / (g + 1.0) + g6 / cl * ul
        return (rl * math.pow(c, 2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul),
                vl, pl * math.pow(c, 2.0 * g / (g - 1.0)))
    if p > pr:
        if 0.0 >= ur + cr * math.sqrt(g2 * p / pr + g1):
            return (rr, ur, vr, pr)
        return (rr * (p / pr + g6) / (p / pr * g6 + 1.0), u, vr, p)
    if 0.0 >= ur + cr:
        return (rr, ur, vr, pr)
    if 0.0 < u + cr * math.pow(p / pr, g1):
        return (rr * math.pow(p / pr, 1.0 / g), u, vr, p)
    c = 2.0 / (g + 1.0) - g6 / cr * ur
    return (rr * math.pow(c, 2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur),
            vr, pr * math.pow(c, 2.0 * g / (g - 1.0)))


def euler_sweep_bf(U, direction, dt, g=1.4):
    """One periodic sweep by per-cell recursion.  U: nested (4, ny, nx) numpy."""
    _, ny, nx = U.shape
    fn, ft = (1, 2) if direction == 0 else (2, 1)

    def cons(l, m):
        if direction == 0:
            jj, ii = l, _w(m, nx)
        else:
            jj, ii = _w(m, ny), l
        return (float(U[0, jj, ii]), float(U[fn, jj, ii]), float(U[ft, jj, ii]), float(U[3, jj, ii]))

    def prim(l, m):
        r, mn, mt, e = cons(l, m)
        un, ut = mn / r, mt / r
        p = (g - 1.0) * (e - 0.5 * r * (un * un + ut * ut))
        return (r, un, ut, p, math.sqrt(g * p / r))

    def slope(l, m):
        a0, a1, a2 = prim(l, m - 1), prim(l, m), prim(l, m + 1)
        out = []
        for q in range(4):
            a = a1[q] - a0[q]
            b = a2[q] - a1[q]
            out.append(2.0 * a * b / (a + b) if a * b > 0.0 else 0.0)
        return out

    def faces(l, m):
        r, un, ut, p, c = prim(l, m)
        dr, du, dv, dp = slope(l, m)
        lam = (un - c, un, un, un + c)
        alp = (0.5 * (dp / (c * c) - r * du / c), dr - dp / (c * c), dv,
               0.5 * (dp / (c * c) + r * du / c))
        cp = [0.5 * (1.0 - dt * lam[w]) * alp[w] if lam[w] >= 0.0 else 0.0 for w in range(4)]
        cm = [0.5 * (1.0 + dt * lam[w]) * alp[w] if lam[w] <= 0.0 else 0.0 for w in range(4)]
        plus = (r + (cp[0] + cp[1] + cp[3]), un + (c / r) * (cp[3] - cp[0]), ut + cp[2],
                p + c * c * (cp[0] + cp[3]))
        minus = (r - (cm[0] + cm[1] + cm[3]), un - (c / r) * (cm[3] - cm[0]), ut - cm[2],
                 p - c * c * (cm[0] + cm[3]))
        return plus, minus

    def flux(l, m):       # interface m + 1/2
        r, un, ut, p = riemann0(faces(l, m)[0], faces(l, m + 1)[1], g)
        et = p / (g - 1.0) + 0.5 * r * (un * un + ut * ut)
        return (r * un, r * un * un + p, r * un * ut, un * (et + p))

    V = U.copy()
    nl, n = (ny, nx) if direction == 0 else (nx, ny)
    for l in range(nl):
        for m in range(n):
            Fp, Fm = flux(l, m), flux(l, m - 1)
            c = cons(l, m)
            new = [c[q] - dt * (Fp[q] - Fm[q]) for q in range(4)]
            jj, ii = (l, m) if direction == 0 else (m, l)
            V[0, jj, ii], V[fn, jj, ii], V[ft, jj, ii], V[3, jj, ii] = new
    return V


def euler_smax_bf(U, g=1.4):
    s = 0.0
    _, ny, nx = U.shape
    for j in range(ny):
        for i in range(nx):
            r = float(U[0, j, i])
            u = float(U[1, j, i]) / r
            v = float(U[2, j, i]) / r
            p = (g - 1.0) * (float(U[3, j, i]) - 0.5 * r * (u * u + v * v))
            c = math.sqrt(g * p / r)
            s = max(s, abs(u) + c, abs(v) + c)
    return s


def normalize_bf(u, c, periodic=True):
    """Normalisation example from its definition, with plain loops: flux
    differences along i (the right neighbour of the last cell is the first
    cell, or the last cell itself when not periodic), the row norm over all
    flux vectors of the row, and out = u - c f / norm (0 where the norm is
    0)."""
    nq, nj, ni = len(u), len(u[0]), len(u[0][0])
    out = [[[0.0] * ni for _ in range(nj)] for _ in range(nq)]
    norms = []
    for j in range(nj):
        right = [(i + 1) % ni if periodic else min(i + 1, ni - 1) for i in range(ni)]
        f = [[u[q][j][right[i]] - u[q][j][i] for i in range(ni)] for q in range(nq)]
        s = 0.0
        for i in range(ni):
            for q in range(nq):
                s += f[q][i] * f[q][i]
        n = math.sqrt(s)
        norms.append(n)
        for q in range(nq):
            for i in range(ni):
                out[q][j][i] = u[q][j][i] - c * (f[q][i] / n if n > 0 else 0.0)
    return out, norms
