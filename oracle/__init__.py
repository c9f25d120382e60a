"""FP64 CPU oracle: numpy front-end to liboracle.so.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the library's product path never
imports this package and shares no code with it.

Every function evaluates a chain rule by rule over full intermediate arrays
(the unfused starting point of the paper, Design section "Dataflow"), in FP64.
Functions whose result is not pinned by an independent check say so in their
docstring ("parity unpinned"); all current entry points are pinned by the
tests in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HFAV_ORACLE_LIB points the tests at a deliberately broken build of the
# oracle (tests/test_oracle_mutations.py checks that the pins catch it)
_LIB_PATH = os.environ.get("HFAV_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.oracle_hdiff.argtypes = [_dp, _dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                 _dp, _dp, _dp]
    lib.oracle_riemann.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, _dp, _dp, _dp]
    lib.oracle_riemann_f.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp, _dp]
    lib.oracle_riemann_f.restype = None
    lib.oracle_euler_sweep.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                       C.c_int, C.c_int, _dp]
    lib.oracle_euler_smax.argtypes = [_dp, C.c_int, C.c_int, C.c_double]
    lib.oracle_euler_smax.restype = C.c_double
    lib.oracle_euler_run.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                     C.c_int, C.c_int, _dp]
    lib.oracle_lap7.argtypes = [_dp, _dp, C.c_int, C.c_int, C.c_int]
    lib.oracle_normalize.argtypes = [_dp, _dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, _dp]
    lib.oracle_biharm.argtypes = [_dp, _dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                  _dp, _dp]
    lib.oracle_linear_chain.argtypes = [C.c_int, _ip, _ip, _ip, _dp, _dp, _dp,
                                        C.c_int, C.c_int, C.c_int]
    lib.oracle_mlp_nparams.argtypes = [C.c_int, C.c_int]
    lib.oracle_mlp_nparams.restype = C.c_size_t
    lib.oracle_mlp_forward.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
    lib.oracle_mlp_forward.restype = C.c_int
    lib.oracle_mlp_loss_grad.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp]
    lib.oracle_mlp_loss_grad.restype = C.c_double
    lib.oracle_adam_step.argtypes = [C.c_size_t, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                     C.c_double, C.c_double, C.c_int]
    lib.oracle_adam_step.restype = None
    lib.oracle_num_threads.restype = C.c_int
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_set_threads.restype = None
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


class OracleError(RuntimeError):
    pass


_RC = {1: "bad argument", 2: "out of memory", 3: "non-physical state (rho<=0 or p<=0)",
       4: "Newton pressure clamp active"}


def _check(rc, allow_clamp=False):
    if rc == 0 or (allow_clamp and rc == 4):
        return
    raise OracleError(_RC.get(rc, f"oracle error {rc}"))


# ------------------------------------------------------------------ hdiff
HDIFF_COEFF = 0.025


def hdiff(inp, coeff=HDIFF_COEFF, limiter=True, stages=False):
    """Horizontal-diffusion chain on (nk, nj, ni), periodic in i and j.

    COSMO micro-kernels (Performance section, "COSMO Micro-Kernels"):
    ulapstage -> flux_x, flux_y -> ustage.  Returns out, or
    (out, lap, flx, fly) when `stages` is true.
    """
    a = _f64(inp)
    nk, nj, ni = a.shape
    out = np.empty_like(a)
    lap = np.empty_like(a) if stages else None
    flx = np.empty_like(a) if stages else None
    fly = np.empty_like(a) if stages else None
    _check(_load().oracle_hdiff(_ptr(a), _ptr(out), nk, nj, ni, float(coeff), int(bool(limiter)),
                                _ptr(lap), _ptr(flx), _ptr(fly)))
    return (out, lap, flx, fly) if stages else out


# ------------------------------------------------------------------ euler
GAMMA = 1.4
CFL = 0.5
NEWTON_ITERS = 10
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1


def riemann(WL, WR, gamma=GAMMA, niter=NEWTON_ITERS):
    """Exact Riemann solver sampled at x/t=0 for n problems.

    WL, WR: (n, 4) primitive states (rho, u_normal, u_transverse, p).
    Returns (W, pstar, ustar, nclamp).
    """
    L = _f64(np.atleast_2d(WL))
    R = _f64(np.atleast_2d(WR))
    n = L.shape[0]
    W = np.empty((n, 4))
    ps = np.empty(n)
    us = np.empty(n)
    nclamp = _load().oracle_riemann(n, _ptr(L), _ptr(R), float(gamma), int(niter),
                                    _ptr(W), _ptr(ps), _ptr(us))
    return W, ps, us, nclamp


def riemann_f(WL, WR, p, gamma=GAMMA):
    """The pressure function f(p) = fL(p) + fR(p) + (uR-uL) at given p."""
    L = _f64(np.atleast_2d(WL))
    R = _f64(np.atleast_2d(WR))
    pp = _f64(np.atleast_1d(p))
    f = np.empty(L.shape[0])
    _load().oracle_riemann_f(L.shape[0], _ptr(L), _ptr(R), float(gamma), _ptr(pp), _ptr(f))
    return f


def euler_sweep(U, direction, dt, gamma=GAMMA, bc=BC_PERIODIC, niter=NEWTON_ITERS,
                fluxes=False):
    """One directional Godunov sweep; returns the new state (and fluxes).

    U: (4, ny, nx) conserved (rho, rho u, rho v, E); direction 0 = x, 1 = y.
    """
    V = _f64(U).copy()
    _, ny, nx = V.shape
    n, nl = (nx, ny) if direction == 0 else (ny, nx)
    F = np.empty((4, nl, n + 1)) if fluxes else None
    _check(_load().oracle_euler_sweep(_ptr(V), nx, ny, int(direction), float(dt), float(gamma),
                                      int(bc), int(niter), _ptr(F)), allow_clamp=False)
    return (V, F) if fluxes else V


def euler_smax(U, gamma=GAMMA):
    V = _f64(U)
    _, ny, nx = V.shape
    return _load().oracle_euler_smax(_ptr(V), nx, ny, float(gamma))


def euler_run(U, nsteps, gamma=GAMMA, cfl=CFL, bc=BC_PERIODIC, niter=NEWTON_ITERS):
    """nsteps of the split scheme (x sweep then y sweep with one dt per step).

    Returns (U_final, dts).
    """
    V = _f64(U).copy()
    _, ny, nx = V.shape
    dts = np.empty(nsteps)
    _check(_load().oracle_euler_run(_ptr(V), nx, ny, int(nsteps), float(gamma), float(cfl),
                                    int(bc), int(niter), _ptr(dts)))
    return V, dts


# ------------------------------------------------------------------ lap7 / biharmonic
BIHARM_NU = 1.0 / 128.0


def normalize(u, c=1.0, norms=False, periodic=True):
    """Normalisation example: u (nq, nj, ni); out = u - c * f / |f|_row with
    f the flux differences along i (the row end wraps, or repeats the last
    cell when periodic is False) and |f|_row the norm over the row's flux
    vectors (0 where the row norm is 0).  Returns out (and the row norms)."""
    a = _f64(u)
    nq, nj, ni = a.shape
    out = np.empty_like(a)
    n = np.empty(nj)
    _check(_load().oracle_normalize(_ptr(a), _ptr(out), nq, nj, ni, float(c), int(bool(periodic)), _ptr(n)))
    return (out, n) if norms else out


def lap7(u):
    a = _f64(u)
    o = np.empty_like(a)
    _check(_load().oracle_lap7(_ptr(a), _ptr(o), *a.shape))
    return o


def biharm(u, nu=BIHARM_NU, nsteps=1, stages=False):
    """out = u - nu * L7(L7(u)) on a periodic (nz, ny, nx) box, nsteps times."""
    a = _f64(u)
    out = np.empty_like(a)
    l1 = np.empty_like(a) if stages else None
    l2 = np.empty_like(a) if stages else None
    _check(_load().oracle_biharm(_ptr(a), _ptr(out), *a.shape, float(nu), int(nsteps),
                                 _ptr(l1), _ptr(l2)))
    return (out, l1, l2) if stages else out


# ------------------------------------------------------------------ linear chains
def linear_chain(chain, inp, offsets_fn):
    """Evaluate a random linear star chain (dict from inputs.random_chain).

    inp: (n_in, nz, ny, nx).  offsets_fn(ndim, r) gives the stencil offsets in
    the order the coefficients use.  Returns (f_out, nz, ny, nx).
    """
    stages = chain["stages"]
    f_io = np.array([stages[0]["f_in"]] + [s["f_out"] for s in stages], dtype=np.int32)
    offs, n_off, coeff = [], [], []
    for s in stages:
        o = offsets_fn(chain["ndim"], s["r"])
        n_off.append(len(o))
        offs.extend(o)
        coeff.append(np.asarray(s["coeff"], dtype=np.float64).ravel())
    offs = np.ascontiguousarray(np.array(offs, dtype=np.int32).ravel())
    n_off = np.array(n_off, dtype=np.int32)
    coeff = _f64(np.concatenate(coeff))
    a = _f64(inp)
    _, nz, ny, nx = a.shape
    out = np.empty((int(f_io[-1]), nz, ny, nx))
    ip = lambda x: x.ctypes.data_as(_ip)
    _check(_load().oracle_linear_chain(len(stages), ip(f_io), ip(n_off), ip(offs), _ptr(coeff),
                                       _ptr(a), _ptr(out), nz, ny, nx))
    return out


# ------------------------------------------------------------------ MLP
def mlp_nparams(d, H=64):
    return int(_load().oracle_mlp_nparams(d, H))


def mlp_forward(x, P, H=64):
    X = _f64(x)
    n, d = X.shape
    y = np.empty(n)
    if _load().oracle_mlp_forward(n, d, H, _ptr(X), _ptr(_f64(P)), _ptr(y)) != 0:
        raise ValueError(f"oracle MLP forward supports 1 <= H <= 512 hidden units, got {H}")
    return y


def mlp_loss_grad(x, t, P, H=64):
    X = _f64(x)
    T = _f64(t)
    Pp = _f64(P)
    n, d = X.shape
    if not 1 <= H <= 512:
        raise ValueError(f"oracle MLP gradient supports 1 <= H <= 512 hidden units, got {H}")
    G = np.empty_like(Pp)
    loss = _load().oracle_mlp_loss_grad(n, d, H, _ptr(X), _ptr(T), _ptr(Pp), _ptr(G))
    return loss, G


def adam_step(P, G, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of P (and its moments m, v) at step t >= 1."""
    for a in (P, G, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().oracle_adam_step(P.size, _ptr(P), _ptr(G), _ptr(m), _ptr(v), float(lr), float(b1),
                             float(b2), float(eps), int(t))
