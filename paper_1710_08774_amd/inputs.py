"""Seeded synthetic inputs shared by the HIP path, the oracle and the benches.

This module only draws random numbers and lays them out as arrays; it holds
none of the fused-chain arithmetic.  Every generator takes an explicit seed
(an int or a numpy SeedSequence) so the HIP path and the oracle see
bit-identical inputs.

Workloads (the paper's COSMO and Hydro2D input decks are not available, so
these synthetic inputs stand in for them, Performance section):

* hdiff:  uniform [0,1) field on an (nk, nj, ni) grid (COSMO micro-kernels).
* euler:  Sod-like split along a random-angle line with smooth periodic
          sinusoidal perturbations of the density and pressure (Hydro2D).
* biharm: sum of 8 random Fourier modes plus 1e-6 uniform noise on a cube.
* batch:  many Sod-like grids with independent sides in [64, 1024].
* chain:  random linear star-stencil chains for the tuning cost model.
* norm:   a system of nq fields on rows of i: per row and field a sinusoid of
          random wavenumber, amplitude and phase on a random offset, plus
          small uniform noise; every 17th row constant (zero flux, zero norm).
"""
from __future__ import annotations

import numpy as np

# Base of the per-workload seeds: SeedSequence(BASE_SEED + workload index).
BASE_SEED = 171008774
W_HDIFF, W_EULER, W_PREC, W_BATCH, W_CHAIN, W_NORM = 0, 1, 2, 3, 4, 5


def seed_seq(seed) -> np.random.SeedSequence:
    if isinstance(seed, np.random.SeedSequence):
        return seed
    return np.random.SeedSequence(int(seed))


def rng_for(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_seq(seed)))


# ---------------------------------------------------------------- norm
def norm_input(nq=4, nj=4096, ni=4096, seed=BASE_SEED + W_NORM, noise=1e-2, const_every=17) -> np.ndarray:
    """(nq, nj, ni) float64: u[q, j, i] = b + A sin(2 pi k i / ni + phi) +
    noise * U[-1, 1), with b ~ U[-1, 1), A ~ U[0.1, 2), k ~ U{1..8} and
    phi ~ U[0, 2 pi) drawn per (q, j); rows j = 0 mod const_every hold the
    constant b (their flux and norm are 0)."""
    rng = rng_for(seed)
    b = rng.uniform(-1.0, 1.0, (nq, nj, 1))
    A = rng.uniform(0.1, 2.0, (nq, nj, 1))
    k = rng.integers(1, 9, (nq, nj, 1))
    phi = rng.uniform(0.0, 2 * np.pi, (nq, nj, 1))
    i = np.arange(ni)[None, None, :]
    u = b + A * np.sin(2 * np.pi * k * i / ni + phi) + noise * rng.uniform(-1.0, 1.0, (nq, nj, ni))
    if const_every:
        u[:, ::const_every, :] = b[:, ::const_every, :]
    return np.ascontiguousarray(u)


# ---------------------------------------------------------------- hdiff
def hdiff_input(nk=8, nj=256, ni=256, seed=BASE_SEED + W_HDIFF) -> np.ndarray:
    """Uniform [0,1) field of shape (nk, nj, ni), float64, C order."""
    return rng_for(seed).random((nk, nj, ni))


# ---------------------------------------------------------------- euler
def euler_ic_params(seed):
    """Random line angle and the 4+4 sinusoidal modes of the Sod-like state."""
    rng = rng_for(seed)
    theta = rng.uniform(0.0, np.pi)
    modes = {}
    for name in ("rho", "p"):
        k = rng.integers(1, 9, size=4)
        l = rng.integers(1, 9, size=4)
        phi = rng.uniform(0.0, 2.0 * np.pi, size=4)
        modes[name] = (k, l, phi)
    return theta, modes


def euler_ic(nx=2048, ny=2048, seed=BASE_SEED + W_EULER, gamma=1.4,
             amp=1e-3, split=True, perturb=True, theta=None):
    """Initial conserved state U of shape (4, ny, nx): (rho, rho*u, rho*v, E).

    Cell centres are x=(i+1/2)/nx, y=(j+1/2)/ny.  The signed distance to a
    line through (1/2, 1/2) at angle theta picks the left state (rho=1, p=1)
    where it is negative and the right state (rho=0.125, p=0.1) otherwise.
    Velocities are zero, so E = p/(gamma-1).
    """
    th, modes = euler_ic_params(seed)
    if theta is not None:
        th = theta
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)                      # (ny, nx)
    if split:
        s = (X - 0.5) * np.cos(th) + (Y - 0.5) * np.sin(th)
        left = s < 0.0
        rho = np.where(left, 1.0, 0.125)
        p = np.where(left, 1.0, 0.1)
    else:
        rho = np.ones((ny, nx))
        p = np.ones((ny, nx))
    if perturb:
        for name in ("rho", "p"):
            k, l, phi = modes[name]
            P = np.zeros((ny, nx))
            for m in range(4):
                P += np.sin(2.0 * np.pi * (k[m] * X + l[m] * Y) + phi[m])
            P *= 0.25
            if name == "rho":
                rho = rho * (1.0 + amp * P)
            else:
                p = p * (1.0 + amp * P)
    U = np.empty((4, ny, nx))
    U[0] = rho
    U[1] = 0.0
    U[2] = 0.0
    U[3] = p / (gamma - 1.0)
    return U


def euler_state_from_prim(rho, u, v, p, gamma=1.4):
    """Conserved state from primitive arrays (used to build test inputs)."""
    rho = np.asarray(rho, dtype=np.float64)
    U = np.empty((4,) + rho.shape)
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * v
    U[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return U


def riemann_states(n, seed, gamma=1.4, log_rho=(-1.0, 0.3), log_p=(-1.2, 0.3), du=0.5):
    """n random admissible left/right primitive states (rho, u, ut, p).

    Densities and pressures are log-uniform over the given decades (the
    ranges of a Sod-like problem), velocities uniform in [-du, du].
    Admissible means the vacuum condition 2(cL+cR)/(gamma-1) > uR-uL holds.
    Returns two (n, 4) float64 arrays.
    """
    rng = rng_for(seed)
    out_l = np.empty((n, 4))
    out_r = np.empty((n, 4))
    filled = 0
    while filled < n:
        m = 2 * (n - filled) + 16
        rl = 10.0 ** rng.uniform(*log_rho, m)
        rr = 10.0 ** rng.uniform(*log_rho, m)
        pl = 10.0 ** rng.uniform(*log_p, m)
        pr = 10.0 ** rng.uniform(*log_p, m)
        ul = rng.uniform(-du, du, m)
        ur = rng.uniform(-du, du, m)
        vl = rng.uniform(-du, du, m)
        vr = rng.uniform(-du, du, m)
        cl = np.sqrt(gamma * pl / rl)
        cr = np.sqrt(gamma * pr / rr)
        ok = 2.0 * (cl + cr) / (gamma - 1.0) > (ur - ul) + 0.5
        idx = np.nonzero(ok)[0][: n - filled]
        k = len(idx)
        out_l[filled:filled + k] = np.stack([rl[idx], ul[idx], vl[idx], pl[idx]], 1)
        out_r[filled:filled + k] = np.stack([rr[idx], ur[idx], vr[idx], pr[idx]], 1)
        filled += k
    return out_l, out_r


# ---------------------------------------------------------------- biharmonic
def biharm_modes(seed=BASE_SEED + W_PREC):
    rng = rng_for(seed)
    amps = rng.uniform(0.5, 1.0, 8)
    waves = []
    while len(waves) < 8:
        w = rng.integers(-8, 9, size=3)
        if np.any(w != 0):
            waves.append(w)
    phi = rng.uniform(0.0, 2.0 * np.pi, 8)
    return amps, np.array(waves), phi, rng


def biharm_input(n=512, seed=BASE_SEED + W_PREC, noise=1e-6, shape=None):
    """Smooth field (sum of 8 periodic Fourier modes) plus uniform noise.

    Shape (nz, ny, nx) = (n, n, n) unless `shape` is given; the modes are
    periodic on the given box.  float64.
    """
    nz, ny, nx = shape if shape is not None else (n, n, n)
    amps, waves, phi, rng = biharm_modes(seed)
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    u = np.zeros((nz, ny, nx))
    for m in range(8):
        kx, ky, kz = waves[m]
        u += amps[m] * np.cos(2.0 * np.pi * (kx * i / nx + ky * j / ny + kz * k / nz) + phi[m])
    u += noise * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    return u


# ---------------------------------------------------------------- batch
def batch_sizes(n_grids=512, seed=BASE_SEED + W_BATCH, lo=64, hi=1024):
    """Independent (nx, ny) per grid, uniform integers in [lo, hi]."""
    rng = rng_for(seed)
    nx = rng.integers(lo, hi + 1, size=n_grids)
    ny = rng.integers(lo, hi + 1, size=n_grids)
    return [(int(a), int(b)) for a, b in zip(nx, ny)]


def batch_grid_seeds(n_grids=512, seed=BASE_SEED + W_BATCH):
    """One child SeedSequence per grid for its own Sod-like initial state."""
    return seed_seq(seed).spawn(n_grids)


def batch_ic(n_grids=512, seed=BASE_SEED + W_BATCH, gamma=1.4, sizes=None):
    if sizes is None:
        sizes = batch_sizes(n_grids, seed)
    seeds = batch_grid_seeds(len(sizes), seed)
    return [euler_ic(nx, ny, seed=s, gamma=gamma) for (nx, ny), s in zip(sizes, seeds)]


# ---------------------------------------------------------------- random chains
def star_offsets(ndim, r):
    """Offsets of a star stencil of radius r: centre, then +-1..r on each axis.

    Offsets are (di, dj, dk) triples, i fastest.
    """
    offs = [(0, 0, 0)]
    for ax in range(ndim):
        for d in range(1, r + 1):
            for s in (-d, d):
                o = [0, 0, 0]
                o[ax] = s
                offs.append(tuple(o))
    return offs


def random_chain(rng, ndim=None, dtype=None, dims=None):
    """A random linear star-stencil chain.

    Returns a dict: ndim, dtype ('f32'|'f64'), dims (nx, ny, nz), n_in,
    stages: list of {r, f_in, f_out, coeff: array (f_out, f_in, n_offsets)}.
    Coefficients are uniform in [-1, 1] and scaled so sum |c| = 1 per output.
    """
    if ndim is None:
        ndim = int(rng.integers(2, 4))
    if dtype is None:
        dtype = "f64" if rng.random() < 0.5 else "f32"
    K = int(rng.integers(2, 7))
    f_prev = int(rng.integers(1, 6))
    n_in = f_prev
    stages = []
    for _ in range(K):
        r = int(rng.integers(1, 4))
        f_out = int(rng.integers(1, 6))
        n_off = 1 + 2 * r * ndim
        c = rng.uniform(-1.0, 1.0, size=(f_out, f_prev, n_off))
        c /= np.abs(c).sum(axis=(1, 2), keepdims=True)
        stages.append({"r": r, "f_in": f_prev, "f_out": f_out, "coeff": c})
        f_prev = f_out
    if dims is None:
        if ndim == 2:
            lo, hi = np.log2(128), np.log2(4096)
            d = [int(round(2 ** rng.uniform(lo, hi) / 32.0)) * 32 for _ in range(2)]
            dims = (max(d[0], 32), max(d[1], 32), 1)
        else:
            lo, hi = np.log2(64), np.log2(512)
            d = [int(round(2 ** rng.uniform(lo, hi) / 32.0)) * 32 for _ in range(3)]
            dims = tuple(max(x, 32) for x in d)
    return {"ndim": ndim, "dtype": dtype, "dims": tuple(int(x) for x in dims),
            "n_in": n_in, "stages": stages}


def chain_input(chain, seed):
    """Uniform [-1, 1) input fields for a random chain: (n_in, nz, ny, nx)."""
    nx, ny, nz = chain["dims"]
    rng = rng_for(seed)
    return 2.0 * rng.random((chain["n_in"], nz, ny, nx)) - 1.0
