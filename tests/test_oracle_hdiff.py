"""Pins of the FP64 oracle's horizontal-diffusion chain (COSMO micro-kernels).

The paper names the four kernels (ulapstage, flux_x, flux_y, ustage) without
formulas; these tests fix the oracle to properties the chain must have, not
to the oracle itself.
"""
import math

import numpy as np
import pytest

import oracle
from bruteforce import hdiff_cell
from paper_1710_08774_amd import inputs


def test_constant_preserved_bitwise():
    for c in (0.0, 0.37, 1e6, -3.25):
        a = np.full((2, 9, 7), c)
        out = oracle.hdiff(a)
        assert np.array_equal(out, a)


def test_laplacian_exact_on_quadratics():
    # q = a i^2 + b j^2 + c ij + d i + e j + f : 5-point Laplacian = 2a + 2b
    nk, nj, ni = 1, 16, 16
    j, i = np.meshgrid(np.arange(nj, dtype=float), np.arange(ni, dtype=float), indexing="ij")
    rng = np.random.default_rng(3)
    for _ in range(5):
        a, b, c, d, e, f = rng.integers(-5, 6, 6).astype(float)
        q = a * i * i + b * j * j + c * i * j + d * i + e * j + f
        _, lap, _, _ = oracle.hdiff(q[None], stages=True)
        inner = lap[0, 2:-2, 2:-2]          # away from the periodic wrap
        assert np.all(inner == 2 * a + 2 * b)


def test_linear_ramp_has_zero_laplacian_and_sign():
    # the Laplacian of i^2 is +2 (not -2): pins the sign convention
    ni = 12
    i = np.arange(ni, dtype=float)
    q = np.tile(i * i, (12, 1))[None]
    _, lap, _, _ = oracle.hdiff(q, stages=True)
    assert np.all(lap[0, :, 2:-2] == 2.0)


def test_periodic_mass_conservation():
    a = inputs.hdiff_input(4, 32, 40, seed=11)
    out = oracle.hdiff(a)
    for k in range(a.shape[0]):
        s0 = math.fsum(a[k].ravel())
        s1 = math.fsum(out[k].ravel())
        assert abs(s1 - s0) <= 4 * a[k].size * np.finfo(float).eps * np.abs(a[k]).max()


def test_mirror_and_transpose_symmetry_bitwise():
    a = inputs.hdiff_input(2, 24, 24, seed=5)
    out = oracle.hdiff(a)
    assert np.array_equal(oracle.hdiff(a[:, :, ::-1]), out[:, :, ::-1])
    assert np.array_equal(oracle.hdiff(a[:, ::-1, :]), out[:, ::-1, :])
    at = np.ascontiguousarray(np.swapaxes(a, 1, 2))
    assert np.array_equal(oracle.hdiff(at), np.swapaxes(out, 1, 2))


def test_planes_independent():
    p = inputs.hdiff_input(1, 16, 20, seed=9)[0]
    a = np.stack([p, p, p])
    out = oracle.hdiff(a)
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    b = a.copy()
    b[1] = 0.5
    outb = oracle.hdiff(b)
    assert np.array_equal(outb[0], out[0]) and np.array_equal(outb[1], b[1])


@pytest.mark.parametrize("m,n", [(1, 0), (2, 3), (5, 1)])
def test_fourier_closed_form_without_limiter(m, n):
    N = 32
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u = np.cos(2 * np.pi * (m * i + n * j) / N)[None]
    out = oracle.hdiff(u, limiter=False)
    sig = 4 * np.sin(np.pi * m / N) ** 2 + 4 * np.sin(np.pi * n / N) ** 2
    ref = (1.0 - 0.025 * sig * sig) * u
    assert np.abs(out - ref).max() <= 1e-14


def test_limiter_removes_up_gradient_flux():
    # every limited flux either is zero or points down the gradient
    a = inputs.hdiff_input(1, 16, 16, seed=21)
    _, _, flx, fly = oracle.hdiff(a, stages=True)
    dx = np.roll(a, -1, axis=2) - a
    dy = np.roll(a, -1, axis=1) - a
    assert np.all(flx * dx <= 0.0) and np.all(fly * dy <= 0.0)
    assert np.count_nonzero(flx) > 0 and np.count_nonzero(fly) > 0


@pytest.mark.parametrize("shape", [(1, 8, 8), (2, 8, 8), (1, 5, 7)])
def test_bruteforce_agreement(shape):
    a = inputs.hdiff_input(*shape, seed=sum(shape))
    out = oracle.hdiff(a)
    for k in range(shape[0]):
        for j in range(shape[1]):
            for i in range(shape[2]):
                assert out[k, j, i] == hdiff_cell(a, k, j, i)
