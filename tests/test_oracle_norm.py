"""Pins of the oracle's normalisation chain (Design, "Reductions &
broadcasts & splits"; Performance, "Normalization Example"): flux
differences along i, a per-row norm (a reduction from (j, i) to j), and the
broadcast of that norm back over the row.  The paper gives no formulas for
this example; the definition is the one stated in oracle/hfav_oracle.c."""
import math

import numpy as np
import pytest

import oracle
from bruteforce import normalize_bf
from paper_1710_08774_amd import inputs


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("shape", [(1, 1, 5), (3, 4, 6), (2, 3, 1), (4, 2, 9)])
def test_normalize_bruteforce(shape, periodic):
    u = inputs.rng_for(sum(shape)).random(shape)
    out, n = oracle.normalize(u, 0.7, norms=True, periodic=periodic)
    ref, nref = normalize_bf(u.tolist(), 0.7, periodic=periodic)
    assert np.allclose(out, np.array(ref), rtol=1e-14, atol=1e-15)
    assert np.allclose(n, nref, rtol=1e-14, atol=0)


def test_normalize_transmissive_closed_form():
    """Transmissive row end: the flux telescopes, sum_i f = u(ni-1) - u(0),
    and a linear ramp u = a i has f = a except the last cell (0), so the
    row norm is |a| sqrt(ni - 1) per field."""
    ni = 17
    a = np.array([0.5, -2.0])
    u = a[:, None, None] * np.arange(ni)[None, None, :] + np.zeros((2, 3, ni))
    out, n = oracle.normalize(u, 1.0, norms=True, periodic=False)
    assert np.allclose(n, math.sqrt((a ** 2).sum() * (ni - 1)), rtol=1e-14)
    d = u - out
    assert np.allclose(d[:, :, -1], 0.0, atol=0) and np.allclose(d.sum(axis=2) * n[None, :],
                                                                (u[:, :, -1] - u[:, :, 0]), rtol=1e-13)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_normalize_fourier_norm_closed_form(k):
    """u_q = A_q cos(2 pi k i / ni + phi_j): the flux is a shifted sinusoid
    and sum_i (cos(t + h) - cos t)^2 over whole periods is 2 ni sin^2(h/2)."""
    nq, nj, ni = 3, 5, 64
    A = np.array([0.5, -1.5, 2.0])
    phi = np.linspace(0.0, 2.0, nj)
    i = np.arange(ni)
    u = A[:, None, None] * np.cos(2 * np.pi * k * i[None, None, :] / ni + phi[None, :, None])
    _, n = oracle.normalize(u, 1.0, norms=True)
    expect = math.sqrt((A ** 2).sum() * 2 * ni * math.sin(math.pi * k / ni) ** 2)
    assert np.allclose(n, expect, rtol=1e-13)


def test_normalize_unit_row_norm_and_scaling():
    u = inputs.rng_for(11).random((3, 6, 40))
    c = 0.25
    out = oracle.normalize(u, c)
    d = (u - out) / c
    assert np.allclose((d ** 2).sum(axis=(0, 2)), 1.0, rtol=1e-13)
    lam = -3.5
    out2 = oracle.normalize(lam * u, c)
    assert np.allclose(out2, lam * u + c * d, rtol=1e-13, atol=1e-13)


def test_normalize_translation_rows_and_constant_rows():
    u = inputs.rng_for(12).random((2, 7, 30))
    out = oracle.normalize(u, 0.5)
    assert np.allclose(oracle.normalize(np.roll(u, 5, axis=2), 0.5), np.roll(out, 5, axis=2), rtol=1e-14, atol=1e-15)
    perm = np.array([3, 0, 6, 1, 5, 2, 4])
    assert np.array_equal(oracle.normalize(u[:, perm], 0.5), out[:, perm])
    v = u.copy()
    v[:, 2, :] = 0.75                       # a constant row has zero flux: unchanged
    o2, n2 = oracle.normalize(v, 0.5, norms=True)
    assert n2[2] == 0.0 and np.array_equal(o2[:, 2], v[:, 2])
