"""Pins of the oracle's 7-point Laplacian chain, random linear star chains and
the cost-model MLP (forward, backward, Adam)."""
import math

import numpy as np
import pytest

import oracle
from bruteforce import biharm_cell, linear_chain_cell
from paper_1710_08774_amd import inputs

NU = oracle.BIHARM_NU


# ------------------------------------------------------------ lap7 / biharmonic
def test_biharm_constant_bitwise():
    for c in (0.0, 1.5, -7.0):
        u = np.full((6, 5, 7), c)
        assert np.array_equal(oracle.biharm(u), u)


def test_lap7_exact_on_quadratics_and_biharm_on_quartics():
    n = 16
    k, j, i = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    rng = np.random.default_rng(1)
    for _ in range(4):
        a, b, c, d, e = rng.integers(-4, 5, 5).astype(float)
        q = a * i * i + b * j * j + c * k * k + d * i * j + e * k
        l = oracle.lap7(q)
        assert np.all(l[2:-2, 2:-2, 2:-2] == 2 * (a + b + c))
    # nabla^4 (i^4) = 24, nabla^4 (i^2 j^2) = 8, away from the periodic wrap
    for q, ref in ((i ** 4, 24.0), (i * i * j * j, 8.0), (k ** 4 + 2 * j ** 4, 72.0)):
        _, _, l2 = oracle.biharm(q, stages=True)
        assert np.all(l2[3:-3, 3:-3, 3:-3] == ref)


@pytest.mark.parametrize("w", [(1, 0, 0), (2, 3, 1), (0, 5, 4)])
def test_fourier_closed_form(w):
    nz, ny, nx = 16, 20, 24
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.cos(2 * np.pi * (w[0] * i / nx + w[1] * j / ny + w[2] * k / nz) + 0.3)
    sig = sum(4 * np.sin(np.pi * wi / ni) ** 2 for wi, ni in zip(w, (nx, ny, nz)))
    out = oracle.biharm(u)
    assert np.abs(out - (1 - NU * sig * sig) * u).max() <= 1e-14


def test_biharm_conservation_and_mirror():
    u = inputs.biharm_input(shape=(12, 10, 14), seed=4)
    out = oracle.biharm(u)
    assert abs(math.fsum(out.ravel()) - math.fsum(u.ravel())) <= 1e-12 * u.size * np.abs(u).max() * 1e-2
    for ax in range(3):
        assert np.array_equal(oracle.biharm(np.flip(u, ax).copy()), np.flip(out, ax))
    # swapping x and y keeps the pairing of the first two sums: bitwise
    ut = np.ascontiguousarray(np.swapaxes(u, 1, 2))
    assert np.array_equal(oracle.biharm(ut), np.swapaxes(out, 1, 2))
    # other permutations reorder the three pair sums: equal to round-off
    up = np.ascontiguousarray(np.transpose(u, (2, 1, 0)))
    assert np.abs(oracle.biharm(up) - np.transpose(out, (2, 1, 0))).max() <= 1e-13


def test_biharm_bruteforce_8cube():
    u = inputs.biharm_input(shape=(8, 8, 8), seed=2)
    out = oracle.biharm(u)
    for (k, j, i) in [(0, 0, 0), (7, 7, 7), (3, 0, 5), (1, 6, 2), (4, 4, 4), (0, 7, 1)]:
        assert out[k, j, i] == biharm_cell(u, k, j, i, NU)


def test_biharm_multistep_is_repeated_application():
    u = inputs.biharm_input(shape=(8, 9, 10), seed=3)
    two = oracle.biharm(u, nsteps=2)
    assert np.array_equal(two, oracle.biharm(oracle.biharm(u)))


# ------------------------------------------------------------ linear chains
def _chain(seed, ndim=2, dims=(12, 10, 1)):
    rng = inputs.rng_for(seed)
    return inputs.random_chain(rng, ndim=ndim, dtype="f64", dims=dims)


@pytest.mark.parametrize("seed,ndim,dims", [(1, 2, (12, 10, 1)), (2, 3, (8, 8, 8)),
                                            (3, 2, (9, 7, 1))])
def test_linear_chain_bruteforce(seed, ndim, dims):
    ch = _chain(seed, ndim, dims)
    x = inputs.chain_input(ch, seed + 100)
    out = oracle.linear_chain(ch, x, inputs.star_offsets)
    rng = np.random.default_rng(seed)
    nz = dims[2]
    for _ in range(6):
        o = int(rng.integers(out.shape[0]))
        k, j, i = int(rng.integers(nz)), int(rng.integers(dims[1])), int(rng.integers(dims[0]))
        ref = linear_chain_cell(ch, x, inputs.star_offsets, o, k, j, i)
        assert abs(out[o, k, j, i] - ref) <= 1e-15


def test_linear_chain_linearity():
    ch = _chain(5, 3, (8, 6, 10))
    x = inputs.chain_input(ch, 1)
    y = inputs.chain_input(ch, 2)
    f = lambda z: oracle.linear_chain(ch, z, inputs.star_offsets)
    assert np.abs(f(2.5 * x - 0.75 * y) - (2.5 * f(x) - 0.75 * f(y))).max() <= 1e-13


def test_linear_chain_fourier_symbols():
    # one Fourier mode in one input field: each stage multiplies by its symbol
    ch = _chain(7, 2, (16, 12, 1))
    nx, ny, nz = ch["dims"]
    m = (3, 2, 0)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    e = np.exp(2j * np.pi * (m[0] * i / nx + m[1] * j / ny + m[2] * k / nz))
    vec = np.zeros(ch["n_in"], complex); vec[0] = 1.0
    for s in ch["stages"]:
        offs = inputs.star_offsets(ch["ndim"], s["r"])
        ph = np.array([np.exp(2j * np.pi * (m[0] * o[0] / nx + m[1] * o[1] / ny + m[2] * o[2] / nz))
                       for o in offs])
        vec = np.einsum("ofq,q,f->o", s["coeff"], ph, vec)
    x = np.zeros((ch["n_in"], nz, ny, nx)); x[0] = e.real
    xi = np.zeros_like(x); xi[0] = e.imag
    out = oracle.linear_chain(ch, x, inputs.star_offsets)
    outi = oracle.linear_chain(ch, xi, inputs.star_offsets)
    ref = vec[:, None, None, None] * e[None]
    assert np.abs(out + 1j * outi - ref).max() <= 1e-13


# ------------------------------------------------------------ MLP
def _params(d, H, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.3, oracle.mlp_nparams(d, H))


def test_mlp_zero_weights_gives_bias():
    d, H = 5, 16
    P = np.zeros(oracle.mlp_nparams(d, H)); P[-1] = 0.625
    y = oracle.mlp_forward(np.random.default_rng(0).normal(size=(7, d)), P, H)
    assert np.all(y == 0.625)


def test_mlp_forward_matches_matrix_products():
    d, H, n = 6, 16, 9
    P = _params(d, H, 1)
    x = np.random.default_rng(2).normal(size=(n, d))
    o = 0
    def take(sz, shape):
        nonlocal o
        a = P[o:o + sz].reshape(shape); o += sz; return a
    W1 = take(H * d, (H, d)); b1 = take(H, (H,))
    W2 = take(H * H, (H, H)); b2 = take(H, (H,))
    W3 = take(H * H, (H, H)); b3 = take(H, (H,))
    W4 = take(H, (1, H)); b4 = take(1, (1,))
    h = np.maximum(x @ W1.T + b1, 0)
    h = np.maximum(h @ W2.T + b2, 0)
    h = np.maximum(h @ W3.T + b3, 0)
    ref = (h @ W4.T + b4)[:, 0]
    assert np.allclose(oracle.mlp_forward(x, P, H), ref, rtol=1e-13, atol=1e-14)


def test_mlp_gradient_central_differences():
    d, H, n = 4, 8, 6
    P = _params(d, H, 3)
    x = np.random.default_rng(4).normal(size=(n, d))
    t = np.random.default_rng(5).normal(size=n)
    loss, G = oracle.mlp_loss_grad(x, t, P, H)
    h = 1e-6
    rng = np.random.default_rng(6)
    for q in rng.choice(P.size, 40, replace=False):
        Pp = P.copy(); Pp[q] += h
        Pm = P.copy(); Pm[q] -= h
        fd = (oracle.mlp_loss_grad(x, t, Pp, H)[0] - oracle.mlp_loss_grad(x, t, Pm, H)[0]) / (2 * h)
        assert abs(fd - G[q]) <= 1e-6 * max(1.0, abs(G[q]))
    # closed form: dL/db_out = 2 * mean residual
    r = oracle.mlp_forward(x, P, H) - t
    assert abs(G[-1] - 2 * r.mean()) <= 1e-13
    assert abs(loss - np.mean(r * r)) <= 1e-13


def test_adam_constant_gradient_closed_form():
    P = np.zeros(5); G = np.array([1.0, -2.0, 0.5, 3.0, -0.1])
    m = np.zeros(5); v = np.zeros(5)
    for t in range(1, 11):
        oracle.adam_step(P, G, m, v, t, lr=1e-3, eps=0.0)
    # constant gradient: bias-corrected moments equal g and g^2, step = lr*sign(g)
    assert np.allclose(P, -10e-3 * np.sign(G), rtol=1e-12, atol=0)


def test_mlp_hidden_width_beyond_oracle_limit_is_an_error():
    # the oracle keeps hidden activations on the stack (at most 512 units):
    # a wider network is refused instead of leaving outputs unset
    d, H = 3, 513
    P = np.zeros(oracle.mlp_nparams(d, H))
    x = np.zeros((2, d))
    with pytest.raises(ValueError):
        oracle.mlp_forward(x, P, H)
    with pytest.raises(ValueError):
        oracle.mlp_loss_grad(x, np.zeros(2), P, H)
