"""GPU parity of the normalisation chain (Performance, "Normalization
Example"; Design, "Reductions & broadcasts & splits") against the oracle:
the fused kernel (one workgroup per row, both inner sweeps), every forced
tile configuration of it, and the unfused one-kernel-per-rule path.

FP64 bound: per output field and for the row norms, max|gpu - oracle| /
max|oracle| <= 1e-12 (the row sum is associated differently on each side:
a relative difference of at most (ni + log2 ni) 2^-53 in the sum, half of
it in the norm).  FP32: the element-wise bound derived in
test_norm_f32_elementwise_bound."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, relerr
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12
U32 = 2.0 ** -24


def run_chain(u, dims, c=0.7, mode=H.MODE_AUTO, dtype=H.F64, forced=None, bc=H.BC_PERIODIC, ndim=2):
    """u: (nq, rows, ni) host array; returns (out (nq, rows, ni), norms (rows,), plan info)."""
    nq = u.shape[0]
    chain = H.Chain(H.norm_spec(nq, c, dtype=dtype, ndim=ndim, with_norm=True))
    kw = {}
    if forced is not None:
        kw = dict(config_source=H.CONFIG_FORCED, forced=forced)
    info = chain.plan(dims, boundary=(bc, H.BC_PERIODIC, H.BC_PERIODIC), mode=mode, **kw)
    tdt = torch.float64 if dtype == H.F64 else torch.float32
    d = dev(u, tdt)
    o = torch.full_like(d, float("nan"))
    n = torch.full((u.shape[1],), float("nan"), dtype=tdt, device=d.device)
    ws = torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device=d.device)
    chain.execute([d[q] for q in range(nq)], [o[q] for q in range(nq)] + [n], ws)
    return host(o), host(n), info


def check(u, got, n, c=0.7, periodic=True, tol=TOL):
    ref, nref = oracle.normalize(u, c, norms=True, periodic=periodic)
    for q in range(u.shape[0]):
        assert relerr(got[q], ref[q]) <= tol, (q, relerr(got[q], ref[q]))
    assert relerr(n, nref) <= tol, relerr(n, nref)
    return ref, nref


SHAPES = [(4, 64, 4096), (4, 33, 1000), (1, 20, 3), (3, 17, 4097), (8, 19, 4096), (5, 9, 777),
          (2, 5, 1), (4, 18, 64), (2, 5, 9000), (6, 7, 2000)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_norm_parity(shape, mode):
    nq, nj, ni = shape
    print("norm parity", shape, mode, flush=True)
    u = inputs.norm_input(nq, nj, ni, seed=inputs.BASE_SEED + 50 + ni)
    got, n, info = run_chain(u, (ni, nj), mode=mode)
    assert bool(info.fused) == (mode == H.MODE_FUSED)
    check(u, got, n)


def _reg_configs(nq, ni):
    out = []
    for seg in (1, 2, 4, 8, 16):
        if nq * seg > 32:
            continue
        for blk in (64, 128, 256, 512, 1024):
            if blk * seg >= ni:
                out.append((blk, 1, seg, 0, 0))
    out += [(b, t, seg, v, x) for (b, t, seg, _, x) in out for v in (2, 3)]
    return out + [(b, 1, 0, 1, 0) for b in (64, 128, 256)]


@pytest.mark.parametrize("nq,ni", [(4, 1000), (2, 129), (3, 64), (1, 4096)])
def test_norm_every_forced_config(nq, ni):
    u = inputs.norm_input(nq, 11, ni, seed=inputs.BASE_SEED + 60 + ni)
    ref, nref = oracle.normalize(u, 0.7, norms=True)
    cfgs = _reg_configs(nq, ni)
    assert len(cfgs) >= 4
    for cfg in cfgs:
        print("norm forced", nq, ni, cfg, flush=True)
        got, n, info = run_chain(u, (ni, 11), forced=cfg)
        assert (info.config.block, info.config.seg, info.config.variant) == (cfg[0], cfg[2], cfg[3])
        for q in range(nq):
            assert relerr(got[q], ref[q]) <= TOL, (cfg, q)
        assert relerr(n, nref) <= TOL, cfg


@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
@pytest.mark.parametrize("ni", [1000, 4096, 5, 9000])
def test_norm_transmissive_row_end(mode, ni):
    u = inputs.norm_input(3, 13, ni, seed=inputs.BASE_SEED + 70 + ni)
    got, n, _ = run_chain(u, (ni, 13), mode=mode, bc=H.BC_TRANSMISSIVE)
    check(u, got, n, periodic=False)


@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_norm_3d_rows(mode):
    """ndim 3: the rows are the (k, j) pairs, the row terms (k, j) arrays."""
    nq, ni, nj, nk = 2, 300, 5, 7
    u = inputs.norm_input(nq, nj * nk, ni, seed=inputs.BASE_SEED + 80)
    got, n, info = run_chain(u, (ni, nj, nk), mode=mode, ndim=3)
    assert info.family == 8 or mode == H.MODE_UNFUSED
    check(u, got, n)


@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_norm_zero_norm_rows_are_unchanged(mode):
    """Rows with zero flux (constant rows, and every row when ni = 1) have a
    zero norm; DIV0 then gives 0 and the update leaves u bit for bit."""
    u = inputs.norm_input(4, 40, 500, seed=inputs.BASE_SEED + 90, const_every=3)
    got, n, _ = run_chain(u, (500, 40), mode=mode)
    check(u, got, n)
    assert np.all(n[::3] == 0.0) and np.array_equal(got[:, ::3], u[:, ::3])
    u1 = inputs.norm_input(3, 9, 1, seed=inputs.BASE_SEED + 91)
    g1, n1, _ = run_chain(u1, (1, 9), mode=mode)
    assert np.all(n1 == 0.0) and np.array_equal(g1, u1)


def test_norm_fused_and_unfused_agree_and_unit_norm():
    """The two paths agree to the FP64 bound, and d = (u - out) / c has unit
    norm on every row with a nonzero flux (a property at any size)."""
    nq, nj, ni, c = 4, 48, 3000, 0.3
    u = inputs.norm_input(nq, nj, ni, seed=inputs.BASE_SEED + 92)
    a, na, _ = run_chain(u, (ni, nj), c=c, mode=H.MODE_FUSED)
    b, nb, _ = run_chain(u, (ni, nj), c=c, mode=H.MODE_UNFUSED)
    for q in range(nq):
        assert relerr(a[q], b[q]) <= TOL
    d = (u - a) / c
    rows = (d ** 2).sum(axis=(0, 2))
    nz = na > 0
    assert np.allclose(rows[nz], 1.0, rtol=1e-10) and np.all(rows[~nz] == 0.0)


def test_norm_f32_elementwise_bound():
    """FP32 storage and arithmetic against the FP64 oracle.  Per element,
    with e = 2^-24, U the largest |u| of the row, N = nq ni and K = nq + ni/64
    + 16 (a bound on the depth of any summation order either path uses):
    rounding u costs e|u| and each flux difference 4eU (both inputs and the
    difference); the row sum then errs by at most 2 sum|f| 4eU + K e s, so
    with sum|f| <= sqrt(N) n the norm errs relatively by 4eU sqrt(N)/n +
    (K/2 + 1)e; the quotient (reciprocal and product) adds 2e, the update
    e|out| + e c|d|.  Together:
      |out32 - out| <= e|u| + e|out| + c (4eU/n + |d|(4eU sqrt(N)/n + (K/2+4)e)),
    and e|u| alone on rows whose norm is 0.  Asserted with a factor 2 for
    the second-order terms."""
    nq, nj, ni, c = 4, 40, 4096, 0.7
    u = inputs.norm_input(nq, nj, ni, seed=inputs.BASE_SEED + 93)
    ref, nref = oracle.normalize(u, c, norms=True)
    d = (u - ref) / c
    U = np.abs(u).max(axis=(0, 2))[None, :, None]
    K = nq + ni / 64 + 16
    N = nq * ni
    nn = nref[None, :, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        rel_n = 4 * U32 * U * math.sqrt(N) / nn + (K / 2 + 4) * U32
        b = U32 * np.abs(u) + U32 * np.abs(ref) + c * (4 * U32 * U / nn + np.abs(d) * rel_n)
    b = np.where(nn > 0, b, U32 * np.abs(u))
    for mode in (H.MODE_FUSED, H.MODE_UNFUSED):
        got, n, _ = run_chain(u, (ni, nj), c=c, mode=mode, dtype=H.F32)
        excess = (np.abs(got - ref) / (2 * b + 1e-300)).max()
        print("norm f32 mode", mode, "max err", np.abs(got - ref).max(), "max err / (2 bound)", excess,
              flush=True)
        assert excess <= 1.0


def test_norm_full_size_all_rows():
    """The bench workload, 4 fields x 4096 rows x 4096 cells, in the
    configuration the bench times: every row against the oracle (within
    1e-12 per field and for the norms), and the unit norm of every row's d."""
    nq, nj, ni, c = 4, 4096, 4096, 1.0
    u = inputs.norm_input(nq, nj, ni)
    got, n, info = run_chain(u, (ni, nj), c=c)
    assert info.fused and info.family == 8
    ref, nref = oracle.normalize(u, c, norms=True)
    for q in range(nq):
        assert relerr(got[q], ref[q]) <= TOL
    assert relerr(n, nref) <= TOL
    d = u - got
    s = (d ** 2).sum(axis=(0, 2))
    nz = n > 0
    assert np.allclose(s[nz], 1.0, rtol=1e-10) and np.all(s[~nz] == 0.0)
