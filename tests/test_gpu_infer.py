"""GPU parity of chains created by inference from rule patterns (pattern
variables "q?", "s?"; Implementation, "Inference") against the oracle: the
instantiated chains run the same fused kernels as the hand-written ones."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, hydro_errs, relerr
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from patterns import biharm_patterns, norm_patterns, sweep_patterns

pytestmark = pytest.mark.gpu
TOL = 1e-12


def test_inferred_biharmonic_bitwise():
    u = inputs.biharm_input(40, shape=(24, 36, 40))
    c = H.chain_infer(biharm_patterns())
    info = c.plan((40, 36, 24))
    assert info.fused and info.family == 4
    d = dev(u)
    o = torch.empty_like(d)
    c.execute([d], [o])
    assert np.array_equal(host(o), oracle.biharm(u))


@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_inferred_normalisation(mode):
    nq, nj, ni = 4, 37, 1500
    u = inputs.norm_input(nq, nj, ni, seed=inputs.BASE_SEED + 95)
    c = H.chain_infer(norm_patterns(nq, c=0.6, with_norm=True))
    info = c.plan((ni, nj), mode=mode)
    d = dev(u)
    o = torch.empty_like(d)
    n = torch.empty(nj, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device="cuda")
    c.execute([d[q] for q in range(nq)], [o[q] for q in range(nq)] + [n], ws)
    ref, nref = oracle.normalize(u, 0.6, norms=True)
    got = host(o)
    for q in range(nq):
        assert relerr(got[q], ref[q]) <= TOL
    assert relerr(host(n), nref) <= TOL


@pytest.mark.parametrize("direction", [0, 1])
def test_inferred_godunov_sweep(direction):
    ny, nx = 70, 130
    U = inputs.euler_ic(nx, ny, seed=77, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    c = H.chain_infer(sweep_patterns(direction))
    info = c.plan((nx, ny))
    assert info.fused
    d = dev(U)
    o = torch.empty_like(d)
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    c.execute([d[0], d[1], d[2], d[3], dtt], [o[0], o[1], o[2], o[3]])
    assert max(hydro_errs(host(o), oracle.euler_sweep(U, direction, dt))) <= TOL
