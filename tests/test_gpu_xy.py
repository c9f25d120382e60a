"""Both Godunov sweeps of a step in one kernel (the x-swept state kept on
chip).  The per-cell formulas are the separate sweeps', evaluated in a
different kernel (the compiler may contract multiply-adds differently), so
the results are compared with the two fused sweeps and with the oracle by
the FP64 bound, 1e-12 per physical field."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, hydro_errs
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from paper_1710_08774_amd.euler import EulerStepper

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _xy(U, dt, bc=(H.BC_PERIODIC, H.BC_PERIODIC), forced=None, dtype=torch.float64, precision=H.PREC_NATIVE):
    _, ny, nx = U.shape
    cd = H.F64 if dtype == torch.float64 else H.F32
    c = H.Chain(H.euler_step_spec(dt_source="dt", with_smax=True, dtype=cd))
    kw = dict(config_source=H.CONFIG_FORCED, forced=forced) if forced else {}
    info = c.plan((nx, ny), bc, mode=H.MODE_FUSED, precision=precision, **kw)
    assert info.family == 9 and info.fused
    d = dev(U, dtype)
    o = torch.empty_like(d)
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    sm = torch.zeros(1, dtype=torch.float64, device="cuda")
    c.execute([d[0], d[1], d[2], d[3], dtt], [o[0], o[1], o[2], o[3], sm])
    return host(o), float(host(sm)[0])


def _split(U, dt, bc=(H.BC_PERIODIC, H.BC_PERIODIC), dtype=torch.float64, precision=H.PREC_NATIVE):
    _, ny, nx = U.shape
    cd = H.F64 if dtype == torch.float64 else H.F32
    cx = H.Chain(H.euler_sweep_spec(0, dt_source="dt", dtype=cd))
    cy = H.Chain(H.euler_sweep_spec(1, dt_source="dt", with_smax=True, dtype=cd))
    cx.plan((nx, ny), bc, mode=H.MODE_FUSED, precision=precision)
    cy.plan((nx, ny), bc, mode=H.MODE_FUSED, precision=precision)
    d = dev(U, dtype)
    m = torch.empty_like(d)
    o = torch.empty_like(d)
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    sm = torch.zeros(1, dtype=torch.float64, device="cuda")
    cx.execute([d[0], d[1], d[2], d[3], dtt], [m[0], m[1], m[2], m[3]])
    cy.execute([m[0], m[1], m[2], m[3], dtt], [o[0], o[1], o[2], o[3], sm])
    return host(o), float(host(sm)[0])


@pytest.mark.parametrize("shape", [(64, 64), (70, 130), (37, 61), (5, 300), (300, 5), (1, 40), (2, 3), (120, 59)])
def test_xy_equals_split_sweeps_and_oracle(shape):
    ny, nx = shape
    print("xy", shape, flush=True)
    U = inputs.euler_ic(nx, ny, seed=nx * 7 + ny, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    got, sm = _xy(U, dt)
    ref, smr = _split(U, dt)
    print("xy vs split", max(hydro_errs(got, ref)), flush=True)
    assert max(hydro_errs(got, ref)) <= TOL and abs(sm - smr) <= TOL * smr
    oref = oracle.euler_sweep(oracle.euler_sweep(U, 0, dt), 1, dt)
    assert max(hydro_errs(got, oref)) <= TOL
    assert abs(sm - oracle.euler_smax(oref)) <= TOL * oracle.euler_smax(oref)


@pytest.mark.parametrize("seg", [1, 2, 7, 16, 33, 128])
def test_xy_segment_lengths(seg):
    U = inputs.euler_ic(130, 90, seed=5, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    got, sm = _xy(U, dt, forced=(64, 1, seg, 0, 0))
    ref, smr = _split(U, dt)
    assert max(hydro_errs(got, ref)) <= TOL and abs(sm - smr) <= TOL * smr


@pytest.mark.parametrize("bc", [(H.BC_TRANSMISSIVE, H.BC_TRANSMISSIVE), (H.BC_PERIODIC, H.BC_TRANSMISSIVE),
                                (H.BC_TRANSMISSIVE, H.BC_PERIODIC)])
def test_xy_boundaries(bc):
    ny, nx = 48, 100
    U = inputs.euler_ic(nx, ny, seed=8, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    got, _ = _xy(U, dt, bc=bc)
    # separate sweeps, each with its own axis' boundary
    cx = H.Chain(H.euler_sweep_spec(0, dt_source="dt"))
    cy = H.Chain(H.euler_sweep_spec(1, dt_source="dt"))
    cx.plan((nx, ny), bc, mode=H.MODE_FUSED)
    cy.plan((nx, ny), bc, mode=H.MODE_FUSED)
    d = dev(U)
    m = torch.empty_like(d)
    o = torch.empty_like(d)
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    cx.execute([d[0], d[1], d[2], d[3], dtt], [m[0], m[1], m[2], m[3]])
    cy.execute([m[0], m[1], m[2], m[3], dtt], [o[0], o[1], o[2], o[3]])
    assert max(hydro_errs(got, host(o))) <= TOL
    oref = oracle.euler_sweep(oracle.euler_sweep(U, 0, dt, bc=bc[0]), 1, dt, bc=bc[1])
    assert max(hydro_errs(got, oref)) <= TOL


def test_xy_f32_state_matches_split():
    """FP32 state: both paths round the x-swept state to FP32 and agree to a
    few FP32 units (bound 4 u per physical field, L1); against the FP64
    oracle the two-sweep kernel is then no further off than the split FP32
    path plus that difference (triangle inequality on the same L1 norms)."""
    from gpu_util import hydro_l1_errs
    U = inputs.euler_ic(150, 70, seed=11, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    got, sm = _xy(U, dt, dtype=torch.float32, precision=H.PREC_F32_F64ACC)
    ref, smr = _split(U, dt, dtype=torch.float32, precision=H.PREC_F32_F64ACC)
    d = hydro_l1_errs(got, ref)
    assert max(d.values()) <= 4 * 2.0 ** -24
    oref = oracle.euler_sweep(oracle.euler_sweep(U, 0, dt), 1, dt)
    e_xy, e_split = hydro_l1_errs(got, oref), hydro_l1_errs(ref, oref)
    print("f32 xy vs oracle", e_xy, "split vs oracle", e_split, flush=True)
    for f in e_xy:
        assert e_xy[f] <= e_split[f] + d[f] * (1 + 1e-9)


def test_xy_stepper_twenty_steps():
    """Twenty steps with dt from the fused CFL reduction: one chain per step
    against two chains per step and against the oracle, within 1e-12."""
    nx, ny, steps = 200, 96, 20
    U = inputs.euler_ic(nx, ny)
    a = EulerStepper(nx, ny, fused_step=True)
    b = EulerStepper(nx, ny)
    assert a.ixy.family == 9
    a.load(U)
    b.load(U)
    a.step(steps)
    b.step(steps)
    ga, gb = host(a.state()), host(b.state())
    assert max(hydro_errs(ga, gb)) <= TOL
    ref, _ = oracle.euler_run(U, steps)
    assert max(hydro_errs(ga, ref)) <= TOL
