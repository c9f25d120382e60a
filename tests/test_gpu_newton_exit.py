"""The Riemann solver's Newton loop stops at the first repeated iterate
(a cycle of period 1 to 6, from which every later iterate is known);
configuration variant bit 64 takes all the steps instead.  Same
kernels, same arithmetic per step: the states must agree bit for bit, over
many steps, on every sweep kernel that runs the solver."""
import numpy as np
import pytest
import torch

from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from paper_1710_08774_amd.euler import EulerBatchStepper, EulerStepper

pytestmark = pytest.mark.gpu
ALL = 64


def _all_steps(info):
    c = info.config
    assert not c.variant & ALL
    return (c.block, c.tile_y, c.seg, c.variant | ALL, c.xcd)


@pytest.mark.parametrize("nx,ny,bc,steps", [
    (2048, 2048, H.BC_PERIODIC, 12),     # the benchmarked workload and launch configuration
    (333, 77, H.BC_TRANSMISSIVE, 30),    # ragged segments, the right-end Riemann problem
    (150, 70, H.BC_PERIODIC, 30),
])
def test_split_sweeps_bitwise(nx, ny, bc, steps):
    print("newton exit: split sweeps", nx, ny, bc, steps, flush=True)
    U = inputs.euler_ic(nx, ny, seed=inputs.BASE_SEED + inputs.W_EULER + ny)
    a = EulerStepper(nx, ny, bc=bc)
    b = EulerStepper(nx, ny, bc=bc, forced_x=_all_steps(a.ix), forced_y=_all_steps(a.iy))
    for st in (a, b):
        st.load(U)
        st.step(steps)
    torch.cuda.synchronize()
    assert torch.equal(a.state(), b.state())
    assert torch.equal(a.smax, b.smax)
    assert bool(torch.isfinite(a.state()).all())


@pytest.mark.parametrize("fx,fy", [((256, 1, 0, 0), (64, 1, 16, 0)),      # row kernel, register-window y kernel
                                   ((128, 1, 0, 2), (128, 1, 16, 1))])    # occupancy variants
def test_other_sweep_kernels_bitwise(fx, fy):
    nx, ny = 300, 140
    print("newton exit: other sweep kernels", fx, fy, flush=True)
    U = inputs.euler_ic(nx, ny, seed=inputs.BASE_SEED + 17)
    a = EulerStepper(nx, ny, forced_x=fx, forced_y=fy)
    b = EulerStepper(nx, ny, forced_x=fx[:3] + (fx[3] | ALL,), forced_y=fy[:3] + (fy[3] | ALL,))
    for st in (a, b):
        st.load(U)
        st.step(20)
    torch.cuda.synchronize()
    assert torch.equal(a.state(), b.state())


def test_f32_state_bitwise():
    nx, ny = 256, 192
    print("newton exit: FP32 state", flush=True)
    U = inputs.euler_ic(nx, ny, seed=inputs.BASE_SEED + 18)
    a = EulerStepper(nx, ny, dtype=torch.float32)
    b = EulerStepper(nx, ny, dtype=torch.float32, forced_x=_all_steps(a.ix), forced_y=_all_steps(a.iy))
    for st in (a, b):
        st.load(U)
        st.step(30)
    torch.cuda.synchronize()
    assert torch.equal(a.state(), b.state())


def test_two_sweep_kernel_bitwise():
    nx, ny = 200, 96
    print("newton exit: two-sweep kernel", flush=True)
    U = inputs.euler_ic(nx, ny, seed=inputs.BASE_SEED + 19)
    a = EulerStepper(nx, ny, fused_step=True)
    b = EulerStepper(nx, ny, fused_step=True, forced_xy=_all_steps(a.ixy))
    for st in (a, b):
        st.load(U)
        st.step(20)
    torch.cuda.synchronize()
    assert torch.equal(a.state(), b.state())


def test_batch_bitwise():
    sizes = inputs.batch_sizes(20, seed=23, lo=8, hi=200)
    print("newton exit: batch", len(sizes), flush=True)
    states = inputs.batch_ic(sizes=sizes, seed=23)
    a = EulerBatchStepper(sizes)
    b = EulerBatchStepper(sizes, forced_x=_all_steps(a.ix), forced_y=_all_steps(a.iy))
    for bt in (a, b):
        bt.load(states)
        bt.step(10)
    torch.cuda.synchronize()
    assert torch.equal(a.U[0], b.U[0])
    assert bool(torch.isfinite(a.U[0]).all())
