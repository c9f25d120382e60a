"""Hydro sweeps written over their state (Design, "In/out chaining"): the
in-place stepper (one state; before each sweep the cells around every
segment boundary are saved) against the stepper with two states, bit for
bit: the same kernels evaluate the same arithmetic, only where some inputs
are read from differs."""
import pytest
import torch

from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from paper_1710_08774_amd.euler import EulerStepper

pytestmark = pytest.mark.gpu
P, T = H.BC_PERIODIC, H.BC_TRANSMISSIVE


@pytest.mark.parametrize("nx,ny,bc,fx,fy,steps", [
    (2048, 2048, P, None, None, 6),                          # the benchmarked workload and configuration
    (333, 77, T, None, None, 20),
    (150, 70, P, None, None, 20),
    (100, 64, P, (64, 1, 0, 3), (256, 1, 1, 3), 10),         # whole rows (one segment wrapping onto itself); 1-row y segments
    (97, 41, T, (64, 1, 1, 3), (256, 1, 2, 3), 10),          # 1-cell and 2-row segments: clamps onto neighbours' cells
    (130, 90, T, (64, 1, 64, 3), (256, 1, 7, 3), 10),        # ragged last segments
])
def test_in_place_equals_two_states(nx, ny, bc, fx, fy, steps):
    print("in-place hydro", nx, ny, bc, fx, fy, steps, flush=True)
    U = inputs.euler_ic(nx, ny, seed=inputs.BASE_SEED + 61 + nx)
    a = EulerStepper(nx, ny, bc=bc, forced_x=fx, forced_y=fy)
    b = EulerStepper(nx, ny, bc=bc, forced_x=fx, forced_y=fy, in_place=True)
    assert b.ix.fused and b.iy.fused
    for ch in (b.cx, b.cy):
        assert all(al["handling"] == "segment_halo_copies" for al in ch.plan_json()["aliases"])
    for st in (a, b):
        st.load(U)
        st.step(steps)
    torch.cuda.synchronize()
    assert b.U[0].data_ptr() == b.U[1].data_ptr()
    assert torch.equal(a.state(), b.state())
    assert torch.equal(a.smax, b.smax)
    assert bool(torch.isfinite(b.state()).all())


def test_in_place_f32_state():
    nx, ny = 256, 192
    U = inputs.euler_ic(nx, ny, seed=inputs.BASE_SEED + 62)
    a = EulerStepper(nx, ny, dtype=torch.float32)
    b = EulerStepper(nx, ny, dtype=torch.float32, in_place=True)
    for st in (a, b):
        st.load(U)
        st.step(20)
    torch.cuda.synchronize()
    assert torch.equal(a.state(), b.state())


def test_in_place_footprint_halves_the_state():
    nx = ny = 2048
    a = EulerStepper(nx, ny)
    b = EulerStepper(nx, ny, in_place=True)
    state = 4 * nx * ny * 8
    assert a.footprint_bytes() == 2 * state
    # one state plus the saved segment halos: 4 cells x 4 fields per line
    # and boundary (y: ceil(2048 / seg) boundaries of 2048 columns)
    ws = max(b.ix.workspace_bytes, b.iy.workspace_bytes)
    assert b.footprint_bytes() == state + ws
    nsg = -(-ny // b.iy.config.seg)
    assert ws == 4 * nsg * 4 * nx * 8
    assert b.footprint_bytes() < 0.65 * a.footprint_bytes()
