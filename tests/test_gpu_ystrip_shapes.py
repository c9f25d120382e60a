"""Tile shapes of the strip kernels (y: columns x rows per chunk 64 x 2/4/8,
32 x 8, 16 x 16, 8 x 32; x: rows x cells per chunk 1 x 64/128/256, 2 x 32)
give the same bits: a cell's arithmetic does not depend on how lanes and
waves are laid over the tile, nor on the segment length (each segment
recomputes its halo with the same formulas).  Ragged tiles and segments,
one-row and one-column grids, both boundaries; the in-place 16 x 16 y strip
and 2 x 32 x strip against two states."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import host, hydro_errs
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from paper_1710_08774_amd.euler import EulerStepper
from test_gpu_parity import TOL64, _sweep_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(256, 32, 23, 3), (256, 16, 63, 3), (256, 16, 47, 3), (256, 16, 15, 3), (256, 16, 1, 3),
          (256, 8, 95, 3), (256, 8, 31, 3), (512, 64, 15, 3), (128, 1, 7, 3)]


@pytest.mark.parametrize("size", [(300, 70), (17, 130), (1, 40), (129, 1), (256, 256)])
@pytest.mark.parametrize("bc", [H.BC_PERIODIC, H.BC_TRANSMISSIVE])
def test_y_strip_shapes_bitwise(size, bc):
    nx, ny = size
    U = inputs.euler_ic(nx, ny, seed=nx + 7 * ny, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    ref = _sweep_gpu(U, 1, dt, H.MODE_FUSED, bc=bc, forced=(256, 1, 15, 3))
    assert max(hydro_errs(ref, oracle.euler_sweep(U, 1, dt, bc=bc))) <= TOL64
    for cfg in SHAPES:
        print("y strip", size, bc, cfg, flush=True)
        got = _sweep_gpu(U, 1, dt, H.MODE_FUSED, bc=bc, forced=cfg)
        assert np.array_equal(got, ref), cfg


def test_y_strip_16x16_run_and_cfl_bitwise():
    """30 steps with the CFL reduction fused into the 16 x 16 strip: the
    same state and dt slots as the 64 x 4 strip, and within 1e-12 of the
    oracle."""
    nx, ny = 200, 333
    U = inputs.euler_ic(nx, ny, seed=105)
    a = EulerStepper(nx, ny, forced_y=(256, 1, 15, 3))
    b = EulerStepper(nx, ny, forced_y=(256, 16, 47, 3))
    a.load(U)
    b.load(U)
    a.step(30)
    b.step(30)
    assert torch.equal(a.state(), b.state()) and torch.equal(a.smax, b.smax)
    ref, _ = oracle.euler_run(U, 30)
    assert max(hydro_errs(host(b.state()), ref)) <= TOL64


@pytest.mark.parametrize("bc", [H.BC_PERIODIC, H.BC_TRANSMISSIVE])
def test_y_strip_16x16_in_place_bitwise(bc):
    nx, ny = 300, 200
    U = inputs.euler_ic(nx, ny, seed=106)
    cfg = (256, 16, 47, 3)
    a = EulerStepper(nx, ny, bc=bc, forced_y=cfg)
    b = EulerStepper(nx, ny, bc=bc, forced_y=cfg, in_place=True)
    assert b.iy.fused and b.iy.config.tile_y == 16 and b.iy.workspace_bytes > 0
    a.load(U)
    b.load(U)
    a.step(10)
    b.step(10)
    assert torch.equal(a.state(), b.state())


XSHAPES = [(64, 2, 191, 3), (64, 2, 31, 3), (64, 2, 0, 3), (64, 2, 1, 3), (128, 1, 100, 3), (256, 1, 255, 3)]


@pytest.mark.parametrize("size", [(300, 70), (17, 131), (1, 40), (129, 1), (400, 3)])
@pytest.mark.parametrize("bc", [H.BC_PERIODIC, H.BC_TRANSMISSIVE])
def test_x_strip_shapes_bitwise(size, bc):
    nx, ny = size
    U = inputs.euler_ic(nx, ny, seed=3 * nx + ny, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    ref = _sweep_gpu(U, 0, dt, H.MODE_FUSED, bc=bc, forced=(64, 1, 191, 3))
    assert max(hydro_errs(ref, oracle.euler_sweep(U, 0, dt, bc=bc))) <= TOL64
    for cfg in XSHAPES:
        print("x strip", size, bc, cfg, flush=True)
        got = _sweep_gpu(U, 0, dt, H.MODE_FUSED, bc=bc, forced=cfg)
        assert np.array_equal(got, ref), cfg


@pytest.mark.parametrize("bc", [H.BC_PERIODIC, H.BC_TRANSMISSIVE])
def test_x_strip_2x32_in_place_bitwise(bc):
    nx, ny = 400, 131
    U = inputs.euler_ic(nx, ny, seed=107)
    cfg = (64, 2, 191, 3)
    a = EulerStepper(nx, ny, bc=bc, forced_x=cfg)
    b = EulerStepper(nx, ny, bc=bc, forced_x=cfg, in_place=True)
    assert b.ix.fused and b.ix.config.tile_y == 2 and b.ix.workspace_bytes > 0
    a.load(U)
    b.load(U)
    a.step(10)
    b.step(10)
    assert torch.equal(a.state(), b.state())
