"""The one-launch batch step (both sweeps of every grid in one persistent
launch, y items waiting on per-grid counters of the x items): bit for bit
against the per-sweep batch, which runs the same strip bodies; through a
HIP graph; at the batched workload's full sizes; and the bounded wait's
give-up path, forced from the host."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import host, hydro_errs
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from paper_1710_08774_amd.euler import EulerBatchStepper

pytestmark = pytest.mark.gpu

# one cell, single rows and columns, rows of exactly one and two x
# segments, bands of 4 rows with 1..3 left over, tiles past 64 columns
EDGE = [(1, 1), (1, 5), (70, 1), (191, 4), (192, 3), (383, 9), (64, 64), (65, 129), (5, 300)]


def _same(a, b, sizes, what):
    for g in range(len(sizes)):
        assert np.array_equal(host(a.grid(g)), host(b.grid(g))), (what, g, sizes[g])
    assert torch.equal(a.smax, b.smax), what


@pytest.mark.parametrize("bc", [H.BC_PERIODIC, H.BC_TRANSMISSIVE])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_step_batch_matches_per_sweep_batch_bitwise(bc, dtype):
    sizes = inputs.batch_sizes(24, seed=13, lo=8, hi=260) + EDGE
    states = inputs.batch_ic(sizes=sizes, seed=13)
    a = EulerBatchStepper(sizes, dtype=dtype, bc=bc)
    b = EulerBatchStepper(sizes, dtype=dtype, bc=bc, fused_step=True)
    assert b.ixy.workspace_bytes > 0
    a.load(states)
    b.load(states)
    for k in range(3):
        a.step(2)
        b.step(2)
        assert b.step_status() == 0
        _same(a, b, sizes, k)


def test_step_batch_every_newton_step_bitwise():
    """Configuration bit 64 (every Newton step) gives the same bits."""
    sizes = inputs.batch_sizes(10, seed=21, lo=16, hi=200) + [(1, 1), (191, 4)]
    states = inputs.batch_ic(sizes=sizes, seed=21)
    a = EulerBatchStepper(sizes, fused_step=True)
    b = EulerBatchStepper(sizes, fused_step=True, forced_xy=(256, 1, 15, 3 | 64, 0))
    a.load(states)
    b.load(states)
    a.step(4)
    b.step(4)
    _same(a, b, sizes, "newton")


def test_step_batch_graph_replays_match_eager():
    sizes = inputs.batch_sizes(12, seed=5, lo=16, hi=120) + [(1, 1), (191, 4)]
    states = inputs.batch_ic(sizes=sizes, seed=5)
    eager = EulerBatchStepper(sizes, fused_step=True)
    eager.load(states)
    graphed = EulerBatchStepper(sizes, fused_step=True)
    graphed.load(states)
    graphed.capture(4)
    for rep in range(3):
        graphed.replay()
        eager.step(4)
        # unrelated eager work and a synchronisation between replays
        torch.cuda.synchronize()
        junk = torch.ones(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert graphed.step_status() == 0
        _same(graphed, eager, sizes, rep)
        assert float(junk) == float(1 << 20)


def test_step_batch_512_grids_matches_per_sweep_batch():
    """The batched workload's real sizes (512 grids, sides 64..1024): every
    cell bit for bit against the per-sweep batch after 2 steps, and three
    seeded grids against the oracle."""
    sizes = inputs.batch_sizes(512)
    states = inputs.batch_ic(sizes=sizes)
    a = EulerBatchStepper(sizes)
    a.load(states)
    a.step(2)
    torch.cuda.synchronize()
    ref_state, ref_smax = a.U[a.cur].clone(), a.smax.clone()
    del a
    b = EulerBatchStepper(sizes, fused_step=True)
    b.load(states)
    b.step(2)
    assert b.step_status() == 0
    assert torch.equal(b.U[b.cur], ref_state)
    assert torch.equal(b.smax, ref_smax)
    rng = np.random.default_rng(inputs.BASE_SEED + 9)
    for g in rng.choice(len(sizes), 3, replace=False):
        ref, _ = oracle.euler_run(states[g], 2)
        assert max(hydro_errs(host(b.grid(g)), ref)) <= 1e-12, (int(g), sizes[g])


def test_step_batch_give_up_sets_status_and_nan_slot():
    """Variant bit 128: every y item awaits a count the x items never reach
    and gives up after 64 polls; the launch still ends, the status word says
    so, and every grid's CFL slot holds NaN."""
    sizes = [(64, 64), (100, 37), (1, 1), (300, 5)]
    states = inputs.batch_ic(sizes=sizes, seed=2)
    b = EulerBatchStepper(sizes, fused_step=True, forced_xy=(256, 1, 15, 3 | 128, 0))
    b.load(states)
    b.step(1)
    assert b.step_status() == 1
    assert bool(torch.isnan(b.smax[1]).all())
    # a correct plan on the same buffers runs clean again
    c = EulerBatchStepper(sizes, fused_step=True)
    c.load(states)
    c.step(1)
    assert c.step_status() == 0
    assert bool(torch.isfinite(c.smax[1]).all())
