"""Batched persistent sweeps over many uneven grids, and HIP-graph capture."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import host, hydro_errs
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from paper_1710_08774_amd.euler import EulerBatchStepper, EulerStepper

pytestmark = pytest.mark.gpu


def _sizes(n, seed, lo=8, hi=200):
    return inputs.batch_sizes(n, seed=seed, lo=lo, hi=hi)


def test_batch_matches_single_grid_bitwise():
    sizes = _sizes(24, 11) + [(1, 5), (70, 1), (64, 64), (65, 129)]
    states = inputs.batch_ic(sizes=sizes, seed=11)
    # the batch runs the single-grid strip bodies: one wave per 191-cell row
    # segment, 4-row strips over 64 columns x 11-row segments
    bt = EulerBatchStepper(sizes, forced_y=(256, 1, 11, 3))
    bt.load(states)
    bt.step(4)
    torch.cuda.synchronize()
    for g, (nx, ny) in enumerate(sizes):
        st = EulerStepper(nx, ny, forced_x=(64, 1, 191, 3), forced_y=(256, 1, 11, 3))
        st.load(states[g])
        st.step(4)
        assert np.array_equal(host(bt.grid(g)), host(st.state())), (g, nx, ny)


def test_batch_per_grid_dt_and_oracle_parity():
    sizes = _sizes(16, 3, lo=32, hi=160)
    states = inputs.batch_ic(sizes=sizes, seed=3)
    bt = EulerBatchStepper(sizes)
    bt.load(states)
    bt.step(10)
    torch.cuda.synchronize()
    for g, U in enumerate(states):
        ref, _ = oracle.euler_run(U, 10)
        assert max(hydro_errs(host(bt.grid(g)), ref)) <= 1e-12, g
    # every grid advanced with its own time step
    assert len(set(np.round(host(bt.smax[0]), 12))) > 1


def test_graph_replays_match_eager():
    sizes = _sizes(12, 5, lo=16, hi=120)
    states = inputs.batch_ic(sizes=sizes, seed=5)
    eager = EulerBatchStepper(sizes)
    eager.load(states)
    graphed = EulerBatchStepper(sizes)
    graphed.load(states)
    graphed.capture(4)
    for rep in range(3):
        graphed.replay()
        eager.step(4)
        # unrelated eager work and a synchronisation between replays
        torch.cuda.synchronize()
        junk = torch.ones(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for g in range(len(sizes)):
            assert np.array_equal(host(graphed.grid(g)), host(eager.grid(g))), (rep, g)
        assert float(junk) == float(1 << 20)


def test_batch_config_workload_sizes_two_steps():
    # the batched workload's real sizes (sides 64..1024), 512 grids, checked on
    # a seeded sample of 6 grids against the oracle
    sizes = inputs.batch_sizes(512)
    states = inputs.batch_ic(sizes=sizes)
    bt = EulerBatchStepper(sizes)
    bt.load(states)
    bt.step(2)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for g in rng.choice(512, 6, replace=False):
        ref, _ = oracle.euler_run(states[g], 2)
        assert max(hydro_errs(host(bt.grid(g)), ref)) <= 1e-12, g


def test_batch_errors():
    c = H.Chain(H.hdiff_spec())
    with pytest.raises(H.HfavError) as e:
        c.plan_batch([(8, 8)])
    assert e.value.code in (H.EUNSUP,)
    cx = H.Chain(H.euler_sweep_spec(0))
    with pytest.raises(H.HfavError) as e:
        cx.plan_batch([(8, 0)])
    assert e.value.code == H.EINVAL
