"""In-place execution on the GPU (Design, "In/out chaining"): the goal is
written over its axiom's buffer; results must equal the oracle's (which
never aliases) bit for bit for the linear chains, within 1e-12 for the
normalisation chain."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, relerr
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs

pytestmark = pytest.mark.gpu
Z = (0, 0, 0)


def _ws(info):
    return torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("shape,cfg", [
    ((3, 70, 200), None),                     # default tiles
    ((2, 70, 200), (64, 1, 7, 4, 0)),         # ragged x tiles and row segments
    ((2, 65, 256), (256, 1, 64, 1, -1)),      # one x tile: the halo wraps onto itself
    ((1, 33, 130), (128, 1, 1, 2, 0)),        # one-row segments
    ((2, 5, 300), (512, 1, 64, 8, 0)),        # one segment; the DPP bit is ignored in place
    ((4, 130, 96), (64, 1, 16, 18, 8)),       # full last tile, XCD order, store hint ignored
])
def test_hdiff_in_place_bitwise(shape, cfg):
    nk, nj, ni = shape
    print("hdiff in place", shape, cfg, flush=True)
    a = inputs.hdiff_input(nk, nj, ni, seed=ni + nj)
    ref = oracle.hdiff(a)
    c = H.Chain(H.hdiff_spec())
    c.alias("out", "u")
    kw = dict(config_source=H.CONFIG_FORCED, forced=cfg) if cfg else {}
    info = c.plan((ni, nj, nk), mode=H.MODE_FUSED, **kw)
    assert c.plan_json()["aliases"][0]["handling"] == "tile_halo_copies"
    u = dev(a)
    c.execute([u], [u], _ws(info))
    assert np.array_equal(host(u), ref)


def test_hdiff_in_place_repeated_steps():
    """Five in-place applications equal five applications of the oracle."""
    a = inputs.hdiff_input(2, 40, 100, seed=9)
    ref = a
    for _ in range(5):
        ref = oracle.hdiff(ref)
    c = H.Chain(H.hdiff_spec())
    c.alias("out", "u")
    info = c.plan((100, 40, 2), mode=H.MODE_FUSED)
    u = dev(a)
    ws = _ws(info)
    for _ in range(5):
        c.execute([u], [u], ws)
    assert np.array_equal(host(u), ref)


@pytest.mark.parametrize("ni", [4096, 1000, 20000])
def test_norm_in_place(ni):
    nq, nj = 3, 21
    u0 = inputs.norm_input(nq, nj, ni, seed=inputs.BASE_SEED + 96 + ni)
    ref = oracle.normalize(u0, 0.7)
    c = H.Chain(H.norm_spec(nq, 0.7))
    for q in range(nq):
        c.alias(f"out{q}", f"u{q}")
    info = c.plan((ni, nj))
    assert info.fused == (ni <= 16384)
    u = dev(u0)
    c.execute([u[q] for q in range(nq)], [u[q] for q in range(nq)], _ws(info))
    got = host(u)
    for q in range(nq):
        assert relerr(got[q], ref[q]) <= 1e-12


@pytest.mark.parametrize("mode", [H.MODE_AUTO, H.MODE_UNFUSED])
def test_biharm_in_place_unfused(mode):
    a = inputs.biharm_input(24, shape=(20, 24, 28))
    c = H.Chain(H.biharm_spec())
    c.alias("out", "u")
    info = c.plan((28, 24, 20), mode=mode)
    assert not info.fused
    u = dev(a)
    c.execute([u], [u], _ws(info))
    assert np.array_equal(host(u), oracle.biharm(a))


def test_neighbour_reads_in_place_use_the_saved_copy():
    spec = H.ChainSpec(ndim=2, axioms=[("u", 2)], goals=["out"],
                       rules=[H.Rule("STAR", [("u", (1, 0, 0)), ("u", (-1, 0, 0))], ["out"], [1.0, -1.0])])
    a = inputs.rng_for(3).random((30, 50))
    ref = np.roll(a, -1, axis=1) - np.roll(a, 1, axis=1)
    c = H.Chain(spec)
    c.alias("out", "u")
    info = c.plan((50, 30))
    assert c.plan_json()["aliases"][0]["handling"] == "full_copy"
    u = dev(a)
    c.execute([u], [u], _ws(info))
    assert np.array_equal(host(u), ref)
