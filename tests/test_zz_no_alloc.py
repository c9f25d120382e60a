"""hfav_execute_noalloc (workspace in the library's static device array)
against hfav_execute (a caller's workspace).  Both run the same kernels, so
the goals must agree bit for bit; the linear chains are also compared with
the oracle bit for bit.  Each case makes two calls in a row on one device,
the second on a smaller grid, so the second call finds the first one's
leftovers in the static array."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs, tune

pytestmark = pytest.mark.gpu


def _ws(info):
    return torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device="cuda")


def test_unfused_hdiff_two_sizes():
    for nk, nj, ni in ((8, 128, 160), (3, 64, 96)):
        print("noalloc unfused hdiff", (nk, nj, ni), flush=True)
        a = inputs.hdiff_input(nk, nj, ni, seed=ni + nj)
        c = H.Chain(H.hdiff_spec())
        info = c.plan((ni, nj, nk), mode=H.MODE_UNFUSED)
        assert not info.fused and 0 < info.workspace_bytes <= H.STATIC_WORKSPACE_BYTES
        u = dev(a)
        y_ws, y_na = torch.full_like(u, np.nan), torch.full_like(u, np.nan)
        c.execute([u], [y_ws], _ws(info))
        c.execute_noalloc([u], [y_na])
        got = host(y_na)
        assert np.array_equal(got, host(y_ws))
        assert np.array_equal(got, oracle.hdiff(a))


def test_in_place_hdiff_two_sizes():
    """The saved tile halos live in the static array."""
    for nk, nj, ni in ((4, 130, 300), (2, 40, 100)):
        print("noalloc in-place hdiff", (nk, nj, ni), flush=True)
        a = inputs.hdiff_input(nk, nj, ni, seed=nk + ni)
        c = H.Chain(H.hdiff_spec())
        c.alias("out", "u")
        info = c.plan((ni, nj, nk), mode=H.MODE_FUSED)
        assert info.fused and info.workspace_bytes > 0
        u_ws, u_na = dev(a), dev(a)
        c.execute([u_ws], [u_ws], _ws(info))
        c.execute_noalloc([u_na], [u_na])
        got = host(u_na)
        assert np.array_equal(got, host(u_ws))
        assert np.array_equal(got, oracle.hdiff(a))


def _star_chain(ndim, dims, seed):
    for k in range(1000):
        ch = inputs.random_chain(inputs.rng_for(seed + 1000 * k), ndim=ndim, dtype="f64", dims=dims)
        if ch["stages"][0]["f_in"] <= 3:
            return ch
    raise AssertionError("no chain drawn")


def test_star_chain_two_sizes():
    """The fused star groups read their coefficient table from the static
    array; the second chain has other coefficients on a smaller grid."""
    for dims, seed in (((96, 64, 48), 5), ((64, 32, 32), 6)):
        ch = _star_chain(3, dims, inputs.BASE_SEED + 700 + seed)
        print("noalloc star chain", tune.chain_dims(ch), len(ch["stages"]), flush=True)
        x = inputs.chain_input(ch, seed)
        c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
        info = c.plan(tune.chain_dims(ch), mode=H.MODE_FUSED)
        assert info.fused and info.workspace_bytes > 0
        xs = [torch.tensor(x[f], dtype=torch.float64, device="cuda") for f in range(x.shape[0])]
        nout = ch["stages"][-1]["f_out"]
        y_ws = [torch.full_like(xs[0], np.nan) for _ in range(nout)]
        y_na = [torch.full_like(xs[0], np.nan) for _ in range(nout)]
        c.execute(xs, y_ws, _ws(info))
        c.execute_noalloc(xs, y_na)
        got = np.stack([host(y) for y in y_na])
        assert np.array_equal(got, np.stack([host(y) for y in y_ws]))
        ref = oracle.linear_chain(ch, x, inputs.star_offsets)
        assert np.array_equal(got, ref)


def test_unfused_full_copy_alias_two_sizes():
    """An in-place goal read at neighbour offsets: the saved copy of the
    whole axiom lives in the static array."""
    spec = H.ChainSpec(ndim=2, axioms=[("u", 2)], goals=["out"],
                       rules=[H.Rule("STAR", [("u", (1, 0, 0)), ("u", (-1, 0, 0))], ["out"], [1.0, -1.0])])
    for nj, ni in ((90, 130), (30, 50)):
        print("noalloc full-copy alias", (nj, ni), flush=True)
        a = inputs.rng_for(ni).random((nj, ni))
        c = H.Chain(spec)
        c.alias("out", "u")
        info = c.plan((ni, nj))
        assert info.workspace_bytes > 0
        u_ws, u_na = dev(a), dev(a)
        c.execute([u_ws], [u_ws], _ws(info))
        c.execute_noalloc([u_na], [u_na])
        got = host(u_na)
        assert np.array_equal(got, host(u_ws))
        assert np.array_equal(got, np.roll(a, -1, axis=1) - np.roll(a, 1, axis=1))


def test_unfused_hydro_sweep_two_sizes():
    """One unfused x sweep of the hydro chain (prim, slopes, trace, Riemann,
    flux and update as separate kernels over full intermediates in the
    static array; dt from the CFL reduction of the state)."""
    for nx, ny in ((96, 64), (64, 40)):
        print("noalloc unfused hydro x sweep", (nx, ny), flush=True)
        U = inputs.euler_ic(nx, ny, seed=inputs.BASE_SEED + inputs.W_EULER + nx)
        st = torch.tensor(U, dtype=torch.float64, device="cuda")
        smax = torch.zeros(1, dtype=torch.float64, device="cuda")
        sm = H.Chain(H.smax_spec(1.4, H.F64))
        sm.plan((nx, ny))
        sm.execute(list(st), [smax[0]])
        c = H.Chain(H.euler_sweep_spec(0, 1.4, 10, 0.5, "smax", False, H.F64))
        info = c.plan((nx, ny), mode=H.MODE_UNFUSED)
        assert not info.fused and 0 < info.workspace_bytes <= H.STATIC_WORKSPACE_BYTES
        o_ws = torch.full_like(st, np.nan)
        o_na = torch.full_like(st, np.nan)
        c.execute(list(st) + [smax[0]], list(o_ws), _ws(info))
        c.execute_noalloc(list(st) + [smax[0]], list(o_na))
        got = host(o_na)
        assert np.isfinite(got).all()
        assert np.array_equal(got, host(o_ws))


def test_batch_step_two_batches():
    """The one-launch batch step: its control block (cursors, per-grid
    counters, the deal of grids to XCDs) and the x-swept state live in the
    static array; the step's own first launch zeroes what must start at
    zero, so the second call does not see the first one's counters."""
    for sizes in ([(64, 64), (100, 37), (1, 1), (300, 5), (191, 4)], [(40, 30), (7, 9)]):
        print("noalloc batch step", sizes, flush=True)
        states = inputs.batch_ic(sizes=sizes, seed=len(sizes))
        c = H.Chain(H.euler_step_spec(with_smax=True))
        info = c.plan_batch(sizes)
        assert 0 < info.workspace_bytes <= H.STATIC_WORKSPACE_BYTES
        off = [c.batch_offset(g) for g in range(len(sizes))]
        packed = np.zeros((4, off[-1] + sizes[-1][0] * sizes[-1][1]))
        for g, ((nx, ny), U) in enumerate(zip(sizes, states)):
            packed[:, off[g]:off[g] + nx * ny] = np.asarray(U).reshape(4, -1)
        u = dev(packed)
        sm = H.Chain(H.smax_spec())
        sm.plan_batch(sizes)
        smax0 = torch.zeros(len(sizes), dtype=torch.float64, device="cuda")
        sm.execute(list(u), [smax0])
        o_ws, o_na = torch.full_like(u, np.nan), torch.full_like(u, np.nan)
        s_ws, s_na = torch.full_like(smax0, np.nan), torch.full_like(smax0, np.nan)
        ws = _ws(info)
        c.execute(list(u) + [smax0], list(o_ws) + [s_ws], ws)
        c.execute_noalloc(list(u) + [smax0], list(o_na) + [s_na])
        torch.cuda.synchronize()
        assert int(ws[:4].cpu().view(torch.int32)[0]) == 0
        got = host(o_na)
        assert np.isfinite(got).all()
        assert np.array_equal(got, host(o_ws))
        assert torch.equal(s_na, s_ws)


def test_oversized_plan_is_refused_and_enqueues_nothing():
    nk, nj, ni = 12, 512, 512
    c = H.Chain(H.hdiff_spec())
    info = c.plan((ni, nj, nk), mode=H.MODE_UNFUSED)
    assert info.workspace_bytes > H.STATIC_WORKSPACE_BYTES
    u = torch.zeros((nk, nj, ni), dtype=torch.float64, device="cuda")
    y = torch.full_like(u, 7.0)
    rc = c.execute_noalloc_status([u], [y], torch.cuda.current_stream().cuda_stream)
    assert rc == H.ESIZE
    assert "static workspace" in H.last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
