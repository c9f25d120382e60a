"""GPU parity: the HIP fused and unfused paths against the FP64 CPU oracle.

Every case calls the library through the C ABI (the ctypes binding) on
seeded inputs shared with the oracle.  FP64 tolerance: 1e-12 normwise
relative error per output field.  The bandwidth-bound chains evaluate each
rule in the oracle's operation order without FMA contraction, so they are
also required to match bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, hydro_errs, relerr
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs
from paper_1710_08774_amd.euler import EulerStepper

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


# ------------------------------------------------------------------ hdiff
HDIFF_SHAPES = [(1, 8, 8), (3, 13, 7), (2, 65, 3), (1, 1, 40), (2, 100, 300), (8, 256, 256)]


@pytest.mark.parametrize("shape", HDIFF_SHAPES)
@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_hdiff_parity(shape, mode):
    nk, nj, ni = shape
    a = inputs.hdiff_input(nk, nj, ni, seed=sum(shape) + 7)
    ref = oracle.hdiff(a)
    c = H.Chain(H.hdiff_spec())
    info = c.plan((ni, nj, nk), mode=mode)
    assert info.fused == (mode == H.MODE_FUSED)
    u = dev(a)
    out = torch.empty_like(u)
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda") if info.workspace_bytes else None
    c.execute([u], [out], ws)
    got = host(out)
    assert relerr(got, ref) <= TOL64
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("block,seg", [(64, 1), (64, 7), (128, 16), (512, 64)])
@pytest.mark.parametrize("variant", [0, 1, 4, 8, 9, 12, 18, 26])
def test_hdiff_tile_configs(block, seg, variant):
    # variants 8-12: neighbours along the lane axis by DPP lane shifts;
    # + 16: non-temporal output stores
    a = inputs.hdiff_input(2, 70, 200, seed=3)
    ref = oracle.hdiff(a)
    c = H.Chain(H.hdiff_spec())
    c.plan((200, 70, 2), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=(block, 1, seg, variant))
    u = dev(a)
    out = torch.empty_like(u)
    c.execute([u], [out])
    assert np.array_equal(host(out), ref)


@pytest.mark.parametrize("shape", [(1, 8, 8), (3, 13, 7), (2, 65, 3), (2, 100, 300)])
def test_hdiff_dpp_parity_ragged(shape):
    nk, nj, ni = shape
    a = inputs.hdiff_input(nk, nj, ni, seed=sum(shape) + 11)
    ref = oracle.hdiff(a)
    for block in (64, 256):
        c = H.Chain(H.hdiff_spec())
        c.plan((ni, nj, nk), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=(block, 1, 5, 8))
        u = dev(a)
        out = torch.empty_like(u)
        c.execute([u], [out])
        assert np.array_equal(host(out), ref), block


def test_hdiff_f32_error_bound():
    a = inputs.hdiff_input(2, 64, 96, seed=4)
    a32 = a.astype(np.float32).astype(np.float64)
    ref = oracle.hdiff(a32)
    c = H.Chain(H.hdiff_spec(dtype=H.F32))
    c.plan((96, 64, 2))
    u = dev(a, torch.float32)
    out = torch.empty_like(u)
    c.execute([u], [out])
    assert relerr(host(out), ref) <= 4e-7


# ------------------------------------------------------------------ euler, one sweep
def _sweep_gpu(U, direction, dt, mode, bc=H.BC_PERIODIC, forced=None):
    _, ny, nx = U.shape
    c = H.Chain(H.euler_sweep_spec(direction, dt_source="dt"))
    src = H.CONFIG_FORCED if forced else H.CONFIG_DEFAULT
    info = c.plan((nx, ny), (bc, bc), mode=mode, config_source=src, forced=forced)
    d = dev(U)
    o = torch.empty_like(d)
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda") if info.workspace_bytes else None
    c.execute([d[0], d[1], d[2], d[3], dtt], [o[0], o[1], o[2], o[3]], ws)
    return host(o)


@pytest.mark.parametrize("shape", [(8, 8), (48, 64), (37, 100), (5, 300), (130, 3)])
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_euler_sweep_parity(shape, direction, mode):
    ny, nx = shape
    U = inputs.euler_ic(nx, ny, seed=nx * 31 + ny, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    ref = oracle.euler_sweep(U, direction, dt)
    got = _sweep_gpu(U, direction, dt, mode)
    assert max(hydro_errs(got, ref)) <= TOL64


@pytest.mark.parametrize("direction,cfg", [(0, (64, 1, 0, 0)), (0, (256, 1, 0, 0)),
                                           (1, (128, 1, 3, 0)), (1, (256, 1, 64, 0)), (1, (64, 1, 1, 0)),
                                           (0, (64, 1, 0, 3)), (0, (256, 1, 0, 3)), (1, (256, 1, 16, 3)),
                                           (1, (128, 1, 5, 3)), (1, (512, 1, 64, 3)), (1, (256, 1, 1, 3)),
                                           (1, (512, 1, 127, 3)), (1, (512, 1, 31, 3)), (1, (128, 1, 3, 3)),
                                           (1, (256, 1, 15, 3)), (1, (256, 1, 7, 3)), (1, (256, 1, 3, 3)),
                                           (0, (256, 1, 255, 3)), (0, (128, 1, 100, 3)), (0, (64, 1, 63, 3)),
                                           (0, (256, 1, 1, 3)), (0, (128, 1, 299, 3))])
def test_euler_sweep_tile_configs(direction, cfg):
    U = inputs.euler_ic(300, 70, seed=12, amp=0.05)
    dt = 0.5 / oracle.euler_smax(U)
    ref = oracle.euler_sweep(U, direction, dt)
    got = _sweep_gpu(U, direction, dt, H.MODE_FUSED, forced=cfg)
    assert max(hydro_errs(got, ref)) <= TOL64


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("strip", [False, True])
def test_euler_transmissive_sweep(direction, strip):
    n = 128
    x = (np.arange(n) + 0.5) / n
    rho = np.where(x < 0.5, 1.0, 0.125)
    p = np.where(x < 0.5, 1.0, 0.1)
    if direction == 0:
        U = inputs.euler_state_from_prim(np.tile(rho, (3, 1)), 0.0, 0.0, np.tile(p, (3, 1)))
    else:
        U = inputs.euler_state_from_prim(np.tile(rho[:, None], (1, 3)), 0.0, 0.0, np.tile(p[:, None], (1, 3)))
    for mode in (H.MODE_FUSED, H.MODE_UNFUSED):
        V = U.copy()
        W = U.copy()
        for _ in range(10):
            dt = 0.5 / oracle.euler_smax(V)
            V = oracle.euler_sweep(V, direction, dt, bc=oracle.BC_TRANSMISSIVE)
            forced = ((256, 1, 16, 3) if strip else None) if mode == H.MODE_FUSED else None
            W = _sweep_gpu(W, direction, dt, mode, bc=H.BC_TRANSMISSIVE, forced=forced)
        assert max(hydro_errs(W, V)) <= TOL64


def test_euler_constant_state_bitwise():
    U = inputs.euler_state_from_prim(np.full((40, 70), 0.7), 0.3, -0.4, 1.9)
    for d in (0, 1):
        for mode in (H.MODE_FUSED, H.MODE_UNFUSED):
            assert np.array_equal(_sweep_gpu(U, d, 0.1, mode), U)


# ------------------------------------------------------------------ euler, time stepping
@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_euler_run_parity(mode):
    nx, ny, steps = 96, 80, 30
    U = inputs.euler_ic(nx, ny, seed=101)
    ref, dts = oracle.euler_run(U, steps)
    st = EulerStepper(nx, ny, mode=mode)
    st.load(U)
    st.step(steps)
    got = host(st.state())
    assert max(hydro_errs(got, ref)) <= TOL64


@pytest.mark.parametrize("shape", [(96, 80), (200, 33)])
@pytest.mark.parametrize("ycfg", [(256, 1, 16, 3), (512, 1, 15, 3)])
def test_euler_run_parity_strip_kernels(shape, ycfg):
    # both sweeps as LDS-ring strips, the CFL reduction fused into the y strip
    nx, ny = shape
    U = inputs.euler_ic(nx, ny, seed=102)
    ref, _ = oracle.euler_run(U, 30)
    st = EulerStepper(nx, ny, forced_x=(256, 1, 0, 3), forced_y=ycfg)
    st.load(U)
    st.step(30)
    assert max(hydro_errs(host(st.state()), ref)) <= TOL64


def test_euler_multiwave_strips_short_segments():
    """Multi-wave strips (4-wave x blocks, 8-row y strips) over many short
    segments: each segment's prologue reads the ring slot that its first
    chunk's last cell takes, so the two must be ordered by a barrier (a
    race there corrupted the first updated cell of some segments)."""
    nx, ny = 1024, 768
    U = inputs.euler_ic(nx, ny, seed=104)
    ref, _ = oracle.euler_run(U, 3)
    st = EulerStepper(nx, ny, forced_x=(256, 1, 63, 3), forced_y=(512, 1, 7, 3))
    st.load(U)
    st.step(3)
    assert max(hydro_errs(host(st.state()), ref)) <= TOL64


def test_euler_config_workload_two_steps_full_size():
    # the benchmark configuration (2048^2, FP64, periodic), compared in full
    nx = ny = 2048
    U = inputs.euler_ic(nx, ny)
    ref, _ = oracle.euler_run(U, 2)
    st = EulerStepper(nx, ny)
    st.load(U)
    st.step(2)
    got = host(st.state())
    assert max(hydro_errs(got, ref)) <= TOL64


def test_euler_hundred_steps_parity():
    nx, ny = 256, 192
    U = inputs.euler_ic(nx, ny, seed=7)
    ref, _ = oracle.euler_run(U, 100)
    st = EulerStepper(nx, ny)
    st.load(U)
    st.step(100)
    assert max(hydro_errs(host(st.state()), ref)) <= TOL64


def test_fused_matches_unfused_stepper():
    nx, ny = 150, 70
    U = inputs.euler_ic(nx, ny, seed=9)
    a = EulerStepper(nx, ny, mode=H.MODE_FUSED)
    b = EulerStepper(nx, ny, mode=H.MODE_UNFUSED)
    a.load(U)
    b.load(U)
    a.step(10)
    b.step(10)
    # identical rule bodies; the two paths differ only in where the compiler
    # forms fused multiply-adds (about one rounding per rule evaluation),
    # which ten steps grow to the 1e-14 level
    assert max(hydro_errs(host(a.state()), host(b.state()))) <= 1e-13


def test_smax_reduction_matches_oracle():
    U = inputs.euler_ic(333, 77, seed=2, amp=0.05)
    st = EulerStepper(333, 77)
    st.load(U)
    torch.cuda.synchronize()
    assert abs(float(st.smax[0]) - oracle.euler_smax(U)) <= 1e-15 * oracle.euler_smax(U)


# ------------------------------------------------------------------ Riemann solver alone
def _riemann_gpu(WL, WR, gamma=1.4):
    """One EULER_RIEMANN rule over a 1 x n periodic row: interface m reads the
    plus face at m and the minus face at m+1, so minus[m+1] = WR[m]."""
    n = len(WL)
    z, e = (0, 0, 0), (1, 0, 0)
    plus, minus, gst = [f"p{q}" for q in range(4)], [f"m{q}" for q in range(4)], [f"g{q}" for q in range(4)]
    spec = H.ChainSpec(ndim=2, axioms=[(t, 2) for t in plus + minus], goals=gst,
                       rules=[H.Rule("EULER_RIEMANN", [(t, z) for t in plus] + [(t, e) for t in minus], gst,
                                     [gamma, oracle.NEWTON_ITERS])])
    c = H.Chain(spec)
    info = c.plan((n, 1), mode=H.MODE_UNFUSED)
    ins = [dev(WL[:, q][None, :]) for q in range(4)] + [dev(np.roll(WR[:, q], 1)[None, :]) for q in range(4)]
    outs = [torch.empty((1, n), dtype=torch.float64, device="cuda") for _ in range(4)]
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda") if info.workspace_bytes else None
    c.execute(ins, outs, ws)
    return np.stack([host(o)[0] for o in outs], axis=1)


def _extreme_riemann_states():
    """Double rarefactions whose star pressure falls 10..40 decades below the
    side pressures (including vacuum generation, where the pressure floor
    holds), and shock tubes with pressure jumps of up to 35 decades."""
    rng = inputs.rng_for(inputs.BASE_SEED + 99)
    L, R = [], []
    for s in np.linspace(3.0, 5.5, 40):                  # u = s c on each side
        pk = 10.0 ** rng.uniform(15, 30)
        c = np.sqrt(1.4 * pk)
        L.append((1.0, -s * c, 0.3, pk))
        R.append((1.0, s * c, -0.2, pk))
    for d in np.linspace(5, 35, 31):
        L.append((1.0, 0.0, 0.0, 10.0 ** (d / 2)))
        R.append((10.0 ** rng.uniform(-2, 2), 0.0, 0.0, 10.0 ** (-d / 2)))
    return np.array(L), np.array(R)


def test_riemann_rule_parity():
    """The device Riemann solver against the oracle's, problem by problem,
    on admissible random states and on extreme pressure ratios (the latter
    reach the exact power-of-two range reduction of the seventh-root)."""
    WL, WR = inputs.riemann_states(4096, seed=inputs.BASE_SEED + 98)
    XL, XR = _extreme_riemann_states()
    WL, WR = np.concatenate([WL, XL]), np.concatenate([WR, XR])
    ref, ps, _, _ = oracle.riemann(WL, WR)
    assert np.isfinite(ref).all()
    x = np.minimum(ps / WL[:, 3], ps / WR[:, 3])
    assert x.min() < 1e-35                               # the range-reduced branch is exercised
    got = _riemann_gpu(WL, WR)
    vscale = np.maximum.reduce([np.abs(WL[:, 1]), np.abs(WR[:, 1]), np.sqrt(1.4 * WL[:, 3] / WL[:, 0]),
                                np.sqrt(1.4 * WR[:, 3] / WR[:, 0])])
    for q, scale in ((0, np.abs(ref[:, 0])), (1, vscale), (2, np.abs(ref[:, 2]) + vscale), (3, np.abs(ref[:, 3]))):
        err = np.abs(got[:, q] - ref[:, q]) / scale
        assert err.max() <= TOL64, (q, int(err.argmax()), float(err.max()))


# ------------------------------------------------------------------ biharmonic
@pytest.mark.parametrize("shape", [(8, 8, 8), (5, 9, 70), (20, 33, 130), (64, 64, 64)])
@pytest.mark.parametrize("mode", [H.MODE_FUSED, H.MODE_UNFUSED])
def test_biharm_parity(shape, mode):
    nz, ny, nx = shape
    u = inputs.biharm_input(shape=shape, seed=nx + ny + nz)
    ref = oracle.biharm(u)
    c = H.Chain(H.biharm_spec())
    info = c.plan((nx, ny, nz), mode=mode)
    d = dev(u)
    o = torch.empty_like(d)
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda") if info.workspace_bytes else None
    c.execute([d], [o], ws)
    got = host(o)
    assert relerr(got, ref) <= TOL64
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 37, 38, 42])
@pytest.mark.parametrize("depth,seg", [(1, 5), (4, 6), (2, 17)])
def test_biharm_tile_variants(variant, depth, seg):
    # ragged tiles in x and y, segments that do not divide nz, every
    # prefetch depth; variants 6-9 own 2 or 4 points per lane, variants
    # 10-14 keep the z windows in registers
    shape = (17, 40, 150)
    u = inputs.biharm_input(shape=shape, seed=5)
    ref = oracle.biharm(u)
    c = H.Chain(H.biharm_spec())
    c.plan((150, 40, 17), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=(256, depth, seg, variant))
    d = dev(u)
    o = torch.empty_like(d)
    c.execute([d], [o])
    assert np.array_equal(host(o), ref)


@pytest.mark.parametrize("variant", [6, 7, 8, 9, 13])
def test_biharm_f32_tile_variants_equal_default(variant):
    """Every tile shape evaluates the same expression per point in the same
    order, so FP32 results equal the default tiles' bit for bit (here with
    ragged 128- and 256-wide tiles)."""
    shape = (9, 50, 300)
    u = inputs.biharm_input(shape=shape, seed=6)
    d = dev(u, torch.float32)
    outs = []
    for cfg in ((1024, 2, 7, 5), (1024, 2, 7, variant)):
        c = H.Chain(H.biharm_spec(dtype=H.F32))
        c.plan((300, 50, 9), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
        o = torch.empty_like(d)
        c.execute([d], [o])
        outs.append(host(o))
    assert np.array_equal(outs[0], outs[1])
    assert relerr(outs[1], oracle.biharm(u.astype(np.float32).astype(np.float64))) <= 1e-6


@pytest.mark.parametrize("dtype,nx", [(H.F32, 150), (H.F32, 301), (H.F64, 151)])
@pytest.mark.parametrize("variant", [6, 7, 8, 9])
def test_biharm_large_tiles_scalar_fetch(dtype, nx, variant):
    """The 1024-lane tiles (2 or 4 points per lane) on rows whose length is
    not a multiple of 4, with ragged tiles in x and y: the same results as
    the 64 x 16 tiles (FP32: bit for bit; FP64: also the oracle bit for
    bit)."""
    shape = (7, 37, nx)
    u = inputs.biharm_input(shape=shape, seed=nx + variant)
    tdt = torch.float32 if dtype == H.F32 else torch.float64
    d = dev(u, tdt)
    outs = []
    for cfg in ((1024, 2, 5, 5), (1024, 2, 5, variant)):
        c = H.Chain(H.biharm_spec(dtype=dtype))
        c.plan((nx, 37, 7), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
        o = torch.empty_like(d)
        c.execute([d], [o])
        outs.append(host(o))
    assert np.array_equal(outs[0], outs[1])
    if dtype == H.F64:
        assert np.array_equal(outs[1], oracle.biharm(u))


@pytest.mark.parametrize("dtype", [H.F32, H.F64])
def test_biharm_unaligned_buffers(dtype):
    """Buffers that do not start on a 16-byte boundary give the results of
    aligned buffers."""
    shape = (6, 20, 64)
    nz, ny, nx = shape
    u = inputs.biharm_input(shape=shape, seed=44)
    tdt = torch.float32 if dtype == H.F32 else torch.float64
    n = nx * ny * nz
    big = torch.zeros(n + 1, dtype=tdt, device="cuda")
    big[1:] = torch.as_tensor(u.reshape(-1), dtype=tdt)
    obig = torch.zeros(n + 1, dtype=tdt, device="cuda")
    d = dev(u, tdt)
    o = torch.empty_like(d)
    c = H.Chain(H.biharm_spec(dtype=dtype))
    c.plan((nx, ny, nz), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=(1024, 2, 4, 7))
    c.execute([d], [o])
    c.execute([big[1:]], [obig[1:]])
    assert np.array_equal(host(obig[1:]).reshape(shape), host(o))
    if dtype == H.F64:
        assert np.array_equal(host(o), oracle.biharm(u))


def test_biharm_f32_error_bound():
    shape = (32, 32, 32)
    u = inputs.biharm_input(shape=shape, seed=8)
    u32 = u.astype(np.float32).astype(np.float64)
    ref_a = oracle.biharm(u32)    # arithmetic error only
    ref_b = oracle.biharm(u)      # end to end
    c = H.Chain(H.biharm_spec(dtype=H.F32))
    c.plan((32, 32, 32))
    d = dev(u, torch.float32)
    o = torch.empty_like(d)
    c.execute([d], [o])
    got = host(o)
    assert relerr(got, ref_a) <= 1e-6
    assert relerr(got, ref_b) <= 1e-6


def test_hdiff_graph_replays_match_eager():
    """Executions captured in a HIP graph give the eager result on every
    replay, with unrelated eager work and synchronisations between replays."""
    a = inputs.hdiff_input(8, 256, 256, seed=31)
    ref = oracle.hdiff(a)
    c = H.Chain(H.hdiff_spec())
    c.plan((256, 256, 8))
    u = dev(a)
    o = torch.empty_like(u)
    c.execute([u], [o])
    eager = host(o)
    assert np.array_equal(eager, ref)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        for _ in range(3):
            c.execute([u], [o])
    for rep in range(3):
        o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        junk = torch.ones(1 << 20, device="cuda").sum()
        assert np.array_equal(host(o), eager), rep
        assert float(junk) == float(1 << 20)


def _lap7_edge(u):
    """7-point Laplacian with transmissive (edge-copy) boundaries, in the
    kernels' reference order (e, w, n, s, t, b: ((e + w) + (n + s)) + (t + b)
    - 6 c, every operation rounded)."""
    p = np.pad(u, 1, mode="edge")
    c = p[1:-1, 1:-1, 1:-1]
    e, w = p[1:-1, 1:-1, 2:], p[1:-1, 1:-1, :-2]
    n, s = p[1:-1, 2:, 1:-1], p[1:-1, :-2, 1:-1]
    t, b = p[2:, 1:-1, 1:-1], p[:-2, 1:-1, 1:-1]
    return ((e + w) + (n + s)) + (t + b) - 6.0 * c


@pytest.mark.parametrize("shape", [(5, 9, 70), (3, 4, 513), (4, 11, 1), (2, 3, 2), (6, 17, 1030)])
def test_biharm_unfused_transmissive_bitwise(shape):
    """The unfused path (two cells per lane in FP64; per-cell loads at row
    ends, at clamped references and on one- or two-cell rows) with
    transmissive boundaries on every axis, bit for bit against a direct
    evaluation in the same order."""
    nz, ny, nx = shape
    u = inputs.biharm_input(shape=shape, seed=nx + 3 * ny)
    nu = 1.0 / 128.0
    ref = u - nu * _lap7_edge(_lap7_edge(u))
    c = H.Chain(H.biharm_spec(nu))
    info = c.plan((nx, ny, nz), (H.BC_TRANSMISSIVE,) * 3, mode=H.MODE_UNFUSED)
    d = dev(u)
    o = torch.empty_like(d)
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda")
    c.execute([d], [o], ws)
    assert np.array_equal(host(o), ref)
