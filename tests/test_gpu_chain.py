"""Random linear star chains (fused groups, every configuration) and the
cost-model MLP kernels against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import host, relerr
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs, tune

pytestmark = pytest.mark.gpu


U32 = 2.0 ** -24


def _run(ch, cfg=None, mode=H.MODE_FUSED, seed=0):
    x = inputs.chain_input(ch, seed)
    tdt = torch.float64 if ch["dtype"] == "f64" else torch.float32
    c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
    dims = tune.chain_dims(ch)
    if cfg is None:
        info = c.plan(dims, mode=mode)
    else:
        info = c.plan(dims, mode=mode, config_source=H.CONFIG_FORCED, forced=cfg)
    xs = [torch.tensor(x[f], dtype=tdt, device="cuda") for f in range(x.shape[0])]
    ys = [torch.empty_like(xs[0]) for _ in range(ch["stages"][-1]["f_out"])]
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda") if info.workspace_bytes else None
    c.execute(xs, ys, ws)
    got = np.stack([host(y) for y in ys])
    xin = x if ch["dtype"] == "f64" else x.astype(np.float32).astype(np.float64)
    ref = oracle.linear_chain(ch, xin, inputs.star_offsets)
    return got, ref, info, xin


def f32_abs_bound(ch, xin):
    """Absolute error bound of an FP32 evaluation of a linear star chain
    against the exact chain on the same (FP32-representable) input.

    Stage k forms each output as a sum of n_k = f_in (1 + 2 r nd) products
    c x with sum |c| = 1.  With the coefficients rounded to FP32 (|c^ - c|
    <= u |c|) and the products and n_k - 1 sums rounded (an inner product is
    within gamma_n sum |c^||x^| of its exact value, gamma_n = n u / (1 - n u);
    Higham, Accuracy and Stability of Numerical Algorithms, section 3.1), the
    error of stage k is its input's error (the map has infinity norm sum |c|
    = 1) plus (u + gamma_{n_k} (1 + u)) times the input's largest value, which
    never exceeds M0 = max |x| plus the error so far (a stage cannot grow the
    largest value).  Summed over the stages: (1 + O(n u)) sum_k (n_k + 1) u
    M0; the factor 1.01 covers the second-order terms (n u < 1e-4 here)."""
    nd = ch["ndim"]
    nk = [st["f_in"] * (1 + 2 * st["r"] * nd) for st in ch["stages"]]
    return 1.01 * sum(n + 1 for n in nk) * U32 * float(np.abs(xin).max())


def check_fields(ch, got, ref, xin, what=""):
    """Per output field: FP64 within 1e-12 normwise relative (and reported
    bitwise), FP32 within the derived absolute bound."""
    assert got.shape == ref.shape
    if ch["dtype"] == "f64":
        errs = [relerr(got[q], ref[q]) for q in range(ref.shape[0])]
        assert max(errs) <= 1e-12, (what, errs)
        return errs
    b = f32_abs_bound(ch, xin)
    for q in range(ref.shape[0]):
        e = float(np.abs(got[q] - ref[q]).max())
        assert e <= b, (what, q, e, b)
    return [relerr(got[q], ref[q]) for q in range(ref.shape[0])]


def _small_chains(n, seed):
    return tune.random_chains(n, seed, max_cells=40000)


def _chain_where(ndim, dtype, dims, seed, ok):
    for k in range(1000):
        ch = inputs.random_chain(inputs.rng_for(seed + 1000 * k), ndim=ndim, dtype=dtype, dims=dims)
        if ok(ch):
            return ch
    raise AssertionError("no chain drawn")


def _deep_chain(ndim, dtype, dims, seed):
    """First seeded chain with at least 4 stages and a stage of radius 3
    (long warm-up, the widest halos)."""
    return _chain_where(ndim, dtype, dims, seed,
                        lambda ch: len(ch["stages"]) >= 4 and max(st["r"] for st in ch["stages"]) == 3)


def _all_tiles_chain(ndim, dtype, dims, seed):
    """First seeded chain of at least 3 stages, one of radius >= 2, whose
    fully fused group fits LDS with every tile shape."""
    def ok(ch):
        if len(ch["stages"]) < 3 or max(st["r"] for st in ch["stages"]) < 2:
            return False
        cands = H.Chain(H.star_chain_spec(ch, inputs.star_offsets)).candidates(tune.chain_dims(ch))
        K = len(ch["stages"])
        return {cfg[3] for cfg in cands if cfg[1] == K} == {0, 1, 2, 3}
    return _chain_where(ndim, dtype, dims, seed, ok)


@pytest.mark.parametrize("k", range(8))
def test_star_chain_default_parity(k):
    ch = _small_chains(8, 77)[k]
    got, ref, info, xin = _run(ch)
    assert info.fused and info.family == 5
    check_fields(ch, got, ref, xin, f"chain {k}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_star_chain_every_configuration(ndim, dtype):
    """Every feasible configuration (fused group depth, tile shape, segment
    length) of a deep chain on a grid whose streamed axis holds at least
    three segments of every segment length plus a ragged last one (389 =
    3 x 128 + 5), with ragged tiles across: the warm-up of the segments
    after the first is compared with the oracle for every tile shape."""
    dims = (150, 389, 1) if ndim == 2 else (40, 26, 389)
    ch = _all_tiles_chain(ndim, dtype, dims, 40 + ndim)
    c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
    cands = c.candidates(tune.chain_dims(ch))
    assert len(cands) >= 3
    assert {cfg[3] for cfg in cands} == {0, 1, 2, 3}          # every tile shape
    nstream = dims[1] if ndim == 2 else dims[2]
    assert all(nstream >= 3 * cfg[2] for cfg in cands)        # >= 3 segments each
    for cfg in cands:
        got, ref, info, xin = _run(ch, cfg)
        check_fields(ch, got, ref, xin, cfg)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim,dims", [(2, (128, 640, 1)), (3, (64, 64, 128))])
def test_star_chain_at_study_sizes(ndim, dims, dtype):
    """Chains at sizes the cost-model study times (2-D 128..4096^2, 3-D
    64..512^3), in the planner's default configuration and in the
    unfused path, per output field."""
    ch = _deep_chain(ndim, dtype, dims, 60 + ndim)
    for mode in (H.MODE_FUSED, H.MODE_UNFUSED):
        got, ref, info, xin = _run(ch, mode=mode)
        assert bool(info.fused) == (mode == H.MODE_FUSED)
        errs = check_fields(ch, got, ref, xin, mode)
        print(f"star chain {ndim}-D {dims} {dtype} mode {mode}: per-field rel err {errs}", flush=True)


def test_star_chain_fp64_bitwise_to_the_oracle():
    """Without multiply-add contraction the fused stages round each product
    and sum in the oracle's order, so FP64 results are equal bit for bit."""
    ch = _deep_chain(3, "f64", (40, 26, 101), 80)
    got, ref, _, _ = _run(ch)
    assert np.array_equal(got, ref)


def test_star_chain_unfused_parity():
    ch = _small_chains(3, 5)[1]
    got, ref, info, xin = _run(ch, mode=H.MODE_UNFUSED)
    assert not info.fused
    check_fields(ch, got, ref, xin)


def test_star_chain_graph_capture_on_first_execute():
    """hfav_execute allocates nothing: a star chain is captured in a HIP
    graph on its first call (the coefficient table was staged by the plan),
    and each replay, with eager work in between, matches an eager run."""
    ch = _deep_chain(2, "f64", (160, 96, 1), 90)
    x = inputs.chain_input(ch, 3)
    c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
    info = c.plan(tune.chain_dims(ch), mode=H.MODE_FUSED)
    xs = [torch.tensor(x[f], device="cuda") for f in range(x.shape[0])]
    ys = [torch.zeros_like(xs[0]) for _ in range(ch["stages"][-1]["f_out"])]
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        c.execute(xs, ys, ws, stream=side)
    ref = oracle.linear_chain(ch, x, inputs.star_offsets)
    for rep in range(3):
        for y in ys:
            y.fill_(rep + 1.0)
        ws.fill_(7)                              # the replay must re-upload the coefficients
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = np.stack([host(y) for y in ys])
        check_fields(ch, got, ref, x, f"replay {rep}")


def test_binding_refuses_mismatched_tensors():
    """Wrong element type, too few elements or a strided view are refused
    by the binding before any launch."""
    c = H.Chain(H.hdiff_spec())
    c.plan((64, 32, 2))
    u = torch.zeros((2, 32, 64), dtype=torch.float64, device="cuda")
    o = torch.empty_like(u)
    for bad in (u.float(), u[:1], torch.zeros((2, 32, 128), dtype=torch.float64, device="cuda")[..., ::2]):
        with pytest.raises(H.HfavError) as e:
            c.execute([bad], [o])
        assert e.value.code == H.EINVAL
    c.execute([u], [o])
    torch.cuda.synchronize()


# ------------------------------------------------------------------ MLP kernels
def _mlp_case(n=96, d=H.COST_FEATURES, Hh=64, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d))
    t = rng.normal(size=n)
    P = tune.init_params(d, Hh, seed).astype(np.float64)
    P[H.mlp_nparams(d, Hh) - 1] = 0.3
    return X, t, P


def test_mlp_forward_and_gradients_vs_oracle():
    d, Hh = H.COST_FEATURES, 64
    X, t, P = _mlp_case()
    n = X.shape[0]
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    Pd = torch.tensor(P, dtype=torch.float32, device="cuda")
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    ws = torch.empty(H.mlp_workspace_bytes(n, d, Hh), dtype=torch.uint8, device="cuda")
    H.mlp_forward(Xd, Pd, y, ws, Hh)
    P32 = P.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    yref = oracle.mlp_forward(X32, P32, Hh)
    assert relerr(host(y), yref) <= 1e-5
    G = torch.empty_like(Pd)
    loss = torch.zeros(1, device="cuda")
    H.mlp_loss_grad(Xd, td, Pd, G, loss, ws, Hh)
    lref, gref = oracle.mlp_loss_grad(X32, t.astype(np.float32).astype(np.float64), P32, Hh)
    assert abs(float(loss) - lref) <= 1e-5 * abs(lref)
    g = host(G)
    # per tensor: W1 b1 W2 b2 W3 b3 W4 b4
    sizes = [Hh * d, Hh, Hh * Hh, Hh, Hh * Hh, Hh, Hh, 1]
    o = 0
    for sz in sizes:
        assert relerr(g[o:o + sz], gref[o:o + sz]) <= 1e-4, (o, sz)
        o += sz


def test_mlp_adam_step_vs_oracle():
    rng = np.random.default_rng(4)
    n = 1000
    P = rng.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    Pd = torch.tensor(P, dtype=torch.float32, device="cuda")
    md = torch.zeros_like(Pd)
    vd = torch.zeros_like(Pd)
    for step in range(1, 6):
        Gs = rng.normal(size=n)
        oracle.adam_step(P, Gs.copy(), m, v, step)
        H.mlp_adam(Pd, torch.tensor(Gs, dtype=torch.float32, device="cuda"), md, vd, step)
    assert np.abs(host(Pd) - P).max() <= 1e-6


def test_mlp_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(300, H.COST_FEATURES)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    _, _, _, hist = tune.train(X, y, iters=1500)
    assert hist[-1][1] < 0.2 * hist[0][1]


def test_cost_model_gains_over_default():
    # reduced study: train on timings of seeded chains, evaluate on held-out
    # chains; the model's choices must beat the planner's default
    train_chains = tune.random_chains(24, tune.TRAIN_SEED, max_cells=1 << 20)
    rec = tune.collect(train_chains, reps=2)
    X = np.array([r["features"] for r in rec], dtype=np.float32)
    params, mean, std, _ = tune.train(X, tune.targets(rec), iters=2000)
    ev = tune.evaluate(tune.random_chains(12, tune.TEST_SEED, max_cells=1 << 20), params, mean, std, reps=2)
    s = tune.summarize(ev)
    print("cost model (reduced study):", s, flush=True)
    assert s["gain_over_default_geomean"] > 1.0
    assert s["regret_mean"] < s["default_regret_mean"]


def test_family_autotuner_database_and_tuned_parity(tmp_path):
    """The family autotuner times its space, the database it writes steers
    hfav_plan(CONFIG_TUNED), and the tuned kernels match the oracle."""
    import json
    from gpu_util import hydro_errs
    from paper_1710_08774_amd.euler import EulerStepper
    space = [(64, 1, 8, 0, 0), (128, 1, 16, 8, -1), (256, 1, 32, 2, 0)]
    res, default_ms = tune.tune_family("hdiff", (200, 70, 2), H.F64, reps=2, space=space)
    assert len(res) == 3 and default_ms > 0
    assert all(ms > 0 for ms, _ in res) and res[0][0] <= res[-1][0]
    db = tune.build_db([("euler_y", H.F64, (96, 80, 1))], reps=1)
    db["entries"].append({"family": "hdiff", "family_id": 1, "dtype": "f64", "dims": [200, 70, 2],
                          "config": list(res[0][1])})
    path = tmp_path / "db.json"
    path.write_text(json.dumps(db))
    assert tune.load_db(str(path)) == 2
    try:
        a = inputs.hdiff_input(2, 70, 200, seed=21)
        c = H.Chain(H.hdiff_spec())
        info = c.plan((200, 70, 2), config_source=H.CONFIG_TUNED)
        assert info.config_source == H.CONFIG_TUNED
        assert (info.config.block, info.config.seg, info.config.variant, info.config.xcd) == \
            (res[0][1][0], res[0][1][2], res[0][1][3], res[0][1][4])
        u = torch.tensor(a, device="cuda")
        out = torch.empty_like(u)
        c.execute([u], [out])
        assert np.array_equal(host(out), oracle.hdiff(a))
        # the hydro stepper with the tuned y configuration
        U = inputs.euler_ic(96, 80, seed=22)
        st = EulerStepper(96, 80, config_source=H.CONFIG_TUNED)
        assert st.iy.config_source == H.CONFIG_TUNED
        assert [st.iy.config.block, st.iy.config.tile_y, st.iy.config.seg, st.iy.config.variant,
                st.iy.config.xcd] == db["entries"][0]["config"]
        st.load(U)
        st.step(5)
        ref, _ = oracle.euler_run(U, 5)
        assert max(hydro_errs(host(st.state()), ref)) <= 1e-12
    finally:
        H.tuning_clear()
