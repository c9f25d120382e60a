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
    return got, ref, info


def _small_chains(n, seed):
    return tune.random_chains(n, seed, max_cells=40000)


@pytest.mark.parametrize("k", range(8))
def test_star_chain_default_parity(k):
    ch = _small_chains(8, 77)[k]
    got, ref, info = _run(ch)
    assert info.fused and info.family == 5
    tol = 1e-12 if ch["dtype"] == "f64" else 2e-6
    assert relerr(got, ref) <= tol


@pytest.mark.parametrize("ndim", [2, 3])
def test_star_chain_every_configuration(ndim):
    rng = inputs.rng_for(ndim + 40)
    dims = (150, 70, 1) if ndim == 2 else (40, 24, 20)
    ch = inputs.random_chain(rng, ndim=ndim, dtype="f64", dims=dims)
    c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
    cands = c.candidates(tune.chain_dims(ch))
    assert len(cands) >= 3
    for cfg in cands:
        got, ref, info = _run(ch, cfg)
        assert relerr(got, ref) <= 1e-12, cfg


def test_star_chain_unfused_parity():
    ch = _small_chains(3, 5)[1]
    got, ref, info = _run(ch, mode=H.MODE_UNFUSED)
    assert not info.fused
    assert relerr(got, ref) <= (1e-12 if ch["dtype"] == "f64" else 2e-6)


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
