"""Cost-model host side (no GPU): candidate sets, feature vectors, and the
installed network's host forward pass against the FP64 oracle."""
import numpy as np

import oracle
from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs, tune


def _chains(n=12, seed=5):
    return tune.random_chains(n, seed)


def test_candidates_feasible_and_deterministic():
    for ch in _chains():
        c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
        dims = tune.chain_dims(ch)
        a = c.candidates(dims)
        assert a == c.candidates(dims) and len(a) >= 3
        K = len(ch["stages"])
        assert all(1 <= cfg[1] <= K and cfg[2] in (32, 64, 128) and 0 <= cfg[3] <= 3 for cfg in a)
        # every candidate plans as a fused configuration
        for cfg in a[:6]:
            info = c.plan(dims, mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
            assert info.fused and info.config.tile_y == cfg[1]


def test_features_shape_and_values():
    ch = _chains(1, 9)[0]
    c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
    dims = tune.chain_dims(ch)
    cfg = c.candidates(dims)[0]
    f = np.array(c.features(dims, cfg))
    assert f.shape == (H.COST_FEATURES,) and np.all(np.isfinite(f))
    assert f[0] == len(ch["stages"]) and f[1] == (ch["ndim"] == 3)
    assert f[6] == sum(s["r"] for s in ch["stages"])


def test_installed_model_matches_oracle_forward():
    ch = _chains(1, 3)[0]
    c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
    dims = tune.chain_dims(ch)
    d, Hh = H.COST_FEATURES, 16
    P = np.random.default_rng(1).normal(0, 0.3, oracle.mlp_nparams(d, Hh))
    mean = np.random.default_rng(2).normal(0, 1, d)
    std = np.random.default_rng(3).uniform(0.5, 2, d)
    H.costmodel_set(P.astype(np.float32).tolist(), Hh, mean.tolist(), std.tolist())
    try:
        for cfg in c.candidates(dims)[:5]:
            f = np.array(c.features(dims, cfg), dtype=np.float64)
            ref = oracle.mlp_forward(((f - mean.astype(np.float32)) / std.astype(np.float32))[None],
                                     P.astype(np.float32).astype(np.float64), Hh)[0]
            assert abs(c.predict(dims, cfg) - ref) <= 1e-4 * max(1.0, abs(ref))
        # the planner then picks the candidate with the smallest prediction
        info = c.plan(dims, mode=H.MODE_FUSED, config_source=H.CONFIG_MODEL)
        assert info.config_source == H.CONFIG_MODEL
        preds = {(k[1], k[2], k[3]): c.predict(dims, k) for k in c.candidates(dims)}
        chosen = (info.config.tile_y, info.config.seg, info.config.variant)
        assert preds[chosen] == min(preds.values())
    finally:
        H.costmodel_set(None, 0, None, None)
    assert c.plan(dims, mode=H.MODE_FUSED, config_source=H.CONFIG_MODEL).config_source == H.CONFIG_DEFAULT


def test_shipped_tuning_db_and_costmodel_load():
    """The MI355X tuning database and trained network shipped with the
    package install and drive CONFIG_TUNED / CONFIG_MODEL plans."""
    from paper_1710_08774_amd import tune
    try:
        n = tune.load_default_db()
        assert n >= 8
        c = H.Chain(H.hdiff_spec())
        assert c.plan((2048, 2048, 64), config_source=H.CONFIG_TUNED).config_source == H.CONFIG_TUNED
        m = tune.load_costmodel()
        assert m["hidden"] == 64 and len(m["params"]) == H.mlp_nparams(len(m["mean"]), 64)
        rng = inputs.rng_for(inputs.BASE_SEED + 123)
        ch = inputs.random_chain(rng)
        sc = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
        dims = tuple(ch["dims"]) if ch["ndim"] == 3 else tuple(ch["dims"][:2])
        info = sc.plan(dims, mode=H.MODE_FUSED, config_source=H.CONFIG_MODEL)
        assert info.config_source == H.CONFIG_MODEL
        cands = [tuple(x) for x in sc.candidates(dims)]
        pred = [sc.predict(dims, k) for k in cands]
        assert all(np.isfinite(pred))
        best = cands[int(np.argmin(pred))]
        assert (info.config.tile_y, info.config.seg, info.config.variant) == (best[1], best[2], best[3])
    finally:
        H.tuning_clear()
        H.costmodel_set(None, 0, None, None)
