"""Autotuners, the tuning database, and the learned cost model.

* `tune_family` times every configuration of a fixed kernel family (hdiff,
  the 7-point chain, the two hydro sweeps) at one shape; `build_db` runs it
  over (family, dtype, shape) buckets and writes the tuning database (JSON),
  `load_db` installs a database into the planner's tuning table, which
  `hfav_plan(..., HFAV_CONFIG_TUNED)` reads (nearest shape bucket);
* `autotune`  times every feasible configuration of a star chain (exhaustive
  search, the reference the model's regret is measured against);
* `collect`   builds a training set of (features, log time per cell) from the
  autotuner's timings on seeded random chains;
* `train`     fits the cost-model MLP on the GPU with the library's own
  forward, backward and Adam kernels (full-batch Adam on z-scored features);
* `study`     trains on one seeded set of chains and reports, on held-out
  chains, the regret of the model's choice against exhaustive search and its
  gain over the planner's default configuration.

Timing uses HIP events on the stream the chain runs on.
Command line: python -m paper_1710_08774_amd.tune {db,study} --help
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import hfav as H
from . import inputs

TRAIN_SEED = inputs.BASE_SEED + inputs.W_CHAIN          # training chains
TEST_SEED = inputs.BASE_SEED + inputs.W_CHAIN + 1       # held-out chains
HIDDEN = 64


def chain_dims(ch):
    return tuple(ch["dims"]) if ch["ndim"] == 3 else tuple(ch["dims"][:2])


# ------------------------------------------------------------------ families
FAMILY_ID = {"hdiff": 1, "euler_x": 2, "euler_y": 3, "lap7_chain": 4, "euler_y_batch": 7, "norm": 8,
             "euler_xy": 9}
NORM_FIELDS = 4      # the normalisation family is tuned with 4 fields (the tuning key has no field count)
DTYPE_NAME = {H.F64: "f64", H.F32: "f32"}


def family_space(family):
    """Configurations (block, tile_y, seg, variant, xcd) searched per family."""
    out = []
    if family == "hdiff":
        for blk in (64, 128, 256, 512):
            for seg in (4, 8, 16, 32, 64, 128):
                for var in (0, 1, 2, 4, 8, 10, 18):
                    for xcd in (0, -1):
                        out.append((blk, 1, seg, var, xcd))
    elif family == "lap7_chain":
        for var in (1, 2, 5, 6, 7, 8, 9, 10, 13, 37, 38):
            for seg in (64, 128):
                for depth in (2, 4):
                    for xcd in (0, 8):
                        out.append((1024, depth, seg, var, xcd))
    elif family == "euler_x":
        for blk in (64, 128, 256):
            for var in (0, 1, 3):
                out.append((blk, 1, 0, var, 0))
        # row segments of the strip kernel (64 k - 1 cells)
        for blk, seg in ((64, 63), (64, 127), (64, 191), (64, 255), (128, 127), (128, 255), (256, 255), (256, 511)):
            out.append((blk, 1, seg, 3, 0))
    elif family == "euler_y":
        for blk in (64, 128, 256):
            for seg in (8, 16, 32):
                for var in (0, 1):
                    out.append((blk, 1, seg, var, 0))
        # LDS-ring strips of 64 columns x block/64 rows per chunk; a segment
        # of seg rows takes seg + 1 chunk rows, so segments of C k - 1 rows
        # leave no idle chunk row
        for seg in (3, 7, 11, 15, 19, 23, 31, 63, 127):
            out.append((256, 1, seg, 3, 0))
        for seg in (31, 63, 127):
            out.append((512, 1, seg, 3, 0))
        for seg in (7, 15):
            out.append((128, 1, seg, 3, 0))
    elif family == "norm":
        # only the configurations covering the row are feasible; the tuner
        # skips the others
        for blk in (64, 128, 256, 512, 1024):
            for seg in (1, 2, 4, 8, 16):
                for var in (0, 2, 3):
                    out.append((blk, 1, seg, var, 0))
        for blk in (64, 128, 256):
            out.append((blk, 1, 0, 1, 0))
    elif family == "euler_xy":
        for seg in (4, 8, 12, 16, 24, 32):
            for xcd in (0, -1):
                out.append((64, 1, seg, 0, xcd))
    else:
        raise ValueError(f"no search space for family {family!r}")
    return out


def _event_ms(fn, reps):
    import torch
    fn()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_family(family, dims, dtype=H.F64, reps=5, space=None):
    """Time every configuration of `family` at `dims` (x, y[, z]).

    Returns (results sorted by time as [(ms, config)], default_ms)."""
    import torch
    space = family_space(family) if space is None else space
    tdt = torch.float64 if dtype == H.F64 else torch.float32
    res = []
    if family in ("hdiff", "lap7_chain"):
        nx, ny, nz = dims
        spec = H.hdiff_spec(dtype=dtype) if family == "hdiff" else H.biharm_spec(dtype=dtype)
        g = torch.Generator(device="cuda").manual_seed(0)
        u = torch.rand((nz, ny, nx), dtype=tdt, device="cuda", generator=g)
        o = torch.empty_like(u)
        c = H.Chain(spec)
        for cfg in space:
            c.plan((nx, ny, nz), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
            res.append((_event_ms(lambda: c.execute([u], [o]), reps), tuple(cfg)))
        c.plan((nx, ny, nz), mode=H.MODE_FUSED)
        default_ms = _event_ms(lambda: c.execute([u], [o]), reps)
    elif family in ("euler_x", "euler_y"):
        from .euler import EulerStepper
        nx, ny = dims[0], dims[1]
        U = inputs.euler_ic(nx, ny)
        x = family == "euler_x"
        for cfg in space:
            st = EulerStepper(nx, ny, dtype=tdt, **({"forced_x": cfg} if x else {"forced_y": cfg}))
            st.load(U)
            res.append((_event_ms(st.sweep_x if x else st.sweep_y, reps), tuple(cfg)))
        st = EulerStepper(nx, ny, dtype=tdt)
        st.load(U)
        default_ms = _event_ms(st.sweep_x if x else st.sweep_y, reps)
    elif family == "norm":
        ni, nrows = dims[0], dims[1]
        g = torch.Generator(device="cuda").manual_seed(0)
        u = torch.rand((NORM_FIELDS, nrows, ni), dtype=tdt, device="cuda", generator=g)
        o = torch.empty_like(u)
        c = H.Chain(H.norm_spec(NORM_FIELDS, dtype=dtype))
        args = ([u[q] for q in range(NORM_FIELDS)], [o[q] for q in range(NORM_FIELDS)])
        for cfg in space:
            try:
                c.plan((ni, nrows), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
            except H.HfavError:
                continue                                  # does not cover the row
            res.append((_event_ms(lambda: c.execute(*args), reps), tuple(cfg)))
        c.plan((ni, nrows), mode=H.MODE_FUSED)
        default_ms = _event_ms(lambda: c.execute(*args), reps)
    elif family == "euler_xy":
        from .euler import EulerStepper
        nx, ny = dims[0], dims[1]
        U = inputs.euler_ic(nx, ny)
        for cfg in space:
            st = EulerStepper(nx, ny, dtype=tdt, fused_step=True, forced_xy=cfg)
            st.load(U)
            res.append((_event_ms(st.step, reps), tuple(cfg)))
        st = EulerStepper(nx, ny, dtype=tdt, fused_step=True)
        st.load(U)
        default_ms = _event_ms(st.step, reps)
    else:
        raise ValueError(f"no autotuner for family {family!r}")
    res.sort(key=lambda r: r[0])
    return res, default_ms


# default buckets: the workload sizes and one smaller shape per family
DB_BUCKETS = [
    ("hdiff", H.F64, (2048, 2048, 64)), ("hdiff", H.F64, (256, 256, 8)), ("hdiff", H.F32, (2048, 2048, 64)),
    ("lap7_chain", H.F64, (512, 512, 512)), ("lap7_chain", H.F32, (512, 512, 512)),
    ("lap7_chain", H.F64, (128, 128, 128)),
    ("euler_x", H.F64, (2048, 2048, 1)), ("euler_x", H.F64, (512, 512, 1)),
    ("euler_y", H.F64, (2048, 2048, 1)), ("euler_y", H.F64, (512, 512, 1)),
    ("euler_y", H.F64, (128, 128, 1)),
    ("norm", H.F64, (4096, 4096, 1)), ("norm", H.F64, (1024, 16384, 1)), ("norm", H.F32, (4096, 4096, 1)),
    ("euler_xy", H.F64, (2048, 2048, 1)), ("euler_xy", H.F64, (512, 512, 1)),
]
# size buckets of the batched y sweep (centres, log2-nearest assignment)
BATCH_BUCKETS = ((128, 128, 1), (362, 362, 1), (724, 724, 1))


def tune_batch(sizes=None, segs=(15, 31, 47, 63, 95, 127, 191, 255), reps=8, dtype=H.F64, log=None, start=63):
    """Segment length of the batched y items (64 columns x seg rows, 4-row
    strips) per size bucket, chosen by timing the whole batch in its faster
    form, the one-launch time step (its load balance depends on the mix):
    coordinate descent over the buckets from `start` rows everywhere, two
    rounds.  Returns database entries for HFAV_FAMILY_EULER_Y_BATCH (used by
    both batch forms)."""
    import torch
    from .euler import EulerBatchStepper
    sizes = inputs.batch_sizes(512) if sizes is None else sizes
    states = inputs.batch_ic(sizes=sizes)
    tdt = torch.float64 if dtype == H.F64 else torch.float32
    bt = EulerBatchStepper(sizes, dtype=tdt, fused_step=True)
    bt.load(states)
    # every trial starts from the same state (later steps of this flow cost
    # more): device copies of the initial state and its CFL slots
    u0, s0 = bt.U[0].clone(), bt.smax.clone()

    def timed(choice):
        H.tuning_clear()
        for centre, seg in zip(BATCH_BUCKETS, choice):
            H.tuning_add(FAMILY_ID["euler_y_batch"], dtype, centre, (256, 1, seg, 3, 0))
        bt.ixy = bt.cxy.plan_batch(bt.sizes, config_source=H.CONFIG_TUNED)
        bt.U[0].copy_(u0)
        bt.smax.copy_(s0)
        bt.cur = bt.slot = 0
        return _event_ms(bt.step, reps)

    choice = [start] * len(BATCH_BUCKETS)
    best = timed(choice)
    base = best
    for _ in range(2):
        for b in range(len(BATCH_BUCKETS)):
            for seg in segs:
                if seg == choice[b]:
                    continue
                trial = list(choice)
                trial[b] = seg
                ms = timed(trial)
                if ms < best:
                    best, choice = ms, trial
    H.tuning_clear()
    if log:
        log(f"db: euler_y_batch {len(sizes)} grids: segments {choice} per bucket, {best:.3f} ms per step "
            f"({start} everywhere: {base:.3f} ms)")
    return [{"family": "euler_y_batch", "family_id": FAMILY_ID["euler_y_batch"], "dtype": DTYPE_NAME[dtype],
             "dims": list(c), "config": [256, 1, seg, 3, 0], "ms": best, "default_ms": base,
             "n_configs": len(segs) * len(BATCH_BUCKETS), "search_s": 0.0}
            for c, seg in zip(BATCH_BUCKETS, choice)]


def build_db(buckets=None, reps=5, log=None, batch=None):
    """Autotune every (family, dtype, shape) bucket and the batch's segment
    lengths (by default only with the full bucket list); returns the
    database."""
    entries = []
    for family, dtype, dims in (DB_BUCKETS if buckets is None else buckets):
        t0 = time.time()
        res, default_ms = tune_family(family, dims, dtype, reps)
        best_ms, best = res[0]
        entries.append({"family": family, "family_id": FAMILY_ID[family], "dtype": DTYPE_NAME[dtype],
                        "dims": list(dims), "config": list(best), "ms": best_ms, "default_ms": default_ms,
                        "n_configs": len(res), "search_s": time.time() - t0})
        if log:
            log(f"db: {family} {DTYPE_NAME[dtype]} {dims}: best {best} {best_ms:.4f} ms "
                f"(default {default_ms:.4f} ms, {len(res)} configs)")
    if batch or (batch is None and buckets is None):
        entries += tune_batch(log=log)
    return {"version": 1, "entries": entries}


HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_DB = os.path.join(HERE, "tuning_db.json")            # MI355X autotuner results
REPORT_DIR = os.environ.get("HFAV_REPORT_DIR", "reports")    # where new tables and studies are written
DEFAULT_COSTMODEL = os.path.join(HERE, "costmodel_mi355x.json")  # MI355X-trained network


def load_default_db():
    """Install the shipped MI355X tuning database; returns its entry count."""
    return load_db(DEFAULT_DB)


def load_costmodel(path=DEFAULT_COSTMODEL):
    """Install a trained cost-model network (JSON with params, mean, std,
    hidden) so that hfav_plan(..., HFAV_CONFIG_MODEL) uses it."""
    with open(path) as f:
        m = json.load(f)
    H.costmodel_set(m["params"], int(m["hidden"]), m["mean"], m["std"])
    return m


def load_db(db):
    """Install a tuning database (dict or JSON path) into the planner's table."""
    if isinstance(db, str):
        with open(db) as f:
            db = json.load(f)
    H.tuning_clear()
    for e in db["entries"]:
        dtype = H.F64 if e["dtype"] == "f64" else H.F32
        dims = list(e["dims"]) + [1] * (3 - len(e["dims"]))
        H.tuning_add(int(e["family_id"]), dtype, dims, tuple(e["config"]))
    return H.tuning_size()


def cfg_key(cfg):
    """Configuration identity: (stages per group, segment, tile shape)."""
    return (int(cfg[1]), int(cfg[2]) if cfg[2] > 0 else 32, int(cfg[3]))


class ChainRun:
    """Device buffers and a planned handle for timing one random chain."""

    def __init__(self, ch, seed=0):
        import torch
        self.torch = torch
        self.ch = ch
        self.chain = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
        self.dims = chain_dims(ch)
        nx, ny, nz = ch["dims"]
        tdt = torch.float64 if ch["dtype"] == "f64" else torch.float32
        g = torch.Generator(device="cuda").manual_seed(int(seed))
        self.x = [torch.rand((nz, ny, nx), dtype=tdt, device="cuda", generator=g) for _ in range(ch["n_in"])]
        self.y = [torch.empty((nz, ny, nx), dtype=tdt, device="cuda") for _ in range(ch["stages"][-1]["f_out"])]
        self.ws = None
        self.cells = nx * ny * nz

    def plan(self, cfg=None, source=H.CONFIG_DEFAULT):
        if cfg is not None:
            info = self.chain.plan(self.dims, mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
        else:
            info = self.chain.plan(self.dims, mode=H.MODE_FUSED, config_source=source)
        need = int(info.workspace_bytes)
        if need and (self.ws is None or self.ws.numel() < need):
            self.ws = None
            self.torch.cuda.empty_cache()
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device="cuda")
        return info

    def run(self):
        self.chain.execute(self.x, self.y, self.ws)

    def time(self, reps=3):
        torch = self.torch
        self.run()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            self.run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def free(self):
        self.x = self.y = self.ws = None
        self.torch.cuda.empty_cache()


def autotune(run: ChainRun, reps=3):
    """Exhaustive search: ms of every feasible configuration."""
    out = []
    for cfg in run.chain.candidates(run.dims):
        run.plan(cfg)
        out.append((cfg, run.time(reps)))
    return out


def random_chains(n, seed, max_cells=None):
    rng = inputs.rng_for(seed)
    chains = []
    while len(chains) < n:
        ch = inputs.random_chain(rng)
        nx, ny, nz = ch["dims"]
        if max_cells and nx * ny * nz > max_cells:
            # keep the chain's structure, shrink the grid to the cap
            s = (max_cells / float(nx * ny * nz)) ** (1.0 / ch["ndim"])
            d = [max(32, int(x * s) // 32 * 32) for x in (nx, ny, nz)[:ch["ndim"]]]
            ch["dims"] = tuple(d) + ((1,) if ch["ndim"] == 2 else ())
        chains.append(ch)
    return chains


def collect(chains, reps=3, log=None):
    """Training records: one per (chain, configuration)."""
    rec = []
    t0 = time.time()
    for ci, ch in enumerate(chains):
        run = ChainRun(ch, seed=ci)
        for cfg, ms in autotune(run, reps):
            rec.append({"chain": ci, "cfg": list(cfg), "ms": ms, "cells": run.cells,
                        "features": run.chain.features(run.dims, cfg)})
        run.free()
        if log and (ci + 1) % 10 == 0:
            log(f"collect: {ci + 1}/{len(chains)} chains, {len(rec)} timings, {time.time() - t0:.0f} s")
    return rec


def targets(rec):
    """log of nanoseconds per cell"""
    return np.array([math.log(r["ms"] * 1e6 / r["cells"]) for r in rec], dtype=np.float32)


def init_params(d, Hh=HIDDEN, seed=0):
    """He-normal weights, zero biases, in the library's flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for nin, nout in ((d, Hh), (Hh, Hh), (Hh, Hh), (Hh, 1)):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / nin), nout * nin))
        parts.append(np.zeros(nout))
    return np.concatenate(parts).astype(np.float32)


def train(X, y, Hh=HIDDEN, iters=3000, lr=1e-3, seed=0, log=None):
    """Full-batch Adam on the GPU through the library's MLP kernels.

    Returns (params, mean, std, loss history)."""
    import torch
    X = np.asarray(X, dtype=np.float32)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-6] = 1.0
    Xn = (X - mean) / std
    n, d = Xn.shape
    dev = "cuda"
    Xd = torch.tensor(Xn, device=dev)
    td = torch.tensor(np.asarray(y, dtype=np.float32), device=dev)
    P = torch.tensor(init_params(d, Hh, seed), device=dev)
    G = torch.zeros_like(P)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    loss = torch.zeros(1, device=dev)
    ws = torch.empty(H.mlp_workspace_bytes(n, d, Hh), dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    hist = []
    for it in range(1, iters + 1):
        H.mlp_loss_grad(Xd, td, P, G, loss, ws, Hh, s)
        H.mlp_adam(P, G, m, v, it, lr=lr, stream=s)
        if it % 100 == 0 or it == 1:
            hist.append((it, float(loss)))
            if log and it % 1000 == 0:
                log(f"train: iter {it} loss {hist[-1][1]:.4f}")
    return P.cpu().numpy(), mean, std, hist


def evaluate(chains, params, mean, std, reps=3, log=None):
    """Regret of the model's choice vs exhaustive search, and its gain over
    the planner's default, on each chain."""
    H.costmodel_set(params.tolist(), HIDDEN, mean.tolist(), std.tolist())
    out = []
    t0 = time.time()
    for ci, ch in enumerate(chains):
        run = ChainRun(ch, seed=1000 + ci)
        t_search = time.time()
        table = {cfg_key(c): ms for c, ms in autotune(run, reps)}
        t_search = time.time() - t_search
        best = min(table.values())
        t_model = time.time()
        im = run.plan(source=H.CONFIG_MODEL)
        t_model = time.time() - t_model
        km = cfg_key((im.config.block, im.config.tile_y, im.config.seg, im.config.variant))
        idf = run.plan(source=H.CONFIG_DEFAULT)
        kd = cfg_key((idf.config.block, idf.config.tile_y, idf.config.seg, idf.config.variant))
        ms_model = table.get(km)
        ms_def = table.get(kd)
        if ms_model is None:
            run.plan((256, km[0], km[1], km[2]))
            ms_model = run.time(reps)
        if ms_def is None:
            run.plan((256, kd[0], kd[1], kd[2]))
            ms_def = run.time(reps)
        out.append({"chain": ci, "best_ms": best, "model_ms": ms_model, "default_ms": ms_def,
                    "regret": ms_model / best - 1.0, "gain_over_default": ms_def / ms_model,
                    "default_regret": ms_def / best - 1.0, "n_configs": len(table),
                    "search_s": t_search, "model_plan_s": t_model,
                    "model_cfg": km, "default_cfg": kd})
        run.free()
        if log and (ci + 1) % 20 == 0:
            log(f"evaluate: {ci + 1}/{len(chains)} chains, {time.time() - t0:.0f} s")
    H.costmodel_set(None, 0, None, None)
    return out


def summarize(ev):
    reg = np.array([e["regret"] for e in ev])
    dreg = np.array([e["default_regret"] for e in ev])
    gain = np.array([e["gain_over_default"] for e in ev])
    return {"chains": len(ev), "regret_mean": float(reg.mean()), "regret_p90": float(np.percentile(reg, 90)),
            "regret_median": float(np.median(reg)), "default_regret_mean": float(dreg.mean()),
            "gain_over_default_geomean": float(np.exp(np.log(gain).mean())),
            "model_picks_best_frac": float(np.mean(reg < 1e-9)),
            "search_seconds_total": float(sum(e["search_s"] for e in ev)),
            "model_plan_seconds_total": float(sum(e["model_plan_s"] for e in ev))}


def study(n_train, n_test, reps=3, iters=3000, max_cells=None, log=print):
    train_chains = random_chains(n_train, TRAIN_SEED, max_cells)
    rec = collect(train_chains, reps, log)
    X = np.array([r["features"] for r in rec], dtype=np.float32)
    y = targets(rec)
    params, mean, std, hist = train(X, y, iters=iters, log=log)
    test_chains = random_chains(n_test, TEST_SEED, max_cells)
    ev = evaluate(test_chains, params, mean, std, reps, log)
    return {"train_timings": len(rec), "train_chains": n_train, "loss_history": hist,
            "summary": summarize(ev), "per_chain": ev,
            "model": {"params": params.tolist(), "mean": mean.tolist(), "std": std.tolist(), "hidden": HIDDEN}}


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1710_08774_amd.tune")
    sub = ap.add_subparsers(dest="cmd", required=True)
    dbp = sub.add_parser("db", help="autotune the kernel families and write the tuning database")
    dbp.add_argument("--reps", type=int, default=5)
    dbp.add_argument("--out", default=os.path.join(REPORT_DIR, "tuning_db.json"))
    dbp.add_argument("--families", nargs="*", default=None,
                     help="tune only these families (default: all, plus the batch segments)")
    dbp.add_argument("--merge", default=None,
                     help="database whose entries of the other families are kept")
    st = sub.add_parser("study", help="train on seeded chains, report regret on held-out chains")
    st.add_argument("--train-chains", type=int, default=60)
    st.add_argument("--test-chains", type=int, default=200)
    st.add_argument("--reps", type=int, default=3)
    st.add_argument("--iters", type=int, default=3000)
    st.add_argument("--max-cells", type=int, default=0, help="cap grid cells per chain (0: none)")
    st.add_argument("--out", default=os.path.join(REPORT_DIR, "costmodel_study.json"))
    a = ap.parse_args(argv)
    if a.cmd == "db":
        buckets, batch = None, None
        if a.families:
            buckets = [b for b in DB_BUCKETS if b[0] in a.families]
            batch = "euler_y_batch" in a.families
        db = build_db(buckets=buckets, reps=a.reps, log=lambda m: print(m, flush=True), batch=batch)
        if a.merge:
            with open(a.merge) as f:
                old = json.load(f)
            tuned = set(a.families or FAMILY_ID)
            db["entries"] = [e for e in old["entries"] if e["family"] not in tuned] + db["entries"]
        os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
        with open(a.out, "w") as f:
            json.dump(db, f, indent=1)
        print(json.dumps({"entries": len(db["entries"]), "out": a.out}), flush=True)
        return 0
    if a.cmd == "study":
        res = study(a.train_chains, a.test_chains, a.reps, a.iters, a.max_cells or None,
                    log=lambda m: print(m, flush=True))
        os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
        with open(a.out, "w") as f:
            json.dump(res, f)
        print(json.dumps({"train_timings": res["train_timings"], **res["summary"]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
