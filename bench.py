"""Benchmark: fused vs unfused split Godunov hydro chain on one MI355X.

Workload: 2-D compressible Euler, directionally split Godunov step (prim ->
van Leer slopes -> characteristic trace -> exact Riemann solver with 10
Newton iterations -> flux -> conservative update, x sweep then y sweep,
fused CFL reduction), FP64, 2048 x 2048 cells, periodic, gamma 1.4, CFL 0.5,
Sod-like seeded initial state (synthetic stand-in for the Hydro2D input).
A step is one x sweep plus one y sweep.  The state is resident in HBM
before the timed region; dt stays on the device.  Each timed run is preceded
by a clock warm-up (the K steps from the initial state, repeated for
CLOCK_WARMUP_S, reported in the line), then the W warm-up steps from the
initial state, then exactly K timed steps from the initial state.

Prints ONE JSON line.  `value` is fused cell-updates/s (cells x steps / s).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the oracle's OpenMP threads stay next to each other (set before any
# library starts an OpenMP runtime)
os.environ.setdefault("OMP_PROC_BIND", "close")

METRIC = "cell-updates/s + % of 8 TB/s HBM, fused vs unfused on one MI355X"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
NX = NY = 2048
# Algorithmic FP64 operations per cell per sweep of the chain (each add, sub,
# mul, div, sqrt and pow counted once): prim 13, slopes 28, trace 70, exact
# Riemann solver with 10 Newton steps 311, flux 16, update 12.
FLOPS_PER_CELL_SWEEP = 450
COMPULSORY_BYTES_PER_CELL_SWEEP = 64      # 4 FP64 fields read once, written once


def kernel_source_hash():
    """Hash of the sweep kernels' sources and of the default launch
    configurations (tune.cpp): either changes the traffic per launch."""
    h = hashlib.sha256()
    for f in ("k_euler.hip", "euler_common.h", "ops.h", "tune.cpp"):
        with open(os.path.join(ROOT, "paper_1710_08774_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(kernel):
    """The committed rocprofv3 counter figures of one sweep kernel (HBM bytes
    per launch, VALU busy, VALU instructions per 64 cells), or {} when the
    kernel source or its default configuration changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", "euler_sweeps_2048_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except OSError:
        return {}
    if d.get("source_hash") != kernel_source_hash():
        return {}
    return d.get("kernels", {}).get(kernel) or {}


def load_traffic(kernel):
    """HBM bytes per launch from the committed counters, or None."""
    return load_counters(kernel).get("hbm_bytes_per_launch")


CLOCK_WARMUP_S = 0.25


def clock_warmup(st, U0d, steps, seconds=CLOCK_WARMUP_S):
    """Repeat the timed run's `steps` steps from the initial state U0d (a
    device tensor), untimed, for `seconds`.  The GPU raises its clock over
    the first tens of milliseconds of sustained work: measured, 20-step
    blocks from the initial state took 0.347 ms per step right after 5
    warm-up steps and 0.28 once the GPU had been busy for ~50 ms.  Repeating
    the timed steps themselves keeps the kernels' statistics over the whole
    run (a profiler's average) those of the timed steps."""
    import torch
    n = 0
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        st.load(U0d)
        st.step(steps)
        torch.cuda.synchronize()
        n += steps
    return {"seconds": seconds, "steps": n, "block": steps}


def run_gpu(mode, steps, warmup, U0, timing=True, dtype=None, in_place=False):
    import torch
    from paper_1710_08774_amd import hfav as H
    from paper_1710_08774_amd.euler import EulerStepper

    st = EulerStepper(NX, NY, mode=mode, dtype=dtype or torch.float64, in_place=in_place)
    # the initial state stays on the device: the reloads are device copies,
    # so the GPU does not idle between the phases below
    U0d = torch.as_tensor(U0, dtype=dtype or torch.float64).cuda()
    clock = clock_warmup(st, U0d, steps)
    st.load(U0d)
    st.step(warmup)
    st.load(U0d)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # two events per step on the launch stream: before the x sweep and
    # between the sweeps; the end of a step is the start of the next (one
    # more event after the last step)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)] if timing else None
    end = torch.cuda.Event(enable_timing=True) if timing else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        if timing:
            evs[s][0].record(stream)
        st.sweep_x()
        if timing:
            evs[s][1].record(stream)
        st.sweep_y()
        st.slot = 1 - st.slot
    if timing:
        end.record(stream)
    t_enq = time.perf_counter()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # host time to enqueue the steps: near ms_per_step, the GPU waited on the host
    out = {"ms_per_step": (t1 - t0) * 1e3 / steps, "seconds": t1 - t0,
           "host_enqueue_ms_per_step": (t_enq - t0) * 1e3 / steps}
    if timing:
        nxt = [evs[s + 1][0] for s in range(steps - 1)] + [end]
        out["x_ms"] = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
        out["y_ms"] = sum(e[1].elapsed_time(n) for e, n in zip(evs, nxt)) / steps
    out["state_finite"] = bool(torch.isfinite(st.state()).all())
    out["clock_warmup"] = clock
    out["info_fused"] = int(st.ix.fused and st.iy.fused)
    # kernel names of the fused sweeps (variant 3 selects the strip kernels)
    out["x_kernel"] = "euler_x_strip_kernel" if st.ix.config.variant == 3 else "euler_x_kernel"
    out["y_kernel"] = "euler_y_strip_kernel" if st.iy.config.variant == 3 else "euler_y_kernel"
    # (block, tile_y, seg, variant): tile_y is the y strip's columns per workgroup
    out["x_config"] = [st.ix.config.block, st.ix.config.tile_y, st.ix.config.seg, st.ix.config.variant]
    out["y_config"] = [st.iy.config.block, st.iy.config.tile_y, st.iy.config.seg, st.iy.config.variant]
    out["footprint_bytes"] = st.footprint_bytes()
    return out


def run_xy(steps, warmup, U0, seg=None):
    """The hydro workload with both sweeps of a step in one kernel (the
    x-swept state on chip; 64 compulsory bytes per cell-step instead of 128),
    timed like the split path: host clock around `steps` steps."""
    import torch
    from paper_1710_08774_amd import hfav as H
    from paper_1710_08774_amd.euler import EulerStepper

    forced = (64, 1, seg, 0, 0) if seg else None
    st = EulerStepper(NX, NY, fused_step=True, forced_xy=forced)
    st.load(U0)
    st.step(warmup)
    st.load(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    cells = NX * NY
    return {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3),
            # one read and one write of the state per step: a sweep's 64 B per cell
            "compulsory_GBs": COMPULSORY_BYTES_PER_CELL_SWEEP * cells / (ms * 1e-3) / 1e9,
            "config": [st.ixy.config.block, st.ixy.config.seg], "state_finite": bool(torch.isfinite(st.state()).all())}


def event_times(fn, reps, warmup=3):
    """Median and mean ms of `reps` executions of fn after `warmup` ones,
    each bracketed by its own pair of HIP events on the current stream."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    t = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return t[len(t) // 2], sum(t) / len(t)


def event_times_rot(fns, reps, warmup=3):
    """As event_times, cycling through the callables `fns` (the same work on
    different buffer sets) so that consecutive executions do not find their
    inputs in the 256 MB Infinity Cache."""
    import torch
    stream = torch.cuda.current_stream()
    for q in range(warmup):
        fns[q % len(fns)]()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for q, (e0, e1) in enumerate(ev):
        e0.record(stream)
        fns[q % len(fns)]()
        e1.record(stream)
    torch.cuda.synchronize()
    t = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return t[len(t) // 2], sum(t) / len(t)


def time_chain(spec, dims, mode, reps, inputs_fn, sets=2):
    """Median and mean ms per hfav_execute of a single-axiom, single-goal
    chain (3 warm-up executions, then `reps` each timed with HIP events on
    the stream the chain is launched on), rotating over `sets` input/output
    buffer sets."""
    import torch
    from paper_1710_08774_amd import hfav as H

    c = H.Chain(spec)
    info = c.plan(dims, mode=mode)
    bufs = []
    for _ in range(sets):
        u = inputs_fn()
        bufs.append((u, torch.empty_like(u)))
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device="cuda") if info.workspace_bytes else None
    fns = [(lambda u=u, o=o: c.execute([u], [o], ws)) for u, o in bufs]
    med, mean = event_times_rot(fns, reps)
    del bufs, fns, ws
    return med, mean, info


def copy_ceiling(nbytes, reps=20, pattern=None, sets=2):
    """Read+write GB/s of plain device copies of `nbytes` (the bytes a chain
    reads and writes once): a flat copy, and, when `pattern` gives the
    geometry of a stencil kernel's tiles and segments, a copy in that
    order.  Median of `reps` event-timed copies, rotating buffer sets."""
    import torch
    from paper_1710_08774_amd import hfav as H

    bufs = [(torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1),
             torch.empty(nbytes, dtype=torch.uint8, device="cuda")) for _ in range(sets)]
    out = {"bytes_each_way": nbytes}
    flat = [(lambda a=a, b=b: H.copy_probe(a, b, H.COPY_FLAT, nbytes=nbytes)) for a, b in bufs]
    ms, _ = event_times_rot(flat, reps)
    out["flat_GBs"] = 2 * nbytes / (ms * 1e-3) / 1e9
    if pattern is not None:
        seg = [(lambda a=a, b=b: H.copy_probe(a, b, H.COPY_SEGMENTS, **pattern)) for a, b in bufs]
        ms, _ = event_times_rot(seg, reps)
        out["pattern"] = dict(pattern)
        out["pattern_GBs"] = 2 * nbytes / (ms * 1e-3) / 1e9
    del bufs
    torch.cuda.empty_cache()
    return out


# tile extents (x, y) of the 7-point chain's tile-shape variants
LAP7_TILES = {1: (32, 8), 2: (64, 8), 3: (128, 2), 4: (32, 4), 5: (64, 16), 6: (64, 32), 7: (128, 16),
              10: (64, 16), 11: (64, 8), 12: (32, 8), 13: (128, 8), 14: (32, 16)}


def chain_copy_pattern(name, info, dims, es):
    """Segment-copy geometry with the same tiles and segments as the fused
    kernel of a bandwidth-bound chain."""
    nx, ny, nz = dims
    cfg = info.config
    if name == "hdiff":            # a row piece of `block` cells streamed down `seg` rows
        return {"slab_bytes": nx * es, "slabs": ny * nz, "row_bytes": nx * es, "band_bytes": cfg.block * es,
                "tile_rows": 1, "seg": cfg.seg, "access_bytes": es}
    var = cfg.variant & 31
    if var == 8:
        tx, ty = (128, 32) if es == 4 else (64, 32)
    elif var == 9:
        tx, ty = (256, 16) if es == 4 else (64, 32)
    else:
        tx, ty = LAP7_TILES.get(var, (64, 16))
    return {"slab_bytes": nx * ny * es, "slabs": nz, "row_bytes": nx * es, "band_bytes": tx * es,
            "tile_rows": ty, "seg": cfg.seg, "access_bytes": es}


def bandwidth_chains(reps=20, which=("hdiff", "biharm64", "biharm32"), unfused=True):
    """Fused vs unfused throughput of the bandwidth-bound chains at sizes whose
    working sets are far larger than the caches."""
    import torch
    from paper_1710_08774_amd import hfav as H

    out = {}
    g = torch.Generator(device="cuda")
    for name in which:
        if name == "hdiff":
            dims, spec, es = (2048, 2048, 64), H.hdiff_spec(), 8
            mk = lambda: torch.rand((64, 2048, 2048), dtype=torch.float64, device="cuda", generator=g.manual_seed(1))
        elif name == "biharm64":
            dims, spec, es = (512, 512, 512), H.biharm_spec(), 8
            mk = lambda: torch.rand((512, 512, 512), dtype=torch.float64, device="cuda", generator=g.manual_seed(2))
        else:
            dims, spec, es = (512, 512, 512), H.biharm_spec(dtype=H.F32), 4
            mk = lambda: torch.rand((512, 512, 512), dtype=torch.float32, device="cuda", generator=g.manual_seed(3))
        cells = dims[0] * dims[1] * dims[2]
        ms, ms_mean, info = time_chain(spec, dims, H.MODE_FUSED, reps, mk)
        gbs = 2 * es * cells / (ms * 1e-3) / 1e9
        ceil = copy_ceiling(es * cells, reps, chain_copy_pattern(name, info, dims, es))
        r = {"dims": list(dims), "dtype": "f64" if es == 8 else "f32", "fused_ms": ms, "fused_ms_mean": ms_mean,
             "fused_cell_updates_per_s": cells / (ms * 1e-3), "fused_GBs": gbs,
             "fused_frac_of_8TBs": gbs / HBM_PEAK_GBS,
             "copy_ceiling": ceil,
             "fused_frac_of_flat_copy": gbs / ceil["flat_GBs"],
             "fused_frac_of_pattern_copy": gbs / ceil["pattern_GBs"],
             "buffer_sets": 2,
             "bytes_per_cell_fused": info.bytes_per_cell_fused,
             "config": [info.config.block, info.config.tile_y, info.config.seg, info.config.variant]}
        if unfused:
            ums, _, uinfo = time_chain(spec, dims, H.MODE_UNFUSED, max(2, reps // 3), mk)
            r.update({"unfused_ms": ums, "unfused_cell_updates_per_s": cells / (ums * 1e-3),
                      "fused_over_unfused": ums / ms, "bytes_per_cell_unfused": uinfo.bytes_per_cell_unfused})
        out[name] = r
        torch.cuda.empty_cache()
    return out


def norm_chain(reps=20, nq=4, nj=4096, ni=4096, unfused=True):
    """Normalisation chain (flux differences, row norm, broadcast division,
    update) on nq FP64 fields of nj rows x ni cells, fused (one workgroup per
    row, both inner sweeps) and unfused (one kernel per rule), timed with HIP
    events on the launch stream.  Compulsory bytes: each u read once and
    each out written once, 2 nq 8 B per cell."""
    import torch
    from paper_1710_08774_amd import hfav as H
    from paper_1710_08774_amd import inputs

    u0 = torch.as_tensor(inputs.norm_input(nq, nj, ni)).to("cuda")
    sets = [(u0, torch.empty_like(u0)), (u0.clone(), torch.empty_like(u0))]
    cells = nj * ni
    out = {"fields": nq, "rows": nj, "cells_per_row": ni, "dtype": "f64", "buffer_sets": len(sets)}
    for mode, name in ((H.MODE_FUSED, "fused"), (H.MODE_UNFUSED, "unfused")):
        if mode == H.MODE_UNFUSED and not unfused:
            continue
        c = H.Chain(H.norm_spec(nq))
        info = c.plan((ni, nj), mode=mode)
        ws = torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device="cuda")
        fns = [(lambda u=u, o=o: c.execute([u[q] for q in range(nq)], [o[q] for q in range(nq)], ws))
               for u, o in sets]
        n = reps if mode == H.MODE_FUSED else max(2, reps // 4)
        ms, ms_mean = event_times_rot(fns, n)
        out[name + "_ms"] = ms
        out[name + "_ms_mean"] = ms_mean
        out[name + "_cell_updates_per_s"] = cells / (ms * 1e-3)
        out["bytes_per_cell_" + name] = info.bytes_per_cell_fused if mode == H.MODE_FUSED \
            else info.bytes_per_cell_unfused
        if mode == H.MODE_FUSED:
            gbs = 2 * nq * 8 * cells / (ms * 1e-3) / 1e9
            ceil = copy_ceiling(nq * 8 * cells, reps)
            out.update({"fused_GBs": gbs, "fused_frac_of_8TBs": gbs / HBM_PEAK_GBS, "copy_ceiling": ceil,
                        "fused_frac_of_flat_copy": gbs / ceil["flat_GBs"],
                        "config": [info.config.block, info.config.seg, info.config.variant],
                        "nests": info.n_nests, "outer_of_nest": list(info.outer_of_nest[:info.n_nests])})
        del ws
    if "unfused_ms" in out:
        out["fused_over_unfused"] = out["unfused_ms"] / out["fused_ms"]
    del u0, sets
    torch.cuda.empty_cache()
    return out


def hdiff_in_place(reps=20, dims=(2048, 2048, 64)):
    """Horizontal diffusion written over its input (declared alias): the
    halo columns and rows at tile boundaries are saved by a copy kernel, the
    fused kernel then runs in place.  Footprint: one field plus the saved
    halos, against two fields out of place."""
    import torch
    from paper_1710_08774_amd import hfav as H

    ni, nj, nk = dims
    g = torch.Generator(device="cuda").manual_seed(4)
    u = torch.rand((nk, nj, ni), dtype=torch.float64, device="cuda", generator=g)
    c = H.Chain(H.hdiff_spec())
    c.alias("out", "u")
    info = c.plan(dims, mode=H.MODE_FUSED)
    ws = torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device="cuda")
    ms, ms_mean = event_times(lambda: c.execute([u], [u], ws), reps)
    cells = ni * nj * nk
    field = cells * 8
    out = {"dims": list(dims), "dtype": "f64", "ms": ms, "ms_mean": ms_mean, "cell_updates_per_s": cells / (ms * 1e-3),
           "compulsory_GBs": 2 * field / (ms * 1e-3) / 1e9,
           "footprint_bytes_in_place": field + info.workspace_bytes, "footprint_bytes_out_of_place": 2 * field,
           "halo_copy_bytes": info.workspace_bytes,
           "config": [info.config.block, info.config.seg, info.config.variant]}
    del u, ws
    torch.cuda.empty_cache()
    return out


def hdiff_config_shape(execs=1000):
    """The horizontal-diffusion chain at 256x256x8 FP64: its 8 MiB working set
    stays in the caches and one execution is shorter than a launch, so the
    rate is labelled effective, launch-inclusive (host clock over back-to-back
    executions) and amortised over `execs` executions replayed from one HIP
    graph."""
    import torch
    from paper_1710_08774_amd import hfav as H

    nk, nj, ni = 8, 256, 256
    cells = nk * nj * ni
    c = H.Chain(H.hdiff_spec())
    info = c.plan((ni, nj, nk))
    g = torch.Generator(device="cuda").manual_seed(0)
    u = torch.rand((nk, nj, ni), dtype=torch.float64, device="cuda", generator=g)
    o = torch.empty_like(u)
    c.execute([u], [o])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(execs):
        c.execute([u], [o])
    torch.cuda.synchronize()
    launch_s = (time.perf_counter() - t0) / execs
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=side):
        for _ in range(execs):
            c.execute([u], [o])
    graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    graph_s = e0.elapsed_time(e1) * 1e-3 / execs
    return {"shape": [nk, nj, ni], "label": "effective (8 MiB working set, cache-resident)",
            "executions": execs, "config": [info.config.block, info.config.seg, info.config.variant],
            "launch_inclusive_us": launch_s * 1e6, "graph_amortised_us": graph_s * 1e6,
            "effective_cell_updates_per_s_launch_inclusive": cells / launch_s,
            "effective_cell_updates_per_s_graph": cells / graph_s,
            "effective_GBs_graph": 16 * cells / graph_s / 1e9}


def batched_grids(steps=50, loop_steps=4):
    """512 independent grids of uneven sizes (sides 64..1024), each with its
    own dt: the batched persistent sweeps with `steps` steps captured in one
    HIP graph, against a loop of per-grid fused launches, and against the
    one-launch step (both sweeps of every grid in one persistent launch per
    step, the same segments; its final state compared bit for bit)."""
    import torch
    from paper_1710_08774_amd import hfav as H
    from paper_1710_08774_amd import inputs, tune
    from paper_1710_08774_amd.euler import EulerBatchStepper, EulerStepper

    # per-size-bucket segment lengths of the batched y sweep from the
    # autotuner's database
    tune.load_default_db()
    sizes = inputs.batch_sizes(512)
    states = inputs.batch_ic(sizes=sizes)
    cells = sum(nx * ny for nx, ny in sizes)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    bt = EulerBatchStepper(sizes, config_source=H.CONFIG_TUNED)
    one = EulerBatchStepper(sizes, config_source=H.CONFIG_TUNED, fused_step=True)
    assert one.y_segments() == bt.y_segments()
    segs = {}
    for (nx, ny), sg in zip(sizes, bt.y_segments()):
        b = "64-255" if max(nx, ny) < 256 else ("256-511" if max(nx, ny) < 512 else "512-1024")
        segs.setdefault(b, set()).add(int(sg))
    segs = {b: sorted(v) for b, v in sorted(segs.items())}
    H.tuning_clear()
    bt.load(states)
    bt.step(2)
    bt.capture(steps)
    torch.cuda.synchronize()
    e0.record(stream)
    bt.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / steps
    finite = bool(torch.isfinite(bt.U[0]).all())
    one.load(states)
    one.step(2)
    one.capture(steps)
    torch.cuda.synchronize()
    e0.record(stream)
    one.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_one = e0.elapsed_time(e1) / steps
    one_status = one.step_status()
    one_equal = bool(torch.equal(one.U[one.cur], bt.U[bt.cur]) and torch.equal(one.smax, bt.smax))
    del bt, one
    torch.cuda.empty_cache()
    loop = []
    for (nx, ny), U in zip(sizes, states):
        st = EulerStepper(nx, ny)
        st.load(U)
        loop.append(st)
    for st in loop:
        st.step(1)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(loop_steps):
        for st in loop:
            st.step(1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1) / loop_steps
    del loop
    torch.cuda.empty_cache()
    return {"grids": len(sizes), "cells": cells, "steps_graphed": steps, "ms_per_step": ms_batch,
            "cell_updates_per_s": cells / (ms_batch * 1e-3), "compulsory_GBs": 128 * cells / (ms_batch * 1e-3) / 1e9,
            "loop_of_per_grid_launches": {"ms_per_step": ms_loop, "cell_updates_per_s": cells / (ms_loop * 1e-3),
                                          "steps": loop_steps},
            "batched_over_loop": ms_loop / ms_batch, "state_finite": finite,
            "y_segments_by_bucket": segs,
            "one_launch_step": {"ms_per_step": ms_one, "cell_updates_per_s": cells / (ms_one * 1e-3),
                                "per_sweep_over_one_launch": ms_batch / ms_one,
                                "bitwise_equal_to_per_sweep": one_equal, "status": one_status}}


def cpu_model():
    """CPU model name and logical CPU count, as lscpu and nproc report them."""
    import subprocess
    model = "unknown"
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except (OSError, subprocess.SubprocessError, ValueError):
        nproc = os.cpu_count()
    return model, nproc


def cpu_baseline(U0, steps_all=4, steps_one=1, runs=3):
    """The FP64 oracle on the host, on the workload itself (the 2048^2 state
    from its initial condition): `runs` timed runs of `steps_all` steps on
    all the oracle's OpenMP threads and of `steps_one` step on one thread
    (OMP_PROC_BIND=close), the median of each."""
    import statistics
    import oracle
    cores = oracle.num_threads()

    def median_rate(steps, threads):
        oracle.set_threads(threads)
        try:
            ts = []
            for _ in range(runs):
                t0 = time.perf_counter()
                oracle.euler_run(U0, steps)
                ts.append(time.perf_counter() - t0)
        finally:
            oracle.set_threads(cores)
        med = statistics.median(ts)
        return NX * NY * steps / med, med, ts

    v_all, t_all, _ = median_rate(steps_all, cores)
    v_one, t_one, _ = median_rate(steps_one, 1)
    model, nproc = cpu_model()
    return {"value": v_all, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, {NX}x{NY} hydro chain, {steps_all} steps from the initial state on "
                      f"{cores} OpenMP threads (OMP_PROC_BIND={os.environ.get('OMP_PROC_BIND')}), "
                      f"median of {runs} runs ({t_all:.2f} s each)",
            "cpu": model, "nproc": nproc,
            "single_thread": {"value": v_one, "unit": "cell-updates/s", "cores": 1,
                              "sample": f"the same workload, {steps_one} step on 1 thread, median of {runs} "
                                        f"runs ({t_one:.2f} s each)"}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-unfused", action="store_true")
    ap.add_argument("--no-timing-events", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--xy-seg", type=int, default=0,
                    help="with --only euler_xy: one segment length instead of the sweep over 8..64")
    ap.add_argument("--no-aux", action="store_true",
                    help="skip the bandwidth-bound chains and the FP32 hydro variant")
    ap.add_argument("--only", choices=["hdiff", "biharm64", "biharm32", "batch", "hdiff_small", "norm",
                                       "hdiff_in_place", "euler_xy"],
                    default=None,
                    help="only time one bandwidth-bound chain, or the batched grids (for profiling)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the chains would shard along the slowest axis with one halo exchange per chain; "
              "that path is not built)", file=sys.stderr)
        return 2
    import torch
    from paper_1710_08774_amd import hfav as H
    from paper_1710_08774_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    H.lib()
    if a.copy_probe_mib:
        n = a.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "launches": 3}), flush=True)
        return 0
    if a.only == "hdiff_small":
        print(json.dumps({"workload": "hdiff_256x256x8", **hdiff_config_shape()}), flush=True)
        return 0
    if a.only == "euler_xy":
        U0 = inputs.euler_ic(NX, NY)
        segs = (a.xy_seg,) if a.xy_seg else (8, 16, 32, 64)
        res = {str(sg): run_xy(a.steps, a.warmup, U0, sg) for sg in segs}
        print(json.dumps({"workload": "euler2d_xy_2048x2048", "by_segment": res}), flush=True)
        return 0
    if a.only == "hdiff_in_place":
        print(json.dumps({"workload": "hdiff_in_place_64x2048x2048", **hdiff_in_place(reps=a.steps)}), flush=True)
        return 0
    if a.only == "norm":
        print(json.dumps({"workload": "norm_4x4096x4096_f64", **norm_chain(reps=a.steps,
                                                                            unfused=not a.no_unfused)}),
              flush=True)
        return 0
    if a.only == "batch":
        print(json.dumps({"workload": "batch", **batched_grids()}), flush=True)
        return 0
    if a.only:
        res = bandwidth_chains(reps=a.steps, which=(a.only,), unfused=not a.no_unfused)
        print(json.dumps({"workload": a.only, **res[a.only]}), flush=True)
        return 0
    U0 = inputs.euler_ic(NX, NY)
    timing = not a.no_timing_events
    fused = run_gpu(H.MODE_FUSED, a.steps, a.warmup, U0, timing)
    unf = None if a.no_unfused else run_gpu(H.MODE_UNFUSED, a.steps, a.warmup, U0, timing)
    cells = NX * NY
    value = cells / (fused["ms_per_step"] * 1e-3)
    line = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "clock_warmup": fused["clock_warmup"],
        "ms_per_step": fused["ms_per_step"],
        "host_enqueue_ms_per_step": fused["host_enqueue_ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "euler2d-split-godunov-exact-riemann-2048x2048-f64", "grid": [NX, NY],
                   "gamma": 1.4, "cfl": 0.5, "newton_iters": 10,
                   "newton_stop": "exact: stops once every lane's iterate repeats, result bit for bit that of 10 steps",
                   "boundary": "periodic",
                   "initial_state": "Sod-like split on a seeded random-angle line + 1e-3 sinusoidal modes",
                   "path": "fused (one kernel per sweep, CFL reduction fused into the y sweep)"},
        "hbm_compulsory": {
            "bytes_per_cell_step": 2 * COMPULSORY_BYTES_PER_CELL_SWEEP,
            "achieved_GBs": 2 * COMPULSORY_BYTES_PER_CELL_SWEEP * cells / (fused["ms_per_step"] * 1e-3) / 1e9,
            "frac_of_8TBs": 2 * COMPULSORY_BYTES_PER_CELL_SWEEP * cells / (fused["ms_per_step"] * 1e-3) / 1e9
            / HBM_PEAK_GBS},
    }
    if unf is not None:
        line["unfused"] = {"value": cells / (unf["ms_per_step"] * 1e-3), "ms_per_step": unf["ms_per_step"],
                           "x_ms": unf.get("x_ms"), "y_ms": unf.get("y_ms")}
        line["fused_over_unfused"] = unf["ms_per_step"] / fused["ms_per_step"]
    if timing:
        kx, ky = fused["x_ms"], fused["y_ms"]
        dom, dur = (fused["x_kernel"], kx) if kx >= ky else (fused["y_kernel"], ky)
        flops = FLOPS_PER_CELL_SWEEP * cells
        achieved = flops / (dur * 1e-3) / 1e12
        line["roofline"] = {"bound": "alu", "kernel": dom, "achieved": achieved,
                            "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": load_traffic(dom),
                            "avg_launch_ms": dur, "x_sweep_ms": kx, "y_sweep_ms": ky,
                            "flops_per_launch": flops, "x_config": fused["x_config"],
                            "y_config": fused["y_config"],
                            # issue-side view of the same kernel from the committed counters:
                            # the flop count above weighs a divide or a 1/7 power as one
                            "valu_busy": load_counters(dom).get("valu_busy"),
                            "valu_instr_per_64_cells": load_counters(dom).get("valu_instr_per_64_cells")}
    if not a.no_aux:
        aux = bandwidth_chains()
        f32 = run_gpu(H.MODE_FUSED, a.steps, a.warmup, U0, False, dtype=torch.float32)
        aux["euler_f32_state_f64_riemann"] = {
            "ms_per_step": f32["ms_per_step"], "cell_updates_per_s": cells / (f32["ms_per_step"] * 1e-3),
            "compulsory_GBs": 64 * cells / (f32["ms_per_step"] * 1e-3) / 1e9}
        ip = run_gpu(H.MODE_FUSED, a.steps, a.warmup, U0, True, in_place=True)
        aux["euler_in_place"] = {
            "ms_per_step": ip["ms_per_step"], "cell_updates_per_s": cells / (ip["ms_per_step"] * 1e-3),
            "x_ms": ip.get("x_ms"), "y_ms": ip.get("y_ms"),
            "footprint_bytes_in_place": ip["footprint_bytes"], "footprint_bytes_two_states": fused["footprint_bytes"],
            "note": "one state; each sweep first saves the cells around its segment boundaries, then writes over it"}
        aux["batch_512_grids"] = batched_grids()
        aux["hdiff_256x256x8"] = hdiff_config_shape()
        aux["norm_4x4096x4096"] = norm_chain()
        aux["hdiff_in_place_64x2048x2048"] = hdiff_in_place()
        aux["euler_xy_one_kernel_per_step"] = run_xy(a.steps, a.warmup, U0)
        line["aux"] = aux
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(U0)
    line["state_finite"] = fused["state_finite"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
