"""Host-side planner tests (no GPU): chain validation, fusion, extents,
windows and footprints against the structural figures the paper states
(tests/golden/plan_pins.json), error codes, determinism."""
import json
import os

import pytest

from paper_1710_08774_amd import hfav as H
from paper_1710_08774_amd import inputs

PINS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "plan_pins.json")))
Z = (0, 0, 0)


def star(refs, out, coeffs=None):
    return H.Rule("STAR", refs, [out], coeffs or [1.0] * len(refs))


def test_laplace3_window_is_three_values():
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["out"], rules=[
        star([("a", Z)], "v"),
        star([("v", (-1, 0, 0)), ("v", Z), ("v", (1, 0, 0))], "out", [1.0, -2.0, 1.0])])
    c = H.Chain(spec)
    c.plan((64, 8))
    v = c.terms()["v"]
    assert v["storage"] == PINS["laplace3_1d"]["storage"]
    assert v["window"] == PINS["laplace3_1d"]["window"] and v["window_axis"] == 0


def test_laplace5_window_and_reuse_order():
    refs = [("v", (0, -1, 0)), ("v", (1, 0, 0)), ("v", Z), ("v", (0, 1, 0)), ("v", (-1, 0, 0))]
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["out"], rules=[
        star([("a", Z)], "v"), star(refs, "out", [0.25, 0.25, -1.0, 0.25, 0.25])])
    c = H.Chain(spec)
    info = c.plan((32, 32))
    v = c.terms()["v"]
    pin = PINS["laplace5_2d"]
    assert v["storage"] == pin["storage"] and v["window_axis"] == 1 and v["window"] == pin["window_rows"]
    reuse = [t for t in c.plan_json()["terms"] if t["name"] == "v"][0]["reuse"]
    assert [r[:2] for r in reuse] == pin["reuse_order_ij"]
    assert info.footprint_contracted == 3 * 32


def test_grouping_and_minkowski_extents():
    # cell read at five displacements forms one group; aux is separate
    refs = [("cell", (1, 0, 0)), ("cell", (-1, 0, 0)), ("cell", (0, 1, 0)), ("cell", (0, -1, 0)),
            ("cell", Z), ("aux", (1, 0, 0))]
    spec = H.ChainSpec(ndim=2, axioms=[("cell", 2), ("aux", 2)], goals=["out"], rules=[
        star(refs, "w"), star([("w", (2, 0, 0)), ("w", (0, -1, 0))], "out")])
    c = H.Chain(spec)
    c.plan((16, 16))
    t = c.terms()
    # extent of cell = extent of w (i in [0,2], j in [-1,0]) + the 5-point star
    assert t["w"]["lo"] == (0, -1, 0) and t["w"]["hi"] == (2, 0, 0)
    assert t["cell"]["lo"] == (-1, -2, 0) and t["cell"]["hi"] == (3, 1, 0)
    assert t["aux"]["lo"] == (1, -1, 0) and t["aux"]["hi"] == (3, 0, 0)


def test_cosmo_chain_contraction():
    pin = PINS["cosmo_hdiff"]
    c = H.Chain(H.hdiff_spec())
    ni, nj, nk = 256, 256, 8
    info = c.plan((ni, nj, nk))
    t = c.terms()
    assert info.n_nests == pin["nests"]
    assert (t["lap"]["storage"], t["lap"]["window_axis"], t["lap"]["window"]) == ("outer", 1, pin["lap_rows"])
    assert (t["fly"]["storage"], t["fly"]["window_axis"], t["fly"]["window"]) == ("outer", 1, pin["fly_rows"])
    assert (t["flx"]["storage"], t["flx"]["window_axis"], t["flx"]["window"]) == ("inner", 0, pin["flx_elems"])
    assert t["u"]["storage"] == "full" and t["out"]["storage"] == "full"
    assert info.footprint_contracted == 5 * ni + 2
    assert info.footprint_unfused == 3 * ni * nj * nk
    assert t["u"]["lo"] == (-2, -2, 0) and t["u"]["hi"] == (2, 2, 0)      # halo 2
    assert info.family == 1 and info.fused == 1
    assert info.bytes_per_cell_fused == 16.0


@pytest.mark.parametrize("direction", [0, 1])
def test_hydro_pass_one_nest_windows_at_most_five(direction):
    pin = PINS["hydro2d_pass"]
    c = H.Chain(H.euler_sweep_spec(direction, with_smax=direction == 1))
    info = c.plan((128, 96))
    assert info.n_nests == pin["nests"]
    assert info.max_window == pin["max_window"]
    terms = c.terms()
    for name, t in terms.items():
        if t["kind"] == 1:
            assert t["storage"] in ("inner", "outer", "register", "scalar"), name
            assert t["window"] <= 5
        if t["kind"] in (0, 2) and t["rank"] == 2:
            assert t["storage"] == "full"
    ax = 0 if direction == 0 else 1
    assert terms["w_r"]["window_axis"] == ax and terms["w_r"]["window"] == 5
    assert terms["F_r"]["window"] == 2
    js = c.plan_json()
    assert len(js["nests"]) == 1 and js["nests"][0]["prologue"] == [0]     # dt broadcast
    assert info.family == (2 if direction == 0 else 3)
    assert info.bytes_per_cell_fused == 64.0
    assert info.bytes_per_cell_unfused == (528.0 if direction == 0 else 560.0)


def test_concave_dataflow_splits_into_two_nests():
    # CFL reduction of the state feeding (through dt) a sweep of the same state
    spec = H.euler_sweep_spec(0, dt_source="smax")
    rules = list(spec.rules)
    axioms = [a for a in spec.axioms if a[0] != "smax"]
    rules.insert(0, H.Rule("EULER_SMAX", [(a, Z) for a in H.EULER_AXIOMS], ["smax"], [1.4], H.REDUCE_MAX))
    c = H.Chain(H.ChainSpec(ndim=2, axioms=axioms, goals=spec.goals, rules=rules))
    info = c.plan((64, 64))
    assert info.n_nests == PINS["normalization_split"]["nests"]
    js = c.plan_json()
    # nest 0: the reduction (rule 0) with the rules that do not need dt
    # (prim 2, slope 3) in its steady state and dt (rule 1) in its epilogue;
    # the trace needs dt, so it starts nest 1
    assert js["nests"][0]["steady"] == [0, 2, 3] and js["nests"][0]["epilogue"] == [1]
    assert js["nests"][1]["steady"][0] == 4
    t = c.terms()
    assert t["smax"]["storage"] == "scalar"
    # terms crossing the split stay full arrays; those inside a nest contract
    assert t["w_r"]["storage"] == "full" and t["d_p"]["storage"] == "full"
    assert t["F_r"]["storage"] == "inner"
    assert info.family == 0 and info.fused == 0          # falls back to the unfused path


def test_independent_chains_fuse():
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2), ("b", 2)], goals=["x", "y"], rules=[
        star([("a", (1, 0, 0)), ("a", Z)], "x"), star([("b", (0, 1, 0))], "y")])
    info = H.Chain(spec).plan((8, 8))
    assert info.n_nests == 1


def test_loop_order_changes_windows():
    c = H.Chain(H.hdiff_spec(loop_order="jik"))   # i is the middle axis, k innermost
    c.plan((32, 32, 4))
    t = c.terms()
    assert t["lap"]["window_axis"] == 1 and t["lap"]["window"] == 3   # j outermost varying
    assert t["flx"]["storage"] == "outer" and t["flx"]["window_axis"] == 0


def test_dead_rules_are_pruned_and_plan_is_deterministic():
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[
        star([("a", Z)], "x"), star([("a", (1, 0, 0))], "dead")])
    c = H.Chain(spec)
    i1 = c.plan((16, 16))
    j1 = c.plan_json()
    i2 = c.plan((16, 16))
    assert j1 == c.plan_json()
    assert i1.n_rules == 1 and i1.nest_of_rule[1] == -1
    assert list(i1.rule_order[:1]) == [0]


def test_unfused_workspace_layout():
    c = H.Chain(H.euler_sweep_spec(0))
    info = c.plan((100, 10), mode=H.MODE_UNFUSED)
    # 25 grid intermediates (prim 5, slopes 4, faces 8, Godunov state 4,
    # fluxes 4) of 1000 doubles, 256-byte aligned, plus the 0-D dt
    assert info.fused == 0
    assert info.workspace_bytes == 25 * ((8000 + 255) // 256 * 256) + 256


# ----------------------------------------------------------------- errors
def code(fn):
    try:
        fn()
    except H.HfavError as e:
        return e.code
    return H.OK


def test_error_duplicate_producer():
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[
        star([("a", Z)], "x"), star([("a", (1, 0, 0))], "x")])
    assert code(lambda: H.Chain(spec)) == H.EDUP
    spec2 = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[
        star([("a", Z)], "x"), star([("x", Z)], "a")])
    assert code(lambda: H.Chain(spec2)) == H.EDUP
    spec3 = H.ChainSpec(ndim=2, axioms=[("a", 2), ("a", 2)], goals=["x"], rules=[star([("a", Z)], "x")])
    assert code(lambda: H.Chain(spec3)) == H.EDUP


def test_error_cycle():
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[
        star([("a", Z), ("y", Z)], "x"), star([("x", (1, 0, 0))], "y")])
    assert code(lambda: H.Chain(spec)) == H.ECYCLE


def test_error_unsatisfiable():
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["nope"], rules=[star([("a", Z)], "x")])
    assert code(lambda: H.Chain(spec)) == H.EUNSAT
    spec2 = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[star([("ghost", Z)], "x")])
    assert code(lambda: H.Chain(spec2)) == H.EUNSAT


def test_error_invalid():
    bad_arity = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"],
                            rules=[H.Rule("HDIFF_LAP", [("a", Z)], ["x"])])
    assert code(lambda: H.Chain(bad_arity)) == H.EINVAL
    bad_op = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[H.Rule(999, [("a", Z)], ["x"])])
    assert code(lambda: H.Chain(bad_op)) == H.EINVAL
    bad_nd = H.ChainSpec(ndim=4, axioms=[("a", 4)], goals=["x"], rules=[star([("a", Z)], "x")])
    assert code(lambda: H.Chain(bad_nd)) == H.EINVAL
    bad_off = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[star([("a", (0, 0, 1))], "x")])
    assert code(lambda: H.Chain(bad_off)) == H.EINVAL
    scalar_as_grid = H.ChainSpec(ndim=2, axioms=[("a", 0)], goals=["x"], rules=[star([("a", Z)], "x")])
    assert code(lambda: H.Chain(scalar_as_grid)) == H.EINVAL
    c = H.Chain(H.hdiff_spec())
    assert code(lambda: c.plan((0, 4, 4))) == H.EINVAL
    assert code(lambda: c.plan((4, 4, 4), boundary=(7, 0, 0))) == H.EINVAL
    c2 = H.Chain(H.euler_sweep_spec(0))
    assert code(lambda: c2.plan((8, 8, 2))) == H.EINVAL       # nz must be 1 for a 2-D chain


def test_error_unsupported_fused_mode():
    spec = H.ChainSpec(ndim=2, axioms=[("a", 2)], goals=["x"], rules=[star([("a", Z)], "x")])
    c = H.Chain(spec)
    assert code(lambda: c.plan((8, 8), mode=H.MODE_FUSED)) == H.EUNSUP
    assert c.plan((8, 8), mode=H.MODE_AUTO).fused == 0
    c64 = H.Chain(H.hdiff_spec())
    assert code(lambda: c64.plan((8, 8, 1), precision=H.PREC_F32_F64ACC)) == H.EUNSUP


def test_execute_errors_before_any_device_call():
    c = H.Chain(H.hdiff_spec())
    assert c.execute_status([0x10000], [0x20000]) == H.ENOPLAN      # no plan yet
    c.plan((16, 16, 2))
    # output overlapping the input
    assert c.execute_status([0x10000], [0x10000 + 64]) == H.EALIAS
    assert c.execute_status([0], [0x20000]) == H.EINVAL               # null pointer
    cu = H.Chain(H.hdiff_spec())
    cu.plan((16, 16, 2), mode=H.MODE_UNFUSED)
    assert cu.execute_status([0x10000], [0x900000], None) == H.ENOPLAN  # workspace missing
    assert "workspace" in H.last_error()


def test_forced_config_validation():
    c = H.Chain(H.hdiff_spec())
    assert code(lambda: c.plan((8, 8, 1), config_source=H.CONFIG_FORCED, forced=(0, 1, 1, 0))) == H.EINVAL
    info = c.plan((8, 8, 1), config_source=H.CONFIG_FORCED, forced=(128, 1, 7, 2))
    assert (info.config.block, info.config.seg, info.config.variant) == (128, 7, 2)
    assert info.config_source == H.CONFIG_FORCED


def test_tuning_table_nearest_entry():
    H.tuning_clear()
    H.tuning_add(1, H.F64, (256, 256, 8), (64, 1, 16, 1))
    H.tuning_add(1, H.F64, (2048, 2048, 64), (512, 1, 128, 4))
    c = H.Chain(H.hdiff_spec())
    small = c.plan((300, 200, 4), config_source=H.CONFIG_TUNED)
    big = c.plan((1800, 2100, 32), config_source=H.CONFIG_TUNED)
    assert small.config.block == 64 and big.config.block == 512
    assert small.config_source == H.CONFIG_TUNED
    H.tuning_clear()
    assert c.plan((300, 200, 4), config_source=H.CONFIG_TUNED).config_source == H.CONFIG_DEFAULT


def test_tuning_db_load_drives_tuned_plans(tmp_path):
    import json
    from paper_1710_08774_amd import tune
    db = {"version": 1, "entries": [
        {"family": "hdiff", "family_id": 1, "dtype": "f64", "dims": [2048, 2048, 64],
         "config": [512, 1, 64, 2, -1]},
        {"family": "euler_y", "family_id": 3, "dtype": "f64", "dims": [512, 512, 1],
         "config": [128, 1, 32, 0, 0]},
        {"family": "lap7_chain", "family_id": 4, "dtype": "f32", "dims": [512, 512, 512],
         "config": [1024, 4, 128, 13, 8]}]}
    path = tmp_path / "db.json"
    path.write_text(json.dumps(db))
    assert tune.load_db(str(path)) == 3
    c = H.Chain(H.hdiff_spec())
    i = c.plan((2000, 1900, 60), config_source=H.CONFIG_TUNED)
    assert (i.config.block, i.config.seg, i.config.variant, i.config.xcd) == (512, 64, 2, -1)
    assert i.config_source == H.CONFIG_TUNED
    y = H.Chain(H.euler_sweep_spec(1))
    i = y.plan((500, 520), config_source=H.CONFIG_TUNED)
    assert (i.config.block, i.config.seg, i.config.variant) == (128, 32, 0)
    b = H.Chain(H.biharm_spec(dtype=H.F32))
    i = b.plan((500, 500, 500), config_source=H.CONFIG_TUNED)
    assert (i.config.tile_y, i.config.variant, i.config.xcd) == (4, 13, 8)
    # an entry of another dtype is not used
    b64 = H.Chain(H.biharm_spec())
    assert b64.plan((500, 500, 500), config_source=H.CONFIG_TUNED).config_source == H.CONFIG_DEFAULT
    H.tuning_clear()


def test_family_search_spaces_plan():
    from paper_1710_08774_amd import tune
    for fam, spec, dims in (("hdiff", H.hdiff_spec(), (64, 48, 2)), ("lap7_chain", H.biharm_spec(), (40, 36, 20)),
                            ("euler_x", H.euler_sweep_spec(0), (64, 48)), ("euler_y", H.euler_sweep_spec(1), (64, 48))):
        c = H.Chain(spec)
        space = tune.family_space(fam)
        assert len(space) == len(set(space)) >= 9
        for cfg in space:
            info = c.plan(dims, mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
            assert info.fused and H.FAMILY[info.family] == fam
    # the two-sweep family: every configuration plans
    c = H.Chain(H.euler_step_spec())
    for cfg in tune.family_space("euler_xy"):
        assert c.plan((64, 48), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg).family == 9
    # the normalisation family: exactly the configurations covering the row plan
    c = H.Chain(H.norm_spec(tune.NORM_FIELDS))
    ok = 0
    for cfg in tune.family_space("norm"):
        blk, _, seg, var, _ = cfg
        fits = var == 1 or (blk * seg >= 1000 and tune.NORM_FIELDS * seg <= 32)
        try:
            info = c.plan((1000, 8), mode=H.MODE_FUSED, config_source=H.CONFIG_FORCED, forced=cfg)
            assert fits and info.family == 8
            ok += 1
        except H.HfavError as e:
            assert not fits and e.code == H.EUNSUP
    assert ok >= 9


def test_random_star_chain_plans():
    rng = inputs.rng_for(5)
    for _ in range(10):
        ch = inputs.random_chain(rng)
        c = H.Chain(H.star_chain_spec(ch, inputs.star_offsets))
        nx, ny, nz = ch["dims"]
        info = c.plan((nx, ny, nz) if ch["ndim"] == 3 else (nx, ny))
        assert info.n_nests == 1
        halo = sum(s["r"] for s in ch["stages"])
        t = c.terms()
        assert t["x0"]["lo"][0] == -halo and t["x0"]["hi"][0] == halo


def test_batch_segments_from_tuning_buckets():
    c = H.Chain(H.euler_sweep_spec(1, dt_source="smax", with_smax=True))
    H.tuning_clear()
    try:
        H.tuning_add(7, H.F64, (128, 128, 1), (64, 1, 8, 1, 0))
        H.tuning_add(7, H.F64, (724, 724, 1), (64, 1, 32, 1, 0))
        c.plan_batch([(100, 120), (700, 800), (90, 1000)], config_source=H.CONFIG_TUNED)
        b = c.plan_json()["batch"]
        assert b["grids"] == 3 and b["y_seg"][:2] == [8, 32]
        c.plan_batch([(100, 120), (700, 800)])
        assert c.plan_json()["batch"]["y_seg"] == [15, 15]
        c.plan_batch([(100, 120)], config_source=H.CONFIG_FORCED, forced=(64, 1, 5, 1))
        assert c.plan_json()["batch"]["y_seg"] == [5]
    finally:
        H.tuning_clear()


def test_two_sweep_step_chain_fuses_into_one_nest():
    """x sweep then y sweep as one chain: equal-rank nests fuse (Design,
    "Fusing iteration nests"); the x-swept state is needed at rows j-2 ..
    j+2 of the y sweep (a 5-row window), and the step's compulsory traffic
    halves from 128 to 64 bytes per cell."""
    c = H.Chain(H.euler_step_spec(with_smax=True))
    info = c.plan((256, 128))
    assert H.FAMILY[info.family] == "euler_xy" and info.fused and info.n_nests == 1
    assert info.bytes_per_cell_fused == 64.0
    t = c.terms()
    for f in ("rho_x", "mx_x", "my_x", "E_x"):
        assert (t[f]["storage"], t[f]["window_axis"], t[f]["window"]) == ("outer", 1, 5)
    assert (info.config.block, info.config.seg, info.config.xcd) == (64, 4, -1)
    big = H.Chain(H.euler_step_spec()).plan((2048, 2048))
    assert (big.config.seg, big.config.xcd) == (12, -1)
    i32 = H.Chain(H.euler_step_spec(dtype=H.F32)).plan((64, 64), precision=H.PREC_F32_F64ACC, mode=H.MODE_FUSED)
    assert i32.family == 9
    # the y sweep reading another dt than the x sweep is not the fused family
    bad = H.euler_step_spec(dt_source="dt")
    bad.rules[-1].inputs[-1] = ("dt2", (0, 0, 0))
    bad.axioms.append(("dt2", 0))
    assert H.Chain(bad).plan((64, 64)).family == 0


# ------------------------------------------------------------ T-P8: fuse_inest
def _closure(n, edges):
    r = [[False] * n for _ in range(n)]
    for a, b in edges:
        r[a][b] = True
    for k in range(n):
        for a in range(n):
            if r[a][k]:
                for b in range(n):
                    if r[k][b]:
                        r[a][b] = True
    return r


# two rank-2 nests with all three phases: A = (0 | 1 | 2), B = (3 | 4 | 5)
_A = (2, [0], [1], [2])
_B = (2, [3], [4], [5])


def test_fuse_inest_equal_rank_phase_by_phase():
    """Design "Fusion": equal-rank nests fuse phase by phase when no ordering
    check fails; forward dependences between them (A's phases feeding B's
    same or later phases) do not prevent it."""
    for edges in ([], [(1, 4)], [(0, 3), (0, 4), (1, 4), (1, 5), (2, 5), (0, 5)]):
        got = H.fuse_nests(6, _closure(6, edges), [_A, _B])
        assert got == [(2, [0, 3], [1, 4], [2, 5])], edges


@pytest.mark.parametrize("which,edge", [
    ("A.prologue <= B.steady", (4, 0)),    # B's steady state feeds A's prologue
    ("B.prologue <= A.steady", (1, 3)),    # A's steady state feeds B's prologue
    ("A.steady <= B.epilogue", (5, 1)),    # B's epilogue feeds A's steady state
    ("B.steady <= A.epilogue", (2, 4)),    # A's epilogue feeds B's steady state
])
def test_fuse_inest_each_ordering_check_alone_splits(which, edge):
    """Each of the four equal-rank checks violated alone (the other three
    hold) leaves the nests unfused: the walk closes A and starts B."""
    got = H.fuse_nests(6, _closure(6, [edge]), [_A, _B])
    assert got == [_A, _B], which


def test_fuse_inest_unequal_rank_placement():
    """Lower-rank nest (rule 6, rank 1) against a rank-2 nest H = (0 | 1 | 2):
    prologue when it can precede H's steady state and epilogue, epilogue
    when H's prologue and steady state can precede it, else unfusable."""
    Hn = (2, [0], [1], [2])
    L = (1, [], [6], [])
    assert H.fuse_nests(7, _closure(7, []), [Hn, L]) == [(2, [6, 0], [1], [2])]
    assert H.fuse_nests(7, _closure(7, [(6, 1)]), [Hn, L]) == [(2, [6, 0], [1], [2])]   # broadcast
    assert H.fuse_nests(7, _closure(7, [(1, 6)]), [Hn, L]) == [(2, [0], [1], [2, 6])]   # reduction
    # the reduction feeds H's own epilogue: placed in the epilogue ahead of it
    assert H.fuse_nests(7, _closure(7, [(1, 6), (6, 2)]), [Hn, L]) == [(2, [0], [1], [6, 2])]
    # H's prologue feeds the broadcast: placed in the prologue after it
    assert H.fuse_nests(7, _closure(7, [(0, 6), (6, 1)]), [Hn, L]) == [(2, [0, 6], [1], [2])]
    # reached from H's epilogue and feeding H's steady state: unfusable
    assert H.fuse_nests(7, _closure(7, [(2, 6), (6, 1)]), [Hn, L]) == [Hn, L]
    # the walk: an unfusable nest closes the fusing nest, and the next
    # equal-rank nest joins the new one
    C = (1, [], [7], [])
    got = H.fuse_nests(8, _closure(8, [(2, 6), (6, 1)]), [Hn, L, C])
    assert got == [Hn, (1, [], [6, 7], [])]


def test_fuse_nests_rejects_bad_arguments():
    with pytest.raises(H.HfavError) as e:
        H.fuse_nests(2, _closure(2, []), [(2, [], [5], [])])
    assert e.value.code == H.EINVAL


def test_binding_checks_tensor_arguments_before_the_call():
    """The binding refuses tensors that are not device tensors of the
    plan's element type and size before anything reaches the library."""
    import torch
    c = H.Chain(H.hdiff_spec())
    c.plan((64, 32, 2))
    u = torch.zeros((2, 32, 64), dtype=torch.float64)
    with pytest.raises(H.HfavError) as e:
        c.execute([u], [torch.zeros_like(u)])
    assert e.value.code == H.EINVAL and "cuda" in str(e.value)
    with pytest.raises(H.HfavError) as e:
        c.execute([u], [])
    assert e.value.code == H.EINVAL
