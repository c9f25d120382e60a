"""Planner on the normalisation chain (host only): reductions along i,
broadcasts of a row term, and the split they force (Design, "Fusing
iteration nests", "Reductions & broadcasts & splits"; Performance,
"Normalization Example": five full visits of the (j, i) space become two).
"""
import pytest

from paper_1710_08774_amd import hfav as H

Z = (0, 0, 0)


def _plan(spec, dims, **kw):
    c = H.Chain(spec)
    info = c.plan(dims, **kw)
    return c, info


def test_norm_split_into_two_sweeps_of_one_outer_nest():
    c, info = _plan(H.norm_spec(4), (4096, 4096))
    nq = 4
    # rules: flux x4, SUMSQ, SUM_I, SQRT, DIV0 x4, AXPY x4
    assert info.n_rules == 3 + 3 * nq
    assert info.n_nests == 2
    assert list(info.outer_of_nest[:2]) == [0, 0]
    nest = [info.nest_of_rule[r] for r in range(info.n_rules)]
    phase = [info.phase_of_rule[r] for r in range(info.n_rules)]
    assert nest[:nq + 2] == [0] * (nq + 2) and phase[:nq + 2] == [1] * (nq + 2)
    assert nest[nq + 2] == 0 and phase[nq + 2] == 2          # the root: epilogue of sweep 1
    assert nest[nq + 3:] == [1] * (2 * nq) and phase[nq + 3:] == [1] * (2 * nq)
    t = c.terms()
    for q in range(nq):
        f = t[f"f{q}"]
        assert (f["storage"], f["window_axis"], f["window"]) == ("outer", 1, 1)   # one row
        assert t[f"d{q}"]["storage"] == "register"
    assert t["e"]["storage"] == "register"
    assert t["s"]["rank"] == 1 and t["s"]["storage"] == "register"
    assert t["n"]["rank"] == 1 and t["n"]["storage"] == "register"
    assert H.FAMILY[info.family] == "norm" and info.fused
    assert info.bytes_per_cell_fused == 2 * nq * 8
    # unfused: flux (u, u -> f), SUMSQ (f x4 -> e), SUM_I (e), DIV0 (f -> d), AXPY (u, d -> out)
    assert info.bytes_per_cell_unfused == 8 * (nq * 2 + (nq + 1) + 1 + nq * 2 + nq * 3)
    assert info.footprint_unfused == (2 * nq + 1) * 4096 * 4096 + 2 * 4096
    assert info.footprint_contracted == nq * 4096 + nq + 1 + 2      # f rows, d, e, s, n
    j = c.plan_json()
    assert [n["outer"] for n in j["nests"]] == [0, 0]
    assert j["nests"][0]["epilogue"] == [nq + 2]


def test_norm_row_goal_and_3d_rows():
    c, info = _plan(H.norm_spec(3, with_norm=True), (1000, 37))
    assert c.terms()["n"]["storage"] == "full" and info.family == 8
    c3, info3 = _plan(H.norm_spec(2, ndim=3), (128, 16, 8))
    assert info3.n_nests == 2 and list(info3.outer_of_nest[:2]) == [0, 0] and info3.family == 8
    assert c3.terms()["s"]["rank"] == 2
    assert c3.terms()["f0"]["window_axis"] == 1          # the slab of j: one row of i


def test_norm_default_configs_cover_the_row():
    for nq, ni, expect in [(4, 4096, (512, 8, 3)), (1, 4096, (256, 16, 3)), (8, 4096, (1024, 4, 3)),
                           (4, 100, (128, 1, 3)), (4, 1, (64, 1, 3)), (4, 9000, (256, 0, 1))]:
        _, info = _plan(H.norm_spec(nq), (ni, 8))
        cfg = info.config
        assert (cfg.block, cfg.seg, cfg.variant) == expect, (nq, ni)
    _, info = _plan(H.norm_spec(4, dtype=H.F32), (4096, 8))
    assert (info.config.block, info.config.seg, info.config.variant) == (512, 8, 2)


def test_norm_loop_order_with_i_outer_is_not_fused():
    """With i outermost the reduction along i is not an inner sweep: no
    shared outer loop, f stays a full array, no fused family."""
    c, info = _plan(H.norm_spec(2, loop_order="ij"), (64, 64))
    assert info.n_nests == 2 and list(info.outer_of_nest[:2]) == [0, 1]
    assert c.terms()["f0"]["storage"] == "full" and c.terms()["n"]["storage"] == "full"
    assert info.family == 0 and not info.fused
    assert info.workspace_bytes > 0
    with pytest.raises(H.HfavError):
        c.plan((64, 64), mode=H.MODE_FUSED)


def test_norm_unfused_workspace_holds_rows_and_grids():
    c, info = _plan(H.norm_spec(2), (300, 20), mode=H.MODE_UNFUSED)
    es = 8
    grid, row = 300 * 20 * es, 20 * es
    rnd = lambda b: (b + 255) // 256 * 256
    # f0, f1, e, d0, d1 grids; s, n rows
    assert info.workspace_bytes == 5 * rnd(grid) + 2 * rnd(row)
    assert not info.fused


def test_norm_forced_config_must_cover_the_row():
    c = H.Chain(H.norm_spec(4))
    with pytest.raises(H.HfavError) as e:
        c.plan((4096, 8), config_source=H.CONFIG_FORCED, forced=(256, 1, 8, 0, 0))
    assert e.value.code == H.EUNSUP
    info = c.plan((2048, 8), config_source=H.CONFIG_FORCED, forced=(256, 1, 8, 0, 0))
    assert (info.config.block, info.config.seg) == (256, 8)
    info = c.plan((5000, 8), config_source=H.CONFIG_FORCED, forced=(128, 1, 0, 1, 0))
    assert info.config.variant == 1


def _spec(rules, axioms, goals, ndim=2):
    return H.ChainSpec(ndim=ndim, axioms=axioms, goals=goals, rules=rules)


@pytest.mark.parametrize("bad", [
    # row-term reference with an offset
    [H.Rule("SUM_I", [("x", Z)], ["s"], reduce=H.REDUCE_SUM),
     H.Rule("DIV0", [("x", Z), ("s", (0, 1, 0))], ["y"])],
    # SUM_I without the SUM reduction
    [H.Rule("SUM_I", [("x", Z)], ["s"]), H.Rule("DIV0", [("x", Z), ("s", Z)], ["y"])],
    # a row term where a grid is needed
    [H.Rule("SUM_I", [("x", Z)], ["s"], reduce=H.REDUCE_SUM), H.Rule("DIV0", [("s", Z), ("x", Z)], ["y"])],
    [H.Rule("SUM_I", [("x", Z)], ["s"], reduce=H.REDUCE_SUM), H.Rule("AXPY", [("x", Z), ("s", Z)], ["y"], [1.0])],
    # SUM_I reads its input at offset 0 only
    [H.Rule("SUM_I", [("x", (1, 0, 0))], ["s"], reduce=H.REDUCE_SUM), H.Rule("DIV0", [("x", Z), ("s", Z)], ["y"])],
    # the MAX reduction belongs to EULER_SMAX
    [H.Rule("SQRT", [("x", Z)], ["y"], reduce=H.REDUCE_MAX)],
])
def test_rank_rules_are_validated(bad):
    with pytest.raises(H.HfavError) as e:
        H.Chain(_spec(bad, [("x", 2)], ["y"]))
    assert e.value.code == H.EINVAL


def test_row_axiom_broadcast_and_sqrt_of_grid():
    """A row term may also be an axiom (broadcast input); SQRT also works on
    grids.  Ranks: rule over rows = ndim - 1."""
    spec = _spec([H.Rule("DIV0", [("x", Z), ("r", Z)], ["y"]), H.Rule("SQRT", [("y", Z)], ["z"]),
                  H.Rule("SQRT", [("r", Z)], ["rr"])],
                 [("x", 2), ("r", 1)], ["z", "rr"])
    c, info = _plan(spec, (50, 6))
    t = c.terms()
    assert t["r"]["rank"] == 1 and t["rr"]["rank"] == 1 and t["z"]["rank"] == 2
    assert info.family == 0
    bad = _spec([H.Rule("SQRT", [("x", Z)], ["y"])], [("x", 0)], ["y"])
    with pytest.raises(H.HfavError):
        H.Chain(bad)


def test_broadcast_goes_into_the_prologue():
    """A rule over rows (rank ndim - 1) whose result a grid rule broadcasts
    along i is fused into the prologue of the grid nest (Design,
    "Reductions & broadcasts & splits"); a reduction's finalisation goes
    into the epilogue (the norm root above)."""
    spec = _spec([H.Rule("SQRT", [("r", Z)], ["n"]), H.Rule("DIV0", [("x", Z), ("n", Z)], ["y"])],
                 [("x", 2), ("r", 1)], ["y"])
    c, info = _plan(spec, (50, 6))
    assert info.n_nests == 1
    assert [info.phase_of_rule[r] for r in range(2)] == [0, 1]
    assert c.terms()["n"]["storage"] == "register"
    j = c.plan_json()
    assert j["nests"][0]["prologue"] == [0] and j["nests"][0]["steady"] == [1]
