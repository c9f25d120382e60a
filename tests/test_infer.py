"""Rule inference from patterns (Implementation, "Inference"): pattern
variables in term names ("q?"), instantiation backward from the goals,
rollback of failed candidates, and equivalence of inferred chains with the
hand-written ones (same plan: family, nests, storage classes)."""
import pytest

from paper_1710_08774_amd import hfav as H
from patterns import R, Z, biharm_patterns, norm_patterns, sweep_patterns


def _shape(chain, dims):
    info = chain.plan(dims)
    terms = chain.terms()
    return info, terms


def test_paper_laplace_example_two_applications():
    """The paper's 5-point Laplace rule applied to its own output: the goal
    laplace(laplace(cell)) needs two applications, bound to cell and to
    laplace(cell)."""
    refs = [("q?", o) for o in (Z, (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0))]
    spec = H.ChainSpec(ndim=2, axioms=[("cell", 2)], goals=["laplace(laplace(cell))"],
                       rules=[R("HDIFF_LAP", refs, ["laplace(q?)"])])
    c = H.chain_infer(spec)
    c.plan((32, 16))
    j = c.plan_json()
    assert [r["binding"] for r in j["rules"]] == ["q?=cell", "q?=laplace(cell)"]
    assert [r["out"] for r in j["rules"]] == [["laplace(cell)"], ["laplace(laplace(cell))"]]
    assert j["rules"][1]["in"][1] == ["laplace(cell)", 1, 0, 0]
    t = c.terms()
    # the inner Laplacian is needed at j-1, j, j+1: a window of three rows
    assert t["laplace(cell)"]["window"] == 3 and t["laplace(cell)"]["storage"] == "outer"


def test_biharmonic_inferred_equals_hand_written():
    a, b = H.chain_infer(biharm_patterns()), H.Chain(H.biharm_spec())
    ia, ta = _shape(a, (64, 48, 40))
    ib, tb = _shape(b, (64, 48, 40))
    assert ia.family == ib.family == 4 and ia.fused and ia.n_nests == ib.n_nests == 1
    assert ia.bytes_per_cell_fused == ib.bytes_per_cell_fused
    assert ta["lap(u)"]["window"] == tb["lap1"]["window"]
    assert ta["lap(lap(u))"]["storage"] == tb["lap2"]["storage"]
    assert [r["binding"] for r in a.plan_json()["rules"]] == ["q?=u", "q?=lap(u)", "q?=u"]


@pytest.mark.parametrize("with_norm", [False, True])
def test_normalisation_inferred_equals_hand_written(with_norm):
    a = H.chain_infer(norm_patterns(4, with_norm=with_norm))
    b = H.Chain(H.norm_spec(4, with_norm=with_norm))
    ia, ta = _shape(a, (4096, 512))
    ib, tb = _shape(b, (4096, 512))
    assert ia.family == ib.family == 8 and ia.n_nests == ib.n_nests == 2
    assert list(ia.outer_of_nest[:2]) == list(ib.outer_of_nest[:2]) == [0, 0]
    assert (ia.config.block, ia.config.seg, ia.config.variant) == (ib.config.block, ib.config.seg,
                                                                  ib.config.variant)
    assert ia.bytes_per_cell_unfused == ib.bytes_per_cell_unfused
    for q in range(4):
        assert ta[f"flux(u{q})"]["storage"] == tb[f"f{q}"]["storage"] == "outer"
        assert ta[f"dir(u{q})"]["storage"] == tb[f"d{q}"]["storage"]
    assert ta["norm"]["storage"] == tb["n"]["storage"]
    rules = a.plan_json()["rules"]
    assert len(rules) == 3 + 3 * 4
    binds = sorted(r["binding"] for r in rules if r["pattern"] == 2)     # the flux pattern
    assert binds == [f"q?=u{q}" for q in range(4)]


def test_backtracking_takes_the_next_candidate():
    """The first rule for g(x) needs h(x), which nothing derives: it is
    rolled back and the second rule is used."""
    spec = H.ChainSpec(ndim=2, axioms=[("x", 2)], goals=["g(x)"], rules=[
        R("AXPY", [("q?", Z), ("h(q?)", Z)], ["g(q?)"], [1.0]),
        R("STAR", [("q?", (1, 0, 0))], ["g(q?)"], [2.0]),
    ])
    c = H.chain_infer(spec)
    c.plan((8, 8))
    rules = c.plan_json()["rules"]
    assert len(rules) == 1 and rules[0]["pattern"] == 1 and rules[0]["op"] == H.OP["STAR"]


def test_shared_terms_are_derived_once():
    spec = H.ChainSpec(ndim=2, axioms=[("x", 2)], goals=["a(x)", "b(x)"], rules=[
        R("STAR", [("s(q?)", Z)], ["a(q?)"], [1.0]),
        R("STAR", [("s(q?)", (1, 0, 0))], ["b(q?)"], [1.0]),
        R("STAR", [("q?", Z), ("q?", (0, 1, 0))], ["s(q?)"], [0.5, 0.5]),
    ])
    c = H.chain_infer(spec)
    c.plan((8, 8))
    outs = [r["out"][0] for r in c.plan_json()["rules"]]
    assert outs == ["s(x)", "a(x)", "b(x)"]


def test_multi_output_rule_binds_every_output():
    """EULER_FLUX has four outputs; deriving one instantiates all four."""
    gst = ["gr(q?)", "gun(q?)", "gut(q?)", "gp(q?)"]
    spec = H.ChainSpec(ndim=2, axioms=[("s", 2)], goals=["fE(s)", "fr(s)"], rules=[
        R("EULER_FLUX", [(g, Z) for g in gst], ["fr(q?)", "fmn(q?)", "fmt(q?)", "fE(q?)"], [1.4]),
        R("STAR", [("q?", Z)], ["gr(q?)"], [1.0]), R("STAR", [("q?", Z)], ["gun(q?)"], [0.1]),
        R("STAR", [("q?", Z)], ["gut(q?)"], [0.2]), R("STAR", [("q?", Z)], ["gp(q?)"], [1.0]),
    ])
    c = H.chain_infer(spec)
    c.plan((8, 8))
    rules = c.plan_json()["rules"]
    assert sum(r["op"] == H.OP["EULER_FLUX"] for r in rules) == 1
    assert rules[-1]["out"] == ["fr(s)", "fmn(s)", "fmt(s)", "fE(s)"]


@pytest.mark.parametrize("rules,axioms,goals,code", [
    # nothing derives the goal
    ([R("STAR", [("q?", Z)], ["f(q?)"], [1.0])], ["x"], ["g(x)"], H.EUNSAT),
    # endless recursion f(x) <- f(f(x)) <- ... stops at the depth bound
    ([R("STAR", [("f(q?)", Z)], ["f(q?)"], [1.0])], ["x"], ["f(x)"], H.EUNSAT),
    ([R("STAR", [("f(f(q?))", Z)], ["f(q?)"], [1.0])], ["x"], ["f(x)"], H.EUNSAT),
    # malformed patterns and variable scoping
    ([R("STAR", [("q??", Z)], ["f(q?)"], [1.0])], ["x"], ["f(x)"], H.EINVAL),
    ([R("STAR", [("q?", Z)], ["f(q?r?)"], [1.0])], ["x"], ["f(x)"], H.EINVAL),
    ([R("STAR", [("r?", Z)], ["f(q?)"], [1.0])], ["x"], ["f(x)"], H.EINVAL),
    ([R("EULER_FLUX", [("q?", Z)] * 4, ["a(q?)", "b(r?)", "c(q?)", "d(q?)"], [1.4])], ["x"], ["a(x)"], H.EINVAL),
    # goals and axioms must be concrete
    ([R("STAR", [("q?", Z)], ["f(q?)"], [1.0])], ["x"], ["f(q?)"], H.EINVAL),
    ([R("STAR", [("q?", Z)], ["f(q?)"], [1.0])], ["x?"], ["f(x)"], H.EINVAL),
])
def test_inference_errors(rules, axioms, goals, code):
    spec = H.ChainSpec(ndim=2, axioms=[(a, 2) for a in axioms], goals=goals, rules=rules)
    with pytest.raises(H.HfavError) as e:
        H.chain_infer(spec)
    assert e.value.code == code


def test_variable_matches_balanced_subterms_only():
    """q? binds a balanced subterm: "pair(q?,r?)" splits "pair(f(a,b),c)"
    at the top-level comma only."""
    spec = H.ChainSpec(ndim=2, axioms=[("c", 2), ("f(a,b)", 2)], goals=["pair(f(a,b),c)"], rules=[
        R("AXPY", [("q?", Z), ("r?", Z)], ["pair(q?,r?)"], [1.0])])
    c = H.chain_infer(spec)
    c.plan((8, 8))
    r = c.plan_json()["rules"][0]
    assert r["binding"] == "q?=f(a,b),r?=c"


@pytest.mark.parametrize("direction", [0, 1])
def test_godunov_sweep_inferred_matches_the_sweep_family(direction):
    """The sweep written once for any state s?: inference instantiates the
    six multi-output rules for s? = s and the planner recognises the fused
    sweep, as for the hand-written chain."""
    a = H.chain_infer(sweep_patterns(direction))
    b = H.Chain(H.euler_sweep_spec(direction, dt_source="dt"))
    ia, ib = a.plan((256, 128)), b.plan((256, 128))
    assert ia.family == ib.family == (2 if direction == 0 else 3) and ia.fused
    assert ia.n_rules == ib.n_rules == 6 and ia.n_nests == ib.n_nests == 1
    assert all(r["binding"] == "s?=s" for r in a.plan_json()["rules"])
    assert ia.bytes_per_cell_unfused == ib.bytes_per_cell_unfused
