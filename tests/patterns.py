"""Rule patterns (pattern variables "q?", "s?") for the inference tests:
the biharmonic update, the normalisation chain and one Godunov sweep, each
written once for any field or state and instantiated by hfav_chain_infer."""
from paper_1710_08774_amd import hfav as H

Z = (0, 0, 0)
R = H.Rule


def lap7_pattern(out="lap(q?)"):
    refs = [("q?", o) for o in (Z, (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))]
    return R("LAP7", refs, [out])


def biharm_patterns(nu=1.0 / 128.0, dtype=H.F64):
    """update(u) = u - nu lap(lap(u))."""
    return H.ChainSpec(ndim=3, dtype=dtype, axioms=[("u", 3)], goals=["update(u)"], rules=[
        R("AXPY", [("q?", Z), ("lap(lap(q?))", Z)], ["update(q?)"], [-nu]),
        lap7_pattern(),
    ])


def norm_patterns(nq=4, c=1.0, dtype=H.F64, with_norm=False):
    us = [f"u{q}" for q in range(nq)]
    return H.ChainSpec(ndim=2, dtype=dtype, axioms=[(u, 2) for u in us],
                       goals=[f"normalize({u})" for u in us] + (["norm"] if with_norm else []), rules=[
        R("AXPY", [("q?", Z), ("dir(q?)", Z)], ["normalize(q?)"], [-c]),
        R("DIV0", [("flux(q?)", Z), ("norm", Z)], ["dir(q?)"]),
        R("STAR", [("q?", (1, 0, 0)), ("q?", Z)], ["flux(q?)"], [1.0, -1.0]),
        R("SQRT", [("rowsum", Z)], ["norm"]),
        R("SUM_I", [("sumsq", Z)], ["rowsum"], reduce=H.REDUCE_SUM),
        R("SUMSQ", [(f"flux({u})", Z) for u in us], ["sumsq"]),
    ])


FIELDS = ("rho", "mx", "my", "E")


def sweep_patterns(direction=0, gamma=1.4, niter=10):
    """One Godunov sweep of any state s?: its conserved fields are rho(s?),
    mx(s?), my(s?), E(s?), the swept state is xsweep(s?) (or ysweep(s?)),
    dt a 0-D axiom.  Goals: the four fields of the swept state "s"."""
    e = (1, 0, 0) if direction == 0 else (0, 1, 0)
    me = tuple(-x for x in e)
    sw = "xsweep" if direction == 0 else "ysweep"
    cons = [f"{f}(s?)" for f in FIELDS]
    mn, mt = (cons[1], cons[2]) if direction == 0 else (cons[2], cons[1])
    prim = [f"{w}(s?)" for w in ("r", "un", "ut", "p", "c")]
    slopes = [f"d{w}(s?)" for w in ("r", "un", "ut", "p")]
    plus = [f"fp{w}(s?)" for w in ("r", "un", "ut", "p")]
    minus = [f"fm{w}(s?)" for w in ("r", "un", "ut", "p")]
    gst = [f"g{w}(s?)" for w in ("r", "un", "ut", "p")]
    flx = [f"F{w}(s?)" for w in ("r", "mn", "mt", "E")]
    new = [f"{f}({sw}(s?))" for f in FIELDS]
    gmn, gmt = (new[1], new[2]) if direction == 0 else (new[2], new[1])
    rules = [
        R("EULER_UPDATE", [(cons[0], Z), (mn, Z), (mt, Z), (cons[3], Z)] + [(f, Z) for f in flx] +
          [(f, me) for f in flx] + [("dt", Z)], [new[0], gmn, gmt, new[3]]),
        R("EULER_FLUX", [(w, Z) for w in gst], flx, [gamma]),
        R("EULER_RIEMANN", [(w, Z) for w in plus] + [(w, e) for w in minus], gst, [gamma, niter]),
        R("EULER_TRACE", [(w, Z) for w in prim] + [(d, Z) for d in slopes] + [("dt", Z)], plus + minus),
        R("EULER_SLOPE", [(w, o) for w in prim[:4] for o in (me, Z, e)], slopes),
        R("EULER_PRIM", [(cons[0], Z), (mn, Z), (mt, Z), (cons[3], Z)], prim, [gamma]),
    ]
    axioms = [(f"{f}(s)", 2) for f in FIELDS] + [("dt", 0)]
    goals = [f"{f}({sw}(s))" for f in FIELDS]
    return H.ChainSpec(ndim=2, axioms=axioms, goals=goals, rules=rules)
