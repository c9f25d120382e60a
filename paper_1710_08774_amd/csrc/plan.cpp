// Planner: iteration nests, fusion, extents, contraction, kernel family.
//
//  * one perfect iteration nest per rule call site, of the rule's rank
//    (Design, "Iteration nests"; call sites are already grouped per rule);
//  * fuse_inest_dag: walk the nests in topological order keeping a "fusing"
//    nest; a nest that cannot be fused splits the DAG and starts a new one
//    (Design, "Fusing the iteration nest DAG");
//  * fuse_inest: equal ranks fuse phase by phase under the four dataflow
//    ordering checks; a lower-rank nest goes into the prologue (broadcast) or
//    the epilogue (after the steady state) of the higher one, otherwise it is
//    unfusable (Design, "Fusing iteration nests", "Reductions & broadcasts &
//    splits");
//  * extents of every grid term are Minkowski sums of the offsets through
//    which the goals reach it (Design, "Variables and storage");
//  * the window of an intermediate is the span of its extent along the
//    outermost axis in which it varies: slabs of that axis ("outer"
//    rotation) or elements when only the innermost axis varies ("inner"
//    rotation) (Design, "Contraction").
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <sstream>
#include <string>

#include "internal.h"
#include "kernels.h"

namespace {

struct Reach {
    int n;
    std::vector<char> m;   // m[a*n+b]: rule b depends on rule a (path a -> b)
    bool path(int a, int b) const { return m[(size_t)a * n + b] != 0; }
};

Reach reachability(const hfav_chain *c) {
    const int n = (int)c->rules.size();
    Reach R{n, std::vector<char>((size_t)n * n, 0)};
    // direct edges producer -> consumer, then closure in topological order
    for (int pos = (int)c->topo.size() - 1; pos >= 0; --pos) {
        int a = c->topo[pos];
        for (int b : c->topo) {
            if (b == a) continue;
            bool direct = false;
            for (const HRef &ref : c->rules[b].in)
                if (c->terms[ref.term].producer == a) direct = true;
            if (direct) {
                R.m[(size_t)a * n + b] = 1;
                for (int x = 0; x < n; ++x)
                    if (R.m[(size_t)b * n + x]) R.m[(size_t)a * n + x] = 1;
            }
        }
    }
    return R;
}

// (R <= S | D): every rule of R can be ordered before every rule of S,
// i.e. no rule of S reaches a rule of R.
bool dataflow_le(const Reach &D, const std::vector<int> &R, const std::vector<int> &S) {
    for (int s : S)
        for (int r : R)
            if (s == r || D.path(s, r)) return false;
    return true;
}

std::vector<int> all_phases(const HNest &N) {
    std::vector<int> v = N.prologue;
    v.insert(v.end(), N.steady.begin(), N.steady.end());
    v.insert(v.end(), N.epilogue.begin(), N.epilogue.end());
    return v;
}

void append(std::vector<int> &a, const std::vector<int> &b) { a.insert(a.end(), b.begin(), b.end()); }

// Returns false when the pair is unfusable.
bool fuse_inest(const Reach &D, const HNest &A, const HNest &B, HNest &out) {
    if (A.rank == B.rank) {
        if (dataflow_le(D, A.prologue, B.steady) && dataflow_le(D, B.prologue, A.steady) &&
            dataflow_le(D, A.steady, B.epilogue) && dataflow_le(D, B.steady, A.epilogue)) {
            out.rank = A.rank;
            out.prologue = A.prologue; append(out.prologue, B.prologue);
            out.steady = A.steady; append(out.steady, B.steady);
            out.epilogue = A.epilogue; append(out.epilogue, B.epilogue);
            return true;
        }
        return false;
    }
    const HNest &lo = A.rank < B.rank ? A : B;
    const HNest &hi = A.rank < B.rank ? B : A;
    const std::vector<int> lo_all = all_phases(lo);
    std::vector<int> hi_body = hi.steady;
    append(hi_body, hi.epilogue);
    std::vector<int> hi_head = hi.prologue;
    append(hi_head, hi.steady);
    const bool before = dataflow_le(D, lo_all, hi_body);
    const bool after = dataflow_le(D, hi_head, lo_all);
    out = hi;
    // inside the phase that receives it, the lower nest goes ahead of the
    // prologue's own rules and after the epilogue's, unless the dataflow
    // between them asks for the other order
    auto merge = [&](const std::vector<int> &phase, bool lo_first, std::vector<int> &dst) {
        const bool lo_before = dataflow_le(D, lo_all, phase), lo_after = dataflow_le(D, phase, lo_all);
        if (!lo_before && !lo_after) return false;
        if (lo_before && (lo_first || !lo_after)) {
            dst = lo_all;
            append(dst, phase);
        } else {
            dst = phase;
            append(dst, lo_all);
        }
        return true;
    };
    if (before && merge(hi.prologue, true, out.prologue)) return true;    // broadcast: prologue
    if (after && merge(hi.epilogue, false, out.epilogue)) return true;    // after the steady state: epilogue
    out = HNest{};
    return false;
}

// fuse_inest_dag: walk the nests in the given (topological) order keeping
// one fusing nest; a nest that cannot join it closes it and starts the next
std::vector<HNest> fuse_inest_dag(const Reach &D, const std::vector<HNest> &initial) {
    std::vector<HNest> nests;
    if (initial.empty()) return nests;
    HNest cur = initial[0];
    for (size_t q = 1; q < initial.size(); ++q) {
        HNest fused;
        if (fuse_inest(D, cur, initial[q], fused)) cur = fused;
        else {                          // split: close the fusing nest
            nests.push_back(cur);
            cur = initial[q];
        }
    }
    nests.push_back(cur);
    return nests;
}

int phase_of(const HNest &N, int r) {
    if (std::find(N.prologue.begin(), N.prologue.end(), r) != N.prologue.end()) return 0;
    if (std::find(N.steady.begin(), N.steady.end(), r) != N.steady.end()) return 1;
    return 2;
}

const char *storage_name(int s) {
    switch (s) {
    case HFAV_STORE_FULL: return "full";
    case HFAV_STORE_REGISTER: return "register";
    case HFAV_STORE_INNER: return "inner";
    case HFAV_STORE_OUTER: return "outer";
    default: return "scalar";
    }
}

// ------------------------------------------------------------ family match
// Reference checks used by the matchers.
bool ref_is(const hfav_chain *c, const HRef &r, int term, int di, int dj, int dk) {
    return r.term == term && r.off[0] == di && r.off[1] == dj && r.off[2] == dk;
}
int prod_out(const hfav_chain *c, int rule, int pos) { return c->rules[rule].out[pos]; }

std::vector<int> live_rules(const hfav_chain *c) { return c->topo; }

int find_op(const hfav_chain *c, int op) {
    int found = -1;
    for (int r : c->topo)
        if (c->rules[r].op == op) {
            if (found >= 0) return -2;   // more than one
            found = r;
        }
    return found;
}

bool is_inter(const hfav_chain *c, int t) { return c->terms[t].kind == TK_INTER; }

bool match_hdiff(const hfav_chain *c, HPlan &p) {
    if (c->topo.size() != 4) return false;
    int rl = find_op(c, HFAV_OP_HDIFF_LAP), rx = find_op(c, HFAV_OP_HDIFF_FLX);
    int ry = find_op(c, HFAV_OP_HDIFF_FLY), ro = find_op(c, HFAV_OP_HDIFF_OUT);
    if (rl < 0 || rx < 0 || ry < 0 || ro < 0) return false;
    const HRule &L = c->rules[rl], &X = c->rules[rx], &Y = c->rules[ry], &O = c->rules[ro];
    const int u = L.in[0].term, lap = L.out[0], flx = X.out[0], fly = Y.out[0];
    if (c->terms[u].kind != TK_AXIOM || c->terms[u].rank != c->ndim) return false;
    if (!is_inter(c, lap) || !is_inter(c, flx) || !is_inter(c, fly)) return false;
    if (!(ref_is(c, L.in[0], u, 0, 0, 0) && ref_is(c, L.in[1], u, 1, 0, 0) && ref_is(c, L.in[2], u, -1, 0, 0) &&
          ref_is(c, L.in[3], u, 0, 1, 0) && ref_is(c, L.in[4], u, 0, -1, 0)))
        return false;
    if (!(ref_is(c, X.in[0], lap, 0, 0, 0) && ref_is(c, X.in[1], lap, 1, 0, 0) && ref_is(c, X.in[2], u, 0, 0, 0) &&
          ref_is(c, X.in[3], u, 1, 0, 0)))
        return false;
    if (!(ref_is(c, Y.in[0], lap, 0, 0, 0) && ref_is(c, Y.in[1], lap, 0, 1, 0) && ref_is(c, Y.in[2], u, 0, 0, 0) &&
          ref_is(c, Y.in[3], u, 0, 1, 0)))
        return false;
    if (!(ref_is(c, O.in[0], u, 0, 0, 0) && ref_is(c, O.in[1], flx, 0, 0, 0) && ref_is(c, O.in[2], flx, -1, 0, 0) &&
          ref_is(c, O.in[3], fly, 0, 0, 0) && ref_is(c, O.in[4], fly, 0, -1, 0)))
        return false;
    if (c->goals.size() != 1 || c->goals[0] != O.out[0]) return false;
    if (p.opts.boundary[0] != HFAV_BC_PERIODIC || p.opts.boundary[1] != HFAV_BC_PERIODIC) return false;
    p.fam_in = {u};
    p.fam_out = {O.out[0]};
    p.fam_param = {O.param[0]};
    return true;
}

// The rules of one directional Godunov sweep (prim, slope, trace, Riemann,
// flux, update) wired as the sweep computes: the direction d from the slope
// stencil, dt the 0-D term the trace and the update read.  The prim inputs
// are grid terms at offset 0 (axioms or another sweep's outputs).
bool sweep_ok(const hfav_chain *c, int rp, int rs, int rt, int rr, int rf, int ru, int &d, int &dt) {
    const HRule &P = c->rules[rp], &S = c->rules[rs], &T = c->rules[rt], &R = c->rules[rr];
    const HRule &F = c->rules[rf], &U = c->rules[ru];
    d = -1;
    for (int ax = 0; ax < 2; ++ax)
        if (S.in[2].off[ax] == 1) d = ax;
    if (d < 0) return false;
    int e[3] = {0, 0, 0};
    e[d] = 1;
    for (int q = 0; q < 4; ++q)
        if (c->terms[P.in[q].term].rank != 2 || !ref_is(c, P.in[q], P.in[q].term, 0, 0, 0)) return false;
    for (int q = 0; q < 4; ++q) {
        int w = P.out[q];
        if (!(ref_is(c, S.in[3 * q], w, -e[0], -e[1], 0) && ref_is(c, S.in[3 * q + 1], w, 0, 0, 0) &&
              ref_is(c, S.in[3 * q + 2], w, e[0], e[1], 0)))
            return false;
    }
    for (int q = 0; q < 5; ++q)
        if (!ref_is(c, T.in[q], P.out[q], 0, 0, 0)) return false;
    for (int q = 0; q < 4; ++q)
        if (!ref_is(c, T.in[5 + q], S.out[q], 0, 0, 0)) return false;
    dt = T.in[9].term;
    for (int q = 0; q < 4; ++q) {
        if (!ref_is(c, R.in[q], T.out[q], 0, 0, 0)) return false;
        if (!ref_is(c, R.in[4 + q], T.out[4 + q], e[0], e[1], 0)) return false;
        if (!ref_is(c, F.in[q], R.out[q], 0, 0, 0)) return false;
        if (!ref_is(c, U.in[q], P.in[q].term, 0, 0, 0)) return false;
        if (!ref_is(c, U.in[4 + q], F.out[q], 0, 0, 0)) return false;
        if (!ref_is(c, U.in[8 + q], F.out[q], -e[0], -e[1], 0)) return false;
    }
    if (U.in[12].term != dt) return false;
    const double g = P.param[0];
    if (R.param[0] != g || F.param[0] != g) return false;
    if (R.param[1] < 0 || R.param[1] > 64 || R.param[1] != (double)(int)R.param[1]) return false;
    for (int r : {rp, rs, rt, rr, rf})
        for (int t : c->rules[r].out)
            if (!is_inter(c, t)) return false;
    return true;
}

// dt of a sweep family: a 0-D axiom, or a 0-D rule cfl/smax of an axiom
bool sweep_dt(const hfav_chain *c, HPlan &p, int dt, int rd) {
    if (rd >= 0) {
        const HRule &Dr = c->rules[rd];
        if (Dr.out[0] != dt || c->terms[Dr.in[0].term].kind != TK_AXIOM) return false;
        p.fam_dt_term = Dr.in[0].term;
        p.fam_dt_mode = 1;
        p.fam_cfl = Dr.param[0];
        return true;
    }
    if (c->terms[dt].kind != TK_AXIOM) return false;
    p.fam_dt_term = dt;
    p.fam_dt_mode = 0;
    return true;
}

// Directionally split Godunov sweep along axis d.
bool match_euler(const hfav_chain *c, HPlan &p, int &dir) {
    if (c->ndim != 2) return false;
    int rp = find_op(c, HFAV_OP_EULER_PRIM), rs = find_op(c, HFAV_OP_EULER_SLOPE);
    int rt = find_op(c, HFAV_OP_EULER_TRACE), rr = find_op(c, HFAV_OP_EULER_RIEMANN);
    int rf = find_op(c, HFAV_OP_EULER_FLUX), ru = find_op(c, HFAV_OP_EULER_UPDATE);
    int rm = find_op(c, HFAV_OP_EULER_SMAX), rd = find_op(c, HFAV_OP_EULER_DT);
    if (rp < 0 || rs < 0 || rt < 0 || rr < 0 || rf < 0 || ru < 0 || rm == -2 || rd == -2) return false;
    size_t expect = 6 + (rm >= 0) + (rd >= 0);
    if (c->topo.size() != expect) return false;
    const HRule &P = c->rules[rp], &R = c->rules[rr], &U = c->rules[ru];
    int d = -1, dt = -1;
    if (!sweep_ok(c, rp, rs, rt, rr, rf, ru, d, dt)) return false;
    for (int q = 0; q < 4; ++q)
        if (c->terms[P.in[q].term].kind != TK_AXIOM) return false;
    const double g = P.param[0];
    // dt: an axiom, or a 0-D rule from an smax axiom
    if (!sweep_dt(c, p, dt, rd)) return false;
    // goals are the 4 updated fields
    for (int q = 0; q < 4; ++q)
        if (c->terms[U.out[q]].kind != TK_GOAL) return false;
    p.fam_smax_goal = -1;
    if (rm >= 0) {
        const HRule &M = c->rules[rm];
        if (M.param[0] != g) return false;
        const bool ok0 = ref_is(c, M.in[0], U.out[0], 0, 0, 0) && ref_is(c, M.in[3], U.out[3], 0, 0, 0);
        const bool ok12 = (ref_is(c, M.in[1], U.out[1], 0, 0, 0) && ref_is(c, M.in[2], U.out[2], 0, 0, 0)) ||
                          (ref_is(c, M.in[1], U.out[2], 0, 0, 0) && ref_is(c, M.in[2], U.out[1], 0, 0, 0));
        if (!ok0 || !ok12 || c->terms[M.out[0]].kind != TK_GOAL) return false;
        p.fam_smax_goal = M.out[0];
    }
    if (c->goals.size() != 4u + (rm >= 0)) return false;
    p.fam_in = {P.in[0].term, P.in[1].term, P.in[2].term, P.in[3].term};
    p.fam_out = {U.out[0], U.out[1], U.out[2], U.out[3]};
    p.fam_param = {g, R.param[1]};
    dir = d;
    return true;
}

// Both sweeps of a time step: an x sweep of the axioms (rho, mx, my, E)
// whose updated state, in the y frame (rho, my, mx, E), feeds a y sweep with
// the same dt, gamma and Newton count; the x-swept state stays an
// intermediate.  Optional CFL reduction of the new state as a 0-D goal.
bool match_euler_xy(const hfav_chain *c, HPlan &p) {
    if (c->ndim != 2) return false;
    static const int ops[6] = {HFAV_OP_EULER_PRIM, HFAV_OP_EULER_SLOPE, HFAV_OP_EULER_TRACE,
                               HFAV_OP_EULER_RIEMANN, HFAV_OP_EULER_FLUX, HFAV_OP_EULER_UPDATE};
    std::vector<int> by[6];
    int rd = -1, rm = -1, other = 0;
    for (int r : c->topo) {
        const int op = c->rules[r].op;
        int k = -1;
        for (int q = 0; q < 6; ++q)
            if (ops[q] == op) k = q;
        if (k >= 0) by[k].push_back(r);
        else if (op == HFAV_OP_EULER_DT && rd < 0) rd = r;
        else if (op == HFAV_OP_EULER_SMAX && rm < 0) rm = r;
        else ++other;
    }
    if (other) return false;
    for (int q = 0; q < 6; ++q)
        if (by[q].size() != 2) return false;
    // chain each sweep's rules from its prim rule by dataflow
    auto chain_from = [&](int rp, int *id) {
        id[0] = rp;
        auto find = [&](int k, int pos, int term) {
            for (int r : by[k])
                if (c->rules[r].in[pos].term == term) return r;
            return -1;
        };
        id[1] = find(1, 1, c->rules[rp].out[0]);
        id[2] = find(2, 0, c->rules[rp].out[0]);
        if (id[2] < 0) return false;
        id[3] = find(3, 0, c->rules[id[2]].out[0]);
        if (id[3] < 0) return false;
        id[4] = find(4, 0, c->rules[id[3]].out[0]);
        if (id[4] < 0) return false;
        id[5] = find(5, 4, c->rules[id[4]].out[0]);
        return id[1] >= 0 && id[5] >= 0;
    };
    int X[6], Y[6];
    int px = by[0][0], py = by[0][1];
    if (c->terms[c->rules[px].in[0].term].kind != TK_AXIOM) std::swap(px, py);
    if (!chain_from(px, X) || !chain_from(py, Y)) return false;
    int dx, dy, dtx, dty;
    if (!sweep_ok(c, X[0], X[1], X[2], X[3], X[4], X[5], dx, dtx) ||
        !sweep_ok(c, Y[0], Y[1], Y[2], Y[3], Y[4], Y[5], dy, dty))
        return false;
    if (dx != 0 || dy != 1 || dtx != dty) return false;
    const HRule &Px = c->rules[X[0]], &Ux = c->rules[X[5]], &Py = c->rules[Y[0]], &Uy = c->rules[Y[5]];
    for (int q = 0; q < 4; ++q)
        if (c->terms[Px.in[q].term].kind != TK_AXIOM || !is_inter(c, Ux.out[q])) return false;
    static const int yframe[4] = {0, 2, 1, 3};
    for (int q = 0; q < 4; ++q)
        if (Py.in[q].term != Ux.out[yframe[q]]) return false;
    const double g = Px.param[0];
    if (Py.param[0] != g || c->rules[X[3]].param[1] != c->rules[Y[3]].param[1]) return false;
    if (!sweep_dt(c, p, dtx, rd)) return false;
    for (int q = 0; q < 4; ++q)
        if (c->terms[Uy.out[q]].kind != TK_GOAL) return false;
    p.fam_smax_goal = -1;
    if (rm >= 0) {
        const HRule &M = c->rules[rm];
        if (M.param[0] != g || c->terms[M.out[0]].kind != TK_GOAL) return false;
        // physical order: rho, mx, my, E
        if (!(ref_is(c, M.in[0], Uy.out[0], 0, 0, 0) && ref_is(c, M.in[1], Uy.out[2], 0, 0, 0) &&
              ref_is(c, M.in[2], Uy.out[1], 0, 0, 0) && ref_is(c, M.in[3], Uy.out[3], 0, 0, 0)))
            return false;
        p.fam_smax_goal = M.out[0];
    }
    if (c->goals.size() != 4u + (rm >= 0)) return false;
    for (int ax = 0; ax < 2; ++ax)
        if (p.opts.boundary[ax] != HFAV_BC_PERIODIC && p.opts.boundary[ax] != HFAV_BC_TRANSMISSIVE) return false;
    p.fam_in = {Px.in[0].term, Px.in[1].term, Px.in[2].term, Px.in[3].term};
    p.fam_out = {Uy.out[0], Uy.out[2], Uy.out[1], Uy.out[3]};
    p.fam_param = {g, c->rules[Y[3]].param[1]};
    return true;
}

bool match_smax(const hfav_chain *c, HPlan &p) {
    if (c->topo.size() != 1) return false;
    const HRule &M = c->rules[c->topo[0]];
    if (M.op != HFAV_OP_EULER_SMAX || c->ndim != 2) return false;
    for (int q = 0; q < 4; ++q)
        if (c->terms[M.in[q].term].kind != TK_AXIOM || !ref_is(c, M.in[q], M.in[q].term, 0, 0, 0)) return false;
    p.fam_in = {M.in[0].term, M.in[1].term, M.in[2].term, M.in[3].term};
    p.fam_out = {M.out[0]};
    p.fam_param = {M.param[0]};
    return true;
}

bool match_lap7_chain(const hfav_chain *c, HPlan &p) {
    if (c->ndim != 3 || c->topo.size() != 3) return false;
    const HRule &A = c->rules[c->topo[0]], &B = c->rules[c->topo[1]], &X = c->rules[c->topo[2]];
    if (A.op != HFAV_OP_LAP7 || B.op != HFAV_OP_LAP7 || X.op != HFAV_OP_AXPY) return false;
    const int u = A.in[0].term, l1 = A.out[0], l2 = B.out[0];
    if (c->terms[u].kind != TK_AXIOM || !is_inter(c, l1) || !is_inter(c, l2)) return false;
    auto lap_ok = [&](const HRule &Rl, int src) {
        return ref_is(c, Rl.in[0], src, 0, 0, 0) && ref_is(c, Rl.in[1], src, 1, 0, 0) &&
               ref_is(c, Rl.in[2], src, -1, 0, 0) && ref_is(c, Rl.in[3], src, 0, 1, 0) &&
               ref_is(c, Rl.in[4], src, 0, -1, 0) && ref_is(c, Rl.in[5], src, 0, 0, 1) &&
               ref_is(c, Rl.in[6], src, 0, 0, -1);
    };
    if (!lap_ok(A, u) || !lap_ok(B, l1)) return false;
    if (!ref_is(c, X.in[0], u, 0, 0, 0) || !ref_is(c, X.in[1], l2, 0, 0, 0)) return false;
    if (c->goals.size() != 1 || c->goals[0] != X.out[0]) return false;
    for (int ax = 0; ax < 3; ++ax)
        if (p.opts.boundary[ax] != HFAV_BC_PERIODIC) return false;
    p.fam_in = {u};
    p.fam_out = {X.out[0]};
    p.fam_param = {X.param[0]};
    return true;
}

// Normalisation chain (Performance, "Normalization Example"): per field q
// a flux f_q = STAR(u_q(0), u_q(+i)), e = SUMSQ(f_0 .. f_{nq-1}),
// s = SUM_I(e), n = SQRT(s), d_q = DIV0(f_q, n), out_q = AXPY(u_q, d_q).
// Family parameters per field: coefficient of u(0), of u(+i), the AXPY
// factor.  Fields are numbered in the SUMSQ reference order.
bool match_norm(const hfav_chain *c, HPlan &p) {
    const int nd = c->ndim;
    if (c->order[nd - 1] != 0) return false;
    // one workgroup per row: the row count must fit a launch
    if ((int64_t)p.opts.dims[1] * p.opts.dims[2] >= ((int64_t)1 << 31)) return false;
    if (p.opts.boundary[0] != HFAV_BC_PERIODIC && p.opts.boundary[0] != HFAV_BC_TRANSMISSIVE) return false;
    const int rsq = find_op(c, HFAV_OP_SUMSQ), rsu = find_op(c, HFAV_OP_SUM_I), rrt = find_op(c, HFAV_OP_SQRT);
    if (rsq < 0 || rsu < 0 || rrt < 0) return false;
    const HRule &SQ = c->rules[rsq], &SU = c->rules[rsu], &RT = c->rules[rrt];
    const int nq = (int)SQ.in.size();
    if (nq < 1 || nq > 8 || c->topo.size() != (size_t)(3 + 3 * nq)) return false;
    const int e = SQ.out[0], s = SU.out[0], n = RT.out[0];
    if (!is_inter(c, e) || !is_inter(c, s) || c->terms[s].rank != nd - 1) return false;
    if (SU.in[0].term != e || RT.in[0].term != s) return false;
    if (c->terms[n].kind == TK_GOAL) {
        if (c->goals.size() != (size_t)nq + 1) return false;
    } else if (c->goals.size() != (size_t)nq) {
        return false;
    }
    std::vector<int> u(nq), out(nq), used;
    std::vector<double> prm;
    for (int q = 0; q < nq; ++q) {
        const HRef &fr = SQ.in[q];
        const int f = fr.term;
        if (!ref_is(c, fr, f, 0, 0, 0) || !is_inter(c, f) || c->terms[f].rank != nd) return false;
        for (int g = 0; g < q; ++g)
            if (SQ.in[g].term == f) return false;
        const HRule &F = c->rules[c->terms[f].producer];
        if (F.op != HFAV_OP_STAR || F.in.size() != 2) return false;
        const int uq = F.in[0].term;
        if (c->terms[uq].kind != TK_AXIOM || c->terms[uq].rank != nd || F.in[1].term != uq) return false;
        double c0 = 0.0, cp = 0.0;
        bool have0 = false, havep = false;
        for (int k = 0; k < 2; ++k) {
            if (ref_is(c, F.in[k], uq, 0, 0, 0) && !have0) { c0 = F.param[k]; have0 = true; }
            else if (ref_is(c, F.in[k], uq, 1, 0, 0) && !havep) { cp = F.param[k]; havep = true; }
            else return false;
        }
        // the DIV0 and AXPY rules of this field
        int rd = -1, ra = -1;
        for (int r : c->topo) {
            const HRule &R = c->rules[r];
            if (R.op == HFAV_OP_DIV0 && R.in[0].term == f) {
                if (rd >= 0 || !ref_is(c, R.in[0], f, 0, 0, 0) || R.in[1].term != n) return false;
                rd = r;
            }
        }
        if (rd < 0 || !is_inter(c, c->rules[rd].out[0])) return false;
        const int d = c->rules[rd].out[0];
        for (int r : c->topo) {
            const HRule &R = c->rules[r];
            if (R.op == HFAV_OP_AXPY && R.in[1].term == d) {
                if (ra >= 0 || !ref_is(c, R.in[0], uq, 0, 0, 0) || !ref_is(c, R.in[1], d, 0, 0, 0)) return false;
                ra = r;
            }
        }
        if (ra < 0 || c->terms[c->rules[ra].out[0]].kind != TK_GOAL) return false;
        for (int r : {c->terms[f].producer, rd, ra}) {
            if (std::find(used.begin(), used.end(), r) != used.end()) return false;
            used.push_back(r);
        }
        u[q] = uq;
        out[q] = c->rules[ra].out[0];
        prm.push_back(c0);
        prm.push_back(cp);
        prm.push_back(c->rules[ra].param[0]);
    }
    p.fam_in = u;
    p.fam_out = out;
    p.fam_param = prm;
    p.fam_row_goal = c->terms[n].kind == TK_GOAL ? n : -1;
    return true;
}

size_t esize(int dtype) { return dtype == HFAV_F64 ? 8 : 4; }

void json_int3(std::ostringstream &o, const int *v) { o << "[" << v[0] << "," << v[1] << "," << v[2] << "]"; }

// a name as a JSON string (quotes, backslashes and control characters escaped)
std::string jstr(const std::string &s) {
    std::string o = "\"";
    for (char ch : s) {
        if (ch == '"' || ch == '\\') { o += '\\'; o += ch; }
        else if ((unsigned char)ch < 0x20) { char b[8]; snprintf(b, sizeof b, "\\u%04x", ch); o += b; }
        else o += ch;
    }
    return o + "\"";
}

}  // namespace

static bool star_ref_is(const hfav_chain *c, const HRef &r, int term, int di, int dj, int dk) {
    (void)c;
    return r.term == term && r.off[0] == di && r.off[1] == dj && r.off[2] == dk;
}

// Layered chain of STAR rules: stage k's rules each read every field of
// stage k-1 through the same star stencil of radius r_k, in the canonical
// offset order (centre, then -d, +d for d = 1..r along x, y, z).
bool match_star_chain(const hfav_chain *c, HPlan &p) {
    if (c->topo.empty()) return false;
    for (int r : c->topo)
        if (c->rules[r].op != HFAV_OP_STAR) return false;
    for (int ax = 0; ax < c->ndim; ++ax)
        if (p.opts.boundary[ax] != HFAV_BC_PERIODIC) return false;
    const int nd = c->ndim;
    std::vector<int> depth(c->rules.size(), -1);
    int K = 0;
    for (int r : c->topo) {
        int d = 1;
        for (const HRef &ref : c->rules[r].in) {
            const int pr = c->terms[ref.term].producer;
            if (pr >= 0) d = std::max(d, depth[pr] + 1);
        }
        depth[r] = d;
        K = std::max(K, d);
    }
    if (K > 6) return false;
    // rules of each stage, in descriptor order
    std::vector<std::vector<int>> stage_rules(K + 1);
    for (int r = 0; r < (int)c->rules.size(); ++r)
        if (c->live[r]) stage_rules[depth[r]].push_back(r);
    p.sstages.assign(K, HPlan::StarStage{});
    // field order of stage k-1 = order of first appearance in stage k's first rule
    std::vector<std::vector<int>> fields(K + 1);
    for (int k = 1; k <= K; ++k) {
        const HRule &R0 = c->rules[stage_rules[k][0]];
        std::vector<int> order;
        for (const HRef &ref : R0.in)
            if (std::find(order.begin(), order.end(), ref.term) == order.end()) order.push_back(ref.term);
        fields[k - 1] = order;
    }
    // last stage outputs: rule order
    for (int r : stage_rules[K]) fields[K].push_back(c->rules[r].out[0]);
    for (int k = 0; k <= K; ++k)
        if (fields[k].empty() || fields[k].size() > 5) return false;
    // stage 0 fields are axioms; stage k fields are exactly stage k's outputs
    for (int t : fields[0])
        if (c->terms[t].kind != TK_AXIOM || c->terms[t].rank != nd) return false;
    for (int k = 1; k <= K; ++k) {
        if (fields[k].size() != stage_rules[k].size()) return false;
        for (int t : fields[k]) {
            const int pr = c->terms[t].producer;
            if (pr < 0 || depth[pr] != k) return false;
            if (k < K && c->terms[t].kind != TK_INTER) return false;
            if (k == K && c->terms[t].kind != TK_GOAL) return false;
        }
    }
    if (c->goals.size() != fields[K].size()) return false;
    p.scoeff.clear();
    p.scoff.clear();
    for (int k = 1; k <= K; ++k) {
        const HRule &R0 = c->rules[stage_rules[k][0]];
        const int fin = (int)fields[k - 1].size();
        if ((int)R0.in.size() % fin) return false;
        const int n_off = (int)R0.in.size() / fin;
        const int r = (n_off - 1) / (2 * nd);
        if (r < 1 || r > 3 || 1 + 2 * r * nd != n_off) return false;
        HPlan::StarStage S;
        S.r = r;
        S.fin = fin;
        S.fout = (int)fields[k].size();
        S.in_terms = fields[k - 1];
        S.out_terms = fields[k];
        p.scoff.push_back((int)p.scoeff.size());
        for (int o = 0; o < S.fout; ++o) {
            const HRule &R = c->rules[c->terms[fields[k][o]].producer];
            if ((int)R.in.size() != fin * n_off) return false;
            for (int f = 0; f < fin; ++f) {
                int q = 0;
                auto expect = [&](int dx, int dy, int dz) {
                    const HRef &ref = R.in[f * n_off + q];
                    const bool ok = star_ref_is(c, ref, fields[k - 1][f], dx, dy, dz);
                    ++q;
                    return ok;
                };
                if (!expect(0, 0, 0)) return false;
                for (int ax = 0; ax < nd; ++ax)
                    for (int d = 1; d <= r; ++d) {
                        int m[3] = {0, 0, 0}, pl[3] = {0, 0, 0};
                        m[ax] = -d;
                        pl[ax] = d;
                        if (!expect(m[0], m[1], m[2]) || !expect(pl[0], pl[1], pl[2])) return false;
                    }
                for (int qq = 0; qq < n_off; ++qq) p.scoeff.push_back(R.param[f * n_off + qq]);
            }
        }
        p.sstages[k - 1] = S;
    }
    return true;
}

// LDS bytes of the group of stages [a, b) at a tile shape
size_t star_group_bytes(const hfav_chain *c, const HPlan &p, int a, int b, int tile) {
    hfav::StarGroupLaunch L{};
    L.nstage = b - a;
    L.nd = c->ndim;
    L.tile = tile;
    L.dtype = c->dtype;
    for (int s = a; s < b; ++s) {
        L.st[s - a].r = p.sstages[s].r;
        L.st[s - a].fin = p.sstages[s].fin;
        L.st[s - a].fout = p.sstages[s].fout;
    }
    return hfav::star_group_lds_bytes(L);
}

// split the stages into groups of at most D (D = 0: all); false if a group
// does not fit in LDS
bool star_groups(const hfav_chain *c, HPlan &p, int D, int tile) {
    const int K = (int)p.sstages.size();
    if (D <= 0 || D > K) D = K;
    p.sgroups.clear();
    for (int s = 0; s < K; s += D) {
        const int e = std::min(K, s + D);
        if (star_group_bytes(c, p, s, e, tile) > hfav::SG_MAX_LDS) return false;
        p.sgroups.push_back(s);
    }
    return true;
}


int hfav_plan_impl(hfav_chain *c, const hfav_plan_opts *o, hfav_plan_info *info) {
    if (!c || !o) return hfav_fail(HFAV_EINVAL, "null chain or options");
    HPlan p;
    p.opts = *o;
    const int nd = c->ndim;
    for (int ax = 0; ax < 3; ++ax) {
        if (o->dims[ax] < 1) return hfav_fail(HFAV_EINVAL, "dims must be >= 1");
        if (ax >= nd && o->dims[ax] != 1) return hfav_fail(HFAV_EINVAL, "dims beyond ndim must be 1");
        if (o->boundary[ax] != HFAV_BC_PERIODIC && o->boundary[ax] != HFAV_BC_TRANSMISSIVE)
            return hfav_fail(HFAV_EINVAL, "unknown boundary");
    }
    if ((int64_t)o->dims[0] * o->dims[1] * o->dims[2] > (int64_t)1 << 36)
        return hfav_fail(HFAV_EINVAL, "grid too large");
    if (o->mode < HFAV_MODE_AUTO || o->mode > HFAV_MODE_UNFUSED) return hfav_fail(HFAV_EINVAL, "unknown mode");
    if (o->precision != HFAV_PREC_NATIVE && o->precision != HFAV_PREC_F32_F64ACC)
        return hfav_fail(HFAV_EINVAL, "unknown precision");
    if (o->precision == HFAV_PREC_F32_F64ACC && c->dtype != HFAV_F32)
        return hfav_fail(HFAV_EUNSUP, "F32_F64ACC precision needs an F32 chain");
    const int64_t ncell = (int64_t)o->dims[0] * o->dims[1] * o->dims[2];

    // ---- nests and fusion
    const Reach D = reachability(c);
    std::vector<HNest> initial;
    for (int r : c->topo) {
        HNest n;
        n.rank = c->rules[r].rank;
        n.steady = {r};
        initial.push_back(n);
    }
    p.nests = fuse_inest_dag(D, initial);
    if ((int)p.nests.size() > HFAV_MAX_NESTS) return hfav_fail(HFAV_EUNSUP, "too many nests after fusion");

    // ---- Minkowski extents, backward from the goals
    const int nt = (int)c->terms.size();
    p.terms.assign(nt, HTermPlan{});
    for (HTermPlan &tp : p.terms) {
        tp.has_ext = false;
        tp.window_axis = -1;
        tp.window = 0;
        tp.storage = HFAV_STORE_FULL;
        for (int ax = 0; ax < 3; ++ax) tp.lo[ax] = tp.hi[ax] = 0;
    }
    auto widen = [&](int t, const int *lo_in, const int *hi_in) {
        HTermPlan &tp = p.terms[t];
        // a row term has no i axis: its extent along i is a single point
        int lo[3] = {lo_in[0], lo_in[1], lo_in[2]}, hi[3] = {hi_in[0], hi_in[1], hi_in[2]};
        if (c->terms[t].rank == nd - 1) lo[0] = hi[0] = 0;
        if (!tp.has_ext) {
            tp.has_ext = true;
            for (int ax = 0; ax < 3; ++ax) { tp.lo[ax] = lo[ax]; tp.hi[ax] = hi[ax]; }
        } else {
            for (int ax = 0; ax < 3; ++ax) {
                tp.lo[ax] = std::min(tp.lo[ax], lo[ax]);
                tp.hi[ax] = std::max(tp.hi[ax], hi[ax]);
            }
        }
    };
    const int zero[3] = {0, 0, 0};
    for (int t : c->goals)
        if (c->terms[t].rank > 0) widen(t, zero, zero);
    for (int pos = (int)c->topo.size() - 1; pos >= 0; --pos) {
        const int r = c->topo[pos];
        const HRule &R = c->rules[r];
        if (R.rank == 0) continue;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        bool any = false;
        if (R.reduce == HFAV_REDUCE_NONE) {
            for (int t : R.out) {
                const HTermPlan &tp = p.terms[t];
                if (!tp.has_ext) continue;
                for (int ax = 0; ax < 3; ++ax) {
                    lo[ax] = any ? std::min(lo[ax], tp.lo[ax]) : tp.lo[ax];
                    hi[ax] = any ? std::max(hi[ax], tp.hi[ax]) : tp.hi[ax];
                }
                any = true;
            }
        }
        if (!any) { for (int ax = 0; ax < 3; ++ax) lo[ax] = hi[ax] = 0; }
        for (const HRef &ref : R.in) {
            if (c->terms[ref.term].rank == 0) continue;
            int l2[3], h2[3];
            for (int ax = 0; ax < 3; ++ax) { l2[ax] = lo[ax] + ref.off[ax]; h2[ax] = hi[ax] + ref.off[ax]; }
            widen(ref.term, l2, h2);
        }
    }

    // ---- outer groups.  Fusion above works at the level of the innermost
    // axis; a split there (a reduction along i whose result a later rule
    // broadcasts back along i) need not split the loops outside it (Design,
    // "Fusing iteration nests": equal outer ranks fuse phase by phase, the
    // split happens inside).  Consecutive nests that iterate every outer
    // axis share one outer loop, each outer iteration running their inner
    // sweeps in order, when every term passed from an earlier nest of the
    // group to a later one is needed at the current outer point only: a
    // grid term whose extent is zero along every outer axis, or a row term.
    // A 0-D term (a reduction over the whole space) is complete only after
    // the last outer iteration and always ends the group.  i must be the
    // innermost axis.
    std::vector<int> nest_of(c->rules.size(), -1);
    for (size_t n = 0; n < p.nests.size(); ++n)
        for (int r : all_phases(p.nests[n])) nest_of[r] = (int)n;
    std::vector<int> outer(p.nests.size(), 0);
    {
        const bool i_inner = c->order[nd - 1] == 0;
        int g = 0;
        for (size_t n = 1; n < p.nests.size(); ++n) {
            bool join = i_inner && p.nests[n].rank >= nd - 1 && p.nests[n - 1].rank >= nd - 1;
            for (int r : all_phases(p.nests[n]))
                for (const HRef &ref : c->rules[r].in) {
                    const int pr = c->terms[ref.term].producer;
                    if (!join || pr < 0 || nest_of[pr] == (int)n || outer[nest_of[pr]] != g) continue;
                    const HTermPlan &tp = p.terms[ref.term];
                    if (c->terms[ref.term].rank == 0) join = false;
                    for (int ax = 1; ax < nd; ++ax)
                        if (tp.lo[ax] != 0 || tp.hi[ax] != 0) join = false;
                }
            if (!join) ++g;
            outer[n] = g;
        }
    }

    // ---- storage classes and windows
    const int64_t nrows = (int64_t)o->dims[1] * o->dims[2];
    int64_t fp_un = 0, fp_con = 0;
    int maxw = 0;
    for (int t = 0; t < nt; ++t) {
        const HTerm &T = c->terms[t];
        HTermPlan &tp = p.terms[t];
        if (T.rank == 0) { tp.storage = HFAV_STORE_SCALAR; continue; }
        if (T.kind != TK_INTER) { tp.storage = HFAV_STORE_FULL; continue; }
        if (T.producer < 0 || !c->live[T.producer]) continue;
        const bool rowt = T.rank == nd - 1;
        fp_un += rowt ? nrows : ncell;
        bool same_nest = true, same_outer = true;
        for (int r : c->topo)
            for (const HRef &ref : c->rules[r].in)
                if (ref.term == t) {
                    if (nest_of[r] != nest_of[T.producer]) same_nest = false;
                    if (outer[nest_of[r]] != outer[nest_of[T.producer]]) same_outer = false;
                }
        if (rowt) {                     // one value per outer iteration, or a row array
            if (same_outer) {
                tp.storage = HFAV_STORE_REGISTER;
                tp.window = 1;
                fp_con += 1;
                maxw = std::max(maxw, 1);
            } else {
                fp_con += nrows;
            }
            continue;
        }
        if (!same_nest && same_outer) { // between two inner sweeps: one row slab
            tp.storage = HFAV_STORE_OUTER;
            tp.window_axis = c->order[nd - 2];
            tp.window = 1;
            fp_con += o->dims[0];
            maxw = std::max(maxw, 1);
            continue;
        }
        if (!same_nest) {
            tp.storage = HFAV_STORE_FULL;
            fp_con += ncell;
            continue;
        }
        // outermost axis (in loop order) along which the extent varies
        int wax = -1;
        for (int q = 0; q < nd; ++q) {
            const int ax = c->order[q];
            if (tp.hi[ax] != tp.lo[ax]) { wax = ax; break; }
        }
        if (wax < 0) {
            tp.storage = HFAV_STORE_REGISTER;
            tp.window = 1;
            tp.window_axis = -1;
            fp_con += 1;
        } else {
            tp.window_axis = wax;
            tp.window = tp.hi[wax] - tp.lo[wax] + 1;
            const int inner = c->order[nd - 1];
            if (wax == inner) {
                tp.storage = HFAV_STORE_INNER;
                fp_con += tp.window;
            } else {
                tp.storage = HFAV_STORE_OUTER;
                // a slab of axis wax spans the axes inside it in loop order
                int64_t slab = 1;
                bool inside = false;
                for (int q = 0; q < nd; ++q) {
                    if (inside) slab *= o->dims[c->order[q]];
                    if (c->order[q] == wax) inside = true;
                }
                fp_con += tp.window * slab;
            }
        }
        maxw = std::max(maxw, tp.window);
    }

    // ---- byte counts
    const size_t es = esize(c->dtype);
    double bf = 0.0, bu = 0.0;
    // (grid terms only: 0-D and row terms cost O(1 / ni) bytes per cell)
    for (int t : c->axioms)
        if (c->terms[t].rank == nd) bf += es;
    for (int t : c->goals)
        if (c->terms[t].rank == nd) bf += es;
    for (int r : c->topo) {
        const HRule &R = c->rules[r];
        if (R.rank == 0) continue;
        std::vector<int> seen;
        for (const HRef &ref : R.in)
            if (c->terms[ref.term].rank == nd && std::find(seen.begin(), seen.end(), ref.term) == seen.end())
                seen.push_back(ref.term);
        bu += es * seen.size();
        for (int t : R.out)
            if (c->terms[t].rank == nd) bu += es;
    }

    // ---- kernel family
    int dir = -1;
    if (match_hdiff(c, p)) p.family = HFAV_FAMILY_HDIFF;
    else if (match_euler(c, p, dir)) {
        p.family = dir == 0 ? HFAV_FAMILY_EULER_X : HFAV_FAMILY_EULER_Y;
        if (o->boundary[dir] != HFAV_BC_PERIODIC && o->boundary[dir] != HFAV_BC_TRANSMISSIVE) p.family = 0;
    } else if (match_lap7_chain(c, p)) p.family = HFAV_FAMILY_LAP7_CHAIN;
    else if (match_smax(c, p)) p.family = HFAV_FAMILY_SMAX;
    else if (match_star_chain(c, p)) p.family = HFAV_FAMILY_STAR_CHAIN;
    else if (match_norm(c, p)) p.family = HFAV_FAMILY_NORM;
    else if (match_euler_xy(c, p)) p.family = HFAV_FAMILY_EULER_XY;
    else p.family = HFAV_FAMILY_NONE;
    if (o->precision == HFAV_PREC_F32_F64ACC && p.family != HFAV_FAMILY_EULER_X &&
        p.family != HFAV_FAMILY_EULER_Y && p.family != HFAV_FAMILY_EULER_XY && o->mode == HFAV_MODE_FUSED)
        return hfav_fail(HFAV_EUNSUP, "F32_F64ACC is implemented for the Euler sweeps only");

    bool fused = false;
    if (o->mode == HFAV_MODE_FUSED) {
        if (p.family == HFAV_FAMILY_NONE)
            return hfav_fail(HFAV_EUNSUP, "no fused kernel family matches this chain");
        fused = true;
    } else if (o->mode == HFAV_MODE_AUTO) {
        fused = p.family != HFAV_FAMILY_NONE;
    }
    // the single-rule reduction has no separate unfused form: it is the same kernel
    if (p.family == HFAV_FAMILY_SMAX && o->mode == HFAV_MODE_UNFUSED) fused = false;

    // ---- configuration
    hfav_config cfg = hfav_default_config(p.family, c->dtype, o->dims);
    int src = HFAV_CONFIG_DEFAULT;
    if (o->config_source == HFAV_CONFIG_FORCED) {
        cfg = o->forced;
        if (cfg.block <= 0 || cfg.block > 1024 || cfg.seg < 0 || cfg.seg > 4096 || cfg.variant < 0 ||
            cfg.xcd < -1 || cfg.xcd > 4096)
            return hfav_fail(HFAV_EINVAL, "forced configuration out of range");
        src = HFAV_CONFIG_FORCED;
    } else if (o->config_source == HFAV_CONFIG_TUNED) {
        if (hfav_tuned_config(p.family, c->dtype, o->dims, &cfg)) src = HFAV_CONFIG_TUNED;
    } else if (o->config_source == HFAV_CONFIG_MODEL) {
        if (p.family == HFAV_FAMILY_STAR_CHAIN && star_model_choose(c, p, o->dims, &cfg)) src = HFAV_CONFIG_MODEL;
    }

    // ---- EULER_X / EULER_Y strip kernels: the shapes that are built
    if (p.family == HFAV_FAMILY_EULER_Y && (cfg.variant & 63) == 3 && !hfav::euler_y_strip_ok(cfg))
        return hfav_fail(HFAV_EINVAL, "y strip configuration not built: tile_y columns 64 (or 1) with block 128, "
                                      "256 or 512, or 32, 16, 8 with block 256");
    if (p.family == HFAV_FAMILY_EULER_X && (cfg.variant & 63) == 3 && !hfav::euler_x_strip_ok(cfg))
        return hfav_fail(HFAV_EINVAL, "x strip configuration not built: tile_y rows 1 with block 64, 128 or 256, "
                                      "or 2 with block 64");

    // ---- NORM: block and cells per thread from the field count and the
    // row length (variant 0 holds the row in registers when it fits)
    if (p.family == HFAV_FAMILY_NORM) {
        const int nq = (int)p.fam_in.size();
        if (src == HFAV_CONFIG_FORCED) {
            if (!hfav::norm_config_ok(nq, o->dims[0], cfg))
                return hfav_fail(HFAV_EUNSUP, "forced normalisation configuration does not cover the row");
        } else if (src != HFAV_CONFIG_TUNED || !hfav::norm_config_ok(nq, o->dims[0], cfg)) {
            cfg = hfav::norm_default_config(nq, o->dims[0], c->dtype);
            src = HFAV_CONFIG_DEFAULT;
        }
    }

    // ---- STAR_CHAIN: groups of fused stages (config.tile_y = stages per
    // group, 0 = all; config.variant = tile shape); the default takes the
    // deepest grouping that fits in LDS
    if (fused && p.family == HFAV_FAMILY_STAR_CHAIN) {
        if (src == HFAV_CONFIG_DEFAULT || src == HFAV_CONFIG_TUNED || !star_groups(c, p, cfg.tile_y, cfg.variant)) {
            if (src == HFAV_CONFIG_FORCED)
                return hfav_fail(HFAV_EUNSUP, "forced star-chain configuration does not fit in LDS");
            int D = (int)p.sstages.size();
            while (D > 1 && !star_groups(c, p, D, cfg.variant)) --D;
            if (!star_groups(c, p, D, cfg.variant)) {
                cfg.variant = 0;
                D = (int)p.sstages.size();
                while (D > 1 && !star_groups(c, p, D, 0)) --D;
                if (!star_groups(c, p, D, 0)) fused = false;
            }
            cfg.tile_y = D;
        }
    }

    // ---- in/out chaining (Design, "In/out chaining"): for each declared
    // alias, the axiom's values that a goal reads after the goal may have
    // overwritten them are saved first.  The axiom's Minkowski extent holds
    // the offsets every goal reads it at.
    //  * NORM: a workgroup holds its whole row on chip before writing it:
    //    nothing to save (the two-pass streamed variant would re-read u);
    //  * HDIFF: only the 2-wide halo columns and rows at tile and segment
    //    boundaries are at risk (the LDS ring is the rolling input buffer):
    //    saved by a copy kernel;
    //  * EULER_X / EULER_Y (each goal written over the axiom of the same
    //    field): a strip segment reads the 2 cells on either side of it,
    //    which the neighbouring segments write: the cells around every
    //    segment boundary are saved by a copy kernel (strip kernels only);
    //  * other fused families: not built; AUTO falls back to unfused;
    //  * unfused: safe when the goal's producer is the last rule to read the
    //    axiom and reads it at offset 0 only; otherwise the whole axiom is
    //    copied and every rule reads the copy.
    p.alias_handling.assign(c->alias.size(), HPlan::ALIAS_SAFE);
    p.alias_ws.assign(c->alias.size(), -1);
    bool euler_ip = false;
    if (!c->alias.empty() && fused) {
        const bool norm_ok = p.family == HFAV_FAMILY_NORM && cfg.variant != 1;
        const bool hdiff_ok = p.family == HFAV_FAMILY_HDIFF;
        bool euler_ok = false;
        if (p.family == HFAV_FAMILY_EULER_X || p.family == HFAV_FAMILY_EULER_Y) {
            euler_ok = true;
            for (const auto &pr : c->alias) {
                bool same_field = false;
                for (int q = 0; q < 4; ++q)
                    if (pr.first == p.fam_out[q] && pr.second == p.fam_in[q]) same_field = true;
                euler_ok = euler_ok && same_field;
            }
            // the in-place sweep runs the strip kernel: 64-cell chunks of
            // one row along x, 64 columns x 4 rows or 16 x 16 along y
            const bool ydir = p.family == HFAV_FAMILY_EULER_Y;
            const int sblock = ydir ? 256 : 64;
            auto ip_shape = [&](const hfav_config &k) {
                if ((k.variant & 63) != 3 || k.block != sblock) return false;
                if (ydir) return hfav::euler_y_strip_cols(k) == 64 || hfav::euler_y_strip_cols(k) == 16;
                return hfav::euler_x_strip_rows(k) == 1 || hfav::euler_x_strip_rows(k) == 2;
            };
            if (euler_ok && src != HFAV_CONFIG_FORCED && !ip_shape(cfg)) {
                cfg.variant = 3 | (cfg.variant & 64);
                cfg.block = sblock;
                cfg.tile_y = 1;
                if (ydir && cfg.seg <= 0) cfg.seg = 15;
            }
            euler_ok = euler_ok && ip_shape(cfg);
            euler_ip = euler_ok;
        }
        if (!norm_ok && !hdiff_ok && !euler_ok) {
            if (o->mode == HFAV_MODE_FUSED)
                return hfav_fail(HFAV_EUNSUP, "in-place execution of this fused kernel family or configuration is "
                                              "not built (normalisation with the row on chip, horizontal "
                                              "diffusion, the hydro sweeps' strip kernels with each goal over "
                                              "its own field's axiom)");
            fused = false;
        }
        // in place, wider tiles and longer segments mean fewer boundaries
        // whose halos must be saved (measured at 64 x 2048^2 FP64: 512-wide
        // tiles and 128-row segments halve the saved bytes and the copy time)
        if (hdiff_ok && src == HFAV_CONFIG_DEFAULT) {
            if (o->dims[0] >= 2048) cfg.block = 512;
            if (o->dims[1] >= 1024 && cfg.seg < 128) cfg.seg = 128;
        }
    }

    // ---- workspace layout
    p.ws_off.assign(nt, -1);
    p.ws_bytes = 0;
    if (fused && p.family == HFAV_FAMILY_STAR_CHAIN) {
        p.ws_coeff = 0;
        p.ws_bytes = (p.scoeff.size() * 8 + 255) / 256 * 256;
        // outputs of every group but the last are full arrays
        for (size_t gi = 1; gi < p.sgroups.size(); ++gi)
            for (int t : p.sstages[p.sgroups[gi] - 1].out_terms) {
                p.ws_off[t] = (int64_t)p.ws_bytes;
                p.ws_bytes += ((size_t)ncell * es + 255) / 256 * 256;
            }
    }
    if (!fused) {
        p.ws_coeff = -1;
        for (int t = 0; t < nt; ++t) {
            const HTerm &T = c->terms[t];
            if (T.kind != TK_INTER || T.producer < 0 || !c->live[T.producer]) continue;
            p.ws_off[t] = (int64_t)p.ws_bytes;
            size_t b = T.rank == 0 ? 8 : T.rank == nd - 1 ? (size_t)nrows * es : (size_t)ncell * es;
            p.ws_bytes += (b + 255) / 256 * 256;
        }
    }
    p.exec_order = c->topo;
    for (size_t q = 0; q < c->alias.size(); ++q) {
        const int g = c->alias[q].first, a = c->alias[q].second;
        if (fused) {
            if (p.family == HFAV_FAMILY_NORM) {
                p.alias_handling[q] = HPlan::ALIAS_ROWS_ON_CHIP;
            } else if (euler_ip) {      // one area of saved segment halos serves every pair
                p.alias_handling[q] = HPlan::ALIAS_SEG_HALOS;
                bool first = true;
                for (size_t r = 0; r < q; ++r)
                    if (p.alias_handling[r] == HPlan::ALIAS_SEG_HALOS) {
                        p.alias_ws[q] = p.alias_ws[r];
                        first = false;
                    }
                if (first) {
                    p.alias_ws[q] = (int64_t)p.ws_bytes;
                    p.ws_bytes += (hfav::euler_inplace_bytes(o->dims[0], o->dims[1],
                                                             p.family == HFAV_FAMILY_EULER_X ? 0 : 1, c->dtype, cfg) +
                                   255) / 256 * 256;
                }
            } else {                    // HDIFF: one halo-copy area serves the pair
                p.alias_handling[q] = HPlan::ALIAS_TILE_HALOS;
                p.alias_ws[q] = (int64_t)p.ws_bytes;
                p.ws_bytes += (hfav::hdiff_inplace_bytes(o->dims[0], o->dims[1], o->dims[2], c->dtype, cfg) + 255) /
                              256 * 256;
            }
            continue;
        }
        const int pg = c->terms[g].producer;
        int last = -1;
        bool off0 = true;
        for (size_t pos = 0; pos < p.exec_order.size(); ++pos) {
            const HRule &R = c->rules[p.exec_order[pos]];
            for (const HRef &ref : R.in)
                if (ref.term == a) {
                    last = (int)pos;
                    if (p.exec_order[pos] == pg && (ref.off[0] || ref.off[1] || ref.off[2])) off0 = false;
                }
        }
        const bool safe = last < 0 || (p.exec_order[last] == pg && off0);
        if (!safe) {
            p.alias_handling[q] = HPlan::ALIAS_FULL_COPY;
            p.alias_ws[q] = (int64_t)p.ws_bytes;
            const size_t b = c->terms[a].rank == nd - 1 ? (size_t)nrows * es : (size_t)ncell * es;
            p.ws_bytes += (b + 255) / 256 * 256;
        }
    }

    // ---- info
    hfav_plan_info &I = p.info;
    memset(&I, 0, sizeof(I));
    I.n_rules = (int)c->topo.size();
    for (size_t q = 0; q < c->topo.size(); ++q) I.rule_order[q] = c->topo[q];
    I.n_nests = (int)p.nests.size();
    for (int r = 0; r < HFAV_MAX_RULES; ++r) { I.nest_of_rule[r] = -1; I.phase_of_rule[r] = -1; }
    for (size_t n = 0; n < p.nests.size(); ++n)
        for (int r : all_phases(p.nests[n])) {
            I.nest_of_rule[r] = (int)n;
            I.phase_of_rule[r] = phase_of(p.nests[n], r);
        }
    I.family = p.family;
    I.fused = fused ? 1 : 0;
    I.streamed_axis = (p.family == HFAV_FAMILY_EULER_X || p.family == HFAV_FAMILY_NORM) ? 0
                      : p.family == HFAV_FAMILY_LAP7_CHAIN ? 2 : 1;
    I.config = cfg;
    I.config_source = src;
    I.footprint_unfused = fp_un;
    I.footprint_contracted = fp_con;
    I.max_window = maxw;
    I.bytes_per_cell_fused = bf;
    I.bytes_per_cell_unfused = bu;
    I.workspace_bytes = p.ws_bytes;
    for (size_t n = 0; n < p.nests.size(); ++n) I.outer_of_nest[n] = outer[n];
    p.outer = outer;

    // ---- JSON
    std::ostringstream js;
    js << "{\"family\":" << p.family << ",\"fused\":" << I.fused << ",\"nests\":[";
    for (size_t n = 0; n < p.nests.size(); ++n) {
        const HNest &N = p.nests[n];
        auto lst = [&](const std::vector<int> &v) {
            js << "[";
            for (size_t q = 0; q < v.size(); ++q) js << (q ? "," : "") << v[q];
            js << "]";
        };
        js << (n ? "," : "") << "{\"rank\":" << N.rank << ",\"outer\":" << outer[n] << ",\"prologue\":";
        lst(N.prologue);
        js << ",\"steady\":";
        lst(N.steady);
        js << ",\"epilogue\":";
        lst(N.epilogue);
        js << "}";
    }
    js << "],\"terms\":[";
    for (int t = 0; t < nt; ++t) {
        const HTerm &T = c->terms[t];
        const HTermPlan &tp = p.terms[t];
        js << (t ? "," : "") << "{\"name\":" << jstr(T.name) << ",\"kind\":" << T.kind << ",\"rank\":" << T.rank
           << ",\"lo\":";
        json_int3(js, tp.lo);
        js << ",\"hi\":";
        json_int3(js, tp.hi);
        js << ",\"storage\":\"" << storage_name(tp.storage) << "\",\"window_axis\":" << tp.window_axis
           << ",\"window\":" << tp.window << ",\"reuse\":[";
        // reuse order: the distinct references to the term, in the order a
        // value is visited under the loop order (first visit at the largest
        // offset along the outermost axis); this total order is the longest
        // path of the per-term reuse graph (Design, "Grouping")
        std::vector<std::array<int, 3>> refs;
        for (int r : c->topo)
            for (const HRef &ref : c->rules[r].in)
                if (ref.term == t) {
                    std::array<int, 3> o = {ref.off[0], ref.off[1], ref.off[2]};
                    if (std::find(refs.begin(), refs.end(), o) == refs.end()) refs.push_back(o);
                }
        std::sort(refs.begin(), refs.end(), [&](const std::array<int, 3> &a, const std::array<int, 3> &b) {
            for (int q = 0; q < nd; ++q) {
                const int ax = c->order[q];
                if (a[ax] != b[ax]) return a[ax] > b[ax];
            }
            return false;
        });
        for (size_t q = 0; q < refs.size(); ++q)
            js << (q ? "," : "") << "[" << refs[q][0] << "," << refs[q][1] << "," << refs[q][2] << "]";
        js << "]}";
    }
    js << "],\"rules\":[";
    for (size_t r = 0; r < c->rules.size(); ++r) {
        const HRule &R = c->rules[r];
        js << (r ? "," : "") << "{\"op\":" << R.op << ",\"live\":" << (c->live[r] ? 1 : 0) << ",\"in\":[";
        for (size_t q = 0; q < R.in.size(); ++q)
            js << (q ? "," : "") << "[" << jstr(c->terms[R.in[q].term].name) << "," << R.in[q].off[0] << ","
               << R.in[q].off[1] << "," << R.in[q].off[2] << "]";
        js << "],\"out\":[";
        for (size_t q = 0; q < R.out.size(); ++q) js << (q ? "," : "") << jstr(c->terms[R.out[q]].name);
        js << "]";
        if (r < c->origin.size())
            js << ",\"pattern\":" << c->origin[r].first << ",\"binding\":" << jstr(c->origin[r].second);
        js << "}";
    }
    js << "],\"aliases\":[";
    for (size_t q = 0; q < c->alias.size(); ++q) {
        static const char *hname[] = {"safe", "tile_halo_copies", "full_copy", "rows_on_chip",
                                      "segment_halo_copies"};
        const HTermPlan &tp = p.terms[c->alias[q].second];
        js << (q ? "," : "") << "{\"goal\":" << jstr(c->terms[c->alias[q].first].name)
           << ",\"axiom\":" << jstr(c->terms[c->alias[q].second].name) << ",\"extent_lo\":";
        json_int3(js, tp.lo);
        js << ",\"extent_hi\":";
        json_int3(js, tp.hi);
        js << ",\"handling\":\"" << hname[p.alias_handling[q]] << "\"}";
    }
    js << "],\"footprint_unfused\":" << fp_un << ",\"footprint_contracted\":" << fp_con
       << ",\"max_window\":" << maxw << ",\"bytes_per_cell_fused\":" << bf
       << ",\"bytes_per_cell_unfused\":" << bu << ",\"config\":{\"block\":" << cfg.block
       << ",\"tile_y\":" << cfg.tile_y << ",\"seg\":" << cfg.seg << ",\"variant\":" << cfg.variant
       << ",\"xcd\":" << cfg.xcd
       << "},\"config_source\":" << src << ",\"workspace_bytes\":" << p.ws_bytes << "}";
    p.json = js.str();
    p.valid = true;
    c->plan = p;
    // STAR_CHAIN: the coefficient table travels to the workspace with every
    // execute as an asynchronous copy from pinned host memory, staged here so
    // that execute itself allocates nothing (host memory only; freeing the
    // previous buffer waits for copies still reading it)
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    c->pinned_err.clear();
    if (fused && p.family == HFAV_FAMILY_STAR_CHAIN) {
        const size_t bytes = c->plan.scoeff.size() * sizeof(double);
        const hipError_t e = hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault);
        if (e == hipSuccess) {
            memcpy(c->pinned, c->plan.scoeff.data(), bytes);
            c->pinned_bytes = bytes;
        } else {
            c->pinned = nullptr;
            c->pinned_err = hipGetErrorString(e);
        }
    }
    if (info) *info = I;
    return HFAV_OK;
}

extern "C" int hfav_plan(hfav_chain *chain, const hfav_plan_opts *opts, hfav_plan_info *info) {
    if (chain) chain->plan.valid = false;
    try {
        return hfav_plan_impl(chain, opts, info);
    } catch (...) {
        return hfav_fail(HFAV_EINVAL, "host exception while planning");
    }
}

extern "C" int hfav_plan_batch(hfav_chain *chain, const hfav_plan_opts *opts, int n_grids, const int *dims,
                               hfav_plan_info *info) {
    if (chain) chain->plan.valid = false;
    if (!chain || !opts || !dims) return hfav_fail(HFAV_EINVAL, "null argument");
    if (n_grids < 1 || n_grids > HFAV_MAX_BATCH) return hfav_fail(HFAV_EINVAL, "n_grids out of range");
    if (chain->ndim != 2) return hfav_fail(HFAV_EUNSUP, "batches are implemented for 2-D chains");
    for (int g = 0; g < n_grids; ++g)
        if (dims[2 * g] < 1 || dims[2 * g] > 65535 || dims[2 * g + 1] < 1 || dims[2 * g + 1] > 65535)
            return hfav_fail(HFAV_EINVAL, "batch grid size out of range");
    if (opts->mode == HFAV_MODE_UNFUSED) return hfav_fail(HFAV_EUNSUP, "batches run the fused kernels only");
    if (!chain->alias.empty()) return hfav_fail(HFAV_EUNSUP, "in-place batches are not built");
    hfav_plan_opts o = *opts;
    o.dims[0] = dims[0];
    o.dims[1] = dims[1];
    o.dims[2] = 1;
    o.mode = HFAV_MODE_FUSED;
    int rc;
    try {
        rc = hfav_plan_impl(chain, &o, info);
    } catch (...) {
        rc = hfav_fail(HFAV_EINVAL, "host exception while planning");
    }
    if (rc != HFAV_OK) return rc;
    HPlan &p = chain->plan;
    if (p.family != HFAV_FAMILY_EULER_X && p.family != HFAV_FAMILY_EULER_Y && p.family != HFAV_FAMILY_SMAX &&
        p.family != HFAV_FAMILY_EULER_XY) {
        p.valid = false;
        return hfav_fail(HFAV_EUNSUP, "batches are implemented for the Euler sweeps, the time step of both "
                                      "sweeps and the CFL reduction");
    }
    p.batch = true;
    p.bnx.resize(n_grids);
    p.bny.resize(n_grids);
    p.bseg.resize(n_grids);
    p.boff.resize(n_grids);
    int64_t off = 0;
    for (int g = 0; g < n_grids; ++g) {
        p.bnx[g] = dims[2 * g];
        p.bny[g] = dims[2 * g + 1];
        p.boff[g] = off;
        off += (int64_t)p.bnx[g] * p.bny[g];
        const int gd[3] = {p.bnx[g], p.bny[g], 1};
        // the batched y sweep runs 4-row strips; its segment length per
        // grid comes from the batch entries of the tuning table (nearest
        // size bucket), else 15 (a segment of s rows walks s + 1 chunk rows)
        hfav_config cg{256, 1, 15, 3, 0};
        if (o.config_source == HFAV_CONFIG_FORCED) cg = o.forced;
        else if (o.config_source == HFAV_CONFIG_TUNED)
            hfav_tuned_config(HFAV_FAMILY_EULER_Y_BATCH, chain->dtype, gd, &cg);
        int seg = cg.seg > 0 ? cg.seg : 15;
        p.bseg[g] = seg > 255 ? 255 : seg;
    }
    p.btotal = off;
    // the time step of both sweeps runs as one persistent launch whose y
    // items read the x-swept state from the workspace
    const bool step = p.family == HFAV_FAMILY_EULER_XY;
    if (step) {
        p.ws_bytes = hfav::step_batch_ws_bytes(p.btotal, chain->dtype);
        p.info.workspace_bytes = p.ws_bytes;
        if (info) info->workspace_bytes = p.ws_bytes;
    }
    // record the batch in the plan's JSON: grid count and y segment lengths
    if (!p.json.empty() && p.json.back() == '}') {
        std::ostringstream bj;
        bj << ",\"batch\":{\"grids\":" << n_grids << ",\"y_seg\":[";
        for (int g = 0; g < n_grids; ++g) bj << (g ? "," : "") << (int)p.bseg[g];
        bj << "]";
        if (step) bj << ",\"one_launch_step\":1,\"workspace_bytes\":" << p.ws_bytes;
        bj << "}";
        p.json.insert(p.json.size() - 1, bj.str());
    }
    return HFAV_OK;
}

extern "C" int64_t hfav_batch_offset(const hfav_chain *c, int grid) {
    if (!c || !c->plan.valid || !c->plan.batch || grid < 0 || grid >= (int)c->plan.boff.size()) return -1;
    return c->plan.boff[grid];
}

extern "C" int hfav_plan_term(const hfav_chain *c, int index, hfav_term_info *info) {
    if (!c || !info) return hfav_fail(HFAV_EINVAL, "null argument");
    if (!c->plan.valid) return hfav_fail(HFAV_ENOPLAN, "chain has no plan");
    if (index < 0 || index >= (int)c->terms.size()) return hfav_fail(HFAV_EINVAL, "term index out of range");
    const HTerm &T = c->terms[index];
    const HTermPlan &tp = c->plan.terms[index];
    info->name = T.name.c_str();
    info->kind = T.kind;
    info->rank = T.rank;
    info->producer = T.producer;
    for (int ax = 0; ax < 3; ++ax) { info->ext_lo[ax] = tp.lo[ax]; info->ext_hi[ax] = tp.hi[ax]; }
    info->storage = tp.storage;
    info->window_axis = tp.window_axis;
    info->window = tp.window;
    return HFAV_OK;
}

extern "C" const char *hfav_plan_json(const hfav_chain *c) {
    if (!c || !c->plan.valid) {
        hfav_fail(HFAV_ENOPLAN, "chain has no plan");
        return nullptr;
    }
    return c->plan.json.c_str();
}

// The nest-fusion walk on caller-given nests and dependences (the planner
// applies the same routine to its one-nest-per-rule DAG).
extern "C" int hfav_fuse_nests(int n_rules, const unsigned char *reach, int n, const hfav_nest *nests,
                               hfav_nest *out, int *n_out) {
    if (n_rules < 1 || n_rules > HFAV_MAX_RULES || !reach || n < 0 || (n > 0 && !nests) || !out || !n_out)
        return hfav_fail(HFAV_EINVAL, "hfav_fuse_nests: bad arguments");
    Reach D{n_rules, std::vector<char>((size_t)n_rules * n_rules, 0)};
    for (int a = 0; a < n_rules; ++a)
        for (int b = 0; b < n_rules; ++b) D.m[(size_t)a * n_rules + b] = reach[(size_t)a * n_rules + b] != 0;
    std::vector<HNest> in;
    auto take = [&](int cnt, const int *ids, std::vector<int> &dst) {
        if (cnt < 0 || cnt > HFAV_MAX_RULES) return false;
        for (int q = 0; q < cnt; ++q) {
            if (ids[q] < 0 || ids[q] >= n_rules) return false;
            dst.push_back(ids[q]);
        }
        return true;
    };
    for (int q = 0; q < n; ++q) {
        HNest N;
        N.rank = nests[q].rank;
        if (!take(nests[q].n_prologue, nests[q].prologue, N.prologue) ||
            !take(nests[q].n_steady, nests[q].steady, N.steady) ||
            !take(nests[q].n_epilogue, nests[q].epilogue, N.epilogue))
            return hfav_fail(HFAV_EINVAL, "hfav_fuse_nests: phase count or rule id out of range");
        in.push_back(N);
    }
    const std::vector<HNest> res = fuse_inest_dag(D, in);
    for (size_t q = 0; q < res.size(); ++q) {
        const HNest &N = res[q];
        if (N.prologue.size() > HFAV_MAX_RULES || N.steady.size() > HFAV_MAX_RULES ||
            N.epilogue.size() > HFAV_MAX_RULES)
            return hfav_fail(HFAV_EINVAL, "hfav_fuse_nests: a fused phase exceeds HFAV_MAX_RULES rules");
        hfav_nest &o = out[q];
        memset(&o, 0, sizeof(o));
        o.rank = N.rank;
        o.n_prologue = (int)N.prologue.size();
        o.n_steady = (int)N.steady.size();
        o.n_epilogue = (int)N.epilogue.size();
        std::copy(N.prologue.begin(), N.prologue.end(), o.prologue);
        std::copy(N.steady.begin(), N.steady.end(), o.steady);
        std::copy(N.epilogue.begin(), N.epilogue.end(), o.epilogue);
    }
    *n_out = (int)res.size();
    return HFAV_OK;
}
