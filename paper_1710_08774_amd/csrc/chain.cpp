// Chain intake: copy the descriptor, intern term names, build the dataflow
// graph (rule call sites as vertices, terms as edges, Design "Dataflow") and
// validate it: one producer per term (Related Work), no cycles, every goal
// derivable from the axioms (Implementation, "Inference"), known ops with
// the right arity.  Rules no goal needs are pruned: inference works backward
// from the goals.
#include <cstring>
#include <map>
#include <new>
#include <string>

#include <hip/hip_runtime.h>

#include "internal.h"

static thread_local std::string g_err;

int hfav_fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

extern "C" const char *hfav_last_error(void) { return g_err.c_str(); }
extern "C" const char *hfav_version(void) { return "hfav-mi355x 0.2 (gfx950)"; }
// the tag is also found by scanning the file, before anything loads it
static const char kBuildTag[] = "hfav-build-id:" HFAV_BUILD_ID;
extern "C" const char *hfav_build_id(void) { return kBuildTag + 14; }

static const OpSpec kOps[] = {
    {HFAV_OP_HDIFF_LAP, "HDIFF_LAP", 5, 1, 0, -1, 0},
    {HFAV_OP_HDIFF_FLX, "HDIFF_FLX", 4, 1, 0, -1, 0},
    {HFAV_OP_HDIFF_FLY, "HDIFF_FLY", 4, 1, 0, -1, 0},
    {HFAV_OP_HDIFF_OUT, "HDIFF_OUT", 5, 1, 1, -1, 0},
    {HFAV_OP_EULER_PRIM, "EULER_PRIM", 4, 5, 1, -1, 0},
    {HFAV_OP_EULER_SLOPE, "EULER_SLOPE", 12, 4, 0, -1, 0},
    {HFAV_OP_EULER_TRACE, "EULER_TRACE", 10, 8, 0, 9, 0},
    {HFAV_OP_EULER_RIEMANN, "EULER_RIEMANN", 8, 4, 2, -1, 0},
    {HFAV_OP_EULER_FLUX, "EULER_FLUX", 4, 4, 1, -1, 0},
    {HFAV_OP_EULER_UPDATE, "EULER_UPDATE", 13, 4, 0, 12, 0},
    {HFAV_OP_EULER_SMAX, "EULER_SMAX", 4, 1, 1, -1, 1},
    {HFAV_OP_EULER_DT, "EULER_DT", 1, 1, 1, 0, 1},
    {HFAV_OP_LAP7, "LAP7", 7, 1, 0, -1, 0},
    {HFAV_OP_AXPY, "AXPY", 2, 1, 1, -1, 0},
    {HFAV_OP_STAR, "STAR", -1, 1, 0, -1, 0},
    {HFAV_OP_SUMSQ, "SUMSQ", -1, 1, 0, -1, 0},
    {HFAV_OP_SUM_I, "SUM_I", 1, 1, 0, -1, 0},
    {HFAV_OP_SQRT, "SQRT", 1, 1, 0, -1, 0},
    {HFAV_OP_DIV0, "DIV0", 2, 1, 0, -1, 0},
};

const OpSpec *op_spec(int op) {
    for (const OpSpec &s : kOps)
        if (s.op == op) return &s;
    return nullptr;
}

static int parse_order(const char *s, int ndim, int order[3]) {
    if (!s) {
        if (ndim == 3) { order[0] = 2; order[1] = 1; order[2] = 0; }
        else { order[0] = 1; order[1] = 0; order[2] = 2; }
        return 0;
    }
    if ((int)strlen(s) != ndim) return -1;
    bool seen[3] = {false, false, false};
    for (int q = 0; q < ndim; ++q) {
        int ax = s[q] == 'i' ? 0 : s[q] == 'j' ? 1 : s[q] == 'k' ? 2 : -1;
        if (ax < 0 || ax >= ndim || seen[ax]) return -1;
        seen[ax] = true;
        order[q] = ax;
    }
    if (ndim == 2) order[2] = 2;
    return 0;
}

static int build(const hfav_chain_desc *d, hfav_chain *c) {
    if (d->ndim != 2 && d->ndim != 3) return hfav_fail(HFAV_EINVAL, "ndim must be 2 or 3");
    if (d->dtype != HFAV_F64 && d->dtype != HFAV_F32) return hfav_fail(HFAV_EINVAL, "unknown dtype");
    if (d->n_axiom < 1 || !d->axioms) return hfav_fail(HFAV_EINVAL, "a chain needs at least one axiom");
    if (d->n_goal < 1 || !d->goals) return hfav_fail(HFAV_EINVAL, "a chain needs at least one goal");
    if (d->n_rule < 0 || (d->n_rule > 0 && !d->rules)) return hfav_fail(HFAV_EINVAL, "bad rule list");
    if (d->n_rule > HFAV_MAX_RULES) return hfav_fail(HFAV_EINVAL, "too many rules");
    c->ndim = d->ndim;
    c->dtype = d->dtype;
    if (parse_order(d->loop_order, d->ndim, c->order) != 0)
        return hfav_fail(HFAV_EINVAL, "loop_order must be a permutation of the axis letters");

    std::map<std::string, int> id;
    auto intern = [&](const char *name) -> int {
        auto it = id.find(name);
        if (it != id.end()) return it->second;
        HTerm t;
        t.name = name;
        t.kind = TK_INTER;
        t.rank = -1;
        t.producer = -1;
        t.axiom_slot = -1;
        t.goal_slot = -1;
        t.out_pos = -1;
        c->terms.push_back(t);
        id[name] = (int)c->terms.size() - 1;
        return (int)c->terms.size() - 1;
    };

    for (int a = 0; a < d->n_axiom; ++a) {
        const hfav_term_decl &ax = d->axioms[a];
        if (!ax.name || !*ax.name) return hfav_fail(HFAV_EINVAL, "axiom without a name");
        if (id.count(ax.name)) return hfav_fail(HFAV_EDUP, std::string("axiom declared twice: ") + ax.name);
        if (ax.rank != 0 && ax.rank != d->ndim && ax.rank != d->ndim - 1)
            return hfav_fail(HFAV_EINVAL, std::string("axiom rank must be 0, ndim - 1 or ndim: ") + ax.name);
        int t = intern(ax.name);
        c->terms[t].kind = TK_AXIOM;
        c->terms[t].rank = ax.rank;
        c->terms[t].axiom_slot = a;
        c->axioms.push_back(t);
    }

    for (int r = 0; r < d->n_rule; ++r) {
        const hfav_rule &dr = d->rules[r];
        const OpSpec *sp = op_spec(dr.op);
        if (!sp) return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": unknown op");
        if (dr.n_in < 1 || !dr.in) return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": no inputs");
        if (sp->n_in >= 0 && dr.n_in != sp->n_in)
            return hfav_fail(HFAV_EINVAL, std::string("rule ") + std::to_string(r) + " (" + sp->name +
                                              "): expected " + std::to_string(sp->n_in) + " inputs");
        if (dr.n_out != sp->n_out || !dr.out)
            return hfav_fail(HFAV_EINVAL, std::string("rule ") + std::to_string(r) + " (" + sp->name +
                                              "): expected " + std::to_string(sp->n_out) + " outputs");
        int need_param = sp->op == HFAV_OP_STAR ? dr.n_in : sp->n_param;
        if (dr.n_param < need_param || (dr.n_param > 0 && !dr.param))
            return hfav_fail(HFAV_EINVAL, std::string("rule ") + std::to_string(r) + " (" + sp->name +
                                              "): missing parameters");
        if (sp->op == HFAV_OP_STAR && dr.n_in > HFAV_MAX_STAR_REFS)
            return hfav_fail(HFAV_EINVAL, "STAR rule with more than " + std::to_string(HFAV_MAX_STAR_REFS) +
                                              " references");
        if (sp->out_rank0 && sp->op == HFAV_OP_EULER_SMAX && dr.reduce != HFAV_REDUCE_MAX)
            return hfav_fail(HFAV_EINVAL, "EULER_SMAX must declare reduce = MAX");
        if (sp->op == HFAV_OP_SUM_I && dr.reduce != HFAV_REDUCE_SUM)
            return hfav_fail(HFAV_EINVAL, "SUM_I must declare reduce = SUM");
        if (dr.reduce != HFAV_REDUCE_NONE && sp->op != HFAV_OP_EULER_SMAX && sp->op != HFAV_OP_SUM_I)
            return hfav_fail(HFAV_EINVAL, "only EULER_SMAX and SUM_I reduce");
        if (sp->op == HFAV_OP_SUMSQ && dr.n_in > 24)
            return hfav_fail(HFAV_EINVAL, "SUMSQ rule with more than 24 references");
        HRule h;
        h.op = dr.op;
        h.reduce = dr.reduce;
        for (int q = 0; q < dr.n_param; ++q) h.param.push_back(dr.param[q]);
        for (int q = 0; q < dr.n_in; ++q) {
            if (!dr.in[q].term || !*dr.in[q].term)
                return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": reference without a term");
            HRef ref;
            ref.term = intern(dr.in[q].term);
            for (int ax = 0; ax < 3; ++ax) {
                ref.off[ax] = dr.in[q].off[ax];
                if (ax >= d->ndim && ref.off[ax] != 0)
                    return hfav_fail(HFAV_EINVAL, "offset along an axis the chain does not have");
                if (ref.off[ax] < -8 || ref.off[ax] > 8)
                    return hfav_fail(HFAV_EINVAL, "offsets are limited to [-8, 8]");
            }
            h.in.push_back(ref);
        }
        for (int q = 0; q < dr.n_out; ++q) {
            if (!dr.out[q] || !*dr.out[q])
                return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": output without a name");
            int t = intern(dr.out[q]);
            HTerm &T = c->terms[t];
            if (T.kind == TK_AXIOM)
                return hfav_fail(HFAV_EDUP, std::string("rule produces an axiom: ") + dr.out[q]);
            if (T.producer >= 0)
                return hfav_fail(HFAV_EDUP, std::string("two rules produce ") + dr.out[q]);
            T.producer = r;
            T.out_pos = q;
            h.out.push_back(t);
        }
        c->rules.push_back(h);
    }

    for (int g = 0; g < d->n_goal; ++g) {
        if (!d->goals[g] || !*d->goals[g]) return hfav_fail(HFAV_EINVAL, "goal without a name");
        auto it = id.find(d->goals[g]);
        if (it == id.end() || (c->terms[it->second].producer < 0 && c->terms[it->second].kind != TK_AXIOM))
            return hfav_fail(HFAV_EUNSAT, std::string("goal not derivable: ") + d->goals[g]);
        int t = it->second;
        if (c->terms[t].kind == TK_AXIOM)
            return hfav_fail(HFAV_EINVAL, std::string("a goal cannot be an axiom: ") + d->goals[g]);
        if (c->terms[t].kind == TK_GOAL) return hfav_fail(HFAV_EDUP, std::string("goal listed twice: ") + d->goals[g]);
        c->terms[t].kind = TK_GOAL;
        c->terms[t].goal_slot = g;
        c->goals.push_back(t);
    }

    const int nr = (int)c->rules.size();
    // liveness: backward from the goals
    c->live.assign(nr, false);
    std::vector<int> stack;
    for (int t : c->goals) stack.push_back(c->terms[t].producer);
    while (!stack.empty()) {
        int r = stack.back();
        stack.pop_back();
        if (r < 0 || c->live[r]) continue;
        c->live[r] = true;
        for (const HRef &ref : c->rules[r].in) {
            const HTerm &T = c->terms[ref.term];
            if (T.kind != TK_AXIOM && T.producer < 0)
                return hfav_fail(HFAV_EUNSAT, "term " + T.name + " is read but neither an axiom nor produced");
            if (T.producer >= 0) stack.push_back(T.producer);
        }
    }
    // topological order of live rules (Kahn); leftover rules form a cycle
    std::vector<int> indeg(nr, 0);
    for (int r = 0; r < nr; ++r)
        if (c->live[r])
            for (const HRef &ref : c->rules[r].in) {
                int p = c->terms[ref.term].producer;
                if (p >= 0 && c->live[p]) ++indeg[r];
            }
    std::vector<int> ready;
    for (int r = 0; r < nr; ++r)
        if (c->live[r] && indeg[r] == 0) ready.push_back(r);
    while (!ready.empty()) {
        // lowest descriptor index first: deterministic
        size_t best = 0;
        for (size_t q = 1; q < ready.size(); ++q)
            if (ready[q] < ready[best]) best = q;
        int r = ready[best];
        ready.erase(ready.begin() + best);
        c->topo.push_back(r);
        for (int s = 0; s < nr; ++s) {
            if (!c->live[s]) continue;
            for (const HRef &ref : c->rules[s].in)
                if (c->terms[ref.term].producer == r && --indeg[s] == 0) ready.push_back(s);
        }
    }
    int nlive = 0;
    for (int r = 0; r < nr; ++r) nlive += c->live[r];
    if ((int)c->topo.size() != nlive) return hfav_fail(HFAV_ECYCLE, "the dataflow graph has a cycle");

    // term and rule ranks, in topological order.  Terms are 0-D, grids
    // (rank ndim) or row terms (rank ndim - 1, one value per row of i).
    // Row terms enter only where an op takes them: SQRT's input and DIV0's
    // divisor (a broadcast along i); SUM_I is the reduction that makes one.
    const int nd = c->ndim, row = c->ndim - 1;
    for (int r : c->topo) {
        HRule &R = c->rules[r];
        const OpSpec *sp = op_spec(R.op);
        bool any_grid = false, any_row = false;
        for (size_t q = 0; q < R.in.size(); ++q) {
            const HTerm &T = c->terms[R.in[q].term];
            if (T.rank < 0) return hfav_fail(HFAV_EUNSAT, "term " + T.name + " has no producer before use");
            const bool want0 = (int)q == sp->scalar_in || (sp->op == HFAV_OP_EULER_DT);
            const bool row_ok = (sp->op == HFAV_OP_SQRT) || (sp->op == HFAV_OP_DIV0 && q == 1);
            const std::string where = std::string(sp->name) + ": input " + std::to_string(q);
            if (want0 && T.rank != 0) return hfav_fail(HFAV_EINVAL, where + " must be 0-D");
            if (!want0 && T.rank == 0) return hfav_fail(HFAV_EINVAL, where + " must be a grid term");
            if (T.rank == row && !row_ok) return hfav_fail(HFAV_EINVAL, where + " cannot be a row term");
            if (T.rank == 0 || T.rank == row) {
                for (int ax = 0; ax < 3; ++ax)
                    if (R.in[q].off[ax] != 0)
                        return hfav_fail(HFAV_EINVAL, T.rank == 0 ? "0-D reference with an offset"
                                                                  : "row-term reference with an offset");
            }
            if (T.rank == nd) any_grid = true;
            if (T.rank == row) any_row = true;
        }
        if (sp->op == HFAV_OP_SUM_I)
            for (int ax = 0; ax < 3; ++ax)
                if (R.in[0].off[ax] != 0) return hfav_fail(HFAV_EINVAL, "SUM_I reads its input at offset 0");
        if (sp->op == HFAV_OP_DIV0 && c->terms[R.in[0].term].rank != nd)
            return hfav_fail(HFAV_EINVAL, "DIV0: input 0 must be a grid term");
        R.rank = any_grid ? nd : any_row ? row : 0;
        const int orank = sp->out_rank0 ? 0 : sp->op == HFAV_OP_SUM_I ? row : R.rank;
        for (int t : R.out) c->terms[t].rank = orank;
    }
    return HFAV_OK;
}

extern "C" int hfav_chain_create(const hfav_chain_desc *desc, hfav_chain **out) {
    if (!out) return hfav_fail(HFAV_EINVAL, "null output handle");
    *out = nullptr;
    if (!desc) return hfav_fail(HFAV_EINVAL, "null descriptor");
    hfav_chain *c = new (std::nothrow) hfav_chain();
    if (!c) return hfav_fail(HFAV_EINVAL, "out of host memory");
    int rc;
    try {
        rc = build(desc, c);
    } catch (...) {
        rc = hfav_fail(HFAV_EINVAL, "host exception while building the chain");
    }
    if (rc != HFAV_OK) {
        delete c;
        return rc;
    }
    *out = c;
    g_err.clear();
    return HFAV_OK;
}

hfav_chain::~hfav_chain() {
    if (pinned) (void)hipHostFree(pinned);
}

extern "C" void hfav_chain_destroy(hfav_chain *c) { delete c; }

extern "C" int hfav_chain_alias(hfav_chain *c, const char *goal, const char *axiom) {
    if (!c || !goal || !axiom) return hfav_fail(HFAV_EINVAL, "null argument");
    int g = -1, a = -1;
    for (int t : c->goals)
        if (c->terms[t].name == goal) g = t;
    for (int t : c->axioms)
        if (c->terms[t].name == axiom) a = t;
    if (g < 0) return hfav_fail(HFAV_EINVAL, std::string("not a goal: ") + goal);
    if (a < 0) return hfav_fail(HFAV_EINVAL, std::string("not an axiom: ") + axiom);
    if (c->terms[g].rank != c->terms[a].rank || c->terms[a].rank == 0)
        return hfav_fail(HFAV_EINVAL, "an alias pairs a goal and an axiom of the same nonzero rank");
    for (const auto &pr : c->alias)
        if (pr.first == g || pr.second == a) return hfav_fail(HFAV_EDUP, "goal or axiom already aliased");
    if ((int)c->alias.size() >= HFAV_MAX_ALIASES)
        return hfav_fail(HFAV_EINVAL, "at most " + std::to_string(HFAV_MAX_ALIASES) + " in-place pairs");
    c->alias.push_back({g, a});
    c->plan.valid = false;
    return HFAV_OK;
}

extern "C" int hfav_num_terms(const hfav_chain *c) { return c ? (int)c->terms.size() : 0; }
