// Rule inference from patterns (Implementation, "Inference"): rules whose
// term names contain pattern variables are instantiated backward from the
// goals until every needed term is an axiom, giving the concrete terms and
// rule applications (the inference DAG; its dual, the dataflow DAG, is
// the concrete chain handed to hfav_chain_create).
//
// Term names are expressions such as "flux(u0)" or "laplace(laplace(cell))".
// In a pattern, an identifier ending in '?' ("q?") is a variable: it matches
// any non-empty substring with balanced parentheses, and the same variable
// takes the same value everywhere in one rule.  The spatial pattern
// variables of the paper's notation (i?, j?, k? with integer offsets) are
// the references' offsets relative to the rule's output point.
//
// Search: a needed term is an axiom, or already produced, or the output of
// the first rule (in descriptor order, then output order) that matches it
// and whose inputs can all be derived; a failed candidate is rolled back
// and the next one tried.  A term that is needed while it is being derived
// (a cycle) fails that candidate; derivations deeper than 64 rule
// applications fail (a pattern such as "f(q?)" needing "f(f(q?))" would
// recurse forever).
#include <cctype>
#include <cstring>
#include <map>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace {

enum { MAX_DEPTH = 64 };

struct Seg {
    bool var;
    std::string text;   // literal text or variable name (without '?')
};
using Pattern = std::vector<Seg>;
using Binding = std::map<std::string, std::string>;

bool ident_char(char ch) { return std::isalnum((unsigned char)ch) || ch == '_'; }

// Split a name into literal runs and variables; false on a malformed
// pattern (a '?' that does not end an identifier, or two variables with
// nothing between them).
bool parse(const char *s, Pattern &p) {
    p.clear();
    std::string lit;
    const size_t n = strlen(s);
    for (size_t q = 0; q < n;) {
        if (ident_char(s[q])) {
            size_t e = q;
            while (e < n && ident_char(s[e])) ++e;
            if (e < n && s[e] == '?') {
                if (!lit.empty()) p.push_back({false, lit});
                lit.clear();
                if (!p.empty() && p.back().var) return false;
                p.push_back({true, std::string(s + q, e - q)});
                q = e + 1;
            } else {
                lit.append(s + q, e - q);
                q = e;
            }
        } else {
            if (s[q] == '?') return false;
            lit.push_back(s[q]);
            ++q;
        }
    }
    if (!lit.empty()) p.push_back({false, lit});
    return true;
}

bool has_vars(const Pattern &p) {
    for (const Seg &g : p)
        if (g.var) return true;
    return false;
}

bool balanced(const std::string &s, size_t a, size_t b) {
    int depth = 0;
    for (size_t q = a; q < b; ++q) {
        if (s[q] == '(') ++depth;
        else if (s[q] == ')' && --depth < 0) return false;
    }
    return depth == 0;
}

// Match pattern segments [k, end) against s[pos, end), extending b.
bool match_from(const Pattern &p, size_t k, const std::string &s, size_t pos, Binding &b) {
    if (k == p.size()) return pos == s.size();
    const Seg &g = p[k];
    if (!g.var) {
        if (s.compare(pos, g.text.size(), g.text) != 0) return false;
        return match_from(p, k + 1, s, pos + g.text.size(), b);
    }
    auto it = b.find(g.text);
    if (it != b.end()) {
        if (s.compare(pos, it->second.size(), it->second) != 0) return false;
        return match_from(p, k + 1, s, pos + it->second.size(), b);
    }
    for (size_t e = pos + 1; e <= s.size(); ++e) {
        if (!balanced(s, pos, e)) continue;
        b[g.text] = s.substr(pos, e - pos);
        if (match_from(p, k + 1, s, e, b)) return true;
        b.erase(g.text);
    }
    return false;
}

bool subst(const Pattern &p, const Binding &b, std::string &out) {
    out.clear();
    for (const Seg &g : p) {
        if (!g.var) {
            out += g.text;
            continue;
        }
        auto it = b.find(g.text);
        if (it == b.end()) return false;
        out += it->second;
    }
    return true;
}

struct PRule {
    const hfav_rule *src;
    std::vector<Pattern> in, out;
};

struct Inst {
    int pattern;
    Binding bind;
    std::vector<std::string> in, out;
};

struct Infer {
    std::vector<PRule> rules;
    std::set<std::string> axioms;
    std::vector<Inst> insts;
    std::map<std::string, int> produced;
    std::set<std::string> active;

    void rollback(size_t mark) {
        while (insts.size() > mark) {
            for (const std::string &o : insts.back().out) produced.erase(o);
            insts.pop_back();
        }
    }

    bool derive(const std::string &t, int depth) {
        if (axioms.count(t) || produced.count(t)) return true;
        if (depth >= MAX_DEPTH || active.count(t)) return false;
        active.insert(t);
        for (size_t r = 0; r < rules.size(); ++r) {
            const PRule &R = rules[r];
            for (size_t k = 0; k < R.out.size(); ++k) {
                Binding b;
                if (!match_from(R.out[k], 0, t, 0, b)) continue;
                Inst I;
                I.pattern = (int)r;
                I.bind = b;
                bool ok = true;
                for (const Pattern &po : R.out) {
                    std::string name;
                    if (!subst(po, b, name) || axioms.count(name) || produced.count(name)) ok = false;
                    I.out.push_back(name);
                }
                for (const Pattern &pi : R.in) {
                    std::string name;
                    if (!subst(pi, b, name)) ok = false;
                    I.in.push_back(name);
                }
                if (!ok) continue;
                const size_t mark = insts.size();
                for (const std::string &name : I.in)
                    if (!derive(name, depth + 1)) { ok = false; break; }
                // an input's derivation may have produced one of these outputs
                for (const std::string &name : I.out)
                    if (ok && produced.count(name)) ok = false;
                if (!ok) {
                    rollback(mark);
                    continue;
                }
                for (const std::string &name : I.out) produced[name] = (int)insts.size();
                insts.push_back(I);
                active.erase(t);
                return true;
            }
        }
        active.erase(t);
        return false;
    }
};

}  // namespace

extern "C" int hfav_chain_infer(const hfav_chain_desc *d, hfav_chain **out) {
    if (!out) return hfav_fail(HFAV_EINVAL, "null output handle");
    *out = nullptr;
    if (!d) return hfav_fail(HFAV_EINVAL, "null descriptor");
    if (d->n_axiom < 1 || !d->axioms || d->n_goal < 1 || !d->goals || d->n_rule < 0 ||
        (d->n_rule > 0 && !d->rules))
        return hfav_fail(HFAV_EINVAL, "descriptor needs axioms, goals and a rule list");
    try {
        Infer F;
        for (int a = 0; a < d->n_axiom; ++a) {
            const char *nm = d->axioms[a].name;
            if (!nm || !*nm || strchr(nm, '?')) return hfav_fail(HFAV_EINVAL, "axioms must be concrete names");
            F.axioms.insert(nm);
        }
        for (int r = 0; r < d->n_rule; ++r) {
            const hfav_rule &src = d->rules[r];
            PRule R;
            R.src = &src;
            if (src.n_in < 1 || !src.in || src.n_out < 1 || !src.out)
                return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": needs inputs and outputs");
            std::set<std::string> outvars;
            for (int q = 0; q < src.n_out; ++q) {
                Pattern p;
                if (!src.out[q] || !*src.out[q] || !parse(src.out[q], p))
                    return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": malformed output pattern");
                std::set<std::string> vs;
                for (const Seg &g : p)
                    if (g.var) vs.insert(g.text);
                if (q == 0) outvars = vs;
                else if (vs != outvars)
                    return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) +
                                                      ": every output must use the same variables");
                R.out.push_back(p);
            }
            for (int q = 0; q < src.n_in; ++q) {
                Pattern p;
                if (!src.in[q].term || !*src.in[q].term || !parse(src.in[q].term, p))
                    return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": malformed input pattern");
                for (const Seg &g : p)
                    if (g.var && !outvars.count(g.text))
                        return hfav_fail(HFAV_EINVAL, "rule " + std::to_string(r) + ": input variable " + g.text +
                                                          "? does not occur in the outputs");
                R.in.push_back(p);
            }
            F.rules.push_back(R);
        }
        for (int g = 0; g < d->n_goal; ++g) {
            const char *nm = d->goals[g];
            if (!nm || !*nm || strchr(nm, '?')) return hfav_fail(HFAV_EINVAL, "goals must be concrete names");
            if (F.axioms.count(nm)) return hfav_fail(HFAV_EINVAL, std::string("a goal cannot be an axiom: ") + nm);
            if (!F.derive(nm, 0)) return hfav_fail(HFAV_EUNSAT, std::string("goal not derivable: ") + nm);
        }
        if ((int)F.insts.size() > HFAV_MAX_RULES) return hfav_fail(HFAV_EINVAL, "too many rule applications");
        // the concrete chain: one rule per application, in derivation order
        std::vector<std::vector<hfav_ref>> refs(F.insts.size());
        std::vector<std::vector<const char *>> outs(F.insts.size());
        std::vector<hfav_rule> rules(F.insts.size());
        for (size_t a = 0; a < F.insts.size(); ++a) {
            const Inst &I = F.insts[a];
            const hfav_rule &src = *F.rules[I.pattern].src;
            for (size_t q = 0; q < I.in.size(); ++q) {
                hfav_ref ref;
                ref.term = I.in[q].c_str();
                for (int ax = 0; ax < 3; ++ax) ref.off[ax] = src.in[q].off[ax];
                refs[a].push_back(ref);
            }
            for (const std::string &o : I.out) outs[a].push_back(o.c_str());
            hfav_rule &R = rules[a];
            R = src;
            R.n_in = (int)refs[a].size();
            R.in = refs[a].data();
            R.n_out = (int)outs[a].size();
            R.out = outs[a].data();
        }
        hfav_chain_desc cd = *d;
        cd.n_rule = (int)rules.size();
        cd.rules = rules.empty() ? nullptr : rules.data();
        hfav_chain *c = nullptr;
        const int rc = hfav_chain_create(&cd, &c);
        if (rc != HFAV_OK) return rc;
        // provenance of each concrete rule: pattern index and binding
        c->origin.resize(F.insts.size());
        for (size_t a = 0; a < F.insts.size(); ++a) {
            std::string s;
            for (const auto &kv : F.insts[a].bind) s += (s.empty() ? "" : ",") + kv.first + "?=" + kv.second;
            c->origin[a] = {F.insts[a].pattern, s};
        }
        *out = c;
        return HFAV_OK;
    } catch (...) {
        return hfav_fail(HFAV_EINVAL, "host exception during inference");
    }
}
