// Host-side representation of a chain and its plan.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hfav.h"

struct HRef {
    int term;
    int off[3];
};

struct HRule {
    int op;
    std::vector<HRef> in;
    std::vector<int> out;        // term ids
    std::vector<double> param;
    int reduce;
    int rank;                    // iteration-space rank: 0 (scalar rule), ndim - 1
                                 // (a rule over row terms) or ndim
};

enum { TK_AXIOM = 0, TK_INTER = 1, TK_GOAL = 2 };

struct HTerm {
    std::string name;
    int kind;                    // TK_*
    int rank;
    int producer;                // rule index, -1 for axioms
    int axiom_slot;              // position in the axiom list, -1
    int goal_slot;               // position in the goal list, -1
    int out_pos;                 // output position within its producer
};

// An iteration nest with its three phases (Design, "Iteration nests").
// Perfect nests have only a steady state.
struct HNest {
    int rank;                    // 0 for a scalar nest, ndim - 1 for a nest over rows
    std::vector<int> prologue, steady, epilogue;   // rule indices
};

struct HTermPlan {
    int lo[3], hi[3];            // Minkowski extent
    bool has_ext;
    int storage;
    int window_axis;
    int window;
};

struct HPlan {
    bool valid = false;
    hfav_plan_opts opts{};
    hfav_plan_info info{};
    std::vector<HNest> nests;
    std::vector<int> outer;      // outer group per nest (nests sharing their outer loops)
    std::vector<HTermPlan> terms;
    int family = HFAV_FAMILY_NONE;
    // family bindings: term ids in the family's canonical argument order
    std::vector<int> fam_in, fam_out;
    int fam_dt_term = -1;        // 0-D term feeding dt (axiom), -1
    int fam_dt_mode = 0;         // 0: term is dt, 1: term is smax (dt = cfl/smax)
    double fam_cfl = 0.0;
    int fam_smax_goal = -1;      // 0-D goal of a fused reduction, -1
    std::vector<double> fam_param;
    int fam_row_goal = -1;       // NORM family: the row norm as a goal, -1
    // unfused: workspace offset per term (-1 = not in workspace)
    std::vector<int64_t> ws_off;
    size_t ws_bytes = 0;
    std::vector<int> exec_order; // rule order for the unfused path
    std::string json;
    // STAR_CHAIN family: stages, coefficient table, groups of fused stages
    struct StarStage {
        int r, fin, fout;
        std::vector<int> in_terms, out_terms;   // term ids of the stage's inputs / outputs
    };
    std::vector<StarStage> sstages;
    std::vector<double> scoeff;                 // host copy, (fout, fin, n_off) per stage
    std::vector<int> scoff;                     // first coefficient of each stage
    std::vector<int> sgroups;                   // first stage of each fused group
    int64_t ws_coeff = -1;                      // workspace offset of the coefficient table
    // in/out chaining: per declared alias (goal, axiom) how the plan keeps
    // it correct, and where the saved input values live in the workspace
    enum { ALIAS_SAFE = 0, ALIAS_TILE_HALOS = 1, ALIAS_FULL_COPY = 2, ALIAS_ROWS_ON_CHIP = 3, ALIAS_SEG_HALOS = 4 };
    std::vector<int> alias_handling;
    std::vector<int64_t> alias_ws;              // workspace offset of the saved values, -1
    // batched plans: per-grid sizes, y-pass segment lengths and offsets
    bool batch = false;
    std::vector<int> bnx, bny, bseg;
    std::vector<int64_t> boff;
    int64_t btotal = 0;
};

struct hfav_chain {
    int ndim = 2;
    int order[3] = {2, 1, 0};    // axis ids outermost first (0 = i, 1 = j, 2 = k)
    int dtype = HFAV_F64;
    std::vector<HTerm> terms;
    std::vector<HRule> rules;    // descriptor order
    std::vector<bool> live;      // rule needed for some goal
    std::vector<int> topo;       // topological order of live rules
    std::vector<int> axioms, goals;  // term ids in declaration order
    // declared in/out aliases: (goal term, axiom term) pairs sharing storage
    std::vector<std::pair<int, int>> alias;
    // inferred chains: the pattern rule and variable binding of each rule
    std::vector<std::pair<int, std::string>> origin;
    HPlan plan;
    void *pinned = nullptr;      // pinned host copy of the plan's coefficient table
    size_t pinned_bytes = 0;     // (staged by hfav_plan for STAR_CHAIN plans)
    std::string pinned_err;      // why staging failed (no device at plan time)
    ~hfav_chain();
};

// limits that let hfav_execute run on fixed storage
enum { HFAV_MAX_ALIASES = 16, HFAV_MAX_STAR_REFS = 96 };

// hfav_execute with the workspace chosen (exec.cpp)
int hfav_execute_ws(hfav_chain *c, const void *const *axioms, void *const *goals, void *workspace, void *stream);

// error reporting (thread-local text)
int hfav_fail(int code, const std::string &msg);

// planner entry (plan.cpp)
int hfav_plan_impl(hfav_chain *c, const hfav_plan_opts *o, hfav_plan_info *info);

// op table (chain.cpp)
struct OpSpec {
    int op;
    const char *name;
    int n_in;          // -1 = any (>= 1)
    int n_out;
    int n_param;       // minimum number of params
    int scalar_in;     // index of a 0-D input, -1 none
    int out_rank0;     // 1 if the output is 0-D
};
const OpSpec *op_spec(int op);

// STAR_CHAIN helpers (plan.cpp) and the learned model (costmodel.cpp)
bool match_star_chain(const hfav_chain *c, HPlan &p);
size_t star_group_bytes(const hfav_chain *c, const HPlan &p, int a, int b, int tile);
bool star_groups(const hfav_chain *c, HPlan &p, int D, int tile);
bool star_model_choose(const hfav_chain *c, HPlan &p, const int dims[3], hfav_config *cfg);

// tuning hooks (tune.cpp)
bool hfav_tuned_config(int family, int dtype, const int dims[3], hfav_config *cfg);
hfav_config hfav_default_config(int family, int dtype, const int dims[3]);
