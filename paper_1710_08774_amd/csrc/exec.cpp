// hfav_execute: enqueue the planned chain.  Fused families launch their
// hand-written kernel (plus a one-lane initialisation of a fused reduction
// goal: the "init" phase of a reduction, Design "Reductions & broadcasts &
// splits"); the unfused path launches one kernel per rule in topological
// order with intermediates in the caller's workspace.  No allocation, no
// synchronisation, no device-to-host traffic.
#include <cstring>
#include <string>

#include "internal.h"
#include "kernels.h"

namespace {

struct Bind {
    const hfav_chain *c;
    const void *const *ax;
    void *const *go;
    char *ws;
    // axioms read from a saved copy (fixed storage: executing allocates
    // nothing, not even host memory)
    int nredirect = 0;
    std::pair<int, const void *> redirect[HFAV_MAX_ALIASES];
    const void *ptr(int t) const {
        const HTerm &T = c->terms[t];
        for (int q = 0; q < nredirect; ++q)
            if (redirect[q].first == t) return redirect[q].second;
        if (T.kind == TK_AXIOM) return ax[T.axiom_slot];
        if (T.kind == TK_GOAL) return go[T.goal_slot];
        const int64_t off = c->plan.ws_off[t];
        return off < 0 ? nullptr : ws + off;
    }
    void *wptr(int t) const { return const_cast<void *>(ptr(t)); }
};

int dev_err(hipError_t e, const char *what) {
    if (e == hipSuccess) return HFAV_OK;
    return hfav_fail(HFAV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t term_bytes(const hfav_chain *c, int t) {
    if (c->plan.batch) {
        if (c->terms[t].rank == 0) return 8 * c->plan.bnx.size();
        return (size_t)c->plan.btotal * (c->dtype == HFAV_F64 ? 8 : 4);
    }
    if (c->terms[t].rank == 0) return 8;
    const int *d = c->plan.opts.dims;
    const size_t es = c->dtype == HFAV_F64 ? 8 : 4;
    if (c->terms[t].rank == c->ndim - 1) return (size_t)d[1] * d[2] * es;   // row term
    return (size_t)d[0] * d[1] * d[2] * es;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

int run_batch(const hfav_chain *c, const Bind &B, hipStream_t s) {
    const HPlan &p = c->plan;
    hfav::EulerBatch Bt;
    Bt.n = (int)p.bnx.size();
    Bt.nx = p.bnx.data();
    Bt.ny = p.bny.data();
    Bt.seg = p.bseg.data();
    Bt.workgroups = 0;
    if (p.family == HFAV_FAMILY_SMAX) {
        const void *U[4];
        for (int q = 0; q < 4; ++q) U[q] = B.ptr(p.fam_in[q]);
        double *out = (double *)B.wptr(p.fam_out[0]);
        int rc = dev_err(hfav::launch_fill_batch(out, Bt.n, 0.0, s), "reduction init");
        if (rc) return rc;
        return dev_err(hfav::launch_euler_smax_batch(U, Bt, p.fam_param[0], out, c->dtype, s), "batched smax launch");
    }
    hfav::EulerLaunch L;
    for (int q = 0; q < 4; ++q) { L.in[q] = B.ptr(p.fam_in[q]); L.out[q] = B.wptr(p.fam_out[q]); }
    L.nx = L.ny = 0;
    const bool step = p.family == HFAV_FAMILY_EULER_XY;
    const int dir = p.family == HFAV_FAMILY_EULER_X ? 0 : 1;
    L.bc = p.opts.boundary[step ? 0 : dir];
    L.bcy = p.opts.boundary[1];
    L.gamma = p.fam_param[0];
    L.niter = (int)p.fam_param[1];
    L.dt_src = (const double *)B.ptr(p.fam_dt_term);
    L.dt_mode = p.fam_dt_mode == 1 ? hfav::DT_FROM_SMAX : hfav::DT_VALUE;
    L.cfl = p.fam_cfl;
    L.smax_out = p.fam_smax_goal >= 0 ? (double *)B.wptr(p.fam_smax_goal) : nullptr;
    L.dtype = c->dtype;
    L.precision = p.opts.precision;
    L.cfg = p.info.config;
    if (step) {
        // the configuration's variant bit 128 makes every wait target a
        // count the x items never reach (tests the give-up path)
        const bool test_giveup = (L.cfg.variant & hfav::EULER_STEP_TEST_GIVEUP) != 0;
        return dev_err(hfav::launch_euler_step_batch(L, Bt, B.ws, test_giveup ? 64 : hfav::STEP_BATCH_SPIN_LIMIT,
                                                     test_giveup ? 1u : 0u, s),
                       "batched step launch");
    }
    if (L.smax_out) {
        int rc = dev_err(hfav::launch_fill_batch(L.smax_out, Bt.n, 0.0, s), "reduction init");
        if (rc) return rc;
    }
    return dev_err(hfav::launch_euler_batch(L, Bt, dir == 0, s), "batched sweep launch");
}

int run_fused(const hfav_chain *c, const Bind &B, hipStream_t s) {
    const HPlan &p = c->plan;
    const int *d = p.opts.dims;
    if (p.batch) return run_batch(c, B, s);
    switch (p.family) {
    case HFAV_FAMILY_HDIFF: {
        hfav::HdiffLaunch L;
        L.in = B.ptr(p.fam_in[0]);
        L.out = B.wptr(p.fam_out[0]);
        L.ni = d[0]; L.nj = d[1]; L.nk = d[2];
        L.coeff = p.fam_param[0];
        L.dtype = c->dtype;
        L.cfg = p.info.config;
        L.halo = nullptr;
        for (size_t q = 0; q < c->alias.size(); ++q)
            if (p.alias_handling[q] == HPlan::ALIAS_TILE_HALOS && L.in == L.out) L.halo = B.ws + p.alias_ws[q];
        return dev_err(hfav::launch_hdiff(L, s), "hdiff kernel launch");
    }
    case HFAV_FAMILY_EULER_X:
    case HFAV_FAMILY_EULER_Y: {
        hfav::EulerLaunch L;
        for (int q = 0; q < 4; ++q) { L.in[q] = B.ptr(p.fam_in[q]); L.out[q] = B.wptr(p.fam_out[q]); }
        L.nx = d[0]; L.ny = d[1];
        const int dir = p.family == HFAV_FAMILY_EULER_X ? 0 : 1;
        L.bc = p.opts.boundary[dir];
        L.gamma = p.fam_param[0];
        L.niter = (int)p.fam_param[1];
        L.dt_src = (const double *)B.ptr(p.fam_dt_term);
        L.dt_mode = p.fam_dt_mode == 1 ? hfav::DT_FROM_SMAX : hfav::DT_VALUE;
        L.cfl = p.fam_cfl;
        L.smax_out = p.fam_smax_goal >= 0 ? (double *)B.wptr(p.fam_smax_goal) : nullptr;
        L.dtype = c->dtype;
        L.precision = p.opts.precision;
        L.cfg = p.info.config;
        // in place when some goal is its axiom's buffer: the saved segment
        // halos live in the workspace
        for (size_t q = 0; q < c->alias.size(); ++q)
            if (p.alias_handling[q] == HPlan::ALIAS_SEG_HALOS)
                for (int f = 0; f < 4; ++f)
                    if (L.in[f] == L.out[f]) L.halo = B.ws + p.alias_ws[q];
        if (L.smax_out) {
            int rc = dev_err(hfav::launch_fill_scalar(L.smax_out, 0.0, s), "reduction init");
            if (rc) return rc;
        }
        return dev_err(dir == 0 ? hfav::launch_euler_x(L, s) : hfav::launch_euler_y(L, s), "euler sweep launch");
    }
    case HFAV_FAMILY_LAP7_CHAIN: {
        hfav::Lap7ChainLaunch L;
        L.in = B.ptr(p.fam_in[0]);
        L.out = B.wptr(p.fam_out[0]);
        L.nx = d[0]; L.ny = d[1]; L.nz = d[2];
        L.alpha = p.fam_param[0];
        L.dtype = c->dtype;
        L.cfg = p.info.config;
        return dev_err(hfav::launch_lap7_chain(L, s), "lap7 chain launch");
    }
    case HFAV_FAMILY_STAR_CHAIN: {
        // the coefficient table is copied from the pinned host copy that
        // hfav_plan staged into the workspace on the stream (a capturable
        // async copy)
        const size_t bytes = p.scoeff.size() * 8;
        if (!c->pinned || c->pinned_bytes != bytes)
            return hfav_fail(HFAV_EDEVICE, "coefficient table not staged at plan time: " + c->pinned_err);
        double *coeff = (double *)(B.ws + p.ws_coeff);
        int rc = dev_err(hipMemcpyAsync(coeff, c->pinned, bytes, hipMemcpyHostToDevice, s), "coefficient upload");
        if (rc) return rc;
        const int K = (int)p.sstages.size();
        for (size_t gi = 0; gi < p.sgroups.size(); ++gi) {
            const int a = p.sgroups[gi], b = gi + 1 < p.sgroups.size() ? p.sgroups[gi + 1] : K;
            hfav::StarGroupLaunch L{};
            L.nstage = b - a;
            L.nd = c->ndim;
            L.nx = d[0]; L.ny = d[1]; L.nz = d[2];
            L.seg = p.info.config.seg;
            L.tile = p.info.config.variant;
            L.dtype = c->dtype;
            L.coeff = coeff;
            for (int s2 = a; s2 < b; ++s2) {
                L.st[s2 - a].r = p.sstages[s2].r;
                L.st[s2 - a].fin = p.sstages[s2].fin;
                L.st[s2 - a].fout = p.sstages[s2].fout;
                L.st[s2 - a].coff = p.scoff[s2];
            }
            for (int f = 0; f < p.sstages[a].fin; ++f) L.in[f] = B.ptr(p.sstages[a].in_terms[f]);
            for (int f = 0; f < p.sstages[b - 1].fout; ++f) L.out[f] = B.wptr(p.sstages[b - 1].out_terms[f]);
            rc = dev_err(hfav::launch_star_group(L, s), "star group launch");
            if (rc) return rc;
        }
        return HFAV_OK;
    }
    case HFAV_FAMILY_SMAX: {
        const void *U[4];
        for (int q = 0; q < 4; ++q) U[q] = B.ptr(p.fam_in[q]);
        double *out = (double *)B.wptr(p.fam_out[0]);
        int rc = dev_err(hfav::launch_fill_scalar(out, 0.0, s), "reduction init");
        if (rc) return rc;
        return dev_err(hfav::launch_euler_smax(U, d[0] * d[1] * d[2], p.fam_param[0], out, c->dtype, s),
                       "smax launch");
    }
    case HFAV_FAMILY_EULER_XY: {
        hfav::EulerLaunch L;
        for (int q = 0; q < 4; ++q) { L.in[q] = B.ptr(p.fam_in[q]); L.out[q] = B.wptr(p.fam_out[q]); }
        L.nx = d[0]; L.ny = d[1];
        L.bc = p.opts.boundary[0];
        L.bcy = p.opts.boundary[1];
        L.gamma = p.fam_param[0];
        L.niter = (int)p.fam_param[1];
        L.dt_src = (const double *)B.ptr(p.fam_dt_term);
        L.dt_mode = p.fam_dt_mode == 1 ? hfav::DT_FROM_SMAX : hfav::DT_VALUE;
        L.cfl = p.fam_cfl;
        L.smax_out = p.fam_smax_goal >= 0 ? (double *)B.wptr(p.fam_smax_goal) : nullptr;
        L.dtype = c->dtype;
        L.precision = p.opts.precision;
        L.cfg = p.info.config;
        if (L.smax_out) {
            int rc = dev_err(hfav::launch_fill_scalar(L.smax_out, 0.0, s), "reduction init");
            if (rc) return rc;
        }
        return dev_err(hfav::launch_euler_xy(L, s), "two-sweep kernel launch");
    }
    case HFAV_FAMILY_NORM: {
        hfav::NormLaunch L;
        memset(&L, 0, sizeof(L));
        L.nq = (int)p.fam_in.size();
        for (int q = 0; q < L.nq; ++q) {
            L.u[q] = B.ptr(p.fam_in[q]);
            L.out[q] = B.wptr(p.fam_out[q]);
            L.c0[q] = p.fam_param[3 * q];
            L.cp[q] = p.fam_param[3 * q + 1];
            L.alpha[q] = p.fam_param[3 * q + 2];
        }
        L.norm = p.fam_row_goal >= 0 ? B.wptr(p.fam_row_goal) : nullptr;
        L.ni = d[0];
        L.nrows = d[1] * d[2];
        L.bc = p.opts.boundary[0];
        L.dtype = c->dtype;
        L.cfg = p.info.config;
        return dev_err(hfav::launch_norm(L, s), "normalisation kernel launch");
    }
    default:
        return hfav_fail(HFAV_EUNSUP, "no fused family");
    }
}

int run_unfused(const hfav_chain *c, Bind &B, hipStream_t s) {
    const HPlan &p = c->plan;
    const int *d = p.opts.dims;
    // in/out chaining: save an aliased axiom that a rule reads after its
    // goal is written (or at a neighbour's offset while writing it)
    for (size_t q = 0; q < c->alias.size(); ++q) {
        if (p.alias_handling[q] != HPlan::ALIAS_FULL_COPY) continue;
        const int g = c->alias[q].first, a = c->alias[q].second;
        const void *src = B.ptr(a);
        if (src != B.ptr(g)) continue;          // not actually in place
        void *dst = B.ws + p.alias_ws[q];
        int rc = dev_err(hipMemcpyAsync(dst, src, term_bytes(c, a), hipMemcpyDeviceToDevice, s), "alias copy");
        if (rc) return rc;
        if (B.nredirect >= HFAV_MAX_ALIASES) return hfav_fail(HFAV_EINVAL, "too many in-place pairs");
        B.redirect[B.nredirect++] = {a, dst};
    }
    for (int r : p.exec_order) {
        const HRule &R = c->rules[r];
        if (R.op == HFAV_OP_STAR) {
            const void *ptrs[HFAV_MAX_STAR_REFS];
            int offs[3 * HFAV_MAX_STAR_REFS];
            if (R.in.size() > HFAV_MAX_STAR_REFS) return hfav_fail(HFAV_EINVAL, "star rule with too many references");
            for (size_t q = 0; q < R.in.size(); ++q) {
                ptrs[q] = B.ptr(R.in[q].term);
                for (int ax = 0; ax < 3; ++ax) offs[3 * q + ax] = R.in[q].off[ax];
            }
            hfav::StarRule S;
            S.n_in = (int)R.in.size();
            S.in = ptrs;
            S.off = offs;
            S.coeff = R.param.data();
            S.out = B.wptr(R.out[0]);
            S.nx = d[0]; S.ny = d[1]; S.nz = d[2];
            for (int ax = 0; ax < 3; ++ax) S.bc[ax] = p.opts.boundary[ax];
            S.dtype = c->dtype;
            int rc = dev_err(hfav::launch_star_rule(S, s), "star rule launch");
            if (rc) return rc;
            continue;
        }
        hfav::UnfusedRule U;
        memset(&U, 0, sizeof(U));
        U.op = R.op;
        U.n_in = (int)R.in.size();
        U.n_out = (int)R.out.size();
        for (size_t q = 0; q < R.in.size(); ++q) {
            U.in[q] = B.ptr(R.in[q].term);
            U.in_rank[q] = c->terms[R.in[q].term].rank;
            for (int ax = 0; ax < 3; ++ax) U.off[q][ax] = R.in[q].off[ax];
        }
        for (size_t q = 0; q < R.out.size(); ++q) U.out[q] = B.wptr(R.out[q]);
        U.out_rank = c->terms[R.out[0]].rank;
        for (size_t q = 0; q < R.param.size() && q < hfav::UF_MAX_PARAM; ++q) U.param[q] = R.param[q];
        U.nx = d[0]; U.ny = d[1]; U.nz = d[2];
        for (int ax = 0; ax < 3; ++ax) U.bc[ax] = p.opts.boundary[ax];
        U.dtype = c->dtype;
        U.precision = p.opts.precision;
        U.ndim = c->ndim;
        if (R.op == HFAV_OP_EULER_SMAX) {
            int rc = dev_err(hfav::launch_fill_scalar((double *)U.out[0], 0.0, s), "reduction init");
            if (rc) return rc;
        }
        int rc = dev_err(hfav::launch_unfused_rule(U, s), "rule kernel launch");
        if (rc) return rc;
    }
    return HFAV_OK;
}

}  // namespace

// hfav_execute with the workspace already chosen (the caller's buffer, or
// the library's static array for hfav_execute_noalloc)
int hfav_execute_ws(hfav_chain *c, const void *const *axioms, void *const *goals, void *workspace, void *stream) {
    if (!c) return hfav_fail(HFAV_EINVAL, "null chain");
    if (!c->plan.valid) return hfav_fail(HFAV_ENOPLAN, "hfav_execute before a successful hfav_plan");
    if (!axioms || !goals) return hfav_fail(HFAV_EINVAL, "null axiom or goal array");
    for (size_t q = 0; q < c->axioms.size(); ++q)
        if (!axioms[q]) return hfav_fail(HFAV_EINVAL, "null axiom pointer " + std::to_string(q));
    for (size_t q = 0; q < c->goals.size(); ++q)
        if (!goals[q]) return hfav_fail(HFAV_EINVAL, "null goal pointer " + std::to_string(q));
    if (c->plan.ws_bytes > 0 && !workspace)
        return hfav_fail(HFAV_ENOPLAN, "this plan needs a workspace of " + std::to_string(c->plan.ws_bytes) + " bytes");
    for (size_t g = 0; g < c->goals.size(); ++g) {
        const size_t ng = term_bytes(c, c->goals[g]);
        for (size_t a = 0; a < c->axioms.size(); ++a) {
            if (!overlap(goals[g], ng, axioms[a], term_bytes(c, c->axioms[a]))) continue;
            // a declared in-place pair may share exactly the same buffer
            bool declared = false;
            for (const auto &pr : c->alias)
                if (pr.first == c->goals[g] && pr.second == c->axioms[a]) declared = true;
            if (declared && goals[g] == axioms[a]) continue;
            return hfav_fail(HFAV_EALIAS, "goal " + c->terms[c->goals[g]].name + " overlaps axiom " +
                                              c->terms[c->axioms[a]].name +
                                              (declared ? " other than exactly" : " (declare it with hfav_chain_alias)"));
        }
        for (size_t h = g + 1; h < c->goals.size(); ++h)
            if (overlap(goals[g], ng, goals[h], term_bytes(c, c->goals[h])))
                return hfav_fail(HFAV_EALIAS, "goals " + c->terms[c->goals[g]].name + " and " +
                                                  c->terms[c->goals[h]].name + " overlap");
    }
    Bind B{c, axioms, goals, (char *)workspace};
    hipStream_t s = (hipStream_t)stream;
    try {
        return c->plan.info.fused ? run_fused(c, B, s) : run_unfused(c, B, s);
    } catch (...) {
        return hfav_fail(HFAV_EINVAL, "host exception while executing");
    }
}

extern "C" int hfav_execute(hfav_chain *c, const void *const *axioms, void *const *goals, void *workspace,
                            void *stream) {
    return hfav_execute_ws(c, axioms, goals, workspace, stream);
}
