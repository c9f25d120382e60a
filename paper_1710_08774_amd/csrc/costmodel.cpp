// Learned cost model for the configuration of fused linear star chains:
// candidate configurations, the feature vector of (chain, grid, config), and
// a host FP32 forward pass of the trained network used by hfav_plan.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "../../include/hfav_mlp.h"

namespace {

std::mutex g_mu;
std::vector<float> g_params;     // empty: no model
int g_H = 0;
float g_mean[HFAV_COST_FEATURES], g_std[HFAV_COST_FEATURES];

const int kSegs[3] = {32, 64, 128};

// tile extents of a tile-shape index (2-D chains have TY = 1)
void tile_dims(int nd, int tile, int &tx, int &ty) {
    if (nd == 2) {
        static const int t2[4] = {64, 128, 256, 512};
        tx = t2[tile & 3];
        ty = 1;
    } else {
        static const int x3[4] = {16, 32, 16, 32}, y3[4] = {4, 4, 16, 8};
        tx = x3[tile & 3];
        ty = y3[tile & 3];
    }
}

std::vector<hfav_config> candidates(const hfav_chain *c, HPlan &p) {
    std::vector<hfav_config> out;
    const int K = (int)p.sstages.size();
    for (int D = 1; D <= K; ++D)
        for (int tile = 0; tile < 4; ++tile) {
            if (!star_groups(c, p, D, tile)) continue;
            for (int seg : kSegs) {
                int tx, ty;
                tile_dims(c->ndim, tile, tx, ty);
                out.push_back(hfav_config{tx * ty, D, seg, tile, 0});
            }
        }
    return out;
}

// feature vector; p.sstages must be filled (match_star_chain)
void features(const hfav_chain *c, HPlan &p, const int dims[3], const hfav_config &cfg, float *f) {
    const int K = (int)p.sstages.size();
    const int nd = c->ndim;
    const double es = c->dtype == HFAV_F64 ? 8.0 : 4.0;
    int sumr = 0, maxr = 0, sumf = 0, maxf = 0;
    double macs = 0.0;
    for (const HPlan::StarStage &S : p.sstages) {
        sumr += S.r;
        maxr = std::max(maxr, S.r);
        sumf += S.fout;
        maxf = std::max(maxf, std::max(S.fin, S.fout));
        macs += (double)S.fin * S.fout * (1 + 2 * S.r * nd);
    }
    const int D = cfg.tile_y <= 0 || cfg.tile_y > K ? K : cfg.tile_y;
    star_groups(c, p, D, cfg.variant);
    const int ngroups = (int)p.sgroups.size();
    int tx, ty;
    tile_dims(nd, cfg.variant, tx, ty);
    const int seg = cfg.seg > 0 ? cfg.seg : 32;
    double max_lds = 0.0, halo = 0.0, warm = 0.0, mid_bytes = 0.0;
    for (int g = 0; g < ngroups; ++g) {
        const int a = p.sgroups[g], b = g + 1 < ngroups ? p.sgroups[g + 1] : K;
        max_lds = std::max(max_lds, (double)star_group_bytes(c, p, a, b, cfg.variant));
        int lead = 0;
        for (int s = a; s < b; ++s) lead += p.sstages[s].r;
        // points computed per output point, weighted by the stage's work
        int h = lead;
        for (int s = a; s < b; ++s) {
            h -= p.sstages[s].r;
            const double area = (double)(tx + 2 * h) * (nd == 3 ? ty + 2 * h : 1) / ((double)tx * ty);
            halo += area * p.sstages[s].fin * p.sstages[s].fout * (1 + 2 * p.sstages[s].r * nd);
        }
        warm += 2.0 * lead / seg;
        if (g + 1 < ngroups) mid_bytes += 2.0 * es * p.sstages[b - 1].fout;
    }
    const double cells = (double)dims[0] * dims[1] * dims[2];
    const double io = es * (p.sstages[0].fin + p.sstages[K - 1].fout);
    float v[HFAV_COST_FEATURES] = {
        (float)K,
        (float)(nd == 3),
        (float)(c->dtype == HFAV_F64),
        (float)std::log2((double)dims[0]),
        (float)std::log2((double)dims[1]),
        (float)std::log2((double)dims[2]),
        (float)sumr,
        (float)maxr,
        (float)sumf,
        (float)maxf,
        (float)std::log2(macs),
        (float)io,
        (float)D,
        (float)ngroups,
        (float)(cfg.variant == 0),
        (float)(cfg.variant == 1),
        (float)(cfg.variant == 2),
        (float)(cfg.variant == 3),
        (float)std::log2((double)seg),
        (float)(max_lds / 65536.0),
        (float)std::log2(halo / macs),
        (float)warm,
        (float)mid_bytes,
        (float)std::log2(cells),
    };
    memcpy(f, v, sizeof(v));
}

float forward(const float *x) {
    const int d = HFAV_COST_FEATURES, H = g_H;
    const float *W1 = g_params.data(), *b1 = W1 + (size_t)H * d, *W2 = b1 + H, *b2 = W2 + (size_t)H * H;
    const float *W3 = b2 + H, *b3 = W3 + (size_t)H * H, *W4 = b3 + H, *b4 = W4 + H;
    std::vector<float> z(d), h1(H), h2(H), h3(H);
    for (int i = 0; i < d; ++i) z[i] = (x[i] - g_mean[i]) / g_std[i];
    auto dense = [&](const float *W, const float *b, const float *in, int nin, float *out) {
        for (int o = 0; o < H; ++o) {
            float acc = b[o];
            for (int i = 0; i < nin; ++i) acc += W[(size_t)o * nin + i] * in[i];
            out[o] = acc > 0.f ? acc : 0.f;
        }
    };
    dense(W1, b1, z.data(), d, h1.data());
    dense(W2, b2, h1.data(), H, h2.data());
    dense(W3, b3, h2.data(), H, h3.data());
    float y = b4[0];
    for (int i = 0; i < H; ++i) y += W4[i] * h3[i];
    return y;
}

bool prepare(hfav_chain *c, const int dims[3], HPlan &p) {
    if (!c) return false;
    p.opts = hfav_plan_opts{};
    for (int ax = 0; ax < 3; ++ax) {
        p.opts.dims[ax] = dims[ax];
        p.opts.boundary[ax] = HFAV_BC_PERIODIC;
    }
    return match_star_chain(c, p);
}

}  // namespace

bool star_model_choose(const hfav_chain *c, HPlan &p, const int dims[3], hfav_config *cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_params.empty()) return false;
    const std::vector<hfav_config> cand = candidates(c, p);
    float best = 1e30f;
    bool found = false;
    for (const hfav_config &k : cand) {
        float f[HFAV_COST_FEATURES];
        features(c, p, dims, k, f);
        const float y = forward(f);
        if (y < best) {
            best = y;
            *cfg = k;
            found = true;
        }
    }
    return found;
}

extern "C" int hfav_star_candidates(hfav_chain *c, const int dims[3], hfav_config *out, int max) {
    HPlan p;
    if (!dims || !prepare(c, dims, p)) return -1;
    const std::vector<hfav_config> cand = candidates(c, p);
    const int n = std::min((int)cand.size(), max);
    for (int q = 0; q < n; ++q) out[q] = cand[q];
    return n;
}

extern "C" int hfav_costmodel_features(hfav_chain *c, const int dims[3], const hfav_config *cfg, float *out) {
    HPlan p;
    if (!cfg || !out || !dims) return hfav_fail(HFAV_EINVAL, "null argument");
    if (!prepare(c, dims, p)) return hfav_fail(HFAV_EUNSUP, "not a chain of linear star stages");
    features(c, p, dims, *cfg, out);
    return HFAV_OK;
}

extern "C" int hfav_costmodel_set(const float *params, int H, const float *mean, const float *std) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!params) {
        g_params.clear();
        g_H = 0;
        return HFAV_OK;
    }
    if (H < 1 || H > 1024 || !mean || !std) return hfav_fail(HFAV_EINVAL, "bad model");
    const int d = HFAV_COST_FEATURES;
    const size_t np = (size_t)H * d + H + 2 * ((size_t)H * H + H) + H + 1;
    g_params.assign(params, params + np);
    g_H = H;
    for (int i = 0; i < d; ++i) {
        g_mean[i] = mean[i];
        g_std[i] = std[i] > 0.f ? std[i] : 1.f;
    }
    return HFAV_OK;
}

extern "C" int hfav_costmodel_predict(hfav_chain *c, const int dims[3], const hfav_config *cfg, float *out) {
    float f[HFAV_COST_FEATURES];
    int rc = hfav_costmodel_features(c, dims, cfg, f);
    if (rc != HFAV_OK) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_params.empty()) return hfav_fail(HFAV_ENOPLAN, "no cost model installed");
    *out = forward(f);
    return HFAV_OK;
}
