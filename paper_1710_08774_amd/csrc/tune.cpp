// Tile configurations: built-in defaults per kernel family, a tuning table
// filled from the autotuner's results, and the hook for the learned cost
// model.
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"
#include "../../include/hfav_tune.h"

namespace {
struct Entry {
    int family, dtype;
    int dims[3];
    hfav_config cfg;
};
std::mutex g_mu;
std::vector<Entry> g_table;
}  // namespace

hfav_config hfav_default_config(int family, int dtype, const int dims[3]) {
    hfav_config c{256, 1, 0, 0, 0};
    // measured on MI355X (the autotuner's database at the workload sizes and
    // at smaller shapes); the tuning table refines these per shape
    const double cells = (double)dims[0] * dims[1] * (dims[2] > 0 ? dims[2] : 1);
    switch (family) {
    case HFAV_FAMILY_HDIFF: {
        if (dtype == HFAV_F64) {    // 2 rows in flight, non-temporal stores, one tile range per XCD
            c.block = 256; c.seg = 32; c.variant = 2 + 16; c.xcd = -1;
        } else {
            c.block = 256; c.seg = 128; c.variant = 0; c.xcd = 0;
        }
        // small grids: shorter segments (down to 4 rows), then narrower
        // tiles, until about 2048 workgroups are in flight; short segments
        // prefetch one row (at 256x256x8 FP64: 5.4 us per execution against
        // 8.7 us with 16-row segments)
        auto wgs = [&](const hfav_config &k) {
            return (double)((dims[0] + k.block - 1) / k.block) * ((dims[1] + k.seg - 1) / k.seg) *
                   (dims[2] > 0 ? dims[2] : 1);
        };
        while (wgs(c) < 2048 && c.seg > 4) c.seg /= 2;
        while (wgs(c) < 2048 && c.block > 64) c.block /= 2;
        if (c.seg <= 8) c.variant = 1;
        break;
    }
    case HFAV_FAMILY_EULER_X: {
        // LDS-ring strips, one wave per segment of seg cells of a row (64
        // per chunk; seg = 64k - 1 leaves no chunk lane idle): 191-cell
        // segments while they give at least 16384 workgroups, else 63
        // (2048^2 FP64: 0.153 ms against 0.162 for one 4-wave workgroup
        // per row, whose 2048 workgroups fill 1.6 rounds of the chip).  The
        // wave on 2 rows x 32 cells per chunk instead, with 159-cell
        // segments, where that still gives 8192 workgroups (2048^2 FP64:
        // 0.127-0.128 ms against 0.130-0.132 with 191-cell segments and 0.129
        // for one row x 64 cells; 127-cell segments 0.129, 255 and longer
        // 0.138-0.145; 4 x 16 and 8 x 8 slower, the shorter chunks cost more
        // than the compact patch saves)
        c.block = 64;
        c.variant = 3;
        c.seg = (double)dims[1] * ((dims[0] + 190) / 191) >= 16384 ? 191 : 63;
        if (c.seg == 191 && (double)((dims[1] + 1) / 2) * ((dims[0] + 158) / 159) >= 8192) {
            c.tile_y = 2;
            c.seg = 159;
        }
        break;
    }
    case HFAV_FAMILY_EULER_Y: {
        // LDS-ring strips of 256 lanes.  A segment of seg rows walks seg + 1
        // chunk rows, so seg = Ck - 1 leaves no chunk row idle (C rows per
        // chunk).  Where they still give four rounds of the 1024 resident
        // workgroups (4 per CU): 16 columns x 16 rows per chunk (a wave on a
        // 16 x 4 patch, a chunk barrier per 16 rows) with 63- or 47-row
        // segments (2048^2 FP64: 0.128-0.129 ms at 63 rows, 0.129-0.130 at
        // 47, against 0.139 for 64 x 4 at 19 rows on the same box; 32 x 8
        // and 8 x 32 in between).  Else 64 columns x 4 rows (2- and 8-wave
        // workgroups measured slower) with the longest of 19 and 15 rows that
        // still gives three rounds, else 7, else 3 (2048^2 FP64, 64 x 4: 19
        // rows 0.147-0.149 ms, 15 rows 0.150-0.153, 23 rows 0.151, 31 rows
        // 0.153-0.156; 512^2: 7 rows 0.025 ms against 0.035 with 15).
        c.block = 256;
        const double cols16 = (dims[0] + 15) / 16;
        for (int seg : {63, 47}) {
            if (cols16 * ((dims[1] + seg - 1) / seg) >= 4096) {
                c.tile_y = 16;
                c.seg = seg;
                c.variant = 3;
                return c;
            }
        }
        const double cols = (dims[0] + 63) / 64;
        auto wgs = [&](int seg) { return cols * ((dims[1] + seg - 1) / seg); };
        c.seg = wgs(19) >= 3072 ? 19 : wgs(15) >= 3072 ? 15 : wgs(7) >= 512 ? 7 : 3;
        c.variant = 3;
        break;
    }
    case HFAV_FAMILY_EULER_XY: {
        // one wave per 60 columns x seg rows: the longest segment (fewest
        // halo rows) that still gives about 5000 waves, each XCD a
        // contiguous range of tiles (measured at 2048^2 and 512^2)
        const long long strips = (dims[0] + 59) / 60;
        c.block = 64;
        c.xcd = -1;
        c.seg = 4;
        for (int s : {16, 12, 8})
            if (strips * ((dims[1] + s - 1) / s) >= 5000) { c.seg = s; break; }
        break;
    }
    case HFAV_FAMILY_LAP7_CHAIN:
        if (cells >= 64.0 * 1024 * 1024) {
            // 2 points per lane, 4 planes in flight, runs of 8 tiles per
            // XCD: FP32 128 x 16 tiles, FP64 64 x 32 (less halo re-read
            // than 64 x 16: at 512^3 FP32 0.24 ms against 0.32)
            c.block = 1024; c.seg = 128; c.tile_y = 4; c.xcd = 8;
            c.variant = dtype == HFAV_F32 ? 7 : 6;
        } else {                                // 32 x 8 tiles, 2 planes in flight
            c.block = 256; c.seg = 64; c.variant = 1; c.tile_y = 2;
        }
        break;
    default: break;
    }
    return c;
}

// nearest entry of the same family and dtype, distance in log2 of the dims
bool hfav_tuned_config(int family, int dtype, const int dims[3], hfav_config *cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    double best = 1e30;
    bool found = false;
    for (const Entry &e : g_table) {
        if (e.family != family || e.dtype != dtype) continue;
        double dist = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            double a = std::log2((double)e.dims[ax]), b = std::log2((double)dims[ax]);
            dist += (a - b) * (a - b);
        }
        if (dist < best) {
            best = dist;
            *cfg = e.cfg;
            found = true;
        }
    }
    return found;
}

extern "C" void hfav_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

extern "C" int hfav_tuning_add(int family, int dtype, const int dims[3], const hfav_config *cfg) {
    if (!dims || !cfg || cfg->block <= 0) return HFAV_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Entry e;
    e.family = family;
    e.dtype = dtype;
    for (int ax = 0; ax < 3; ++ax) e.dims[ax] = dims[ax] > 0 ? dims[ax] : 1;
    e.cfg = *cfg;
    g_table.push_back(e);
    return HFAV_OK;
}

extern "C" int hfav_tuning_size(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_table.size();
}
