// Launch interface between the host planner/dispatcher and the HIP kernels.
// Host-only declarations; every launcher enqueues on the given stream and
// returns the HIP error of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/hfav.h"

namespace hfav {

enum { DT_VALUE = 0, DT_FROM_SMAX = 1 };

// One directional Godunov sweep, fused.  Pointers are in the sweep frame:
// in[0..3] = (rho, normal momentum, transverse momentum, E).
struct EulerLaunch {
    const void *in[4];
    void *out[4];
    int nx, ny;            // grid (the sweep runs along x for EULER_X, y for EULER_Y)
    int bc;                // hfav_bc along the sweep axis
    double gamma;
    int niter;
    const double *dt_src;  // dt itself, or smax when dt_mode = DT_FROM_SMAX
    int dt_mode;
    double cfl;
    double *smax_out;      // nullable: fused max(|u|+c,|v|+c) of the updated state
    int dtype;             // hfav_dtype
    int precision;         // hfav_precision
    hfav_config cfg;
    int bcy;               // boundary along y (both sweeps in one kernel)
    // in place (out[q] == in[q]): workspace of euler_inplace_bytes for the
    // cells around the segment boundaries, saved before the sweep; null
    // when not in place.  Strip kernels only (variant 3; x: 64-cell chunks,
    // y: 4-row chunks).
    void *halo = nullptr;
};
// workspace bytes of an in-place sweep along x (dir 0) or y (dir 1)
size_t euler_inplace_bytes(int nx, int ny, int dir, int dtype, const hfav_config &cfg);
// segment length a strip sweep runs with (the configuration's, or its default)
int euler_strip_seg(int n, int dir, const hfav_config &cfg);
// x strip: rows per workgroup (tile_y, 1 when tile_y <= 1), and whether
// the (rows, block) pair is built: 1 x 64/128/256, 2 x 64
int euler_x_strip_rows(const hfav_config &cfg);
bool euler_x_strip_ok(const hfav_config &cfg);
// y strip: columns per workgroup (tile_y, 64 when tile_y <= 1), and whether
// the (columns, block) pair is built: 64 x 128/256/512, 32/16/8 x 256
int euler_y_strip_cols(const hfav_config &cfg);
bool euler_y_strip_ok(const hfav_config &cfg);
hipError_t launch_euler_x(const EulerLaunch &L, hipStream_t s);
// x sweep then y sweep of one time step in one kernel; in/out in the
// physical frame (rho, mx, my, E), bc along x, bcy along y, cfg.seg rows per
// segment
hipError_t launch_euler_xy(const EulerLaunch &L, hipStream_t s);
hipError_t launch_euler_y(const EulerLaunch &L, hipStream_t s);

// Batched sweeps over many grids in packed buffers (grid g at element offset
// sum_{h<g} nx_h*ny_h of every plane); dt_src and smax_out point to arrays
// of one value per grid.
struct EulerBatch {
    int n;
    const int *nx, *ny;   // host arrays, n entries each
    const int *seg;       // y-pass segment length per grid
    int workgroups;       // persistent pool size, 0 = default
};
hipError_t launch_euler_batch(const EulerLaunch &L, const EulerBatch &B, bool x_pass, hipStream_t s);
hipError_t launch_euler_smax_batch(const void *const *U, const EulerBatch &B, double gamma, double *out,
                                   int dtype, hipStream_t s);
hipError_t launch_fill_batch(double *p, int n, double v, hipStream_t s);
// Both sweeps of a time step for every grid of a batch in one persistent
// launch (after a one-workgroup launch that zeroes its control block and
// the CFL slots and deals the grids to the XCDs).  in/out in the physical
// frame (rho, mx, my, E), bc along x, bcy along y, B.seg rows per y item.
// Workspace: the control block (status word at byte 0: bit 0 set when a y
// item gave up waiting for its grid's x items, bit 1 when an XCD's items
// were not all taken; per-grid counters from STEP_BATCH_CNT_OFFSET), then
// the x-swept state.  A y item polls at most spin_limit times; wait_extra
// (0 in use) is added to the count it awaits.
constexpr size_t STEP_BATCH_CTL_BYTES = 4096;
constexpr size_t STEP_BATCH_CNT_OFFSET = 256;
constexpr int STEP_BATCH_SPIN_LIMIT = 1 << 18;
constexpr int EULER_STEP_TEST_GIVEUP = 128;     // configuration variant bit
size_t step_batch_ws_bytes(long long cells, int dtype);
hipError_t launch_euler_step_batch(const EulerLaunch &L, const EulerBatch &B, void *ws, int spin_limit,
                                   unsigned wait_extra, hipStream_t s);

// smax = max over cells of max(|u|+c, |v|+c); *out must hold 0 beforehand.
hipError_t launch_euler_smax(const void *const *U, int n, double gamma, double *out,
                             int dtype, hipStream_t s);
// *p = v for a 0-D term (a fill kernel rather than a memset, so that the
// call can be captured in a graph)
hipError_t launch_fill_scalar(double *p, double v, hipStream_t s);
// *out = cfl / *smax
hipError_t launch_dt_from_smax(const double *smax, double cfl, double *out, hipStream_t s);

struct HdiffLaunch {
    const void *in;
    void *out;
    int ni, nj, nk;
    double coeff;
    int dtype;
    hfav_config cfg;
    // in-place execution (out == in): device scratch for the copies of the
    // at-risk halo columns and rows, hdiff_inplace_bytes() long; null
    // otherwise
    void *halo;
};
hipError_t launch_hdiff(const HdiffLaunch &L, hipStream_t s);
// bytes of the halo copies an in-place hdiff launch needs at this
// configuration (4 columns per x-tile boundary, 4 rows per row segment)
size_t hdiff_inplace_bytes(int ni, int nj, int nk, int dtype, const hfav_config &cfg);

struct Lap7ChainLaunch {
    const void *in;
    void *out;
    int nx, ny, nz;
    double alpha;          // out = u + alpha * lap7(lap7(u))
    int dtype;
    hfav_config cfg;
};
hipError_t launch_lap7_chain(const Lap7ChainLaunch &L, hipStream_t s);

// ---- normalisation chain: one workgroup per row of i (NORM family)
enum { NORM_MAX_Q = 8, NORM_REG_BUDGET = 32 };   // fields; register slots nq * cells per thread
struct NormLaunch {
    const void *u[NORM_MAX_Q];
    void *out[NORM_MAX_Q];
    void *norm;                       // row goal (nrows values), or null
    double c0[NORM_MAX_Q], cp[NORM_MAX_Q], alpha[NORM_MAX_Q];
    int nq, ni, nrows;
    int bc;                           // boundary along i
    int dtype;
    hfav_config cfg;                  // block; seg = cells per thread (variants 0, 2, 3);
                                      // variant 0 registers, 1 two streamed sweeps,
                                      // 2 registers + non-temporal stores, 3 registers
                                      // + non-temporal loads and stores
};
bool norm_config_ok(int nq, int ni, const hfav_config &c);
hfav_config norm_default_config(int nq, int ni, int dtype);
hipError_t launch_norm(const NormLaunch &L, hipStream_t s);

// ---- unfused path: one kernel per rule over full arrays
enum { UF_MAX_IN = 24, UF_MAX_OUT = 8, UF_MAX_PARAM = 4 };
struct UnfusedRule {
    int op;
    int n_in, n_out;
    const void *in[UF_MAX_IN];        // grid inputs (rank > 0) or 0-D pointers
    int off[UF_MAX_IN][3];
    int in_rank[UF_MAX_IN];
    void *out[UF_MAX_OUT];
    int out_rank;                     // 0 for 0-D outputs
    double param[UF_MAX_PARAM];
    int nx, ny, nz;
    int bc[3];
    int dtype;
    int precision;
    int ndim;                         // row terms have rank ndim - 1
};
hipError_t launch_unfused_rule(const UnfusedRule &R, hipStream_t s);

// Generic linear star rule (any number of references), unfused.
struct StarRule {
    int n_in;
    const void *const *in;   // host array of n_in device pointers
    const int *off;          // host array (n_in, 3)
    const double *coeff;     // host array n_in
    void *out;
    int nx, ny, nz;
    int bc[3];
    int dtype;
};
hipError_t launch_star_rule(const StarRule &R, hipStream_t s);

// ---- fused groups of linear star stages
enum { SG_MAX_F = 5, SG_MAX_STAGES = 6, SG_MAX_LDS = 65536 };
struct StarGroupLaunch {
    struct Stage {
        int r, fin, fout;
        int coff;                      // first coefficient of the stage in the device table
        int lds, planes, hx, hy, px, py;   // ring layout (filled by the launcher)
    };
    const void *in[SG_MAX_F];
    void *out[SG_MAX_F];
    const double *coeff;               // device coefficient table
    int nstage, nd;
    int nx, ny, nz;
    int seg;
    int tile;                          // tile-shape index
    int dtype;
    Stage st[SG_MAX_STAGES];
};
hipError_t launch_star_group(StarGroupLaunch &L, hipStream_t s);
size_t star_group_lds_bytes(const StarGroupLaunch &L);

}  // namespace hfav
