/*
 * hfav.h - fused stencil-chain execution on AMD Instinct MI355X (gfx950).
 *
 * A chain is stated the way the paper states its problems (Introduction,
 * "Contributions"; Implementation, "Inference"): AXIOMS are the input arrays,
 * GOALS the outputs, and RULES the kernels, each rule reading named terms at
 * constant relative offsets (the translation-free frame of Design,
 * "Fundamentals") and producing named terms at offset zero.  The library
 *
 *   hfav_chain_create  records and validates the chain (dataflow DAG: rule
 *                      call sites as vertices, terms as edges; Design,
 *                      "Dataflow"; one producer per term, Related Work),
 *   hfav_plan          builds the iteration-nest DAG, fuses it (Design,
 *                      "Fusion", both fuse_inest_dag and fuse_inest), places
 *                      0-D broadcasts and reductions in prologue / epilogue
 *                      phases (Design, "Reductions & broadcasts & splits"),
 *                      derives every term's extent by Minkowski sums of the
 *                      offsets (Design, "Variables and storage"), and the
 *                      rolling-window depth of every intermediate from its
 *                      reuse span (Design, "Contraction"); it then selects a
 *                      hand-written fused gfx950 kernel family and its tile
 *                      configuration, or the unfused one-kernel-per-rule path,
 *   hfav_execute       enqueues the chain on a HIP stream.
 *
 * All functions are thread-compatible (one handle per thread at a time),
 * never abort and never throw; they return an hfav_status.  Strings returned
 * by the library stay valid until the next call on the same thread.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller.
 * Grid terms are dense, C order, innermost axis i (x) fastest:
 * element (i, j, k) of an (nx, ny, nz) grid is at ((k*ny + j)*nx + i).
 * 0-D terms (rank 0) are device pointers to one element.  The element type
 * of every term is the chain's dtype (hfav_chain_desc.dtype); 0-D terms are
 * always double.
 */
#ifndef HFAV_H
#define HFAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef enum {
    HFAV_OK = 0,
    HFAV_EINVAL = 1,   /* null or ill-formed argument, unknown op, wrong arity,
                          bad dims, ndim not in {2,3} */
    HFAV_EUNSAT = 2,   /* a goal (or a rule input) is not derivable from the
                          axioms through the rules (Implementation, "Inference") */
    HFAV_EDUP = 3,     /* two rules produce the same term, or a rule produces an
                          axiom: one producer per term (Related Work) */
    HFAV_ECYCLE = 4,   /* the dataflow graph has a cycle (Design, "Dataflow") */
    HFAV_EUNSUP = 5,   /* valid chain but no kernel can run it in the requested
                          mode / precision */
    HFAV_EALIAS = 6,   /* an output buffer overlaps an input buffer; aliasing is
                          not declared by this interface (Design, "In/out
                          chaining") */
    HFAV_ENOPLAN = 7,  /* execute before a successful plan, or a missing
                          workspace */
    HFAV_EDEVICE = 8,  /* HIP runtime or launch error; text in hfav_last_error */
    HFAV_ESIZE = 9     /* the plan's workspace exceeds the library's static
                          workspace (hfav_execute_noalloc) */
} hfav_status;

/* ------------------------------------------------------------------ enums */
typedef enum { HFAV_F64 = 0, HFAV_F32 = 1 } hfav_dtype;

/* Rule catalogue.  The kernels themselves are compiled into the library; a
 * rule names one and binds its arguments BY POSITION (Implementation: only
 * the function name and argument positions matter).  "in" lists the input
 * references in argument order, "out" the produced terms.  Offsets are
 * (di, dj, dk).  Params are doubles. */
typedef enum {
    /* COSMO horizontal diffusion (Performance, "COSMO Micro-Kernels") */
    HFAV_OP_HDIFF_LAP = 1,   /* in: u(c), u(+i), u(-i), u(+j), u(-j) -> lap
                                lap = (e+w) + (n+s) - 4c                        */
    HFAV_OP_HDIFF_FLX = 2,   /* in: lap(0), lap(+i), u(0), u(+i) -> flx
                                flx = lap(+i)-lap(0); 0 if flx*(u(+i)-u(0)) > 0 */
    HFAV_OP_HDIFF_FLY = 3,   /* same along j: lap(0), lap(+j), u(0), u(+j) -> fly */
    HFAV_OP_HDIFF_OUT = 4,   /* in: u, flx(0), flx(-i), fly(0), fly(-j) -> out;
                                param[0] = coeff;
                                out = u - coeff*((flx-flx(-i)) + (fly-fly(-j)))  */
    /* Directionally split Godunov sweep (Performance, "Hydro2D").  Fields of
     * a sweep are ordered (rho, normal momentum, transverse momentum, E);
     * the same rules with offsets along j and swapped momenta give the y
     * pass, as the paper describes for its dimensionally split operator. */
    HFAV_OP_EULER_PRIM = 10,   /* in: rho, mn, mt, E (offset 0) -> r, un, ut, p, c;
                                  param[0] = gamma (constoprim + eos)             */
    HFAV_OP_EULER_SLOPE = 11,  /* in: r(-1), r(0), r(+1), un(..), ut(..), p(..)
                                  (12 refs, offsets along the sweep) -> dr, dun,
                                  dut, dp (van Leer limited)                       */
    HFAV_OP_EULER_TRACE = 12,  /* in: r, un, ut, p, c, dr, dun, dut, dp, dt (0-D)
                                  -> 4 plus-face values (rho, un, ut, p) at m+1/2,
                                  then 4 minus-face values at m-1/2               */
    HFAV_OP_EULER_RIEMANN = 13,/* in: 4 plus-face values at offset 0, 4 minus-face
                                  values at offset +1 (qleftright) -> Godunov
                                  state (rho, un, ut, p) at x/t = 0;
                                  param[0] = gamma, param[1] = Newton iterations  */
    HFAV_OP_EULER_FLUX = 14,   /* in: Godunov state -> 4 fluxes; param[0] = gamma */
    HFAV_OP_EULER_UPDATE = 15, /* in: 4 conserved (0), 4 fluxes (0), 4 fluxes (-1),
                                  dt (0-D) -> 4 conserved                          */
    HFAV_OP_EULER_SMAX = 16,   /* in: rho, mx, my, E -> smax (0-D, reduce MAX):
                                  max over cells of max(|u|+c, |v|+c); gamma      */
    HFAV_OP_EULER_DT = 17,     /* 0-D: in: smax -> dt = param[0](CFL)/smax        */
    /* Linear stencils */
    HFAV_OP_LAP7 = 20,         /* in: u(0), u(+i), u(-i), u(+j), u(-j), u(+k), u(-k)
                                  -> ((e+w)+(n+s))+(t+b) - 6c                      */
    HFAV_OP_AXPY = 21,         /* in: a, b -> a + param[0]*b                       */
    HFAV_OP_STAR = 22,         /* in: n refs -> sum_q param[q]*ref_q, accumulated
                                  in reference order from zero                    */
    /* Reductions, broadcasts and splits (Design, "Reductions & broadcasts &
     * splits"; the normalisation example of Performance, "Normalization
     * Example").  A ROW TERM has rank ndim - 1: one value per row of the
     * innermost axis i, indexed by the remaining axes (j, or (j, k)), stored
     * as a dense array of dims[1] * dims[2] elements in the chain dtype.
     * References to row terms take no offsets. */
    HFAV_OP_SUMSQ = 30,        /* in: 1..24 grid refs -> sum_q ref_q^2, accumulated
                                  in reference order from zero                    */
    HFAV_OP_SUM_I = 31,        /* in: x (grid, offset 0) -> row term s = sum over i
                                  of x; reduce must be HFAV_REDUCE_SUM (identity
                                  0, any association order: the init, accumulate
                                  and finalise phases of a reduction)             */
    HFAV_OP_SQRT = 32,         /* in: x (grid or row term) -> sqrt(x), same rank  */
    HFAV_OP_DIV0 = 33          /* in: a (grid), b (grid, or row term broadcast
                                  along i) -> a / b, and 0 where b == 0           */
} hfav_op;

typedef enum { HFAV_REDUCE_NONE = 0, HFAV_REDUCE_MAX = 1, HFAV_REDUCE_SUM = 2 } hfav_reduce;
typedef enum { HFAV_BC_PERIODIC = 0, HFAV_BC_TRANSMISSIVE = 1 } hfav_bc;
typedef enum { HFAV_MODE_AUTO = 0, HFAV_MODE_FUSED = 1, HFAV_MODE_UNFUSED = 2 } hfav_mode;
typedef enum {
    HFAV_PREC_NATIVE = 0,     /* all arithmetic in the chain dtype */
    HFAV_PREC_F32_F64ACC = 1  /* F32 storage and arithmetic, except the Riemann
                                 pressure iteration and the conservative update
                                 accumulation, which run in F64 */
} hfav_precision;
typedef enum {
    HFAV_CONFIG_DEFAULT = 0,  /* built-in per-family default */
    HFAV_CONFIG_TUNED = 1,    /* tuning table (hfav_tuning_add), else default */
    HFAV_CONFIG_MODEL = 2,    /* learned cost model (hfav_costmodel_set), else default */
    HFAV_CONFIG_FORCED = 3    /* hfav_plan_opts.forced */
} hfav_config_source;

typedef enum {
    HFAV_FAMILY_NONE = 0,     /* no fused kernel: unfused path */
    HFAV_FAMILY_HDIFF = 1,
    HFAV_FAMILY_EULER_X = 2,
    HFAV_FAMILY_EULER_Y = 3,
    HFAV_FAMILY_LAP7_CHAIN = 4,
    HFAV_FAMILY_STAR_CHAIN = 5,
    HFAV_FAMILY_SMAX = 6,
    HFAV_FAMILY_EULER_Y_BATCH = 7, /* tuning-table key only: the segment length
                                     (config.seg) of one grid's batched y
                                     sweep, by that grid's (nx, ny) */
    HFAV_FAMILY_EULER_XY = 9, /* both sweeps of a time step (x then y, same dt)
                                 in one kernel: the x-swept state stays on
                                 chip (config.seg = rows per segment) */
    HFAV_FAMILY_NORM = 8      /* flux differences along i (STAR, two refs at
                                 di = 0 and +1) of nq <= 8 fields, SUMSQ of the
                                 fluxes, SUM_I, SQRT, one DIV0 and one AXPY per
                                 field; optional row goal: the norm.  One
                                 workgroup per row runs both inner sweeps */
} hfav_family;

typedef enum {
    HFAV_STORE_FULL = 0,       /* full array in HBM (axiom, goal, or split) */
    HFAV_STORE_REGISTER = 1,   /* window of 1: a value in a register */
    HFAV_STORE_INNER = 2,      /* rolling window along the innermost axis only
                                  ("inner" rotation, Design "Contraction") */
    HFAV_STORE_OUTER = 3,      /* rolling window of slabs along an outer axis
                                  ("outer" rotation) */
    HFAV_STORE_SCALAR = 4      /* 0-D term */
} hfav_storage;
/* A row term produced and consumed inside one outer iteration is REGISTER
 * (one value per row); a grid term passed between two inner sweeps of one
 * outer iteration is OUTER with a window of one slab (the row). */

/* --------------------------------------------------------------- the chain */
typedef struct {
    const char *term;   /* term name */
    int off[3];         /* (di, dj, dk) relative offset */
} hfav_ref;

typedef struct {
    int op;                     /* hfav_op */
    int n_in;                   /* number of input references */
    const hfav_ref *in;
    int n_out;                  /* number of produced terms */
    const char *const *out;     /* produced term names (offset 0) */
    int n_param;
    const double *param;
    int reduce;                 /* hfav_reduce: MAX makes the (single) output a
                                   0-D term accumulated over the iteration space
                                   (EULER_SMAX); SUM goes with SUM_I */
} hfav_rule;

typedef struct {
    const char *name;
    int rank;                   /* 0 for a scalar (device pointer to one double),
                                   ndim for a grid, ndim - 1 for a row term */
} hfav_term_decl;

typedef struct {
    int ndim;                   /* 2 or 3 */
    const char *loop_order;     /* axis letters outermost first, e.g. "kji" or
                                   "ji"; NULL means "kji" / "ji" (Design,
                                   "Fundamentals": user-selected global order) */
    int dtype;                  /* hfav_dtype of every grid term */
    int n_axiom;
    const hfav_term_decl *axioms;
    int n_goal;
    const char *const *goals;
    int n_rule;
    const hfav_rule *rules;
} hfav_chain_desc;

typedef struct hfav_chain hfav_chain;   /* opaque */

/* Fused-kernel tile configuration (autotuner / cost-model search space). */
typedef struct {
    int block;      /* threads per workgroup (64, 128, 256, 512, 1024) */
    int tile_y;     /* family-specific second tile parameter (prefetch depth
                       of the 7-point chain; columns per workgroup of the y
                       strip kernel, 8, 16, 32 or 64; rows per workgroup of
                       the x strip kernel, 1 or 2), or 1 */
    int seg;        /* cells streamed per thread along the streamed axis */
    int variant;    /* family-specific kernel variant, 0 = default.
                       EULER_X / EULER_Y: 0 register budget free, 1 at least
                       4 waves per SIMD, 2 at least 5, 3 LDS-ring strip
                       kernel (y: tile_y columns (1: 64) x block / tile_y
                       rows per chunk, 64 x 2, 4 or 8 or 32 x 8, 16 x 16,
                       8 x 32; segments of seg rows; x: tile_y rows (1
                       or 2) x block / tile_y cells per chunk, 1 x 64, 128
                       or 256 or 2 x 32, segments of seg cells, 0 =
                       whole rows; a segment of seg cells walks seg + 1
                       chunk positions); + 64 every Newton step of the
                       Riemann solver is taken (by default the iteration
                       stops once an iterate repeats, with the same
                       result bit for bit).  EULER_XY and the batched
                       sweeps take the + 64 bit too.
                       HDIFF: row prefetch depth 1 -> 1, 2 -> 2, 4 -> 8,
                       otherwise 4; + 8 DPP lane exchange; + 16
                       non-temporal output stores.  LAP7_CHAIN: tile shape
                       (1-5 plane rings, one point per lane; 6-9 plane
                       rings with 2 or 4 points per lane: 64 x 32,
                       128 x 16, FP32 128 x 32 and 256 x 16, FP64 64 x 32
                       for 8 and 9; 10-14 z windows in registers);
                       + 32 non-temporal output stores.  STAR_CHAIN: tile
                       shape.
                       NORM: 0 row in registers (block * seg >= the row,
                       fields * seg <= 32), 1 two streamed sweeps (block
                       64, 128 or 256, any row), 2 and 3 as 0 with
                       non-temporal stores, or loads and stores. */
    int xcd;        /* workgroup order over the 8 XCDs: 0 = hardware order,
                       G > 0 = runs of G consecutive tiles per XCD,
                       -1 = one contiguous range of tiles per XCD */
} hfav_config;

typedef struct {
    int dims[3];                /* nx, ny, nz (nz = 1 for ndim 2) */
    int boundary[3];            /* hfav_bc per axis (i, j, k) */
    int mode;                   /* hfav_mode */
    int precision;              /* hfav_precision */
    int config_source;          /* hfav_config_source */
    hfav_config forced;         /* used when config_source = FORCED */
} hfav_plan_opts;

#define HFAV_MAX_RULES 64
#define HFAV_MAX_NESTS 8

typedef struct {
    int n_rules;                        /* rules kept after pruning dead ones */
    int rule_order[HFAV_MAX_RULES];     /* topological order (descriptor indices) */
    int n_nests;                        /* iteration nests after fusion */
    int nest_of_rule[HFAV_MAX_RULES];   /* nest index per descriptor rule, -1 if pruned */
    int phase_of_rule[HFAV_MAX_RULES];  /* 0 prologue, 1 steady state, 2 epilogue */
    int family;                         /* hfav_family chosen (NONE = unfused) */
    int fused;                          /* 1 if hfav_execute runs a fused kernel */
    int streamed_axis;                  /* axis streamed by the fused kernel (0 i, 1 j, 2 k) */
    hfav_config config;                 /* tile configuration chosen */
    int config_source;                  /* where the configuration came from */
    int64_t footprint_unfused;          /* elements of all intermediates as full arrays */
    int64_t footprint_contracted;       /* elements of all intermediates after contraction */
    int max_window;                     /* largest window depth (slabs or elements) */
    double bytes_per_cell_fused;        /* compulsory HBM bytes per cell: axioms once + goals once */
    double bytes_per_cell_unfused;      /* HBM bytes per cell of the one-kernel-per-rule path */
    size_t workspace_bytes;             /* device workspace hfav_execute needs (0 for most fused) */
    int outer_of_nest[HFAV_MAX_NESTS];  /* nests with the same value share their outer
                                           loops (every axis but i): a split that only
                                           the inner axis needs, such as a reduction
                                           along i feeding a broadcast along i, leaves
                                           one outer nest holding two inner sweeps */
} hfav_plan_info;

typedef struct {
    const char *name;
    int kind;                   /* 0 axiom, 1 intermediate, 2 goal */
    int rank;
    int producer;               /* descriptor rule index, -1 for an axiom */
    int ext_lo[3], ext_hi[3];   /* Minkowski extent relative to the nest point */
    int storage;                /* hfav_storage */
    int window_axis;            /* axis of the rolling window (0 i, 1 j, 2 k), -1 none */
    int window;                 /* window depth: slabs (OUTER) or elements (INNER) */
} hfav_term_info;

/* ------------------------------------------------------------- the calls */

/* Record and validate a chain.  The descriptor and everything it points to
 * are copied; the caller keeps ownership.  Rules not needed for any goal are
 * pruned (inference works backward from the goals).
 * Errors: EINVAL, EUNSAT, EDUP, ECYCLE.  *out is NULL on error. */
int hfav_chain_create(const hfav_chain_desc *desc, hfav_chain **out);

/* Plan the chain for a grid size and boundary: fusion, extents, windows,
 * kernel family and tile configuration.  Host only, deterministic, allocates
 * no device memory (a fused STAR_CHAIN plan stages its coefficient table in
 * pinned host memory, see hfav_execute).  `info` may be NULL.  Re-planning
 * replaces the plan; a graph captured from this chain's executes must not
 * be replayed after a re-plan (it copies from the staging buffer, which
 * re-planning frees).
 * Errors: EINVAL (bad dims / boundary), EUNSUP (mode or precision not
 * available for this chain). */
int hfav_plan(hfav_chain *chain, const hfav_plan_opts *opts, hfav_plan_info *info);

/* Enqueue the planned chain on `stream` (a hipStream_t; NULL = default
 * stream).  axioms[] and goals[] are device pointers in declaration order.
 * `workspace` must hold info.workspace_bytes (it may be NULL when that is 0);
 * it is caller-owned device memory the call may overwrite.  Asynchronous: no
 * device allocation, no synchronisation, no device-to-host read, so it can
 * be captured in a HIP graph, also on its first call.  The STAR_CHAIN
 * family's coefficient table travels with the call as an asynchronous
 * host-to-device copy into the workspace, from a pinned host buffer that
 * hfav_plan allocates and fills (EDEVICE if that allocation failed, e.g.
 * when the plan was made without a device).
 * Kernel faults surface at the caller's next synchronisation.  A goal may
 * share an axiom's buffer only as a pair declared with hfav_chain_alias.
 * Errors: ENOPLAN, EINVAL (null pointer), EALIAS, EDEVICE. */
int hfav_execute(hfav_chain *chain, const void *const *axioms, void *const *goals,
                 void *workspace, void *stream);

/* hfav_execute without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The plan's workspace
 * (info.workspace_bytes) is taken from a static device array of
 * HFAV_STATIC_WORKSPACE_BYTES that the library holds on each device it runs
 * on, from the first call on that device (which looks up the array's
 * address with that device current) until the process ends.  The call
 * itself allocates nothing, device or host, and runs the same kernels as
 * hfav_execute with the same results.  Every call on one device shares that
 * device's array and leaves its contents behind; no part of it has to start
 * at zero (every workspace byte a call reads was written earlier in the same
 * call), so nothing is cleared.  Two calls whose work overlaps on one device
 * (different streams or threads, not ordered by the caller) RACE on the
 * array: order them, e.g. on one stream.  Arguments, ownership and the
 * other errors as hfav_execute.
 * Errors: ESIZE (info.workspace_bytes > HFAV_STATIC_WORKSPACE_BYTES; nothing
 * is enqueued), EDEVICE (no current device, or the array's address could not
 * be found), and those of hfav_execute. */
#define HFAV_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int hfav_execute_noalloc(hfav_chain *chain, const void *const *axioms, void *const *goals, void *stream);

/* Create a chain by inference from rule patterns (Implementation,
 * "Inference").  The descriptor is that of hfav_chain_create, except that
 * rule term names may contain pattern variables: an identifier ending in
 * '?' (as in the paper's "q?") matches any non-empty substring with
 * balanced parentheses, with one value per variable per rule application.
 * Term names are expressions, e.g. a rule with input "q?" and output
 * "laplace(q?)" derives "laplace(laplace(cell))" from the axiom "cell" in
 * two applications.  Offsets are relative to the output point as in
 * hfav_chain_create (the paper's j?-1, i?+1).  Axioms and goals are
 * concrete.  Every variable of a rule must occur in each of its outputs.
 * Working backward from the goals in order, each needed term that is not
 * an axiom or already produced is produced by the first rule (descriptor
 * order, then output order) that matches it and whose inputs can all be
 * derived, trying the next on failure; cycles and derivations deeper than
 * 64 applications fail.  The resulting concrete rules (one per
 * application, in derivation order) are validated as by
 * hfav_chain_create; hfav_plan_json lists each with its pattern index and
 * binding.  Errors: EINVAL (malformed pattern, concrete axioms or goals
 * required, too many applications), EUNSAT (a goal is not derivable), and
 * those of hfav_chain_create.  *out is NULL on error. */
int hfav_chain_infer(const hfav_chain_desc *patterns, hfav_chain **out);

/* Declare that `goal` will be written over `axiom` (the same device
 * buffer passed in both places: an in-place update).  Design, "In/out
 * chaining": by default terminals do not alias; a declared pair lets
 * hfav_execute accept goals[g] == axioms[a] for that pair (exactly the same
 * pointer; any other overlap is still EALIAS).  The next hfav_plan finds
 * which of the axiom's values a goal reads after they may have been
 * overwritten and saves them first: nothing for the normalisation kernel
 * (a row is on chip before it is written), the halo columns and rows at the
 * tile and segment boundaries for the horizontal-diffusion kernel (a copy
 * kernel into the workspace), for the hydro sweeps (each goal over the axiom
 * of its own field; the strip kernels) the cells b-2 .. b+1 around every
 * segment boundary b of every line (a copy kernel into the workspace;
 * batches are not built in place), and for the unfused path nothing when the
 * goal's producer is the last rule to read the axiom and reads it at offset
 * 0 only, else a copy of the whole axiom.  Other fused families fall back
 * to the unfused path (AUTO) or fail with EUNSUP (FUSED).  The plan JSON
 * lists each pair with the axiom's extent and the handling chosen.  The
 * goal and the axiom must have the same nonzero rank; each at most once; at
 * most 16 pairs per chain.
 * Errors: EINVAL, EDUP. */
int hfav_chain_alias(hfav_chain *chain, const char *goal, const char *axiom);

/* Release a chain (NULL is allowed). */
void hfav_chain_destroy(hfav_chain *chain);

/* Text of the last error on this thread ("" if none). */
const char *hfav_last_error(void);

/* Library version string. */
const char *hfav_version(void);

/* Hash of the sources the library was built from (16 hex digits): a binding
 * compares it with the sources it ships with to refuse a stale build. */
const char *hfav_build_id(void);

/* ------------------------------------------------------------- batches */
#define HFAV_MAX_BATCH 640

/* Plan a 2-D Euler sweep chain, a time step of both sweeps (the chain of
 * the EULER_XY family), or the CFL reduction for a batch of independent
 * grids of different sizes, advanced together by persistent kernels: one
 * launch per sweep for all grids, or for the time step ONE launch for both
 * sweeps of all grids.  dims: host array
 * (n_grids, 2) of (nx, ny), each in [1, 65535]; opts.dims is ignored.  Every
 * grid term is then ONE packed device buffer holding grid g at element
 * offset hfav_batch_offset(chain, g), and every 0-D term is a device array of
 * n_grids doubles (one dt / CFL slot per grid).  The y-sweep segment length
 * of each grid (rows per y work item, 1..255; default 15) comes
 * from the configuration source (the tuning table is consulted with that
 * grid's own size; a forced configuration gives every grid its seg).  Host
 * only; allocates nothing.
 *
 * The per-sweep form's work items: x, one wave on 2 rows x 191 cells; y,
 * 16 columns x the grid's segment of rows.
 *
 * The time step in one launch (Design, "Fusing iteration nests": the two
 * sweeps' nests fused; the x-swept state is not contracted across grids'
 * work items, so it lives in the workspace): each execute first deals the
 * grids to the device's XCDs (one launch of one workgroup: snake order over
 * the grid sizes, largest first), then runs every item of a grid on its
 * XCD, so the x-swept state passes through one L2.  Per XCD one atomic
 * cursor hands out the x items of its grids (4 rows x 191 cells) before any
 * y item; a y item of grid g first waits until every x item of g has
 * finished (a bounded number of polls).  info.workspace_bytes = 4096 + 4
 * planes of the packed size, each padded to 256 bytes.  Workspace byte 0
 * holds a 32-bit status word after the step: 0, or bit 0 set when a y item
 * gave up waiting (its cells are not updated and its grid's CFL slot holds
 * NaN), bit 1 when the items of an XCD were not all taken (an XCD that ran
 * no workgroup).  No correct run sets either: every item a y item waits for
 * is already held by a running workgroup, and the hardware deals the
 * 1024 workgroups round robin over the XCDs.  Configuration variant bit
 * 128 makes every wait target a count that is never reached, with 64
 * polls, to test that path.
 * Errors: EINVAL (bad sizes, n_grids not in [1, HFAV_MAX_BATCH]), EUNSUP
 * (chain not an Euler sweep, time step or CFL reduction, unfused mode, or
 * in-place aliases). */
int hfav_plan_batch(hfav_chain *chain, const hfav_plan_opts *opts, int n_grids, const int *dims,
                    hfav_plan_info *info);

/* Element offset of grid g in the packed buffers of a batched plan, or -1. */
int64_t hfav_batch_offset(const hfav_chain *chain, int grid);

/* Per-term plan details (extent, storage class, window), term index in
 * [0, hfav_num_terms).  Errors: ENOPLAN, EINVAL. */
int hfav_num_terms(const hfav_chain *chain);
int hfav_plan_term(const hfav_chain *chain, int index, hfav_term_info *info);

/* The plan as a JSON document (nests, phases, extents, windows, family,
 * configuration); valid until the next call on this thread.  NULL on error. */
const char *hfav_plan_json(const hfav_chain *chain);

/* ------------------------------------------------------- nest fusion */
/* An iteration nest as rule ids per phase (Design, "Iteration nests": a
 * prologue, a steady state and an epilogue around the loops of its rank). */
typedef struct {
    int rank;                           /* rank of the iteration space */
    int n_prologue, n_steady, n_epilogue;
    int prologue[HFAV_MAX_RULES];       /* rule ids in [0, n_rules) */
    int steady[HFAV_MAX_RULES];
    int epilogue[HFAV_MAX_RULES];
} hfav_nest;

/* The nest-fusion walk of the planner (Design, "Fusion": fuse_inest_dag and
 * fuse_inest) on caller-given nests, so that nests a concrete chain never
 * hands the walk (a later nest with its own prologue or epilogue) can be
 * fused too.  nests[0..n) are visited in order with one fusing nest; a nest
 * joins it when fuse_inest allows, otherwise the fusing nest is closed and
 * the nest starts the next one.  Equal ranks fuse phase by phase when
 * (A.prologue <= B.steady), (B.prologue <= A.steady), (A.steady <=
 * B.epilogue) and (B.steady <= A.epilogue) all hold, where (R <= S) means no
 * rule of S is, or depends on, a rule of R.  Unequal ranks: the lower-rank
 * nest goes into the prologue of the higher one if it can precede that
 * nest's steady state and epilogue, else into its epilogue if the higher
 * nest's prologue and steady state can precede it, else the pair is
 * unfusable.  reach: n_rules * n_rules bytes (host), reach[a * n_rules + b]
 * nonzero when rule b depends on rule a through a path of dataflow edges
 * (a transitively closed relation).  out: host array with room for n nests;
 * *n_out receives their number.  Host only, allocates nothing the caller
 * must free.  Errors: EINVAL (null pointer, n_rules not in [1,
 * HFAV_MAX_RULES], a phase count or rule id out of range, a fused phase
 * longer than HFAV_MAX_RULES). */
int hfav_fuse_nests(int n_rules, const unsigned char *reach, int n, const hfav_nest *nests,
                    hfav_nest *out, int *n_out);

#ifdef __cplusplus
}
#endif
#endif /* HFAV_H */
