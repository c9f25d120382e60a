/*
 * hfav_tune.h - tile-configuration sources for hfav_plan.
 *
 * The fused kernel families have a small configuration space (threads per
 * workgroup, tile shape, cells streamed per thread, kernel variant).  A plan
 * picks its configuration from one of three sources (hfav_plan_opts
 * .config_source): the built-in default, the tuning table below (filled
 * from exhaustive autotuner timings), or the learned cost model
 * (hfav_mlp.h).  These calls are host-only and process-wide; they are
 * safe to call from several threads.
 */
#ifndef HFAV_TUNE_H
#define HFAV_TUNE_H

#include "hfav.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Remove every tuning-table entry. */
void hfav_tuning_clear(void);

/* Add the best configuration measured for (family, dtype, dims).  A plan with
 * config_source = HFAV_CONFIG_TUNED takes the entry of the same family and
 * dtype whose dims are nearest in log2 distance; with no such entry it keeps
 * the default.  dims: host array of 3 ints (nx, ny, nz).
 * Errors: HFAV_EINVAL for null pointers or block <= 0. */
int hfav_tuning_add(int family, int dtype, const int dims[3], const hfav_config *cfg);

/* Number of tuning-table entries. */
int hfav_tuning_size(void);

#ifdef __cplusplus
}
#endif
#endif /* HFAV_TUNE_H */
