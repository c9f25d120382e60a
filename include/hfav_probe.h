/*
 * hfav_probe.h - streaming-bandwidth probes.
 *
 * A fused chain reads each input from HBM once and writes each output once
 * (the compulsory traffic of the paper's fused form: Design, "Contraction";
 * Performance, the bandwidth-bound COSMO kernels).  How close a chain gets
 * to that traffic's time is judged against two ceilings: the nominal HBM
 * peak, and what a plain device copy of the same bytes reaches on the same
 * GPU.  These calls enqueue such copies; they compute nothing of a chain.
 */
#ifndef HFAV_PROBE_H
#define HFAV_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    /* bytes/16 lanes, one 16-byte element each, one 256-lane workgroup per
     * 4 KiB, non-temporal loads and stores: the flat streaming ceiling */
    HFAV_COPY_FLAT = 0,
    /* the access pattern of the streaming stencil kernels: the buffer is
     * `slabs` slabs of `slab_bytes`; inside a slab a tile is `tile_rows`
     * runs of `band_bytes`, `row_bytes` apart; a workgroup of 256 lanes
     * copies one tile through `seg` consecutive slabs (4 slabs in flight),
     * each lane moving `access_bytes` (4, 8 or 16) per access */
    HFAV_COPY_SEGMENTS = 1
} hfav_copy_pattern;

typedef struct {
    int pattern;            /* hfav_copy_pattern */
    int64_t bytes;          /* FLAT: bytes to copy (a multiple of 16) */
    int64_t slab_bytes;     /* SEGMENTS: geometry as above; slab_bytes a
                               multiple of row_bytes, row_bytes of band_bytes,
                               band_bytes of access_bytes, (slab_bytes /
                               row_bytes) of tile_rows */
    int64_t slabs;
    int64_t row_bytes;
    int band_bytes;
    int tile_rows;
    int seg;
    int access_bytes;
} hfav_copy_desc;

/* Enqueue a copy of src to dst (device pointers, 16-byte aligned, not
 * overlapping, each holding the bytes the pattern covers: `bytes`, or
 * slabs * slab_bytes) on `stream` (a hipStream_t, NULL = default stream).
 * Asynchronous; allocates nothing.
 * Errors: 1 (HFAV_EINVAL) for a null pointer or an inconsistent geometry,
 * 8 (HFAV_EDEVICE) for a launch error (text in hfav_last_error). */
int hfav_copy_probe(const hfav_copy_desc *desc, const void *src, void *dst, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HFAV_PROBE_H */
