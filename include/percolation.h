/*
 * percolation.h -- C ABI of the gfx950 site-percolation engine: a porous
 * medium drawn site by site and a cluster invaded into it from an invasion
 * point (Tomov, McGuigan, Bennett, Smith, Spiletic 2003, Section 2.3).
 *
 * Medium: an L x L lattice with open boundaries. Site (i, j) draws
 * R = (u + 1) / 2^32, u the 32-bit Philox4x32-10 output word (i*L + j) % 4
 * of counter ((i*L + j) / 4, 0, 0, 2) under key (seed low, seed high), and
 * is a pore iff R <= porosity, i.e. u < floor(porosity * 2^32).
 *
 * Invasion (Section 2.3): the cluster starts at the invasion source (every
 * pore of row 0, or one point) and spreads in passes; pass k takes in every
 * pore that shares an edge with a site already in the cluster. The engine
 * computes each site's arrival pass, the pass in which it joins the cluster,
 * which equals its breadth-first distance through pores from the source; it
 * does not run the passes one by one. The steady state is reached after
 * (max arrival) passes, and the cluster spans when it reaches the far side.
 *
 * Errors are the ISING_* codes of ising.h. Every call that reads results
 * synchronises the context's stream.
 */
#ifndef PERCOLATION_H
#define PERCOLATION_H

#include <stddef.h>
#include <stdint.h>

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PERC_SOURCE_TOP_ROW 0u /* every pore of row 0 starts invaded */
#define PERC_SOURCE_POINT 1u   /* only site (i0, j0), if it is a pore */

typedef struct perc_params {
    uint32_t L;       /* side, 1 <= L <= 65536 */
    double porosity;  /* P in [0, 1] (Section 2.3) */
    uint64_t seed;    /* Philox key */
    uint32_t source;  /* PERC_SOURCE_* */
    uint32_t i0, j0;  /* invasion point (PERC_SOURCE_POINT), each < L */
} perc_params;

typedef struct perc_result {
    uint64_t pores;         /* pore sites in the medium */
    uint64_t invaded;       /* sites in the final cluster */
    int32_t passes;         /* passes to the steady state = max arrival (0 if the cluster is empty) */
    uint32_t spans;         /* bit 0: cluster holds sites of rows 0 and L-1; bit 1: of columns 0 and L-1 */
    /* work measures of the engine (not paper quantities) */
    uint32_t launches;         /* relaxation launches */
    uint32_t pad;
    uint64_t tile_visits;      /* 64 x 64 tiles relaxed, summed over launches */
    uint64_t tile_iterations;  /* breadth-first levels run, summed over tile visits */
    uint64_t arrival_hash;  /* FNV-1a-64 of the int32 arrival map, little-endian row-major (opt-in) */
} perc_result;

typedef struct perc_ctx perc_ctx; /* opaque, library-owned */

/* Create a context for one medium and allocate its device memory (5 bytes
 * per site plus per-tile work lists) on `stream` (NULL: the library creates
 * and owns one). Errors: EINVAL (invalid params, out == NULL), ENOMEM,
 * EDEVICE. *out is NULL on failure. */
int perc_create(const perc_params* params, void* stream, perc_ctx** out);

/* Draw the medium and invade it to the steady state. Synchronises (the
 * engine polls its work list between groups of launches). Running again
 * redraws the same medium and gives the same result. Errors: EINVAL,
 * ESTATE, EDEVICE. */
int perc_run(perc_ctx* ctx);

/* Draw and invade the media of `count` contexts together, with the same
 * results as perc_run on each: every relaxation launch covers the queued
 * tiles of all of them, so many small media fill the GPU (Section 2.3 asks
 * for the porosity from which a spanning cluster exists, a question over
 * many media). Runs on the first context's stream after each context's
 * earlier work. Synchronises. Errors: EINVAL (NULL or repeated contexts,
 * contexts on different devices), ESTATE, ERANGE (more than 2^32 tiles
 * together), ENOMEM, EDEVICE (the first context is poisoned). */
int perc_run_batch(perc_ctx* const* ctxs, size_t count);

/* Change the porosity, seed and invasion source of a context for its next
 * run; params->L must equal the context's side (the buffers are kept).
 * Errors: EINVAL (invalid params or another side), ESTATE. */
int perc_set_params(perc_ctx* ctx, const perc_params* params);

/* Summary of the last run into *out; want_hash != 0 also hashes the arrival
 * map (copies it to the host). Errors: EINVAL, ESTATE (no run yet). */
int perc_result_get(perc_ctx* ctx, perc_result* out, uint32_t want_hash);

/* Copy the medium (row-major uint8, 1 = pore) to `host` of n >= L*L bytes. */
int perc_copy_medium(perc_ctx* ctx, uint8_t* host, size_t n);

/* Copy the arrival map (row-major int32: the arrival pass, -1 for solid or
 * never-invaded sites) to `host` of n >= L*L entries. */
int perc_copy_arrival(perc_ctx* ctx, int32_t* host, size_t n);

/* Release the context and its device memory. NULL is a no-op. */
int perc_destroy(perc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
