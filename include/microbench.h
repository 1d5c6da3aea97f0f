/*
 * microbench.h -- vector-operation and host-transfer micro-benchmarks of
 * the gfx950 engine, the MI355X counterparts of the calibration the paper
 * runs on its GPU (Tomov et al. 2003, Section 4, Table 2: '=' copy,
 * + - * /, sin and cos, log and exp on float vectors of four values per
 * lattice site; Section 6, Table 5: reading and writing a whole lattice
 * and only its border between host and GPU). They measure what a kernel
 * of the engine can expect from HBM, the vector ALUs and the host link.
 *
 * All calls enqueue on `stream` (NULL: the null stream) and return at once;
 * the caller times them. Errors are the ISING_* codes of ising.h.
 */
#ifndef MICROBENCH_H
#define MICROBENCH_H

#include <stddef.h>
#include <stdint.h>

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MB_OP_COPY 0u /* a[k] = c[k] */
#define MB_OP_ADD 1u  /* a[k] = a[k] + c[k] */
#define MB_OP_SUB 2u  /* a[k] = a[k] - c[k] */
#define MB_OP_MUL 3u  /* a[k] = a[k] * c[k] */
#define MB_OP_DIV 4u  /* a[k] = a[k] / c[k] (IEEE single, correctly rounded) */
#define MB_OP_SIN 5u  /* a[k] = sin(a[k]) (device math library, single precision) */
#define MB_OP_COS 6u  /* a[k] = cos(a[k]) */
#define MB_OP_LOG 7u  /* a[k] = log(a[k]) */
#define MB_OP_EXP 8u  /* a[k] = exp(a[k]) */

/* One pass of `op` over n floats: a (device, read and written; only written
 * for MB_OP_COPY) and c (device, read by the first five ops; may be NULL
 * for the others). Both 16-byte aligned. Errors: EINVAL (op, NULL a, NULL
 * c where it is read, misaligned pointers), EDEVICE. */
int mb_vector_op(uint32_t op, float* a, const float* c, size_t n, void* stream);

#define MB_HOST_TO_DEVICE 0u
#define MB_DEVICE_TO_HOST 1u

/* Copy an L x L lattice of `elem` bytes per site, row-major, between host
 * memory and device memory in the given direction: all of it
 * (border == 0), or only its border (border != 0: rows 0 and L-1 and
 * columns 0 and L-1, 4L - 4 sites; the other sites of dst are untouched).
 * Pinned host memory (hipHostMalloc) gives asynchronous copies. Errors:
 * EINVAL (NULL pointers, L == 0, elem == 0, direction), EDEVICE. */
int mb_copy_lattice(void* dst, const void* src, uint32_t L, uint32_t elem, uint32_t direction, int border,
                    void* stream);

/* Philox4x32-10 rate: n_threads threads each evaluate calls_per_thread
 * Philox calls with counter (thread, k, 0, 0) and key (seed low, seed high),
 * k = 0 .. calls_per_thread-1, and write the XOR of all words they drew to
 * out[thread] (device, n_threads uint32). The draw is the one every site
 * update of the Metropolis sweep needs (one call per four sites), so
 * 4 x calls per second is the update rate the draws alone allow. Errors:
 * EINVAL (NULL out, n_threads == 0 or > 2^31), EDEVICE. */
int mb_philox(uint32_t* out, size_t n_threads, uint32_t calls_per_thread, uint64_t seed, void* stream);

#ifdef __cplusplus
}
#endif
#endif
