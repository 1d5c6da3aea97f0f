/*
 * ising.h -- C ABI of the MI355X (gfx950) checkerboard Metropolis engine for
 * the two-dimensional Ising model.
 *
 * The model and the update rule are those of Tomov, McGuigan, Bennett, Smith,
 * Spiletic, "Benchmarking and Implementation of Probability-Based Simulations
 * on Programmable Graphics Cards" (2003), Section 2.2:
 *   - an L x L square lattice of spins s = +1 / -1, here with periodic
 *     boundaries;
 *   - energy E = -J sum_<jk> s_j s_k - h sum_j s_j (the paper's energy is the
 *     case J = 1, h = 0), magnetisation M = #up - #down;
 *   - a random initial state with spin-up probability p;
 *   - checkerboard colouring: one sweep is the pass over colour 0
 *     ((i + j) even, "black") followed by the pass over colour 1;
 *   - Metropolis decision per site: flip if dE < 0, else draw R in [0, 1] and
 *     flip if R <= exp(-dE / T) (Boltzmann constant 1, T in units of J).
 *
 * Choices the paper leaves open, fixed here so that every result is
 * reproducible bit for bit:
 *   - Draws. Philox4x32-10 (Salmon et al., SC 2011). The sites of colour c are
 *     numbered ord = (i*L + j) / 2; the four sites ord = 4q .. 4q+3 share the
 *     call with counter (q, t, c, d) and key (seed & 0xffffffff, seed >> 32)
 *     and take output word ord % 4. t is the absolute sweep index, d = 0 for
 *     Metropolis decisions and d = 1 for the initial state (drawn at t = 0).
 *   - Acceptance. R = (u + 1) / 2^32 for the 32-bit draw u, so the flip
 *     happens iff u < thr(s, n), thr = floor(exp(-dE/T) * 2^32) evaluated in
 *     IEEE double as exp(-(2.0 * s * (J * n + h)) / T) with n the sum of the
 *     four neighbours, and thr = 2^32 when dE <= 0.
 *   - Initial state: up iff u < floor(p_up * 2^32).
 *   - Observables after sweep t: bond sum B_t = sum_{i,j} s(i,j) (s(i,j+1) +
 *     s(i+1,j)) (every edge once) and M_t = sum s, both exact int64; the
 *     energy is E = -J B - h M.
 *   - Canonical lattice bytes: row-major int8, +1 -> 0x01, -1 -> 0xFF.
 *     Lattice hash: FNV-1a 64 over those L*L bytes.
 *
 * Device memory is HIP device memory of the current device; streams are
 * hipStream_t passed as void* (NULL = the library creates its own stream).
 * All sweep calls are asynchronous on the context's stream; calls that return
 * host data synchronise that stream. A context must not be used by two host
 * threads at once. Every entry point returns ISING_OK or a negative error
 * code and never throws. On a HIP error the context is poisoned: later calls
 * return ISING_ESTATE and only ising_destroy is valid.
 */
#ifndef ISING_MI355X_H
#define ISING_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISING_OK 0
#define ISING_EINVAL (-1)      /* bad argument (odd or too large L, T <= 0, NaN, NULL ...) */
#define ISING_ENOMEM (-2)      /* device or host allocation failed */
#define ISING_EDEVICE (-3)     /* a HIP call failed; the context is now poisoned */
#define ISING_ERANGE (-4)      /* sweep index would pass 2^32 - 1, or a buffer is too small */
#define ISING_EUNSUPPORTED (-5) /* valid request the library cannot serve */
#define ISING_ESTATE (-6)      /* context poisoned by an earlier device error */
#define ISING_EIO (-7)         /* a file could not be written (the batch tuning cache) */

#define ISING_MAX_L 65536u     /* counter word 0 holds site/8: L*L/8 must fit 32 bits */

/* Plan selection (ising_params.flags, low byte). AUTO picks per lattice side:
 * the workgroup-resident kernel for small sides, the band-resident plan for
 * sides 192 to 16384 (about one band of rows per compute unit), the fused
 * one-pass sweep by full-row workgroups where a row fits one workgroup, the
 * fused sweep by wave tiles for larger sides, the two-pass in-place sweep
 * otherwise. The others force a path (ISING_EUNSUPPORTED if the side does
 * not fit it). */
#define ISING_PLAN_AUTO 0u
#define ISING_PLAN_TWO_PASS 1u  /* one launch per colour, in place */
#define ISING_PLAN_FUSED 2u     /* one launch per sweep, ping-pong buffers; a wave per tile */
#define ISING_PLAN_RESIDENT 3u  /* one workgroup runs all sweeps of the call */
#define ISING_PLAN_GENERIC 4u   /* per-site draws; the only path for L % 8 != 0 */
#define ISING_PLAN_FUSED_ROWS 5u /* as FUSED, a workgroup per band of whole rows (L/8 <= 16 * 64 * cw) */
#define ISING_PLAN_BANDS 6u      /* the lattice split into bands of whole rows, one workgroup each, all
                                   * resident at once; each band stays in LDS at one bit per site (as
                                   * bytes at sides 512, 1024 and 2048, and 4096 with h != 0) for every
                                   * sweep of a launch, bands trade edge rows after each half-sweep
                                   * (L % 8 == 0, L <= 16384) */
/* Sweeps of one band-plan launch (the lattice crosses HBM once per launch);
 * longer calls are split into launches of this many sweeps. */
#define ISING_BAND_SWEEPS_PER_LAUNCH 512u

/* Model and run parameters (Section 2.2: L x L lattice, coupling J, field h,
 * temperature T, spin-up probability p_up of the initial state). */
typedef struct ising_params {
    uint32_t L;      /* side, even, 2 <= L <= ISING_MAX_L */
    uint32_t flags;  /* ISING_PLAN_* */
    double J;        /* coupling, finite */
    double h;        /* field, finite */
    double T;        /* temperature, finite and > 0 */
    uint64_t seed;   /* Philox key */
    double p_up;     /* in [0, 1] */
} ising_params;

/* Current state summary (Eq. (1) of Section 2.1 is estimated by averaging
 * these over sweeps; see ising_series_averages). */
typedef struct ising_obs {
    uint64_t sweeps_done;  /* absolute sweep index t of the next sweep */
    int64_t bond_sum;      /* B of the current lattice */
    int64_t mag_sum;       /* M of the current lattice */
    double energy;         /* -J B - h M */
    double e_per_site;     /* energy / L^2 */
    double m_per_site;     /* M / L^2 */
    uint64_t lattice_hash; /* FNV-1a 64 of the canonical bytes (if requested) */
    uint64_t series_len;   /* per-sweep (B_t, M_t) pairs pending on the device */
} ising_obs;

/* Averages over a window of the per-sweep series, summed in increasing t in
 * IEEE double (Eq. (1) estimated as a plain time average). */
typedef struct ising_averages {
    uint64_t n;       /* sweeps in the window */
    double e;         /* <E / N> */
    double e2;        /* <(E / N)^2> */
    double m;         /* <M / N> */
    double abs_m;     /* <|M| / N> */
    double m2;        /* <(M / N)^2> */
} ising_averages;

#define ISING_OBS_HASH 1u    /* compute lattice_hash (copies the lattice to the host) */
#define ISING_OBS_SERIES 2u  /* copy out and clear the pending per-sweep series */

typedef struct ising_ctx ising_ctx; /* opaque, library-owned */

/* Bytes of device memory the lattice state of a context for side L uses
 * under the given plan flags (the per-sweep series buffer is separate and
 * library-owned). Returns 0 for an invalid L or a plan that cannot serve it. */
size_t ising_state_bytes(uint32_t L, uint32_t flags);

/* Create a context: validate `params`, allocate its device buffers, build the
 * acceptance table on the host and draw the initial state (Section 2.2) on
 * `stream` (NULL: the library creates and owns a stream). The context starts
 * at sweep t = 0. *out is set to the context, or to NULL on failure.
 * Errors: EINVAL (invalid params or out == NULL), EUNSUPPORTED (forced plan
 * cannot serve L), ENOMEM, EDEVICE. */
int ising_create(const ising_params* params, void* stream, ising_ctx** out);

/* As ising_create, but the lattice state lives in caller-owned device memory
 * `dev_buf` of `bytes` >= ising_state_bytes(L, flags) bytes (for example a
 * PyTorch tensor). The buffer must stay allocated until ising_destroy; its
 * layout is internal (read the lattice with ising_copy_spins). */
int ising_create_in(const ising_params* params, void* dev_buf, size_t bytes, void* stream,
                    ising_ctx** out);

/* Enqueue n full sweeps (colour 0 then colour 1, Section 2.2) on the
 * context's stream, for sweep indices t .. t+n-1, and record (B_t, M_t)
 * after each. Asynchronous. n = 0 is a no-op. Errors: EINVAL (NULL ctx),
 * ERANGE (t + n > 2^32), ESTATE, ENOMEM (series buffer growth), EDEVICE,
 * EUNSUPPORTED (a band-plan context whose stream is being captured into a
 * graph: capture ising_sweep_static instead). */
int ising_sweep(ising_ctx* ctx, uint64_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * n sweeps as ising_sweep, with two differences. The per-sweep pairs
 * (B_t, M_t) are written to the caller's device array series_dev (2 n
 * int64: B_t then M_t for each sweep, oldest first) instead of the
 * context's pending series, which stays as it is. And the sweep kernels'
 * per-tile (fused plan) or per-block (two-pass plan) partial sums go to a
 * fixed device array inside the library of ISING_STATIC_SCRATCH_PAIRS int64
 * pairs (1 MiB; each device that runs this call holds its own copy until the
 * process ends) instead of context memory. No device memory is allocated or
 * freed and nothing is synchronised; the work is enqueued on the context's
 * stream. Every call on one device shares that device's array and leaves
 * its last contents there (the kernels write each slot before they read
 * it): calls that overlap on one device, on any streams, race and must be
 * ordered by the caller. The fused plan needs 2 x its tiles pairs (32768^2
 * with 32-row tiles: 32768), the two-pass plan one per block, the band
 * plan one per band and sweep (its launches are split so that they fit; its
 * edge-row slots were allocated when the plan was set); the resident and
 * per-site plans need none. While the context's stream is being captured
 * into a graph, a band-plan context's sweeps are enqueued as two-pass
 * launches with one word per thread (the same results): a band launch's
 * edge-row tags advance on the host with every launch, which a replayed
 * graph would not do. Errors: EINVAL (NULL ctx or series_dev),
 * ERANGE (t + n > 2^32, or the plan needs more pairs than the array holds:
 * pick taller tiles with ising_plan_set), ESTATE, EDEVICE. */
#define ISING_STATIC_SCRATCH_PAIRS 65536u
int ising_sweep_static(ising_ctx* ctx, uint64_t n, int64_t* series_dev);

/* Synchronise the context's stream and report the current state in *out
 * (may be NULL). With ISING_OBS_HASH the lattice is copied to the host and
 * hashed. With ISING_OBS_SERIES the pending per-sweep series (oldest first)
 * is copied into bond_series / mag_series (host arrays of `capacity`
 * entries; either may be NULL to skip it) and then cleared; ERANGE if
 * capacity is smaller than the pending length (nothing is cleared then). */
int ising_observables(ising_ctx* ctx, ising_obs* out, int64_t* bond_series, int64_t* mag_series,
                      uint64_t capacity, uint32_t want);

/* Start the read-back of a later ising_observables(ctx, ..., want) without
 * waiting: enqueue on the context's stream the device-to-host copies of the
 * pending series (whole) and, with ISING_OBS_HASH, of the lattice, into
 * pinned host memory the context owns. Later ising_observables calls wait
 * for these copies and answer from them as long as no call has changed the
 * lattice or the series since (clearing the series is such a change) and
 * `want` covers what they ask for; otherwise the copies are discarded and
 * the call reads back afresh. A caller that keeps more work queued behind
 * this context's last sweep (a server stepping other requests) thereby
 * waits only for that sweep: copies enqueued later would run after the work
 * queued before them. Errors: EINVAL (NULL ctx, unknown want bits), ESTATE,
 * EUNSUPPORTED (more than 64 MiB to read back, or no pinned memory to be
 * had: call ising_observables alone), EDEVICE. */
int ising_prefetch_observables(ising_ctx* ctx, uint32_t want);

/* Copy the current lattice to host memory `host` of n >= L*L bytes in the
 * canonical layout (row-major int8, +1 / -1). Synchronises. */
int ising_copy_spins(ising_ctx* ctx, int8_t* host, size_t n);

/* Replace the lattice by host canonical bytes (n >= L*L, every byte +1 or
 * -1, else EINVAL) and set the sweep index to t (checkpoint restore; the
 * counter-based draws make a restored run continue exactly). Clears the
 * pending series. Synchronises. */
int ising_load_spins(ising_ctx* ctx, const int8_t* host, size_t n, uint64_t t);

/* Run n_sweeps[k] sweeps on ctxs[k], k < count, together on `stream`
 * (NULL: the library's own stream on the contexts' device, which keeps
 * consecutive batches in stream order), with the batch plan ISING_BATCH_AUTO
 * picks (see ising_sweep_batch_plan): one persistent launch from a captured
 * graph in which each workgroup takes whole lattices, largest work first,
 * and runs all of their sweeps from its local memory, or, when that is
 * predicted slower, graph replays of passes that spread every lattice over
 * the whole GPU. The descriptors are staged through pinned host
 * memory by one copy kernel. A batch with a single lattice to sweep whose
 * side the band-resident plan serves by default (192 to 16384) runs on that
 * plan instead, on the context's stream ordered after `stream`'s earlier
 * work and before its later work (neither batch plan can spread one lattice
 * over the chip). Lattices may differ in L, J, h, T and seed;
 * each must satisfy L % 8 == 0 and have no pending device error. Contexts
 * are validated before anything is launched (all-or-nothing). The results
 * are bit-identical to calling ising_sweep on each context alone.
 * Asynchronous; the contexts' own streams are ordered after it. */
int ising_sweep_batch(ising_ctx* const* ctxs, const uint64_t* n_sweeps, size_t count, void* stream);

/* As ising_sweep_batch with an explicit batch plan:
 * ISING_BATCH_RESIDENT: one persistent launch, each workgroup runs whole
 *   lattices (every sweep) taken from a work queue, largest first. A lattice
 *   of side up to 1072 is held in the workgroup's local memory at one bit
 *   per site for all its sweeps, except that lattices of side up to 256 are
 *   held as bytes when h != 0 or while the batch has fewer lattices than
 *   the launch has workgroups (lower latency per sweep); larger ones are
 *   swept in global memory;
 *   (a single context's ising_sweep under the resident plan runs the same
 *   per-lattice code in one workgroup, launched directly);
 * ISING_BATCH_STEPPED: every sweep is one launch over the tiles of all
 *   lattices, so each lattice is spread over the whole GPU; sweeps are
 *   replayed from a captured graph in groups of 16. When every side is a
 *   multiple of 16 the sweep is one pass (each lattice alternates between
 *   two buffers; a context without its second buffer gets one, L*L bytes,
 *   on first use); otherwise it is a launch per colour, in place;
 * ISING_BATCH_AUTO: the plan predicted faster from the device's rates per
 *   lattice class (see ising_batch_tune): the resident launch's makespan
 *   (lattices handed out largest work first to its workgroups, one per
 *   compute unit) against the stepped plan's summed time, each lattice's
 *   work divided by its class's rate.
 * The stepped plan's tile height (8, 16 or 32 rows, sides that are
 * multiples of 16) is the one predicted fastest the same way. Results are
 * identical for every plan and tile height. */
#define ISING_BATCH_AUTO 0u
#define ISING_BATCH_RESIDENT 1u
#define ISING_BATCH_STEPPED 2u
int ising_sweep_batch_plan(ising_ctx* const* ctxs, const uint64_t* n_sweeps, size_t count, void* stream,
                           uint32_t plan);

/* Batch autotuner (the many-lattice workloads of Section 2.2). The batch
 * plans' speeds depend on the lattices' sides and fields, so ISING_BATCH_AUTO
 * and the stepped tile height are chosen from rates per class: a side band
 * (up to 128, 256, 512, 1072, larger) and whether the field needs the
 * general bit-packed update (h != 0). Rates are site updates per ns: for the
 * resident plan, of one workgroup on one lattice (plus a fixed time per
 * lattice: taking it from the queue and converting it to bits and back);
 * for the stepped plan, of
 * the whole GPU, per tile height (8, 16, 32); plus the stepped plan's least
 * time per sweep. Until a device is tuned, built-in rates measured on an
 * MI355X are used.
 *
 * ising_batch_tune times both plans on `device` with synthetic batches of
 * each class (one lattice per resident workgroup; hot starts, J = 1, T over
 * [1.5, 3.5], h = 0 or 0.05; a few seconds and up to 2 GiB of device
 * memory, freed on return) and keeps the rates for that device in this
 * process. cache_path (NULL: the ISING_TUNE_CACHE environment variable, if
 * set and not empty) names a text file: rates stored there for the same
 * device (architecture, compute units, launch sizes) are loaded instead of
 * timed, unless flags has ISING_TUNE_RETIME; timed rates are written there.
 * *from_cache (optional) is set to 1 when the rates were loaded.
 * Synchronises the device. Errors: EINVAL (bad device or flags), EDEVICE,
 * ENOMEM, EIO (the cache file could not be written; the rates are kept). */
#define ISING_TUNE_RETIME 1u
int ising_batch_tune(int device, const char* cache_path, uint32_t flags, int* from_cache);

typedef struct ising_batch_rate {
    uint32_t max_side;               /* class: sides up to this (the previous class's excluded) */
    uint32_t field;                  /* class: 1 if the table needs the general bit-packed update */
    double resident_per_workgroup;   /* site updates per ns, one resident workgroup */
    double resident_fixed_ns;        /* resident: time per lattice besides its sweeps */
    double stepped[3];               /* site updates per ns, whole GPU, tile rows 8, 16, 32 */
} ising_batch_rate;

/* The rates ISING_BATCH_AUTO uses on `device`: n >= 10 entries, ordered by
 * side band then field; *tuned (optional) 1 if measured on this device in
 * this process; *floor_ns (optional) the stepped plan's least time per
 * sweep. Host only. */
int ising_batch_rates(int device, ising_batch_rate* out, size_t n, int* tuned, double* floor_ns);

/* The batch plan ISING_BATCH_AUTO's model picks for this batch
 * (ISING_BATCH_RESIDENT or ISING_BATCH_STEPPED), the stepped tile height (0
 * when the stepped plan would not use the one-pass walk), and
 * predicted_ns[0], [1] (optional): the predicted resident and stepped
 * times. (A batch with a single lattice to sweep that the band plan serves
 * runs on that plan; see ising_sweep_batch.) Host only. */
int ising_batch_choice(ising_ctx* const* ctxs, const uint64_t* n_sweeps, size_t count, uint32_t* plan,
                       uint32_t* rows, double* predicted_ns);

/* Plain time averages of a series window of n sweeps for an L x L lattice
 * with coupling J and field h (host only, no device work). */
int ising_series_averages(const int64_t* bond_series, const int64_t* mag_series, uint64_t n,
                          uint32_t L, double J, double h, ising_averages* out);

/* Plan the context runs with: ISING_PLAN_* and, for tunable plans, the
 * chunk width in 32-bit words (for the band plan: rows per wave) and the
 * tile or band height in rows. */
int ising_plan_info(const ising_ctx* ctx, uint32_t* plan, uint32_t* chunk_words,
                    uint32_t* rows_per_thread);

/* Force the plan of a context (ISING_PLAN_*; for ISING_PLAN_FUSED also the
 * chunk width cw in {1, 2, 4} words per lane and the tile height rows in
 * {4, 8, 16, 32, 64, 128}; for ISING_PLAN_FUSED_ROWS cw and the band height
 * rows in {8, 16, 32, 64, 128}, with L/8 / (64 cw) <= 16; for
 * ISING_PLAN_BANDS the band height rows >= 1, giving ceil(L / rows) >= 2
 * bands that must all fit the device at once, and cw in {1, 2, 4} rows per
 * wave; 0 picks a default). Switching to the fused plan may allocate a second lattice
 * buffer, to the band plan its edge-row slots. Results do not
 * depend on the plan.
 * Errors: EUNSUPPORTED if the plan cannot serve the context's L. */
int ising_plan_set(ising_ctx* ctx, uint32_t plan, uint32_t cw, uint32_t rows);

/* Autotuner: time `trial_sweeps` sweeps of every plan and fused tile shape
 * that can serve the context's L on a scratch copy of its lattice (the
 * context's own state is untouched), in three interleaved rounds keeping
 * each candidate's fastest; switch the context to the fastest (the default
 * plan for L stays unless another is more than 3% faster) and remember it
 * for later AUTO contexts of the same L in this process. Synchronises. The
 * chosen plan is readable with ising_plan_info. */
int ising_tune(ising_ctx* ctx, uint32_t trial_sweeps);

/* ---- Creutz demon dynamics (Section 2.2) --------------------------------
 * The deterministic checkerboard dynamics the paper cites as the faster,
 * random-number-free alternative to Metropolis sweeps. Every site carries a
 * demon energy d in units of 4J, 0 <= d <= 255 (zero field, J > 0 only).
 * A pass over colour c flips a site iff its demon can pay for the move:
 * e = dE / 4J = s * (sum of the four neighbour spins) / 2, flip iff e <= d
 * and d - e <= 255, then d -= e. A sweep is the colour-0 pass followed by
 * the colour-1 pass; -B + 4 * (demon total) is conserved exactly and the
 * reversed sweep (colour 1 then colour 0) undoes a sweep exactly. The demon
 * total, read as a thermometer, gives the temperature: in equilibrium each
 * demon is Boltzmann-distributed, <d> = 1 / (exp(4J / T) - 1). */

/* Give the context demons: host canonical bytes (row-major L*L, n >= L*L)
 * or, with host == NULL, every demon = fill. Allocates the demon buffer on
 * first use (L*L bytes). Synchronises. Errors: EINVAL (NULL ctx, n too
 * small), EUNSUPPORTED (h != 0 or J <= 0), ENOMEM, ESTATE, EDEVICE. */
int ising_creutz_init(ising_ctx* ctx, const uint8_t* host, size_t n, uint8_t fill);

/* Enqueue n Creutz sweeps (reverse != 0: n reversed sweeps) on the
 * context's stream and record (B, M) after each in the per-sweep series,
 * as ising_sweep does. Draws no random numbers and leaves the Metropolis
 * sweep index t unchanged. Asynchronous. Errors: EINVAL (NULL ctx), ESTATE
 * (no demons: call ising_creutz_init first; or poisoned), ENOMEM, EDEVICE. */
int ising_creutz_sweep(ising_ctx* ctx, uint64_t n, int reverse);

/* Demon total (units of 4J) into *out. Synchronises. Errors as above. */
int ising_demon_sum(ising_ctx* ctx, int64_t* out);

/* Copy the demons to host memory `host` of n >= L*L bytes, canonical
 * row-major layout. Synchronises. */
int ising_copy_demons(ising_ctx* ctx, uint8_t* host, size_t n);

/* Re-initialise a context for new parameters of the same side, keeping its
 * device buffers (a request server reusing contexts instead of freeing and
 * allocating, which would synchronise the device): the result is the same
 * as ising_create with *params, i.e. the acceptance table of (J, h, T), the
 * initial lattice drawn from (seed, p_up) (Section 2.2), sweep index 0 and
 * an empty series. params->L must equal the context's side; the plan is
 * kept (params->flags must be ISING_PLAN_AUTO or the context's plan).
 * Creutz demons, if any, are dropped. Asynchronous on the context's stream.
 * Errors: EINVAL (invalid params, another side or plan), ESTATE (poisoned),
 * EDEVICE. */
int ising_reset(ising_ctx* ctx, const ising_params* params);

/* Make room now for the per-sweep series of `sweeps` further sweeps, so that
 * later ising_sweep and batch calls covering them allocate nothing (growing
 * the series buffer synchronises the context's stream). Errors: EINVAL,
 * ESTATE, ERANGE (the sweep index would pass 2^32), ENOMEM. */
int ising_reserve(ising_ctx* ctx, uint64_t sweeps);

/* Release the context and its library-owned device memory. NULL is a no-op.
 * Synchronises the context's stream first. */
int ising_destroy(ising_ctx* ctx);

/* Static description of an error code. */
const char* ising_strerror(int code);

/* The HIP failure behind the last ISING_EDEVICE this context returned: the
 * failing call and HIP's error name ("" if there was none). The string
 * belongs to the context and lives until ising_destroy. */
const char* ising_device_error(const ising_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
