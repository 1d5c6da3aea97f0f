// C ABI and host runtime of the gfx950 checkerboard Metropolis engine.
// The public contract (model, keying, error behaviour) is in include/ising.h.
#include <hip/hip_runtime.h>

#include <cstdio>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <queue>
#include <vector>

#include "ising.h"
#include "ising_launch.hpp"
#include "ising_creutz.hpp"
#include "ising_runtime.hpp"

using namespace ising;

namespace ising {

// Threshold of the Metropolis decision for spin s (+1/-1) with neighbour sum
// n (Section 2.2, steps 2-4): dE = 2 s (J n + h); accept iff the 32-bit draw
// u < thr, thr = 2^32 for dE <= 0, else floor(exp(-dE/T) * 2^32). Evaluated
// in IEEE double in exactly this order, without contraction.
#pragma clang fp contract(off)
uint64_t metropolis_threshold(double J, double h, double T, int s, int n) {
    const double dE = 2.0 * (double)s * (J * (double)n + h);
    if (dE <= 0.0) return (uint64_t)1 << 32;
    return (uint64_t)std::floor(std::exp(-dE / T) * 4294967296.0);
}

void build_accept_table(double J, double h, double T, AcceptTable* at, bool* exact) {
    std::memset(at, 0, sizeof(*at));
    bool any_zero = false;
    for (int sbit = 0; sbit < 2; ++sbit) {
        for (int nup = 0; nup <= 4; ++nup) {
            const int code = 8 * sbit + nup;
            const uint64_t thr = metropolis_threshold(J, h, T, sbit ? 1 : -1, 2 * nup - 4);
            at->thr_lo[code] = (uint32_t)thr;
            at->thr_hi[code] = (uint32_t)(thr >> 32);
            if (thr == 0) any_zero = true;
            at->thr_m1[code] = thr == 0 ? 0u : (uint32_t)(thr - 1);
        }
    }
    *exact = any_zero;
}

uint64_t fnv1a64(const uint8_t* p, size_t n) {
    uint64_t hsh = 0xcbf29ce484222325ull;
    for (size_t k = 0; k < n; ++k) {
        hsh ^= p[k];
        hsh *= 0x100000001b3ull;
    }
    return hsh;
}

static bool valid_params(const ising_params* p) {
    if (!p) return false;
    if (p->L < 2 || (p->L & 1u) || p->L > ISING_MAX_L) return false;
    if (!std::isfinite(p->J) || !std::isfinite(p->h) || !std::isfinite(p->T) || !(p->T > 0.0)) return false;
    if (!(p->p_up >= 0.0 && p->p_up <= 1.0)) return false;
    if ((p->flags & 0xffu) > ISING_PLAN_BANDS) return false;
    return true;
}

// Plans remembered by the autotuner, by side.
static std::mutex g_tuned_mu;
static std::map<uint32_t, Plan> g_tuned;

// Sides up to this run all their sweeps inside one workgroup by default.
constexpr uint32_t kResidentMaxL = 128;
// Fused tiles wanted per launch (one wave each) before a taller/wider tile is used.
constexpr uint32_t kFusedMinTiles = 16384;
// The autotuner replaces the default plan only when a candidate is faster
// by more than this fraction (timing noise must not flip the choice).
constexpr float kTuneMargin = 0.03f;
// Band plan: sides it serves by default, and sweeps per launch (the
// partials of a launch are bands x sweeps pairs). Its default band height
// gives about one band per compute unit: one band a CU measured fastest
// from 192 to 16384 (fewer bands leave CUs idle, more put unequal numbers of
// bands on CUs; at the small sides a band's half-sweep is bound by the
// latency of its rows and of the edge exchange, not by the chip's rate).
constexpr uint32_t kBandMinDefaultL = 192;
constexpr uint32_t kBandChunk = ISING_BAND_SWEEPS_PER_LAUNCH;
constexpr uint32_t kTuneRounds = 3;

// Full-row fused shape: the widest chunk whose workgroup spans the row in at
// most 16 waves, with the tallest band that still gives 4096 waves (four per
// SIMD on 256 compute units: at 32768^2, 128-row bands, one workgroup per
// compute unit), else the shape with the most waves.
static bool default_fused_rows(uint32_t L, uint32_t* cw_out, uint32_t* rows_out) {
    static const uint32_t cws[3] = {4, 2, 1};
    static const uint32_t rs[5] = {128, 64, 32, 16, 8};
    uint64_t best = 0;
    uint32_t bcw = 0, br = 0;
    for (uint32_t cw : cws) {
        for (uint32_t r : rs) {
            if (!fused_rows_supported(L, cw, r)) continue;
            const uint64_t waves = (uint64_t)(L / 8u / (64u * cw)) * fused_rows_bands(L, r);
            if (waves >= 4096) {
                *cw_out = cw;
                *rows_out = r;
                return true;
            }
            if (waves > best) {
                best = waves;
                bcw = cw;
                br = r;
            }
        }
    }
    if (!best) return false;
    *cw_out = bcw;
    *rows_out = br;
    return true;
}

static uint32_t default_cw(uint32_t L) {
    const uint32_t Hw = L / 8u;
    return (Hw % 4u == 0u) ? 4u : (Hw % 2u == 0u) ? 2u : 1u;
}

// Largest fused tile (cw, rows) that still gives kFusedMinTiles tiles, else
// the one with the most tiles.
static bool default_fused(uint32_t L, uint32_t* cw_out, uint32_t* rows_out) {
    static const uint32_t cws[3] = {4, 2, 1};
    static const uint32_t rs[4] = {64, 32, 16, 8};
    uint32_t best_tiles = 0, bcw = 0, br = 0;
    for (uint32_t cw : cws) {
        for (uint32_t r : rs) {
            if (!fused_supported(L, cw, r)) continue;
            const uint32_t tiles = fused_tiles(L, cw, r);
            if (tiles >= kFusedMinTiles) {
                *cw_out = cw;
                *rows_out = r;
                return true;
            }
            if (tiles > best_tiles) {
                best_tiles = tiles;
                bcw = cw;
                br = r;
            }
        }
    }
    if (!best_tiles) return false;
    *cw_out = bcw;
    *rows_out = br;
    return true;
}

// Band plan geometry: bands of a nominal `rows` rows, `per_wave` rows a wave
// (at most 16 waves a workgroup; a wave runs its rows one after another).
uint32_t band_count(uint32_t L, uint32_t rows) { return (L + rows - 1u) / rows; }
uint32_t band_threads(uint32_t L, uint32_t G, uint32_t per_wave) {
    const uint32_t rows = (L + G - 1u) / G;
    return 64u * std::min<uint32_t>(16u, (rows + per_wave - 1u) / per_wave);
}
uint32_t band_words(uint32_t L) { return (L / 8u + 7u) / 8u; }

// Whether every band of the plan can be resident at once on the current
// device (counted for the kernel variant with more registers).
static bool bands_fit(uint32_t L, uint32_t rows, uint32_t per_wave) {
    const uint32_t G = band_count(L, rows);
    if (G < 2u || G > L) return false;
    const uint32_t cap =
        bands_capacity(band_threads(L, G, per_wave), band_lds_bytes(L, G, band_words(L)), true, band_words(L));
    return cap >= G;
}

static uint32_t band_default_rows(uint32_t L) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    return std::max<uint32_t>(1u, (L + (uint32_t)cus - 1u) / (uint32_t)cus);
}

bool plan_for(uint32_t L, uint32_t kind, uint32_t cw, uint32_t rows, Plan* out) {
    Plan pl{};
    const bool words = (L % 8u) == 0u;
    switch (kind) {
        case ISING_PLAN_GENERIC:
            pl.kind = ISING_PLAN_GENERIC;
            pl.cw = 1;
            break;
        case ISING_PLAN_TWO_PASS:
        case ISING_PLAN_RESIDENT:
            if (!words) return false;
            pl.kind = kind;
            pl.cw = cw ? cw : default_cw(L);
            if (pl.cw != 1 && pl.cw != 2 && pl.cw != 4) return false;
            if ((L / 8u) % pl.cw != 0u) return false;
            break;
        case ISING_PLAN_FUSED:
            pl.kind = ISING_PLAN_FUSED;
            if (cw == 0 && rows == 0) {
                if (!default_fused(L, &pl.cw, &pl.rows)) return false;
            } else {
                uint32_t dcw = 0, dr = 0;
                const bool have = default_fused(L, &dcw, &dr);
                pl.cw = cw ? cw : (have ? dcw : 1);
                pl.rows = rows ? rows : (have ? dr : 8);
                if (!fused_supported(L, pl.cw, pl.rows)) return false;
            }
            break;
        case ISING_PLAN_FUSED_ROWS:
            pl.kind = ISING_PLAN_FUSED_ROWS;
            if (cw == 0 && rows == 0) {
                if (!default_fused_rows(L, &pl.cw, &pl.rows)) return false;
            } else {
                uint32_t dcw = 0, dr = 0;
                const bool have = default_fused_rows(L, &dcw, &dr);
                pl.cw = cw ? cw : (have ? dcw : 1);
                pl.rows = rows ? rows : (have ? dr : 8);
                if (!fused_rows_supported(L, pl.cw, pl.rows)) return false;
            }
            break;
        case ISING_PLAN_BANDS:
            if (!words || band_words(L) > kBandMaxWr) return false;
            pl.kind = ISING_PLAN_BANDS;
            pl.cw = cw ? cw : 1;  // rows a wave
            if (pl.cw != 1 && pl.cw != 2 && pl.cw != 4) return false;
            pl.rows = rows ? rows : band_default_rows(L);
            if (!bands_fit(L, pl.rows, pl.cw)) return false;
            break;
        case ISING_PLAN_AUTO: {
            {
                std::lock_guard<std::mutex> g(g_tuned_mu);
                auto it = g_tuned.find(L);
                if (it != g_tuned.end()) {
                    *out = it->second;
                    return true;
                }
            }
            if (!words) return plan_for(L, ISING_PLAN_GENERIC, 0, 0, out);
            if (L <= kResidentMaxL) return plan_for(L, ISING_PLAN_RESIDENT, 0, 0, out);
            if (L >= kBandMinDefaultL && plan_for(L, ISING_PLAN_BANDS, 0, 0, out)) return true;
            if (plan_for(L, ISING_PLAN_FUSED_ROWS, 0, 0, out)) return true;
            if (plan_for(L, ISING_PLAN_FUSED, 0, 0, out)) return true;
            return plan_for(L, ISING_PLAN_TWO_PASS, 0, 0, out);
        }
        default:
            return false;
    }
    *out = pl;
    return true;
}

}  // namespace ising

// ---------------------------------------------------------------------------
// Context helpers
// ---------------------------------------------------------------------------
int ctx_fail(ising_ctx* ctx, hipError_t e, const char* where) {
    ctx->poisoned = true;
    ctx->last_hip = e;
    std::snprintf(ctx->device_error, sizeof(ctx->device_error), "%.100s: %s (%d)", where ? where : "",
                  hipGetErrorName(e), (int)e);
    (void)hipGetLastError();
    return ISING_EDEVICE;
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return ctx_fail((ctx), e_, #expr); \
    } while (0)

static int ctx_enter(ising_ctx* ctx) {
    if (!ctx) return ISING_EINVAL;
    if (ctx->poisoned) return ISING_ESTATE;
    ++ctx->api_seq;  // the stream may get work the batch engine has not seen
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return ctx_fail(ctx, e, "hipSetDevice");
    return ISING_OK;
}

static Planes planes_of(uint8_t* base, uint32_t L) {
    Planes p;
    const size_t N = (size_t)L * L;
    p.p[0] = base;
    p.p[1] = base + N / 2;
    p.L = L;
    p.H = L / 2;
    p.Hw = L / 8;
    return p;
}

Planes ctx_planes(const ising_ctx* ctx) { return planes_of(ctx->buf[ctx->cur], ctx->L); }
Planes ctx_planes_alt(const ising_ctx* ctx) { return planes_of(ctx->buf[ctx->cur ^ 1], ctx->L); }

// Make room for `more` series entries beyond the pending ones.
int ctx_reserve_series(ising_ctx* ctx, uint64_t more) {
    const uint64_t need = ctx->series_len + more;
    if (need <= ctx->series_cap) return ISING_OK;
    uint64_t cap = ctx->series_cap ? ctx->series_cap : 1024;
    while (cap < need) cap *= 2;
    int64_t* fresh = nullptr;
    if (hipMalloc(&fresh, cap * 2 * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return ISING_ENOMEM;
    }
    if (ctx->series) {
        if (ctx->series_len) {
            HIP_TRY(ctx, hipMemcpyAsync(fresh, ctx->series, ctx->series_len * 2 * sizeof(int64_t),
                                        hipMemcpyDeviceToDevice, ctx->stream));
        }
        // queued work may still write the old buffer (a first buffer needs
        // no wait: nothing queued refers to it)
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(ctx->series);
    }
    ctx->series = fresh;
    ctx->series_cap = cap;
    return ISING_OK;
}

// The band plan's edge-row slots for G bands and its timeout mark (the
// slots only grow; growing waits for the launches that may still use them).
static int ctx_band_slots(ising_ctx* ctx, uint32_t G) {
    if (G > ctx->band_cap) {
        if (ctx->band_cap) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->band_pub) (void)hipFree(ctx->band_pub);
        ctx->band_pub = nullptr;
        ctx->band_cap = 0;
        const size_t words = band_pub_words(G, band_words(ctx->L));
        if (hipMalloc(&ctx->band_pub, words * sizeof(uint64_t)) != hipSuccess) {
            (void)hipGetLastError();
            return ISING_ENOMEM;
        }
        // fresh slots carry tag 0, below every tag a launch waits for
        HIP_TRY(ctx, hipMemsetAsync(ctx->band_pub, 0, words * sizeof(uint64_t), ctx->stream));
        ctx->band_base = 0;
        ctx->band_cap = G;
    }
    if (!ctx->band_err) {
        if (hipMalloc(&ctx->band_err, sizeof(uint32_t)) != hipSuccess ||
            hipHostMalloc(&ctx->band_err_host, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return ISING_ENOMEM;
        }
        *ctx->band_err_host = 0;
        HIP_TRY(ctx, hipMemsetAsync(ctx->band_err, 0, sizeof(uint32_t), ctx->stream));
    }
    return ISING_OK;
}

// Allocate what the context's plan needs: the second lattice buffer for
// ping-pong, partial-sum buffers sized to the plan's tiles or blocks.
int ctx_prepare_plan(ising_ctx* ctx) {
    const size_t N = (size_t)ctx->L * ctx->L;
    const bool pingpong = ctx->plan.kind == ISING_PLAN_FUSED || ctx->plan.kind == ISING_PLAN_FUSED_ROWS;
    if (pingpong && !ctx->buf[1]) {
        if (hipMalloc(&ctx->buf[1], N) != hipSuccess) {
            (void)hipGetLastError();
            return ISING_ENOMEM;
        }
        ctx->owns_buf[1] = true;
    }
    if (ctx->plan.kind == ISING_PLAN_BANDS) {
        const int rc = ctx_band_slots(ctx, band_count(ctx->L, ctx->plan.rows));
        if (rc != ISING_OK) return rc;
    }
    uint32_t need = 0;
    const Planes pl = ctx_planes(ctx);
    if (ctx->plan.kind == ISING_PLAN_FUSED) need = fused_tiles(ctx->L, ctx->plan.cw, ctx->plan.rows);
    if (ctx->plan.kind == ISING_PLAN_FUSED_ROWS) need = fused_rows_bands(ctx->L, ctx->plan.rows);
    if (ctx->plan.kind == ISING_PLAN_TWO_PASS) need = two_pass_blocks(pl, ctx->plan.cw);
    if (need > ctx->part_cap) {
        for (int k = 0; k < 2; ++k) {
            if (ctx->part[k]) (void)hipFree(ctx->part[k]);
            ctx->part[k] = nullptr;
        }
        ctx->part_cap = 0;
        for (int k = 0; k < 2; ++k) {
            if (hipMalloc(&ctx->part[k], (size_t)need * 2 * sizeof(int64_t)) != hipSuccess) {
                (void)hipGetLastError();
                return ISING_ENOMEM;
            }
        }
        ctx->part_cap = need;
    }
    return ISING_OK;
}

static size_t state_bytes_for(uint32_t L, const Plan& pl) {
    const size_t N = (size_t)L * L;
    return (pl.kind == ISING_PLAN_FUSED || pl.kind == ISING_PLAN_FUSED_ROWS) ? 2 * N : N;
}

// n sweeps of either fused plan; series slots ser[0 .. 2n); per-tile (per
// band) partials alternate between part0 and part1 (each n_tiles pairs).
static int sweep_fused(ising_ctx* ctx, uint64_t n, int64_t* ser, int64_t* part0, int64_t* part1) {
    int64_t* const part[2] = {part0, part1};
    const uint32_t k0 = (uint32_t)ctx->p.seed, k1 = (uint32_t)(ctx->p.seed >> 32);
    const uint32_t L = ctx->L, Hw = L / 8u;
    const uint32_t cw = ctx->plan.cw, rows = ctx->plan.rows;
    const bool by_rows = ctx->plan.kind == ISING_PLAN_FUSED_ROWS;
    const uint32_t n_tx = Hw / (64u * cw);
    const uint32_t n_tiles = by_rows ? fused_rows_bands(L, rows) : fused_tiles(L, cw, rows);
    for (uint64_t k = 0; k < n; ++k) {
        const uint32_t t = (uint32_t)(ctx->t + k);
        const Planes src = ctx_planes(ctx), dst = ctx_planes_alt(ctx);
        FusedArgs a{reinterpret_cast<const uint32_t*>(src.p[0]), reinterpret_cast<const uint32_t*>(src.p[1]),
                    reinterpret_cast<uint32_t*>(dst.p[0]), reinterpret_cast<uint32_t*>(dst.p[1]),
                    L, Hw, t, k0, k1, n_tx, n_tiles, part[k & 1]};
        PartialReduce red{nullptr, 0, nullptr};
        if (k > 0) red = PartialReduce{part[(k - 1) & 1], n_tiles, ser + 2 * (k - 1)};
        if (by_rows)
            HIP_TRY(ctx, launch_fused_rows(a, ctx->table, cw, rows, red, ctx->stream));
        else
            HIP_TRY(ctx, launch_fused(a, ctx->table, ctx->exact, cw, rows, red, ctx->stream));
        ctx->cur ^= 1;
    }
    HIP_TRY(ctx, launch_reduce_partials(PartialReduce{part[(n - 1) & 1], n_tiles, ser + 2 * (n - 1)}, ctx->stream));
    return ISING_OK;
}

// The band plan's partials for launches of kBandChunk sweeps, allocated on
// the first ising_sweep (a context that only runs in batches never needs
// them, and ising_sweep_static uses the library's array instead).
static int ctx_band_part(ising_ctx* ctx, uint32_t G) {
    if (ctx->band_part && ctx->band_part_cap >= G) return ISING_OK;
    if (ctx->band_part) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(ctx->band_part);
        ctx->band_part = nullptr;
        ctx->band_part_cap = 0;
    }
    if (hipMalloc(&ctx->band_part, (size_t)kBandChunk * G * 2 * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        ctx->band_part = nullptr;
        return ISING_ENOMEM;
    }
    ctx->band_part_cap = G;
    return ISING_OK;
}

// n sweeps of the band plan with bands of `rows` rows, `per_wave` rows a
// wave: launches of up to `chunk` sweeps, each followed by the sum of its
// bands' partials (at part) into ser.
static int sweep_bands(ising_ctx* ctx, uint64_t n, int64_t* ser, int64_t* part, uint32_t chunk, uint32_t rows,
                       uint32_t per_wave) {
    const uint32_t L = ctx->L, G = band_count(L, rows);
    const Planes pl = ctx_planes(ctx);
    const uint32_t mode = bits_mode(ctx->table);
    BandArgs a{};
    a.p0 = reinterpret_cast<uint32_t*>(pl.p[0]);
    a.p1 = reinterpret_cast<uint32_t*>(pl.p[1]);
    a.L = L;
    a.Hw = L / 8u;
    a.Wr = band_words(L);
    a.k0 = (uint32_t)ctx->p.seed;
    a.k1 = (uint32_t)(ctx->p.seed >> 32);
    a.pub = ctx->band_pub;
    a.part = part;
    a.err = ctx->band_err;
    a.general = mode == 3u;
    a.bl = bits_lattice(ctx->table, L, a.Hw, mode);
    a.at = ctx->table;
    for (uint64_t done = 0; done < n;) {
        const uint32_t m = (uint32_t)std::min<uint64_t>(n - done, chunk);
        if ((uint64_t)ctx->band_base + 2ull * m >= 0xffffffffull) {
            // the tags would wrap: clear every slot and count from 0 again
            HIP_TRY(ctx, launch_bands_clear(ctx->band_pub, band_pub_words(ctx->band_cap, a.Wr), ctx->stream));
            ctx->band_base = 0;
        }
        a.t0 = (uint32_t)(ctx->t + done);
        a.n = m;
        a.base = ctx->band_base;
        HIP_TRY(ctx, launch_bands(a, G, band_threads(L, G, per_wave), ctx->stream));
        // every slot the launch used ends it tagged base + 2 m or base + 2 m - 1
        ctx->band_base += 2u * m;
        HIP_TRY(ctx, launch_bands_reduce(part, G, m, ser + 2 * done, ctx->stream));
        done += m;
    }
    return ISING_OK;
}

// n sweeps of the two-pass plan; per-block partials in part (nb pairs).
// (cw: words per thread, 0 for the context's plan's.)
static int sweep_two_pass(ising_ctx* ctx, uint64_t n, int64_t* ser, int64_t* part, uint32_t cw = 0) {
    const uint32_t k0 = (uint32_t)ctx->p.seed, k1 = (uint32_t)(ctx->p.seed >> 32);
    const Planes pl = ctx_planes(ctx);
    if (!cw) cw = ctx->plan.cw;
    const uint32_t nb = two_pass_blocks(pl, cw);
    for (uint64_t k = 0; k < n; ++k) {
        const uint32_t t = (uint32_t)(ctx->t + k);
        PartialReduce red{nullptr, 0, nullptr};
        if (k > 0) red = PartialReduce{part, nb, ser + 2 * (k - 1)};
        HIP_TRY(ctx, launch_two_pass(pl, ctx->table, ctx->exact, cw, t, k0, k1, part, red, ctx->stream));
    }
    HIP_TRY(ctx, launch_reduce_partials(PartialReduce{part, nb, ser + 2 * (n - 1)}, ctx->stream));
    return ISING_OK;
}

// Sweeps per graph replay of a single context. Only the two-pass plan
// replays graphs: its two short launches per sweep leave small lattices
// bound by launch latency, which a replay cuts (256 x 256: 8.8 -> 6.9 us
// per sweep). The fused plans' one launch per sweep measured no faster
// replayed at 512 to 2048 and 7% slower at 4096, so they launch directly.
constexpr uint32_t kGraphSweeps = 16;

void ctx_drop_graphs(ising_ctx* ctx) {
    if (!ctx->gexec) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
}

// Capture kGraphSweeps sweeps of the two-pass plan into ctx->gexec: each
// sweep writes its partials to a slot of its own and reads its index from
// the header; the last node sums the partials into the series slots the
// header names and advances the header.
static int ctx_build_graph(ising_ctx* ctx) {
    const Planes pl = ctx_planes(ctx);
    const uint32_t pairs = two_pass_blocks(pl, ctx->plan.cw);
    if (!ctx->ghdr) {
        if (hipMalloc(&ctx->ghdr, sizeof(SweepHeader)) != hipSuccess) {
            (void)hipGetLastError();
            ctx->ghdr = nullptr;
            return ISING_ENOMEM;
        }
    }
    const size_t need = (size_t)kGraphSweeps * pairs;
    if (need > ctx->gpart_pairs) {
        ctx_drop_graphs(ctx);  // a captured graph may write the old buffer
        if (ctx->gpart) (void)hipFree(ctx->gpart);
        ctx->gpart = nullptr;
        ctx->gpart_pairs = 0;
        if (hipMalloc(&ctx->gpart, need * 2 * sizeof(int64_t)) != hipSuccess) {
            (void)hipGetLastError();
            ctx->gpart = nullptr;
            return ISING_ENOMEM;
        }
        ctx->gpart_pairs = need;
    }
    const uint32_t k0 = (uint32_t)ctx->p.seed, k1 = (uint32_t)(ctx->p.seed >> 32);
    const PartialReduce none{nullptr, 0, nullptr};
    hipStream_t cap = nullptr;
    HIP_TRY(ctx, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t r = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    hipError_t lr = hipSuccess;
    if (r == hipSuccess) {
        for (uint32_t k = 0; lr == hipSuccess && k < kGraphSweeps; ++k)
            lr = launch_two_pass(pl, ctx->table, ctx->exact, ctx->plan.cw, k, k0, k1, ctx->gpart + 2ull * k * pairs,
                                 none, cap, &ctx->ghdr->t);
        if (lr == hipSuccess) lr = launch_reduce_group(ctx->gpart, pairs, kGraphSweeps, ctx->ghdr, cap);
        hipGraph_t graph = nullptr;
        r = hipStreamEndCapture(cap, &graph);
        if (r == hipSuccess && lr != hipSuccess) r = lr;
        if (r == hipSuccess) r = hipGraphInstantiate(&ctx->gexec, graph, nullptr, nullptr, 0);
        if (r == hipSuccess) ctx->gcur = ctx->cur;
        if (graph) (void)hipGraphDestroy(graph);
    }
    (void)hipStreamDestroy(cap);
    if (r != hipSuccess) return ctx_fail(ctx, r, "capture of the sweep graph");
    return ISING_OK;
}

// The first n - n % kGraphSweeps of n sweeps as graph replays; returns the
// sweeps left for direct launches.
static int sweep_replays(ising_ctx* ctx, uint64_t n, uint64_t* left) {
    *left = n;
    const uint64_t reps = n / kGraphSweeps;
    if (reps == 0 || ctx->plan.kind != ISING_PLAN_TWO_PASS) return ISING_OK;
    if (ctx->gexec && ctx->gcur != (uint32_t)ctx->cur) ctx_drop_graphs(ctx);  // a fused batch or Creutz sweep moved the lattice
    if (!ctx->gexec) {
        const int rc = ctx_build_graph(ctx);
        if (rc != ISING_OK) return rc;
    }
    HIP_TRY(ctx, launch_set_header(ctx->ghdr, (uint32_t)ctx->t, ctx->series + 2 * ctx->series_len, ctx->stream));
    for (uint64_t k = 0; k < reps; ++k) HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
    ctx->t += reps * kGraphSweeps;
    ctx->series_len += reps * kGraphSweeps;
    *left = n - reps * kGraphSweeps;
    return ISING_OK;
}

static int sweep_generic(ising_ctx* ctx, uint64_t n, int64_t* ser) {
    const uint32_t k0 = (uint32_t)ctx->p.seed, k1 = (uint32_t)(ctx->p.seed >> 32);
    HIP_TRY(ctx, launch_zero(ser, 2 * n, ctx->stream));
    const Planes pl = ctx_planes(ctx);
    for (uint64_t k = 0; k < n; ++k) {
        const uint32_t t = (uint32_t)(ctx->t + k);
        HIP_TRY(ctx, launch_generic_sweep(pl, ctx->table, ctx->exact, t, k0, k1, ser + 2 * k, ctx->stream));
    }
    return ISING_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t ising_state_bytes(uint32_t L, uint32_t flags) {
    if (L < 2 || (L & 1u) || L > ISING_MAX_L) return 0;
    Plan pl;
    if (!plan_for(L, flags & 0xffu, 0, 0, &pl)) return 0;
    return state_bytes_for(L, pl);
}

static int create_common(const ising_params* params, void* dev_buf, size_t bytes, void* stream,
                         ising_ctx** out) {
    if (!out) return ISING_EINVAL;
    *out = nullptr;
    if (!valid_params(params)) return ISING_EINVAL;
    Plan plan;
    if (!plan_for(params->L, params->flags & 0xffu, 0, 0, &plan)) return ISING_EUNSUPPORTED;
    const size_t N = (size_t)params->L * params->L;
    const size_t need = state_bytes_for(params->L, plan);
    if (dev_buf && bytes < need) return ISING_EINVAL;

    ising_ctx* ctx = new (std::nothrow) ising_ctx();
    if (!ctx) return ISING_ENOMEM;
    ctx->p = *params;
    ctx->L = params->L;
    ctx->plan = plan;
    build_accept_table(params->J, params->h, params->T, &ctx->table, &ctx->exact);
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return ISING_EDEVICE;
    }
    if (stream) {
        ctx->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return ISING_EDEVICE;
        }
        ctx->owns_stream = true;
    }
    if (dev_buf) {
        ctx->buf[0] = (uint8_t*)dev_buf;
        if (need >= 2 * N) ctx->buf[1] = (uint8_t*)dev_buf + N;
    } else {
        if (hipMalloc(&ctx->buf[0], N) != hipSuccess) {
            (void)hipGetLastError();
            ising_destroy(ctx);
            return ISING_ENOMEM;
        }
        ctx->owns_buf[0] = true;
    }
    if (hipMalloc(&ctx->scratch, 4 * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        ising_destroy(ctx);
        return ISING_ENOMEM;
    }
    // the series buffer is allocated by the first sweep or ising_reserve, so
    // that a caller reserving its whole run allocates it once, with no free
    int rc = ctx_prepare_plan(ctx);
    if (rc != ISING_OK) {
        ising_destroy(ctx);
        return rc;
    }
    const uint64_t pthr = (uint64_t)std::floor(params->p_up * 4294967296.0);
    if (launch_init(ctx_planes(ctx), (ctx->L % 8u) == 0u, (uint32_t)params->seed,
                    (uint32_t)(params->seed >> 32), pthr, ctx->stream) != hipSuccess) {
        ising_destroy(ctx);
        return ISING_EDEVICE;
    }
    *out = ctx;
    return ISING_OK;
}

int ising_create(const ising_params* params, void* stream, ising_ctx** out) {
    return create_common(params, nullptr, 0, stream, out);
}

int ising_create_in(const ising_params* params, void* dev_buf, size_t bytes, void* stream, ising_ctx** out) {
    if (!dev_buf) {
        if (out) *out = nullptr;
        return ISING_EINVAL;
    }
    return create_common(params, dev_buf, bytes, stream, out);
}

int ising_reset(ising_ctx* ctx, const ising_params* params) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (!valid_params(params) || params->L != ctx->L) return ISING_EINVAL;
    const uint32_t kind = params->flags & 0xffu;
    if (kind != ISING_PLAN_AUTO && kind != ctx->plan.kind) return ISING_EINVAL;
    if (ctx->demon || ctx->demon_alt) {
        // earlier work on the context's stream may still read the demons
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->demon) (void)hipFree(ctx->demon);
        if (ctx->demon_alt) (void)hipFree(ctx->demon_alt);
        ctx->demon = nullptr;
        ctx->demon_alt = nullptr;
    }
    // the new initial lattice is drawn on the context's stream, after all of
    // its earlier work; captured sweeps hold the old table and key
    ctx_drop_graphs(ctx);
    ctx->p = *params;
    build_accept_table(params->J, params->h, params->T, &ctx->table, &ctx->exact);
    ctx->cur = 0;
    ctx->t = 0;
    ctx->series_len = 0;
    ++ctx->gen;
    const uint64_t pthr = (uint64_t)std::floor(params->p_up * 4294967296.0);
    HIP_TRY(ctx, launch_init(ctx_planes(ctx), (ctx->L % 8u) == 0u, (uint32_t)params->seed,
                             (uint32_t)(params->seed >> 32), pthr, ctx->stream));
    return ISING_OK;
}

int ising_reserve(ising_ctx* ctx, uint64_t sweeps) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (ctx->t + sweeps > ((uint64_t)1 << 32)) return ISING_ERANGE;
    return ctx_reserve_series(ctx, sweeps);
}

// Whether work enqueued on s is being captured into a graph. The band plan
// must not be captured: each launch's edge-row tags start from a base the
// host advances per launch, so a replayed launch would find the slots
// still holding the previous replay's words under the tags it waits for.
static bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return st != hipStreamCaptureStatusNone;
}

int ising_sweep(ising_ctx* ctx, uint64_t n) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (n == 0) return ISING_OK;
    if (ctx->plan.kind == ISING_PLAN_BANDS && stream_capturing(ctx->stream)) return ISING_EUNSUPPORTED;
    if (ctx->t + n > ((uint64_t)1 << 32)) return ISING_ERANGE;
    rc = ctx_reserve_series(ctx, n);
    if (rc != ISING_OK) return rc;
    ++ctx->gen;
    if (ctx->plan.kind == ISING_PLAN_RESIDENT) {
        // one workgroup runs every sweep from local memory (bytes: a lone
        // lattice's latency, not the chip's throughput, sets the time)
        BatchItem it;
        fill_batch_item(ctx, n, false, it);
        if (bits_fit(ctx->L) && !bytes_fit(ctx->L)) it.bits = bits_mode(ctx->table);
        HIP_TRY(ctx, launch_batch_one(it, ctx->stream));
        ctx->t += n;
        ctx->series_len += n;
        return ISING_OK;
    }
    rc = sweep_replays(ctx, n, &n);
    if (rc != ISING_OK || n == 0) return rc;
    int64_t* ser = ctx->series + 2 * ctx->series_len;
    switch (ctx->plan.kind) {
        case ISING_PLAN_FUSED:
        case ISING_PLAN_FUSED_ROWS: rc = sweep_fused(ctx, n, ser, ctx->part[0], ctx->part[1]); break;
        case ISING_PLAN_TWO_PASS: rc = sweep_two_pass(ctx, n, ser, ctx->part[0]); break;
        case ISING_PLAN_GENERIC: rc = sweep_generic(ctx, n, ser); break;
        case ISING_PLAN_BANDS:
            rc = ctx_band_part(ctx, band_count(ctx->L, ctx->plan.rows));
            if (rc == ISING_OK) rc = sweep_bands(ctx, n, ser, ctx->band_part, kBandChunk, ctx->plan.rows, ctx->plan.cw);
            break;
        default: return ISING_EUNSUPPORTED;
    }
    if (rc != ISING_OK) return rc;
    ctx->t += n;
    ctx->series_len += n;
    return ISING_OK;
}

// Device array for ising_sweep_static: the per-tile (or per-block) partial
// sums of its sweep kernels. One copy per device, for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress
// returned on that device (the array's name is not a device address in host
// code).
static __device__ __align__(256) int64_t scratch[2 * ISING_STATIC_SCRATCH_PAIRS];
static std::mutex g_scratch_mu;
static int64_t* g_scratch_ptr[64] = {};

// The array's address on `dev` (current), looked up on the first call there.
static int64_t* static_scratch(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<int64_t*>(ptr);
    }
    return g_scratch_ptr[dev];
}

int ising_sweep_static(ising_ctx* ctx, uint64_t n, int64_t* series_dev) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (!series_dev) return ISING_EINVAL;
    if (n == 0) return ISING_OK;
    if (ctx->t + n > ((uint64_t)1 << 32)) return ISING_ERANGE;
    uint32_t pairs = 0;  // partial slots the plan's kernels need
    if (ctx->plan.kind == ISING_PLAN_FUSED) pairs = 2 * fused_tiles(ctx->L, ctx->plan.cw, ctx->plan.rows);
    if (ctx->plan.kind == ISING_PLAN_FUSED_ROWS) pairs = 2 * fused_rows_bands(ctx->L, ctx->plan.rows);
    if (ctx->plan.kind == ISING_PLAN_TWO_PASS) pairs = two_pass_blocks(ctx_planes(ctx), ctx->plan.cw);
    // under capture the band plan's sweeps run as two-pass launches
    const bool bands_as_two_pass = ctx->plan.kind == ISING_PLAN_BANDS && stream_capturing(ctx->stream);
    if (ctx->plan.kind == ISING_PLAN_BANDS)
        pairs = bands_as_two_pass ? two_pass_blocks(ctx_planes(ctx), 1) : band_count(ctx->L, ctx->plan.rows);
    if (pairs > ISING_STATIC_SCRATCH_PAIRS) return ISING_ERANGE;
    int64_t* sc = nullptr;
    if (pairs) {
        sc = static_scratch(ctx->device);
        if (!sc) return ctx_fail(ctx, hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    }
    ++ctx->gen;
    switch (ctx->plan.kind) {
        case ISING_PLAN_FUSED:
        case ISING_PLAN_FUSED_ROWS: {
            const uint32_t tiles = pairs / 2;
            rc = sweep_fused(ctx, n, series_dev, sc, sc + 2ull * tiles);
            break;
        }
        case ISING_PLAN_TWO_PASS: rc = sweep_two_pass(ctx, n, series_dev, sc); break;
        case ISING_PLAN_GENERIC: rc = sweep_generic(ctx, n, series_dev); break;
        case ISING_PLAN_BANDS:
            if (bands_as_two_pass)
                rc = sweep_two_pass(ctx, n, series_dev, sc, 1);
            else
                rc = sweep_bands(ctx, n, series_dev, sc,
                                 std::min<uint32_t>(kBandChunk, ISING_STATIC_SCRATCH_PAIRS / pairs), ctx->plan.rows,
                                 ctx->plan.cw);
            break;
        case ISING_PLAN_RESIDENT: {
            BatchItem it;
            fill_batch_item(ctx, n, false, it);
            it.series = series_dev;
            if (bits_fit(ctx->L) && !bytes_fit(ctx->L)) it.bits = bits_mode(ctx->table);
            HIP_TRY(ctx, launch_batch_one(it, ctx->stream));
            rc = ISING_OK;
            break;
        }
        default: return ISING_EUNSUPPORTED;
    }
    if (rc != ISING_OK) return rc;
    ctx->t += n;
    return ISING_OK;
}

int ising_sweep_batch(ising_ctx* const* ctxs, const uint64_t* n_sweeps, size_t count, void* stream) {
    return ising_sweep_batch_plan(ctxs, n_sweeps, count, stream, ISING_BATCH_AUTO);
}

// A batch with one lattice to sweep: the batch plans spread it over too
// few workgroups (the resident plan: one; the stepped plan: one wave per
// tile), so it runs on the band plan at its default band height (whatever
// the context's own plan), ordered like a batch on stream s: after s's
// earlier work and before its later work (s null: the context's stream,
// which every earlier batch of the engine was ordered before).
static int lone_band_batch(ising_ctx* ctx, uint64_t n, hipStream_t s) {
    int rc = ctx_enter(ctx);  // the engine orders this context afresh next time
    if (rc != ISING_OK) return rc;
    Plan bp;
    if (!plan_for(ctx->L, ISING_PLAN_BANDS, 0, 0, &bp)) return ISING_EUNSUPPORTED;
    const uint32_t G = band_count(ctx->L, bp.rows);
    if ((rc = ctx_reserve_series(ctx, n)) != ISING_OK) return rc;
    if ((rc = ctx_band_slots(ctx, G)) != ISING_OK) return rc;
    if ((rc = ctx_band_part(ctx, G)) != ISING_OK) return rc;
    const bool other = s && s != ctx->stream;
    struct Ev {
        hipEvent_t e = nullptr;
        ~Ev() {
            if (e) (void)hipEventDestroy(e);
        }
    } ev;
    if (other) {
        HIP_TRY(ctx, hipEventCreateWithFlags(&ev.e, hipEventDisableTiming));
        HIP_TRY(ctx, hipEventRecord(ev.e, s));
        HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, ev.e, 0));
    }
    ++ctx->gen;
    rc = sweep_bands(ctx, n, ctx->series + 2 * ctx->series_len, ctx->band_part, kBandChunk, bp.rows, bp.cw);
    if (rc != ISING_OK) return rc;
    ctx->t += n;
    ctx->series_len += n;
    if (other) {
        HIP_TRY(ctx, hipEventRecord(ev.e, ctx->stream));
        HIP_TRY(ctx, hipStreamWaitEvent(s, ev.e, 0));
    }
    return ISING_OK;
}

// Whether a batch of one lattice with sweeps goes to lone_band_batch: the
// sides where the band plan is the single-lattice default.
static bool lone_band_fits(const ising_ctx* c) {
    Plan bp;
    return c->L >= kBandMinDefaultL && plan_for(c->L, ISING_PLAN_BANDS, 0, 0, &bp);
}

int ising_sweep_batch_plan(ising_ctx* const* ctxs, const uint64_t* n_sweeps, size_t count, void* stream,
                           uint32_t plan) {
    if (!ctxs || !n_sweeps || plan > ISING_BATCH_STEPPED) return ISING_EINVAL;
    if (count == 0) return ISING_OK;
    int dev = -1;
    for (size_t k = 0; k < count; ++k) {
        ising_ctx* c = ctxs[k];
        if (!c) return ISING_EINVAL;
        if (c->poisoned) return ISING_ESTATE;
        if (c->L % 8u != 0u) return ISING_EUNSUPPORTED;
        if (c->t + n_sweeps[k] > ((uint64_t)1 << 32)) return ISING_ERANGE;
        if (dev < 0) dev = c->device;
        if (c->device != dev) return ISING_EINVAL;
        for (size_t j = 0; j < k; ++j)
            if (ctxs[j] == c) return ISING_EINVAL;  // one context may appear once
    }
    if (hipSetDevice(dev) != hipSuccess) return ISING_EDEVICE;
    if (plan == ISING_BATCH_AUTO) {
        size_t live = 0, only = 0;
        for (size_t k = 0; k < count; ++k)
            if (n_sweeps[k]) {
                ++live;
                only = k;
            }
        if (live == 0) return ISING_OK;
        if (live == 1 && lone_band_fits(ctxs[only]))
            return lone_band_batch(ctxs[only], n_sweeps[only], static_cast<hipStream_t>(stream));
    }
    // the plan (AUTO) and the stepped tile height predicted fastest from
    // the device's per-class rates
    BatchChoice ch;
    const int rc = batch_choose(ctxs, n_sweeps, count, dev, &ch);
    if (rc != ISING_OK) return rc;
    const bool stepped = plan == ISING_BATCH_AUTO ? ch.stepped : plan == ISING_BATCH_STEPPED;
    return engine_run(ctxs, n_sweeps, count, static_cast<hipStream_t>(stream), stepped, ch.rows);
}

static int ensure_canonical(ising_ctx* ctx) {
    if (ctx->canon) return ISING_OK;
    if (hipMalloc(&ctx->canon, (size_t)ctx->L * ctx->L) != hipSuccess) {
        (void)hipGetLastError();
        return ISING_ENOMEM;
    }
    return ISING_OK;
}

// The band plan's edge waits give up only when a neighbouring band stopped
// publishing (the bands were not all resident): the launch's results are
// then not valid. Copy its mark back with a read-back, check it after.
static int enqueue_band_check(ising_ctx* ctx) {
    if (ctx->band_err)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->band_err_host, ctx->band_err, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
    return ISING_OK;
}

static int band_check(ising_ctx* ctx) {
    if (ctx->band_err_host && *ctx->band_err_host)
        return ctx_fail(ctx, hipErrorLaunchTimeOut, "band plan: a wait for a neighbouring band gave up");
    return ISING_OK;
}

int ising_copy_spins(ising_ctx* ctx, int8_t* host, size_t n) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    const size_t N = (size_t)ctx->L * ctx->L;
    if (!host || n < N) return ISING_EINVAL;
    rc = ensure_canonical(ctx);
    if (rc != ISING_OK) return rc;
    HIP_TRY(ctx, launch_to_canonical(ctx_planes(ctx), ctx->canon, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(host, ctx->canon, N, hipMemcpyDeviceToHost, ctx->stream));
    rc = enqueue_band_check(ctx);
    if (rc != ISING_OK) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return band_check(ctx);
}

int ising_load_spins(ising_ctx* ctx, const int8_t* host, size_t n, uint64_t t) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    const size_t N = (size_t)ctx->L * ctx->L;
    if (!host || n < N || t > ((uint64_t)1 << 32)) return ISING_EINVAL;
    for (size_t k = 0; k < N; ++k)
        if (host[k] != 1 && host[k] != -1) return ISING_EINVAL;
    rc = ensure_canonical(ctx);
    if (rc != ISING_OK) return rc;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->canon, host, N, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, launch_from_canonical(ctx_planes(ctx), ctx->canon, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->t = t;
    ctx->series_len = 0;
    ++ctx->gen;
    return ISING_OK;
}

// Pinned host memory of at least `bytes`, kept by the context for reading
// observables back. A device-to-host copy into pinned memory goes to a DMA
// engine and is ordered by its stream alone; a copy into pageable memory is
// staged by the runtime through copy kernels on the stream's hardware queue,
// where it can wait behind other streams' kernels that share the queue.
// Returns nullptr when `bytes` exceeds kMaxHostStage or the allocation fails:
// the caller then reads into pageable memory. The stage only grows, and only
// between calls (each read-back is synchronised before it returns).
static constexpr size_t kMaxHostStage = (size_t)64 << 20;

static void* ctx_host_stage(ising_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->host_stage_bytes) return ctx->host_stage;
    if (bytes > kMaxHostStage) return nullptr;
    const size_t series_bytes = (size_t)ctx->series_cap * 2 * sizeof(int64_t);
    size_t want = std::max<size_t>(bytes, std::min(kMaxHostStage, series_bytes));
    want = std::max<size_t>(want, 4096);
    void* fresh = nullptr;
    if (hipHostMalloc(&fresh, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
    ctx->host_stage = fresh;
    ctx->host_stage_bytes = want;
    return fresh;
}

// Enqueue on the context's stream the copies ising_observables reads: the
// whole pending series into `ser` when `full` (else the current (B, M): the
// last series entry, or a fresh reduction when no sweep is pending) and,
// with ISING_OBS_HASH, the canonical lattice bytes into `bytes`.
static int enqueue_readback(ising_ctx* ctx, uint32_t want, bool full, int64_t* ser, uint8_t* bytes) {
    const uint64_t len = ctx->series_len;
    if (full) {
        HIP_TRY(ctx, hipMemcpyAsync(ser, ctx->series, 2 * len * sizeof(int64_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
    } else if (len) {
        HIP_TRY(ctx, hipMemcpyAsync(ser, ctx->series + 2 * (len - 1), 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
    } else {
        HIP_TRY(ctx, launch_observe(ctx_planes(ctx), ctx->scratch, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(ser, ctx->scratch, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    }
    if (want & ISING_OBS_HASH) {
        const int rc = ensure_canonical(ctx);
        if (rc != ISING_OK) return rc;
        const size_t N = (size_t)ctx->L * ctx->L;
        HIP_TRY(ctx, launch_to_canonical(ctx_planes(ctx), ctx->canon, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(bytes, ctx->canon, N, hipMemcpyDeviceToHost, ctx->stream));
    }
    return enqueue_band_check(ctx);
}

int ising_prefetch_observables(ising_ctx* ctx, uint32_t want) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (want & ~(ISING_OBS_HASH | ISING_OBS_SERIES)) return ISING_EINVAL;
    if (ctx->pre_state == 1) {
        // the stage is about to be rewritten: the earlier read-back must land first
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->pre_state = 0;
    const uint64_t len = ctx->series_len;
    const bool full = (want & ISING_OBS_SERIES) && len;
    const size_t ser_bytes = (full ? 2 * len : 2) * sizeof(int64_t);
    const size_t hash_off = (ser_bytes + 255) & ~(size_t)255;
    const size_t N = (size_t)ctx->L * ctx->L;
    uint8_t* stage = static_cast<uint8_t*>(ctx_host_stage(ctx, (want & ISING_OBS_HASH) ? hash_off + N : ser_bytes));
    if (!stage) return ISING_EUNSUPPORTED;
    rc = enqueue_readback(ctx, want, full, reinterpret_cast<int64_t*>(stage), stage + hash_off);
    if (rc != ISING_OK) return rc;
    ctx->pre_state = 1;
    ctx->pre_full = full;
    ctx->pre_want = want;
    ctx->pre_gen = ctx->gen;
    ctx->pre_hash_off = hash_off;
    return ISING_OK;
}

int ising_observables(ising_ctx* ctx, ising_obs* out, int64_t* bond_series, int64_t* mag_series,
                      uint64_t capacity, uint32_t want) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (want & ~(ISING_OBS_HASH | ISING_OBS_SERIES)) return ISING_EINVAL;
    const uint64_t len = ctx->series_len;
    if ((want & ISING_OBS_SERIES) && (bond_series || mag_series) && capacity < len) return ISING_ERANGE;
    const size_t N = (size_t)ctx->L * ctx->L;
    const bool copy_series = (want & ISING_OBS_SERIES) && len && (bond_series || mag_series);
    const bool hash = (want & ISING_OBS_HASH) != 0;
    std::vector<int64_t> ser_pageable;
    std::vector<uint8_t> bytes_pageable;
    int64_t* ser = nullptr;
    uint8_t* bytes = nullptr;
    bool full = copy_series;
    if (ctx->pre_state == 1) {
        // a prefetched read-back must land before the stage is read or reused
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        ctx->pre_state = 2;
    }
    if (ctx->pre_state == 2) {
        // it answers this call if nothing changed since and it holds
        // everything asked for (and keeps answering until something changes)
        if (ctx->pre_gen == ctx->gen && (want & ~ctx->pre_want) == 0 && (!copy_series || ctx->pre_full)) {
            uint8_t* stage = static_cast<uint8_t*>(ctx->host_stage);
            ser = reinterpret_cast<int64_t*>(stage);
            bytes = stage + ctx->pre_hash_off;
            full = ctx->pre_full;
        } else {
            ctx->pre_state = 0;
        }
    }
    if (!ser) {
        const size_t ser_bytes = (full ? 2 * len : 2) * sizeof(int64_t);
        const size_t hash_off = (ser_bytes + 255) & ~(size_t)255;
        // read back into the context's pinned stage when it fits, else into
        // pageable memory
        uint8_t* stage = static_cast<uint8_t*>(ctx_host_stage(ctx, hash ? hash_off + N : ser_bytes));
        if (!stage) {
            try {
                ser_pageable.resize(ser_bytes / sizeof(int64_t));
                if (hash) bytes_pageable.resize(N);
            } catch (...) {
                return ISING_ENOMEM;
            }
        }
        ser = stage ? reinterpret_cast<int64_t*>(stage) : ser_pageable.data();
        bytes = stage ? stage + hash_off : bytes_pageable.data();
        rc = enqueue_readback(ctx, want, full, ser, bytes);
        if (rc != ISING_OK) return rc;
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    rc = band_check(ctx);
    if (rc != ISING_OK) return rc;
    const uint64_t hsh = hash ? fnv1a64(bytes, N) : 0;
    const int64_t* last = full ? ser + 2 * (len - 1) : ser;
    const int64_t bm[2] = {last[0], last[1]};
    if (copy_series) {
        for (uint64_t k = 0; k < len; ++k) {
            if (bond_series) bond_series[k] = ser[2 * k];
            if (mag_series) mag_series[k] = ser[2 * k + 1];
        }
    }
    if (out) {
        const double N = (double)ctx->L * (double)ctx->L;
        out->sweeps_done = ctx->t;
        out->bond_sum = bm[0];
        out->mag_sum = bm[1];
        out->energy = -ctx->p.J * (double)bm[0] - ctx->p.h * (double)bm[1];
        out->e_per_site = out->energy / N;
        out->m_per_site = (double)bm[1] / N;
        out->lattice_hash = hsh;
        out->series_len = len;
    }
    if (want & ISING_OBS_SERIES) {
        ctx->series_len = 0;
        ++ctx->gen;
    }
    return ISING_OK;
}

int ising_series_averages(const int64_t* bond_series, const int64_t* mag_series, uint64_t n, uint32_t L,
                          double J, double h, ising_averages* out) {
    if (!bond_series || !mag_series || !out || n == 0 || L < 2) return ISING_EINVAL;
    const double N = (double)L * (double)L;
    double se = 0, se2 = 0, sm = 0, sam = 0, sm2 = 0;
    for (uint64_t k = 0; k < n; ++k) {
        const double e = (-J * (double)bond_series[k] - h * (double)mag_series[k]) / N;
        const double m = (double)mag_series[k] / N;
        se += e;
        se2 += e * e;
        sm += m;
        sam += std::fabs(m);
        sm2 += m * m;
    }
    const double dn = (double)n;
    out->n = n;
    out->e = se / dn;
    out->e2 = se2 / dn;
    out->m = sm / dn;
    out->abs_m = sam / dn;
    out->m2 = sm2 / dn;
    return ISING_OK;
}

int ising_plan_info(const ising_ctx* ctx, uint32_t* plan, uint32_t* chunk_words, uint32_t* rows_per_thread) {
    if (!ctx) return ISING_EINVAL;
    if (plan) *plan = ctx->plan.kind;
    if (chunk_words) *chunk_words = ctx->plan.cw;
    if (rows_per_thread) *rows_per_thread = ctx->plan.rows;
    return ISING_OK;
}

int ising_plan_set(ising_ctx* ctx, uint32_t plan, uint32_t cw, uint32_t rows) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (plan == ISING_PLAN_AUTO || plan > ISING_PLAN_BANDS) return ISING_EINVAL;
    Plan pl;
    if (!plan_for(ctx->L, plan, cw, rows, &pl)) return ISING_EUNSUPPORTED;
    ctx_drop_graphs(ctx);
    const Plan old = ctx->plan;
    ctx->plan = pl;
    rc = ctx_prepare_plan(ctx);
    if (rc != ISING_OK) ctx->plan = old;
    return rc;
}

int ising_tune(ising_ctx* ctx, uint32_t trial_sweeps) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (trial_sweeps == 0) return ISING_EINVAL;
    const uint32_t L = ctx->L;
    std::vector<Plan> cands;
    Plan pl;
    if (L % 8u != 0u) {
        plan_for(L, ISING_PLAN_GENERIC, 0, 0, &pl);
        cands.push_back(pl);
    } else {
        static const uint32_t cws[3] = {1, 2, 4};
        static const uint32_t rs[6] = {4, 8, 16, 32, 64, 128};
        for (uint32_t cw : cws)
            for (uint32_t r : rs)
                if (plan_for(L, ISING_PLAN_FUSED, cw, r, &pl)) cands.push_back(pl);
        for (uint32_t cw : cws)
            for (uint32_t r : rs)
                if (r >= 8 && plan_for(L, ISING_PLAN_FUSED_ROWS, cw, r, &pl)) cands.push_back(pl);
        for (uint32_t cw : cws)
            if (plan_for(L, ISING_PLAN_TWO_PASS, cw, 0, &pl)) cands.push_back(pl);
        if (L <= 1024 && plan_for(L, ISING_PLAN_RESIDENT, 0, 0, &pl)) cands.push_back(pl);
        const uint32_t brs[6] = {band_default_rows(L), 2, 4, 8, 16, 32};
        // one row a wave: two or four (fewer waves a SIMD) measured 12-80% slower
        for (uint32_t k = 0; k < 6; ++k) {
            if (k > 0 && brs[k] == brs[0]) continue;
            if (plan_for(L, ISING_PLAN_BANDS, 1, brs[k], &pl)) cands.push_back(pl);
        }
    }
    // scratch context over a copy of the lattice, same table and seed
    ising_params p = ctx->p;
    p.flags = ISING_PLAN_GENERIC;
    ising_ctx* tmp = nullptr;
    rc = ising_create(&p, ctx->stream, &tmp);
    if (rc != ISING_OK) return rc;
    const size_t N = (size_t)L * L;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best_ms = 0.f;
    Plan best = ctx->plan;
    bool have = false;
    // the default plan for this side is timed first and kept unless beaten
    Plan dflt;
    {
        std::lock_guard<std::mutex> g(g_tuned_mu);
        g_tuned.erase(L);  // the default is the untuned AUTO choice
    }
    if (plan_for(L, ISING_PLAN_AUTO, 0, 0, &dflt)) {
        for (size_t k = 0; k < cands.size(); ++k) {
            if (cands[k].kind == dflt.kind && cands[k].cw == dflt.cw && cands[k].rows == dflt.rows) {
                std::swap(cands[0], cands[k]);
                break;
            }
        }
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = ISING_EDEVICE;
    // kTuneRounds interleaved rounds over the candidates; each keeps its
    // fastest round, so a slow outlier (clock ramp, a neighbour's work)
    // does not decide the plan
    std::vector<float> fastest(cands.size(), 0.f);
    for (uint32_t round = 0; rc == ISING_OK && round < kTuneRounds; ++round) {
        for (size_t k = 0; rc == ISING_OK && k < cands.size(); ++k) {
            ctx_drop_graphs(tmp);  // graphs captured for the previous candidate
            tmp->plan = cands[k];
            rc = ctx_prepare_plan(tmp);
            if (rc != ISING_OK) break;
            if (hipMemcpyAsync(tmp->buf[tmp->cur], ctx->buf[ctx->cur], N, hipMemcpyDeviceToDevice, ctx->stream) !=
                hipSuccess) {
                rc = ISING_EDEVICE;
                break;
            }
            tmp->t = ctx->t;
            tmp->series_len = 0;
            // warm-up; a whole graph replay when the trial has one, so that
            // the timed sweeps do not include the capture
            rc = ising_sweep(tmp, trial_sweeps >= kGraphSweeps ? kGraphSweeps : 1);
            if (rc != ISING_OK) break;
            tmp->series_len = 0;
            if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = ISING_EDEVICE;
            if (rc == ISING_OK) rc = ising_sweep(tmp, trial_sweeps);
            if (rc == ISING_OK && hipEventRecord(e1, ctx->stream) != hipSuccess) rc = ISING_EDEVICE;
            if (rc == ISING_OK && hipEventSynchronize(e1) != hipSuccess) rc = ISING_EDEVICE;
            float ms = 0.f;
            if (rc == ISING_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = ISING_EDEVICE;
            if (rc != ISING_OK) break;
            tmp->series_len = 0;
            if (round == 0 || ms < fastest[k]) fastest[k] = ms;
        }
    }
    for (size_t k = 0; rc == ISING_OK && k < cands.size(); ++k) {
        if (!have || fastest[k] < best_ms * (1.0f - kTuneMargin)) {
            best_ms = fastest[k];
            best = cands[k];
            have = true;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ising_destroy(tmp);
    if (rc != ISING_OK) return rc == ISING_EDEVICE ? ctx_fail(ctx, hipErrorUnknown, "autotuner trial context") : rc;
    ctx_drop_graphs(ctx);
    const Plan old = ctx->plan;
    ctx->plan = best;
    rc = ctx_prepare_plan(ctx);
    if (rc != ISING_OK) {
        ctx->plan = old;
        return rc;
    }
    std::lock_guard<std::mutex> g(g_tuned_mu);
    g_tuned[L] = best;
    return ISING_OK;
}

int ising_creutz_init(ising_ctx* ctx, const uint8_t* host, size_t n, uint8_t fill) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    const size_t N = (size_t)ctx->L * ctx->L;
    if (host && n < N) return ISING_EINVAL;
    if (ctx->p.h != 0.0 || !(ctx->p.J > 0.0)) return ISING_EUNSUPPORTED;
    if (!ctx->demon) {
        if (hipMalloc(&ctx->demon, N) != hipSuccess) {
            (void)hipGetLastError();
            ctx->demon = nullptr;
            return ISING_ENOMEM;
        }
    }
    if (!ctx->cpart && ctx->L % 8u == 0u) {
        if (hipMalloc(&ctx->cpart, (size_t)creutz_blocks(ctx_planes(ctx)) * 2 * sizeof(int64_t)) != hipSuccess) {
            (void)hipGetLastError();
            ctx->cpart = nullptr;
            return ISING_ENOMEM;
        }
    }
    const Planes dm = planes_of(ctx->demon, ctx->L);
    if (host) {
        rc = ensure_canonical(ctx);
        if (rc != ISING_OK) return rc;
        HIP_TRY(ctx, hipMemcpyAsync(ctx->canon, host, N, hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(ctx, launch_bytes_from_canonical(dm, reinterpret_cast<const uint8_t*>(ctx->canon), ctx->stream));
    } else {
        HIP_TRY(ctx, launch_fill_u8(ctx->demon, N, fill, ctx->stream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ++ctx->gen;
    return ISING_OK;
}

// Buffers of the fused Creutz sweep: the second spin and demon buffers
// (ping-pong) and per-tile partials for the (cw, rows) tiling.
static int creutz_fused_prepare(ising_ctx* ctx, uint32_t cw, uint32_t rows) {
    const size_t N = (size_t)ctx->L * ctx->L;
    if (!ctx->buf[1]) {
        if (hipMalloc(&ctx->buf[1], N) != hipSuccess) {
            (void)hipGetLastError();
            ctx->buf[1] = nullptr;
            return ISING_ENOMEM;
        }
        ctx->owns_buf[1] = true;
    }
    if (!ctx->demon_alt) {
        if (hipMalloc(&ctx->demon_alt, N) != hipSuccess) {
            (void)hipGetLastError();
            ctx->demon_alt = nullptr;
            return ISING_ENOMEM;
        }
    }
    const uint32_t need = fused_tiles(ctx->L, cw, rows);
    if (need > ctx->cfpart_cap) {
        for (int k = 0; k < 2; ++k) {
            if (ctx->cfpart[k]) (void)hipFree(ctx->cfpart[k]);
            ctx->cfpart[k] = nullptr;
        }
        ctx->cfpart_cap = 0;
        for (int k = 0; k < 2; ++k) {
            if (hipMalloc(&ctx->cfpart[k], (size_t)need * 2 * sizeof(int64_t)) != hipSuccess) {
                (void)hipGetLastError();
                return ISING_ENOMEM;
            }
        }
        ctx->cfpart_cap = need;
    }
    return ISING_OK;
}

// n fused Creutz sweeps; series slots ser[0 .. 2n).
static int creutz_sweep_fused(ising_ctx* ctx, uint64_t n, uint32_t cw, uint32_t rows, int64_t* ser) {
    const uint32_t L = ctx->L, Hw = L / 8u;
    const uint32_t n_tx = Hw / (64u * cw);
    const uint32_t n_tiles = fused_tiles(L, cw, rows);
    for (uint64_t k = 0; k < n; ++k) {
        const Planes src = ctx_planes(ctx), dst = ctx_planes_alt(ctx);
        const Planes ds = planes_of(ctx->demon, L), dd = planes_of(ctx->demon_alt, L);
        CreutzFusedArgs a{reinterpret_cast<const uint32_t*>(src.p[0]), reinterpret_cast<const uint32_t*>(src.p[1]),
                          reinterpret_cast<const uint32_t*>(ds.p[0]), reinterpret_cast<const uint32_t*>(ds.p[1]),
                          reinterpret_cast<uint32_t*>(dst.p[0]), reinterpret_cast<uint32_t*>(dst.p[1]),
                          reinterpret_cast<uint32_t*>(dd.p[0]), reinterpret_cast<uint32_t*>(dd.p[1]),
                          L, Hw, n_tx, n_tiles, ctx->cfpart[k & 1]};
        PartialReduce red{nullptr, 0, nullptr};
        if (k > 0) red = PartialReduce{ctx->cfpart[(k - 1) & 1], n_tiles, ser + 2 * (k - 1)};
        HIP_TRY(ctx, launch_creutz_fused(a, cw, rows, red, ctx->stream));
        ctx->cur ^= 1;
        std::swap(ctx->demon, ctx->demon_alt);
    }
    HIP_TRY(ctx, launch_reduce_partials(PartialReduce{ctx->cfpart[(n - 1) & 1], n_tiles, ser + 2 * (n - 1)},
                                        ctx->stream));
    return ISING_OK;
}

int ising_creutz_sweep(ising_ctx* ctx, uint64_t n, int reverse) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (!ctx->demon) return ISING_ESTATE;
    if (n == 0) return ISING_OK;
    rc = ctx_reserve_series(ctx, n);
    if (rc != ISING_OK) return rc;
    ++ctx->gen;
    int64_t* ser = ctx->series + 2 * ctx->series_len;
    uint32_t cw = 0, rows = 0;
    if (!reverse && ctx->L % 8u == 0u && default_fused(ctx->L, &cw, &rows)) {
        rc = creutz_fused_prepare(ctx, cw, rows);
        if (rc != ISING_OK) return rc;
        rc = creutz_sweep_fused(ctx, n, cw, rows, ser);
        if (rc != ISING_OK) return rc;
        ctx->series_len += n;
        return ISING_OK;
    }
    const Planes pl = ctx_planes(ctx), dm = planes_of(ctx->demon, ctx->L);
    if (ctx->L % 8u == 0u) {
        const uint32_t nb = creutz_blocks(pl);
        for (uint64_t k = 0; k < n; ++k) {
            PartialReduce red{nullptr, 0, nullptr};
            if (k > 0) red = PartialReduce{ctx->cpart, nb, ser + 2 * (k - 1)};
            HIP_TRY(ctx, launch_creutz_sweep(pl, dm, reverse != 0, ctx->cpart, red, ctx->stream));
        }
        HIP_TRY(ctx, launch_reduce_partials(PartialReduce{ctx->cpart, nb, ser + 2 * (n - 1)}, ctx->stream));
    } else {
        for (uint64_t k = 0; k < n; ++k) {
            HIP_TRY(ctx, launch_creutz_sweep_sites(pl, dm, reverse != 0, ctx->stream));
            HIP_TRY(ctx, launch_observe(pl, ser + 2 * k, ctx->stream));
        }
    }
    ctx->series_len += n;
    return ISING_OK;
}

int ising_demon_sum(ising_ctx* ctx, int64_t* out) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    if (!out) return ISING_EINVAL;
    if (!ctx->demon) return ISING_ESTATE;
    HIP_TRY(ctx, launch_demon_sum(ctx->demon, (uint64_t)ctx->L * ctx->L, ctx->scratch + 2, ctx->stream));
    int64_t v = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&v, ctx->scratch + 2, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    *out = v;
    return ISING_OK;
}

int ising_copy_demons(ising_ctx* ctx, uint8_t* host, size_t n) {
    int rc = ctx_enter(ctx);
    if (rc != ISING_OK) return rc;
    const size_t N = (size_t)ctx->L * ctx->L;
    if (!host || n < N) return ISING_EINVAL;
    if (!ctx->demon) return ISING_ESTATE;
    rc = ensure_canonical(ctx);
    if (rc != ISING_OK) return rc;
    HIP_TRY(ctx, launch_bytes_to_canonical(planes_of(ctx->demon, ctx->L), reinterpret_cast<uint8_t*>(ctx->canon),
                                           ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(host, ctx->canon, N, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return ISING_OK;
}

int ising_destroy(ising_ctx* ctx) {
    if (!ctx) return ISING_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    ctx_drop_graphs(ctx);
    if (ctx->ghdr) (void)hipFree(ctx->ghdr);
    if (ctx->gpart) (void)hipFree(ctx->gpart);
    for (int k = 0; k < 2; ++k) {
        if (ctx->owns_buf[k] && ctx->buf[k]) (void)hipFree(ctx->buf[k]);
        if (ctx->part[k]) (void)hipFree(ctx->part[k]);
    }
    if (ctx->series) (void)hipFree(ctx->series);
    if (ctx->demon) (void)hipFree(ctx->demon);
    if (ctx->demon_alt) (void)hipFree(ctx->demon_alt);
    if (ctx->cpart) (void)hipFree(ctx->cpart);
    if (ctx->band_pub) (void)hipFree(ctx->band_pub);
    if (ctx->band_part) (void)hipFree(ctx->band_part);
    if (ctx->band_err) (void)hipFree(ctx->band_err);
    if (ctx->band_err_host) (void)hipHostFree(ctx->band_err_host);
    for (int k = 0; k < 2; ++k)
        if (ctx->cfpart[k]) (void)hipFree(ctx->cfpart[k]);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->canon) (void)hipFree(ctx->canon);
    if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
    if (ctx->owns_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    (void)hipGetLastError();
    delete ctx;
    return ISING_OK;
}

const char* ising_device_error(const ising_ctx* ctx) {
    return ctx ? ctx->device_error : "";
}

const char* ising_strerror(int code) {
    switch (code) {
        case ISING_OK: return "ok";
        case ISING_EINVAL: return "invalid argument";
        case ISING_ENOMEM: return "out of memory";
        case ISING_EDEVICE: return "HIP device error";
        case ISING_ERANGE: return "out of range";
        case ISING_EUNSUPPORTED: return "unsupported by this library";
        case ISING_ESTATE: return "context poisoned by an earlier device error";
        case ISING_EIO: return "file could not be written";
        default: return "unknown error";
    }
}

}  // extern "C"
