// C ABI of the percolation engine (include/percolation.h): context,
// device buffers, and the host loop that relaunches the tile relaxation
// until no tile is queued.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "perc_launch.hpp"
#include "percolation.h"

using namespace perc;

struct perc_ctx {
    perc_params p{};
    uint64_t N = 0;
    uint32_t n_tx = 0, n_ty = 0, n_tiles = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    uint8_t* pore = nullptr;
    uint32_t* arr = nullptr;
    WorkLists w{};
    Stats* stats = nullptr;
    uint32_t* h_len = nullptr;  // pinned: queued-tile count polled between launch groups
    uint32_t grid = 0;
    uint32_t launches = 0;
    bool ran = false;
    bool poisoned = false;
};

namespace {

constexpr uint32_t kLaunchGroup = 8;           // relaxation launches between polls
constexpr uint64_t kMaxLaunches = 1ull << 26;  // far beyond any medium: a guard, not a limit

bool valid(const perc_params* p) {
    if (!p || p->L < 1 || p->L > 65536u) return false;
    if (!(p->porosity >= 0.0 && p->porosity <= 1.0)) return false;
    if (p->source > PERC_SOURCE_POINT) return false;
    if (p->source == PERC_SOURCE_POINT && (p->i0 >= p->L || p->j0 >= p->L)) return false;
    return true;
}

int fail(perc_ctx* c) {
    c->poisoned = true;
    (void)hipGetLastError();
    return ISING_EDEVICE;
}

#define PERC_TRY(c, expr)                     \
    do {                                      \
        if ((expr) != hipSuccess) return fail(c); \
    } while (0)

int enter(perc_ctx* c) {
    if (!c) return ISING_EINVAL;
    if (c->poisoned) return ISING_ESTATE;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c);
    return ISING_OK;
}

template <typename T>
bool dev_alloc(T** p, size_t bytes) {
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    return true;
}

uint64_t fnv1a64(const uint8_t* p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t k = 0; k < n; ++k) {
        h ^= p[k];
        h *= 0x100000001b3ull;
    }
    return h;
}

}  // namespace

extern "C" {

int perc_create(const perc_params* params, void* stream, perc_ctx** out) {
    if (!out) return ISING_EINVAL;
    *out = nullptr;
    if (!valid(params)) return ISING_EINVAL;
    perc_ctx* c = new (std::nothrow) perc_ctx();
    if (!c) return ISING_ENOMEM;
    c->p = *params;
    const uint32_t L = params->L;
    c->N = (uint64_t)L * L;
    c->n_tx = (L + kTile - 1) / kTile;
    c->n_ty = c->n_tx;
    c->n_tiles = c->n_tx * c->n_ty;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return ISING_EDEVICE;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return ISING_EDEVICE;
        }
        c->owns_stream = true;
    }
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    c->grid = std::min<uint32_t>(c->n_tiles, (uint32_t)cus * 8u);
    bool ok = dev_alloc(&c->pore, c->N) && dev_alloc(&c->arr, c->N * sizeof(uint32_t)) &&
              dev_alloc(&c->w.list[0], (size_t)c->n_tiles * 4) && dev_alloc(&c->w.list[1], (size_t)c->n_tiles * 4) &&
              dev_alloc(&c->w.queued[0], (size_t)c->n_tiles * 4) &&
              dev_alloc(&c->w.queued[1], (size_t)c->n_tiles * 4) && dev_alloc(&c->w.len, 3 * sizeof(uint32_t)) &&
              dev_alloc(&c->stats, sizeof(Stats));
    if (ok && hipHostMalloc((void**)&c->h_len, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->h_len = nullptr;
        ok = false;
    }
    if (!ok) {
        perc_destroy(c);
        return ISING_ENOMEM;
    }
    *out = c;
    return ISING_OK;
}

int perc_run(perc_ctx* c) {
    int rc = enter(c);
    if (rc != ISING_OK) return rc;
    const perc_params& p = c->p;
    const uint64_t pthr = (uint64_t)std::floor(p.porosity * 4294967296.0);
    c->ran = false;
    PERC_TRY(c, hipMemsetAsync(c->stats, 0, sizeof(Stats), c->stream));
    PERC_TRY(c, hipMemsetAsync(c->w.queued[0], 0, (size_t)c->n_tiles * 4, c->stream));
    PERC_TRY(c, hipMemsetAsync(c->w.queued[1], 0, (size_t)c->n_tiles * 4, c->stream));
    PERC_TRY(c, launch_draw(c->pore, c->arr, p.L, pthr, (uint32_t)p.seed, (uint32_t)(p.seed >> 32), p.source, p.i0,
                            p.j0, c->stats, c->stream));
    PERC_TRY(c, launch_seed_lists(c->w, c->n_tx, c->n_tiles, p.source, p.i0, p.j0, c->stream));
    uint64_t k = 0;
    for (;;) {
        for (uint32_t g = 0; g < kLaunchGroup; ++g, ++k)
            PERC_TRY(c, launch_relax(c->arr, p.L, c->n_tx, c->n_ty, c->w, k, c->grid, c->stats, c->stream));
        // tiles queued for launch k (its input list length)
        PERC_TRY(c, hipMemcpyAsync(c->h_len, c->w.len + (k % 3), sizeof(uint32_t), hipMemcpyDeviceToHost,
                                   c->stream));
        PERC_TRY(c, hipStreamSynchronize(c->stream));
        if (*c->h_len == 0) break;
        if (k >= kMaxLaunches) return ISING_ERANGE;
    }
    PERC_TRY(c, launch_finish(c->arr, p.L, c->stats, c->stream));
    PERC_TRY(c, hipStreamSynchronize(c->stream));
    c->launches = (uint32_t)std::min<uint64_t>(k, 0xffffffffu);
    c->ran = true;
    return ISING_OK;
}

int perc_copy_medium(perc_ctx* c, uint8_t* host, size_t n) {
    int rc = enter(c);
    if (rc != ISING_OK) return rc;
    if (!host || n < c->N) return ISING_EINVAL;
    if (!c->ran) return ISING_ESTATE;
    PERC_TRY(c, hipMemcpyAsync(host, c->pore, c->N, hipMemcpyDeviceToHost, c->stream));
    PERC_TRY(c, hipStreamSynchronize(c->stream));
    return ISING_OK;
}

int perc_copy_arrival(perc_ctx* c, int32_t* host, size_t n) {
    int rc = enter(c);
    if (rc != ISING_OK) return rc;
    if (!host || n < c->N) return ISING_EINVAL;
    if (!c->ran) return ISING_ESTATE;
    PERC_TRY(c, hipMemcpyAsync(host, c->arr, c->N * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    PERC_TRY(c, hipStreamSynchronize(c->stream));
    return ISING_OK;
}

int perc_result_get(perc_ctx* c, perc_result* out, uint32_t want_hash) {
    int rc = enter(c);
    if (rc != ISING_OK) return rc;
    if (!out) return ISING_EINVAL;
    if (!c->ran) return ISING_ESTATE;
    Stats st{};
    PERC_TRY(c, hipMemcpyAsync(&st, c->stats, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    PERC_TRY(c, hipStreamSynchronize(c->stream));
    perc_result r{};
    r.pores = st.pores;
    r.invaded = st.invaded;
    r.passes = (int32_t)st.max_arrival;
    r.spans = ((st.edges & 3u) == 3u ? 1u : 0u) | ((st.edges & 12u) == 12u ? 2u : 0u);
    r.launches = c->launches;
    r.tile_visits = st.visits;
    r.tile_iterations = st.iterations;
    if (want_hash) {
        std::vector<int32_t> a;
        try {
            a.resize(c->N);
        } catch (...) {
            return ISING_ENOMEM;
        }
        rc = perc_copy_arrival(c, a.data(), a.size());
        if (rc != ISING_OK) return rc;
        r.arrival_hash = fnv1a64(reinterpret_cast<const uint8_t*>(a.data()), a.size() * sizeof(int32_t));
    }
    *out = r;
    return ISING_OK;
}

int perc_destroy(perc_ctx* c) {
    if (!c) return ISING_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->pore);
    (void)hipFree(c->arr);
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(c->w.list[k]);
        (void)hipFree(c->w.queued[k]);
    }
    (void)hipFree(c->w.len);
    (void)hipFree(c->stats);
    if (c->h_len) (void)hipHostFree(c->h_len);
    if (c->owns_stream && c->stream) (void)hipStreamDestroy(c->stream);
    (void)hipGetLastError();
    delete c;
    return ISING_OK;
}

}  // extern "C"
