// C ABI of the percolation engine (include/percolation.h): contexts, device
// buffers, and the host loop that relaunches the tile relaxation until no
// tile of any medium of the run is queued.
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
    uint32_t* queued[2] = {nullptr, nullptr};
    uint32_t* resume = nullptr;
    Stats* stats = nullptr;
    Medium md{};              // this medium's descriptor (host copy)
    Medium* d_md = nullptr;   // ... and on the device, for runs of this medium alone
    WorkLists w{};            // work lists for runs of this medium alone
    uint32_t* h_len = nullptr;  // pinned: queued-entry count polled between launch groups
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

#define PERC_TRY(c, expr)                         \
    do {                                          \
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

uint32_t relax_grid(uint64_t tiles, int device) {
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    return (uint32_t)std::min<uint64_t>(tiles, (uint64_t)cus * 16u);  // one-wave workgroups
}

// Draw and invade the media ctxs[0..count) on stream s, with work lists w
// (capacity: their tiles together), the device media table d_media and a
// relaxation grid of `grid` workgroups. Synchronises s. Errors poison
// ctxs[0].
int run_media(perc_ctx* const* ctxs, size_t count, hipStream_t s, const WorkLists& w, const Medium* d_media,
              uint32_t grid, uint32_t* h_len) {
    perc_ctx* c0 = ctxs[0];
    for (size_t m = 0; m < count; ++m) {
        perc_ctx* c = ctxs[m];
        const perc_params& p = c->p;
        const uint64_t pthr = (uint64_t)std::floor(p.porosity * 4294967296.0);
        c->ran = false;
        PERC_TRY(c0, hipMemsetAsync(c->stats, 0, sizeof(Stats), s));
        PERC_TRY(c0, hipMemsetAsync(c->queued[0], 0, (size_t)c->n_tiles * 4, s));
        PERC_TRY(c0, hipMemsetAsync(c->queued[1], 0, (size_t)c->n_tiles * 4, s));
        PERC_TRY(c0, hipMemsetAsync(c->resume, 0xff, (size_t)c->n_tiles * 4, s));
        PERC_TRY(c0, launch_draw(c->pore, c->arr, p.L, pthr, (uint32_t)p.seed, (uint32_t)(p.seed >> 32), p.source,
                                 p.i0, p.j0, c->stats, s));
    }
    PERC_TRY(c0, launch_reset_lists(w, s));
    for (size_t m = 0; m < count; ++m) {
        const perc_params& p = ctxs[m]->p;
        PERC_TRY(c0, launch_seed(w, d_media, (uint32_t)m, ctxs[m]->n_tx, p.source, p.i0, p.j0, s));
    }
    uint64_t k = 0;
    for (;;) {
        for (uint32_t g = 0; g < kLaunchGroup; ++g, ++k) PERC_TRY(c0, launch_relax(d_media, w, k, grid, s));
        // entries queued for launch k (its input list length)
        PERC_TRY(c0, hipMemcpyAsync(h_len, w.len + (k % 3), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        PERC_TRY(c0, hipStreamSynchronize(s));
        if (*h_len == 0) break;
        if (k >= kMaxLaunches) return ISING_ERANGE;
    }
    for (size_t m = 0; m < count; ++m) PERC_TRY(c0, launch_finish(ctxs[m]->arr, ctxs[m]->p.L, ctxs[m]->stats, s));
    PERC_TRY(c0, hipStreamSynchronize(s));
    for (size_t m = 0; m < count; ++m) {
        ctxs[m]->launches = (uint32_t)std::min<uint64_t>(k, 0xffffffffu);
        ctxs[m]->ran = true;
    }
    return ISING_OK;
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
    c->grid = relax_grid(c->n_tiles, c->device);
    bool ok = dev_alloc(&c->pore, c->N) && dev_alloc(&c->arr, c->N * sizeof(uint32_t)) &&
              dev_alloc(&c->queued[0], (size_t)c->n_tiles * 4) && dev_alloc(&c->queued[1], (size_t)c->n_tiles * 4) &&
              dev_alloc(&c->resume, (size_t)c->n_tiles * 4) &&
              dev_alloc(&c->stats, sizeof(Stats)) && dev_alloc(&c->d_md, sizeof(Medium)) &&
              dev_alloc(&c->w.list[0], (size_t)c->n_tiles * sizeof(uint2)) &&
              dev_alloc(&c->w.list[1], (size_t)c->n_tiles * sizeof(uint2)) &&
              dev_alloc(&c->w.len, 3 * sizeof(uint32_t));
    if (ok && hipHostMalloc((void**)&c->h_len, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->h_len = nullptr;
        ok = false;
    }
    if (ok) {
        c->md = Medium{c->arr, {c->queued[0], c->queued[1]}, c->resume, c->stats, L, c->n_tx, c->n_ty, 0u};
        ok = hipMemcpy(c->d_md, &c->md, sizeof(Medium), hipMemcpyHostToDevice) == hipSuccess;
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
    return run_media(&c, 1, c->stream, c->w, c->d_md, c->grid, c->h_len);
}

int perc_run_batch(perc_ctx* const* ctxs, size_t count) {
    if (!ctxs) return ISING_EINVAL;
    if (count == 0) return ISING_OK;
    uint64_t tiles = 0;
    for (size_t m = 0; m < count; ++m) {
        if (!ctxs[m]) return ISING_EINVAL;
        if (ctxs[m]->poisoned) return ISING_ESTATE;
        if (ctxs[m]->device != ctxs[0]->device) return ISING_EINVAL;
        for (size_t j = 0; j < m; ++j)
            if (ctxs[j] == ctxs[m]) return ISING_EINVAL;  // one context may appear once
        tiles += ctxs[m]->n_tiles;
    }
    if (tiles > 0xffffffffu) return ISING_ERANGE;
    perc_ctx* c0 = ctxs[0];
    int rc = enter(c0);
    if (rc != ISING_OK) return rc;
    hipStream_t s = c0->stream;
    // the run starts after each medium's earlier work on its own stream
    for (size_t m = 1; m < count; ++m)
        if (ctxs[m]->stream != s) PERC_TRY(c0, hipStreamSynchronize(ctxs[m]->stream));
    std::vector<Medium> table(count);
    for (size_t m = 0; m < count; ++m) table[m] = ctxs[m]->md;
    Medium* d_table = nullptr;
    WorkLists w{};
    bool ok = dev_alloc(&d_table, count * sizeof(Medium)) && dev_alloc(&w.list[0], tiles * sizeof(uint2)) &&
              dev_alloc(&w.list[1], tiles * sizeof(uint2)) && dev_alloc(&w.len, 3 * sizeof(uint32_t));
    if (ok) {
        ok = hipMemcpyAsync(d_table, table.data(), count * sizeof(Medium), hipMemcpyHostToDevice, s) == hipSuccess;
        if (!ok) rc = fail(c0);
    } else {
        rc = ISING_ENOMEM;
    }
    if (ok) rc = run_media(ctxs, count, s, w, d_table, relax_grid(tiles, c0->device), c0->h_len);
    (void)hipStreamSynchronize(s);
    (void)hipFree(d_table);
    (void)hipFree(w.list[0]);
    (void)hipFree(w.list[1]);
    (void)hipFree(w.len);
    (void)hipGetLastError();
    return rc;
}

int perc_set_params(perc_ctx* c, const perc_params* params) {
    if (!c) return ISING_EINVAL;
    if (c->poisoned) return ISING_ESTATE;
    if (!valid(params) || params->L != c->p.L) return ISING_EINVAL;
    c->p = *params;
    c->ran = false;
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
        (void)hipFree(c->queued[k]);
    }
    (void)hipFree(c->resume);
    (void)hipFree(c->w.len);
    (void)hipFree(c->stats);
    (void)hipFree(c->d_md);
    if (c->h_len) (void)hipHostFree(c->h_len);
    if (c->owns_stream && c->stream) (void)hipStreamDestroy(c->stream);
    (void)hipGetLastError();
    delete c;
    return ISING_OK;
}

}  // extern "C"
