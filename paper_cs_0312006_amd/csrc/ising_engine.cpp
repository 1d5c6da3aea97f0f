// Batch engine: runs many contexts' sweeps as one persistent, workgroup-
// resident launch (ising_batch.hip), or as stepped sweeps over the tiles of
// every lattice (ising_multi_fused.hip, ising_multi.hip), replayed from
// captured hipGraphs.
//
// Per device the engine owns one staging block (headers, queue order, tile
// starts and lattice descriptors) on the device with a pinned host mirror,
// the stepped plans' per-tile partials, and its own launch stream. A call
// fills the mirror, copies it to the device with one copy kernel on the
// launch stream, and replays the plan's graph, whose kernels read the
// block; the graphs are captured once per buffer generation. The launch is
// ordered after every context's earlier work (an event per context whose
// stream saw other work since the engine last ordered it) and every
// context's later work after the launch (one event, waited on per stream).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "ising.h"
#include "ising_launch.hpp"
#include "ising_runtime.hpp"

using namespace ising;

namespace {

struct Engine {
    std::mutex mu;
    bool ready = false;
    size_t cap = 0;
    uint8_t* d_stage = nullptr;  // staging block on the device and its pinned host mirror
    uint8_t* h_stage = nullptr;
    size_t off_items = 0;
    BatchItem* d_items = nullptr;
    uint32_t* d_order = nullptr;
    BatchHeader* d_hdr = nullptr;
    BatchItem* h_items = nullptr;
    uint32_t* h_order = nullptr;
    BatchHeader* h_hdr = nullptr;
    hipEvent_t staged = nullptr;  // completion of the last staging copies, on the launch stream
    hipEvent_t order_ev = nullptr;
    hipEvent_t done = nullptr;    // completion of the last launch, on the launch stream
    // The launch stream may be a context's stream that is destroyed before
    // the next call, and an event is only waited on from later calls after
    // being relayed to the engine's own stream, which lives as long as the
    // process: these two are the relayed copies.
    hipStream_t relay = nullptr;
    hipEvent_t staged_relay = nullptr;
    hipEvent_t done_relay = nullptr;
    bool staged_pending = false;
    bool launched = false;
    hipStream_t last_stream = nullptr;  // stream of the last launch (meaningful while launched)
    hipStream_t launch = nullptr;  // the engine's own launch stream (calls that name none), never destroyed
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t grid = 0;
    // stepped plan
    uint32_t* d_vbs = nullptr;
    uint32_t* h_vbs = nullptr;
    MultiHeader* d_mhdr = nullptr;
    MultiHeader* h_mhdr = nullptr;
    hipGraph_t mgraph = nullptr;
    hipGraphExec_t mexec = nullptr;
    uint32_t mgrid = 0;
    // stepped plan, fused walk (sides multiple of 16)
    hipGraph_t fgraph = nullptr;
    hipGraphExec_t fexec = nullptr;
    uint32_t fslots = 0;  // waves of the fused walk resident on the GPU at once
    uint32_t fgrid = 0;   // workgroups per launch of the fused walk
    int64_t* d_part = nullptr;  // (B, M) of every tile / virtual block for each sweep of a replay
    size_t part_bytes = 0;
};

constexpr uint32_t kSweepsPerReplay = 16;

constexpr int kMaxDevices = 64;
Engine g_engines[kMaxDevices];

void release_buffers(Engine& e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
    if (e.mexec) (void)hipGraphExecDestroy(e.mexec);
    if (e.mgraph) (void)hipGraphDestroy(e.mgraph);
    e.mexec = nullptr;
    e.mgraph = nullptr;
    if (e.fexec) (void)hipGraphExecDestroy(e.fexec);
    if (e.fgraph) (void)hipGraphDestroy(e.fgraph);
    e.fexec = nullptr;
    e.fgraph = nullptr;
    if (e.d_stage) (void)hipFree(e.d_stage);
    if (e.h_stage) (void)hipHostFree(e.h_stage);
    e.d_stage = nullptr;
    e.h_stage = nullptr;
    e.d_items = nullptr;
    e.d_order = nullptr;
    e.d_hdr = nullptr;
    e.h_items = nullptr;
    e.h_order = nullptr;
    e.h_hdr = nullptr;
    e.d_vbs = nullptr;
    e.h_vbs = nullptr;
    e.d_mhdr = nullptr;
    e.h_mhdr = nullptr;
    e.cap = 0;
}

hipError_t ensure_capacity(Engine& e, size_t count) {
    if (count <= e.cap) return hipSuccess;
    if (e.staged_pending) {
        hipError_t r = hipEventSynchronize(e.staged_relay);
        if (r != hipSuccess) return r;
        e.staged_pending = false;
    }
    // the previous graph may still be running on some stream: drain
    hipError_t r = hipDeviceSynchronize();
    if (r != hipSuccess) return r;
    release_buffers(e);
    size_t cap = 256;
    while (cap < count) cap *= 2;
    // one staging block, [hdr | mhdr | order | vbs | items], so that a call
    // stages its descriptors with a single copy
    static_assert(sizeof(BatchHeader) <= 32 && sizeof(MultiHeader) <= 32, "staging block headers");
    const size_t off_order = 64;
    const size_t off_vbs = off_order + cap * sizeof(uint32_t);
    const size_t off_items = (off_vbs + (cap + 1) * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t bytes = off_items + cap * sizeof(BatchItem);
    if ((r = hipMalloc(&e.d_stage, bytes)) != hipSuccess) return r;
    if ((r = hipHostMalloc(&e.h_stage, bytes, hipHostMallocDefault)) != hipSuccess) return r;
    e.off_items = off_items;
    e.d_hdr = reinterpret_cast<BatchHeader*>(e.d_stage);
    e.d_mhdr = reinterpret_cast<MultiHeader*>(e.d_stage + 32);
    e.d_order = reinterpret_cast<uint32_t*>(e.d_stage + off_order);
    e.d_vbs = reinterpret_cast<uint32_t*>(e.d_stage + off_vbs);
    e.d_items = reinterpret_cast<BatchItem*>(e.d_stage + off_items);
    e.h_hdr = reinterpret_cast<BatchHeader*>(e.h_stage);
    e.h_mhdr = reinterpret_cast<MultiHeader*>(e.h_stage + 32);
    e.h_order = reinterpret_cast<uint32_t*>(e.h_stage + off_order);
    e.h_vbs = reinterpret_cast<uint32_t*>(e.h_stage + off_vbs);
    e.h_items = reinterpret_cast<BatchItem*>(e.h_stage + off_items);
    e.cap = cap;
    return hipSuccess;
}

hipError_t init_engine(Engine& e) {
    if (e.ready) return hipSuccess;
    hipError_t r = hipEventCreateWithFlags(&e.staged, hipEventDisableTiming);
    if (r != hipSuccess) return r;
    r = hipEventCreateWithFlags(&e.order_ev, hipEventDisableTiming);
    if (r != hipSuccess) return r;
    r = hipEventCreateWithFlags(&e.done, hipEventDisableTiming);
    if (r != hipSuccess) return r;
    r = hipEventCreateWithFlags(&e.staged_relay, hipEventDisableTiming);
    if (r != hipSuccess) return r;
    r = hipEventCreateWithFlags(&e.done_relay, hipEventDisableTiming);
    if (r != hipSuccess) return r;
    r = hipStreamCreateWithFlags(&e.relay, hipStreamNonBlocking);
    if (r != hipSuccess) return r;
    r = hipStreamCreateWithFlags(&e.launch, hipStreamNonBlocking);
    if (r != hipSuccess) return r;
    int dev = 0;
    hipDeviceProp_t prop;
    if ((r = hipGetDevice(&dev)) != hipSuccess) return r;
    if ((r = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return r;
    int per_cu = 0;
    if ((r = batch_occupancy(&per_cu)) != hipSuccess) return r;
    if (per_cu < 1) per_cu = 1;
    e.grid = (uint32_t)prop.multiProcessorCount * (uint32_t)per_cu;
    e.mgrid = (uint32_t)prop.multiProcessorCount * 8u;
    e.fslots = multi_fused_wave_slots((uint32_t)prop.multiProcessorCount);
    // the fused walk's launches: four times the workgroups the GPU holds at
    // once (as many workgroups as it holds waves), so that most workgroups
    // start as others finish and take about one tile per wave, rather than
    // each resident wave striding over a fixed share of tiles that differ
    // in height and width
    e.fgrid = e.fslots;
    e.ready = true;
    return hipSuccess;
}

// Capture the single persistent launch into a graph (once per buffer set).
hipError_t ensure_graph(Engine& e, hipStream_t s) {
    if (e.exec) return hipSuccess;
    hipStream_t cap = nullptr;
    hipError_t r = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (r != hipSuccess) return r;
    r = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (r == hipSuccess) {
        hipError_t lr = launch_batch(e.d_items, e.d_order, e.d_hdr, e.grid, cap);
        r = hipStreamEndCapture(cap, &e.graph);
        if (lr != hipSuccess) r = lr;
    }
    if (r == hipSuccess) r = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    (void)s;
    return r;
}

// Capture G sweeps of the stepped plan (one advance node, 2 G passes, one
// reduce of the block partials into the series).
hipError_t ensure_multi_graph(Engine& e) {
    if (e.mexec) return hipSuccess;
    hipStream_t cap = nullptr;
    hipError_t r = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (r != hipSuccess) return r;
    r = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (r == hipSuccess) {
        hipError_t lr = launch_multi_graph_body(e.d_items, e.d_vbs, e.d_mhdr, kSweepsPerReplay, e.mgrid, cap);
        r = hipStreamEndCapture(cap, &e.mgraph);
        if (lr != hipSuccess) r = lr;
    }
    if (r == hipSuccess) r = hipGraphInstantiate(&e.mexec, e.mgraph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    return r;
}

// Room for the stepped plans' partials: G sweeps x `tiles` (B, M) pairs
// (one per tile of the fused walk or virtual block of the two-pass walk).
// The buffer only grows; growing waits for the device, since a queued
// replay may still write the old one.
hipError_t ensure_partials(Engine& e, uint64_t tiles) {
    const size_t need = (size_t)kSweepsPerReplay * tiles * 2 * sizeof(int64_t);
    if (need <= e.part_bytes) return hipSuccess;
    hipError_t r = hipDeviceSynchronize();
    if (r != hipSuccess) return r;
    e.staged_pending = false;
    if (e.d_part) (void)hipFree(e.d_part);
    e.d_part = nullptr;
    e.part_bytes = 0;
    size_t cap = (size_t)1 << 20;
    while (cap < need) cap *= 2;
    if ((r = hipMalloc(&e.d_part, cap)) != hipSuccess) return r;
    e.part_bytes = cap;
    return hipSuccess;
}

// Capture G sweeps of the stepped plan's fused walk (one advance node, G
// launches, one reduce of the tile partials into the series).
hipError_t ensure_fused_graph(Engine& e) {
    if (e.fexec) return hipSuccess;
    hipStream_t cap = nullptr;
    hipError_t r = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (r != hipSuccess) return r;
    r = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (r == hipSuccess) {
        hipError_t lr = launch_multi_fused_graph_body(e.d_items, e.d_vbs, e.d_mhdr, kSweepsPerReplay, e.fgrid, cap);
        r = hipStreamEndCapture(cap, &e.fgraph);
        if (lr != hipSuccess) r = lr;
    }
    if (r == hipSuccess) r = hipGraphInstantiate(&e.fexec, e.fgraph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    return r;
}

}  // namespace

uint32_t engine_resident_slots(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return 0;
    Engine& e = g_engines[dev];
    std::lock_guard<std::mutex> g(e.mu);
    if (init_engine(e) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return e.grid;
}

uint32_t engine_fused_slots(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return 0;
    Engine& e = g_engines[dev];
    std::lock_guard<std::mutex> g(e.mu);
    if (init_engine(e) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return e.fslots;
}

void fill_batch_item(const ising_ctx* c, uint64_t n, bool stepped, BatchItem& it) {
    const Planes pl = ctx_planes(c);
    it.p0 = reinterpret_cast<uint32_t*>(pl.p[0]);
    it.p1 = reinterpret_cast<uint32_t*>(pl.p[1]);
    it.q0 = nullptr;
    it.q1 = nullptr;
    it.series = c->series + 2 * c->series_len;
    it.L = c->L;
    it.Hw = c->L / 8u;
    it.cw = (it.Hw % 4u == 0u) ? 4u : (it.Hw % 2u == 0u) ? 2u : 1u;
    // a lattice too small to give every thread of the resident workgroup a
    // chunk uses one word per thread (latency, not width)
    if (!stepped && (uint64_t)it.L * it.Hw <= 2ull * batch_block_threads()) it.cw = 1u;
    it.t0 = (uint32_t)c->t;
    it.n = (uint32_t)n;
    it.k0 = (uint32_t)c->p.seed;
    it.k1 = (uint32_t)(c->p.seed >> 32);
    it.exact = c->exact ? 1u : 0u;
    it.bits = 0u;
    it.pad = 0;
    it.table = c->table;
}

int engine_run(ising_ctx* const* ctxs, const uint64_t* n, size_t count, hipStream_t s, bool stepped,
               uint32_t rows_wanted) {
    int dev = ctxs[0]->device;
    if (dev < 0 || dev >= kMaxDevices) return ISING_EINVAL;
    // series room first (may synchronise the contexts' streams)
    for (size_t k = 0; k < count; ++k) {
        if (n[k] == 0) continue;
        int rc = ctx_reserve_series(ctxs[k], n[k]);
        if (rc != ISING_OK) return rc;
    }
    Engine& e = g_engines[dev];
    std::lock_guard<std::mutex> g(e.mu);
    hipError_t r = init_engine(e);
    if (r == hipSuccess && !s) s = e.launch;
    if (r == hipSuccess) r = ensure_capacity(e, count);
    if (r != hipSuccess) {
        if (r == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            return ISING_ENOMEM;
        }
        return ctx_fail(ctxs[0], r, "engine: set-up");
    }
    if (e.staged_pending) {  // pinned staging area still being read by the last copy
        if ((r = hipEventSynchronize(e.staged_relay)) != hipSuccess)
            return ctx_fail(ctxs[0], r, "engine: staging wait");
        e.staged_pending = false;
    }
    // the stepped plan walks sides that are multiples of 16 with the fused
    // one-pass kernel, each lattice ping-ponging between its two buffers
    bool fused = stepped;
    for (size_t k = 0; fused && k < count; ++k) fused = multi_fused_supported(ctxs[k]->L);
    if (fused) {
        for (size_t k = 0; k < count; ++k) {
            ising_ctx* c = ctxs[k];
            if (c->buf[1] || n[k] == 0) continue;
            if (hipMalloc(&c->buf[1], (size_t)c->L * c->L) != hipSuccess) {
                (void)hipGetLastError();
                return ISING_ENOMEM;
            }
            c->owns_buf[1] = true;
        }
    }
    std::vector<uint64_t> work(count);
    uint32_t live = 0;
    for (size_t k = 0; k < count; ++k)
        if (n[k]) ++live;
    // A thread updates a bit-packed word with eight Philox blocks where a
    // byte word takes one, so bits trade a lattice's latency for local
    // memory. While the batch leaves workgroups idle, latency decides: a
    // lattice that fits in local memory as bytes stays bytes.
    const bool saturated = live >= e.grid;
    for (size_t k = 0; k < count; ++k) {
        ising_ctx* c = ctxs[k];
        BatchItem& it = e.h_items[k];
        fill_batch_item(c, n[k], stepped, it);
        if (fused && c->buf[1]) {
            const Planes alt = ctx_planes_alt(c);
            it.q0 = reinterpret_cast<uint32_t*>(alt.p[0]);
            it.q1 = reinterpret_cast<uint32_t*>(alt.p[1]);
        }
        // the general (h != 0) bit update costs more per site than the byte
        // kernel: only for lattices that do not fit as bytes
        const uint32_t mode = bits_fit(c->L) ? bits_mode(c->table) : 0u;
        it.bits = (!stepped && mode && (!bytes_fit(c->L) || (saturated && mode != 3u))) ? mode : 0u;
        work[k] = (uint64_t)c->L * c->L * n[k];
    }
    uint64_t max_n = 0;
    for (size_t k = 0; k < count; ++k) max_n = std::max<uint64_t>(max_n, n[k]);
    if (live == 0) return ISING_OK;
    if (!stepped) {
        // longest work first; lattices with no sweeps are left out of the queue
        std::vector<uint32_t> idx(count);
        std::iota(idx.begin(), idx.end(), 0u);
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return work[a] > work[b]; });
        for (size_t k = 0; k < count; ++k) e.h_order[k] = idx[k];
        e.h_hdr->count = live;
        e.h_hdr->head = 0;
    } else {
        // fused walk: the tile height asked for, else the tallest tiles (32
        // rows) that still give every wave slot of the GPU about two tiles
        uint32_t rows = rows_wanted ? rows_wanted : 32u;
        if (fused && !rows_wanted) {
            const uint64_t want = 2ull * e.fslots;
            for (; rows > 8u; rows /= 2u) {
                uint64_t tiles = 0;
                for (size_t k = 0; k < count; ++k)
                    if (n[k]) tiles += multi_fused_tiles(e.h_items[k].L, rows);
                if (tiles >= want) break;
            }
        }
        uint64_t vb = 0;
        for (size_t k = 0; k < count; ++k) {
            e.h_vbs[k] = (uint32_t)vb;
            vb += fused ? multi_fused_tiles(e.h_items[k].L, rows) : multi_vblocks(e.h_items[k].L, e.h_items[k].cw);
        }
        if (vb >= ((uint64_t)1 << 32)) return ISING_ERANGE;
        e.h_vbs[count] = (uint32_t)vb;
        e.h_mhdr->n_items = (uint32_t)count;
        e.h_mhdr->total_vblocks = (uint32_t)vb;
        e.h_mhdr->s_base = 0u - kSweepsPerReplay;  // the graph's first node adds G
        e.h_mhdr->rows = rows;
        if ((r = ensure_partials(e, vb)) != hipSuccess) {
            if (r == hipErrorOutOfMemory) {
                (void)hipGetLastError();
                return ISING_ENOMEM;
            }
            return ctx_fail(ctxs[0], r, "engine: partials");
        }
        e.h_mhdr->part = e.d_part;
    }

    // order the launch after every context's earlier work. A context with
    // no API call since an earlier launch of this engine ordered its stream
    // after that launch has nothing newer on its stream than that launch,
    // which the wait on the previous launch below already covers.
    for (size_t k = 0; k < count; ++k) {
        hipStream_t cs = ctxs[k]->stream;
        if (cs == s) continue;
        if (e.launched && ctxs[k]->engine_seq == ctxs[k]->api_seq) continue;
        if ((r = hipEventRecord(e.order_ev, cs)) != hipSuccess) return ctx_fail(ctxs[k], r, "engine: record order");
        if ((r = hipStreamWaitEvent(s, e.order_ev, 0)) != hipSuccess)
            return ctx_fail(ctxs[k], r, "engine: wait order");
    }
    // the device descriptors may still be read by the previous launch (when
    // both are on the engine's own stream, stream order already waits for it)
    const bool after_own = s == e.launch && e.last_stream == e.launch;
    if (e.launched && !after_own && (r = hipStreamWaitEvent(s, e.done_relay, 0)) != hipSuccess)
        return ctx_fail(ctxs[0], r, "engine: wait previous launch");
    static_assert(sizeof(BatchItem) % 4 == 0, "staging copies whole words");
    r = launch_stage_copy(e.d_stage, e.h_stage, e.off_items + count * sizeof(BatchItem), s);
    if (r != hipSuccess) return ctx_fail(ctxs[0], r, "engine: stage descriptors");
    if ((r = hipEventRecord(e.staged, s)) != hipSuccess || (r = hipStreamWaitEvent(e.relay, e.staged, 0)) != hipSuccess ||
        (r = hipEventRecord(e.staged_relay, e.relay)) != hipSuccess)
        return ctx_fail(ctxs[0], r, "engine: record staged");
    e.staged_pending = true;
    if (!stepped) {
        r = ensure_graph(e, s);
        if (r == hipSuccess) r = hipGraphLaunch(e.exec, s);
    } else if (fused) {
        r = ensure_fused_graph(e);
        const uint64_t replays = (max_n + kSweepsPerReplay - 1) / kSweepsPerReplay;
        for (uint64_t k = 0; r == hipSuccess && k < replays; ++k) r = hipGraphLaunch(e.fexec, s);
    } else {
        r = ensure_multi_graph(e);
        const uint64_t replays = (max_n + kSweepsPerReplay - 1) / kSweepsPerReplay;
        for (uint64_t k = 0; r == hipSuccess && k < replays; ++k) r = hipGraphLaunch(e.mexec, s);
    }
    if (r != hipSuccess) return ctx_fail(ctxs[0], r, stepped ? "engine: stepped graph" : "engine: resident graph");
    if ((r = hipEventRecord(e.done, s)) != hipSuccess || (r = hipStreamWaitEvent(e.relay, e.done, 0)) != hipSuccess ||
        (r = hipEventRecord(e.done_relay, e.relay)) != hipSuccess)
        return ctx_fail(ctxs[0], r, "engine: record done");
    e.launched = true;
    e.last_stream = s;
    // and every context's later work after it
    if ((r = hipEventRecord(e.order_ev, s)) != hipSuccess) return ctx_fail(ctxs[0], r, "engine: record after");
    for (size_t k = 0; k < count; ++k) {
        hipStream_t cs = ctxs[k]->stream;
        if (cs != s && (r = hipStreamWaitEvent(cs, e.order_ev, 0)) != hipSuccess)
            return ctx_fail(ctxs[k], r, "engine: wait after");
        ctxs[k]->engine_seq = ctxs[k]->api_seq;
    }
    for (size_t k = 0; k < count; ++k) {
        if (n[k]) ++ctxs[k]->gen;
        ctxs[k]->t += n[k];
        ctxs[k]->series_len += n[k];
        if (fused && (n[k] & 1u)) ctxs[k]->cur ^= 1;  // an odd number of ping-pong sweeps
    }
    return ISING_OK;
}
