// Internal runtime state shared by the C ABI implementation files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising.h"
#include "ising_bands.hpp"
#include "ising_launch.hpp"

namespace ising {

// How a context runs its sweeps.
struct Plan {
    uint32_t kind = ISING_PLAN_TWO_PASS;  // ISING_PLAN_*
    uint32_t cw = 1;                      // 32-bit words per thread/lane and row
    uint32_t rows = 0;                    // tile height (fused plan)
};

uint64_t metropolis_threshold(double J, double h, double T, int s, int n);
void build_accept_table(double J, double h, double T, AcceptTable* at, bool* exact);
uint64_t fnv1a64(const uint8_t* p, size_t n);

// Plan that can serve side L for the requested ISING_PLAN_* (cw / rows 0 =
// default); false if it cannot.
bool plan_for(uint32_t L, uint32_t kind, uint32_t cw, uint32_t rows, Plan* out);

}  // namespace ising

struct ising_ctx {
    ising_params p{};
    uint32_t L = 0;
    ising::Plan plan{};
    ising::AcceptTable table{};
    bool exact = false;        // some threshold is 0: use the 64-bit compare
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    uint8_t* buf[2] = {nullptr, nullptr};  // lattice buffers (the second only for ping-pong)
    bool owns_buf[2] = {false, false};
    int cur = 0;                 // which buffer holds the current lattice
    int64_t* series = nullptr;   // (B_t, M_t) pairs, series_cap of them
    uint64_t series_cap = 0;
    uint64_t series_len = 0;
    int64_t* part[2] = {nullptr, nullptr};  // per-tile / per-block partials
    uint32_t part_cap = 0;       // pairs per partial buffer
    int64_t* scratch = nullptr;  // 4 int64 for observables
    int8_t* canon = nullptr;     // N bytes, canonical layout staging
    void* host_stage = nullptr;  // pinned host memory the observables are read back into
    size_t host_stage_bytes = 0;
    uint64_t gen = 0;            // bumped by every call that changes the lattice or the series
    uint64_t api_seq = 0;        // bumped by every API call on the context (ctx_enter)
    uint64_t engine_seq = ~0ull;  // api_seq when the batch engine last ordered the stream after its launch
    // a read-back started by ising_prefetch_observables into host_stage:
    // 0 none, 1 copies enqueued, 2 copies landed (valid while gen == pre_gen)
    int pre_state = 0;
    bool pre_full = false;       // the whole series was copied (else only the current (B, M))
    uint32_t pre_want = 0;
    uint64_t pre_gen = 0;
    size_t pre_hash_off = 0;
    uint8_t* demon = nullptr;    // Creutz demons (N bytes, colour-plane layout), once initialised
    uint8_t* demon_alt = nullptr;  // second demon buffer for the fused (ping-pong) Creutz sweep
    int64_t* cpart = nullptr;    // Creutz per-block (B, M) partials
    int64_t* cfpart[2] = {nullptr, nullptr};  // fused Creutz per-tile partials, double-buffered
    uint32_t cfpart_cap = 0;
    // Graph replays of the two-pass plan (kGraphSweeps sweeps each): the
    // instantiated graph, the lattice buffer it was captured on, the device
    // header it reads (sweep index, series slot) and the partials of a
    // replay's sweeps (kGraphSweeps x blocks pairs).
    hipGraphExec_t gexec = nullptr;
    uint32_t gcur = 0;
    ising::SweepHeader* ghdr = nullptr;
    int64_t* gpart = nullptr;
    size_t gpart_pairs = 0;
    // Band-resident plan: tagged edge-row slots for band_cap bands (2 x
    // bands x 2 rows; the tag of the last half-sweep published is
    // band_base, growing across launches), per-band partials of up to
    // kBandChunk sweeps for band_part_cap bands (allocated by the first
    // ising_sweep), the timeout mark of the edge waits and its pinned host
    // copy.
    uint64_t* band_pub = nullptr;
    int64_t* band_part = nullptr;
    uint32_t* band_err = nullptr;
    uint32_t* band_err_host = nullptr;
    uint32_t band_cap = 0;
    uint32_t band_part_cap = 0;
    uint32_t band_base = 0;
    uint64_t t = 0;              // next sweep index
    bool poisoned = false;
    hipError_t last_hip = hipSuccess;
    char device_error[160] = {0};  // failing call and HIP error of the last EDEVICE
};

ising::Planes ctx_planes(const ising_ctx* ctx);
ising::Planes ctx_planes_alt(const ising_ctx* ctx);
int ctx_reserve_series(ising_ctx* ctx, uint64_t more);
int ctx_prepare_plan(ising_ctx* ctx);
// Forget the context's captured sweep graphs (its plan, table or buffers
// changed); waits for its stream when there are any.
void ctx_drop_graphs(ising_ctx* ctx);
// Poison the context after a failed HIP call `where` and return EDEVICE.
int ctx_fail(ising_ctx* ctx, hipError_t e, const char* where = "");

// Batch engine (ising_engine.cpp): run ctxs[k] for n[k] sweeps each on
// stream s, either as one persistent workgroup-resident launch or as the
// stepped multi-lattice graph.
// Run a batch on stream s (nullptr: the engine's own stream on the
// contexts' device), ordered after every context's earlier work and before
// its later work.
// rows: the stepped fused walk's tile height (8, 16 or 32; 0: the engine's
// own choice).
int engine_run(ising_ctx* const* ctxs, const uint64_t* n, size_t count, hipStream_t s, bool stepped,
               uint32_t rows = 0);
// Workgroups of the persistent resident launch on device dev (lattices it
// runs at once); 0 if the engine cannot be set up.
uint32_t engine_resident_slots(int dev);
// Waves of the stepped fused walk resident at once on device dev.
uint32_t engine_fused_slots(int dev);

// Batch plan model (ising_batch_tune.cpp): the plan and stepped tile height
// predicted fastest for a batch, from the device's measured (or built-in)
// per-class rates, with both predictions in ns.
struct BatchChoice {
    bool stepped;
    uint32_t rows;
    double resident_ns, stepped_ns;
};
int batch_choose(ising_ctx* const* ctxs, const uint64_t* n, size_t count, int dev, BatchChoice* out);
// Descriptor of context c for n sweeps from its current state: lattice
// planes, series slots after the pending ones, draw key, table, words per
// thread (stepped or resident). The fused walk's second planes and the
// bit-packing choice are left to the caller (null / 0).
void fill_batch_item(const ising_ctx* c, uint64_t n, bool stepped, ising::BatchItem& it);
