// Launchers of the percolation engine (perc_kernels.hip), shared with its
// runtime (perc_runtime.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace perc {

constexpr uint32_t kTile = 64;               // tile side (sites)
constexpr uint32_t kThreads = 256;           // per workgroup: a 64-wide column of 16-site strips
constexpr uint32_t kStrip = kTile * kTile / kThreads;
constexpr uint32_t kSolid = 0xffffffffu;     // arrival of a solid site (-1 as int32)
constexpr uint32_t kUnreached = 0x7fffffffu; // pore not (yet) invaded

struct Stats {
    unsigned long long pores;
    unsigned long long invaded;
    uint32_t max_arrival;
    uint32_t edges;  // bit 0 row 0, bit 1 row L-1, bit 2 column 0, bit 3 column L-1
    unsigned long long visits;      // tile visits over all relaxation launches
    unsigned long long iterations;  // relaxation iterations summed over visits
};

// Work lists: tiles to relax in a launch. Launch k reads list[k % 2] with
// length len[k % 3], appends to list[(k + 1) % 2] / len[(k + 1) % 3] and
// clears len[(k + 2) % 3]; queued[p][tile] says whether the tile is in
// list p, so no tile is listed twice.
struct WorkLists {
    uint32_t* list[2];
    uint32_t* queued[2];
    uint32_t* len;  // 3 counters
};

hipError_t launch_draw(uint8_t* pore, uint32_t* arr, uint32_t L, uint64_t pthr, uint32_t k0, uint32_t k1,
                       uint32_t source, uint32_t i0, uint32_t j0, Stats* stats, hipStream_t s);
hipError_t launch_seed_lists(const WorkLists& w, uint32_t n_tx, uint32_t n_tiles, uint32_t source, uint32_t i0,
                             uint32_t j0, hipStream_t s);
hipError_t launch_relax(uint32_t* arr, uint32_t L, uint32_t n_tx, uint32_t n_ty, const WorkLists& w, uint64_t k,
                        uint32_t grid, Stats* stats, hipStream_t s);
hipError_t launch_finish(uint32_t* arr, uint32_t L, Stats* stats, hipStream_t s);

}  // namespace perc
