// Launchers of the percolation engine (perc_kernels.hip), shared with its
// runtime (perc_runtime.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace perc {

constexpr uint32_t kTile = 64;               // tile side (sites)
constexpr uint32_t kThreads = 256;           // per workgroup of the draw, seed and finish passes
constexpr uint32_t kRelaxThreads = kTile;    // relaxation: one wave per tile, a lane per tile row
constexpr uint32_t kSolid = 0xffffffffu;     // arrival of a solid site (-1 as int32)
constexpr uint32_t kUnreached = 0x7fffffffu; // pore not (yet) invaded

struct Stats {
    unsigned long long pores;
    unsigned long long invaded;
    uint32_t max_arrival;
    uint32_t edges;  // bit 0 row 0, bit 1 row L-1, bit 2 column 0, bit 3 column L-1
    unsigned long long visits;      // tile visits over all relaxation launches
    unsigned long long iterations;  // breadth-first levels summed over visits
};

// One medium of a run (a run relaxes one or several media together).
struct Medium {
    uint32_t* arr;        // arrival passes, row-major
    uint32_t* queued[2];  // per tile: is it in work list 0 / 1
    uint32_t* resume;     // per tile: level from which its next visit must start (all ones: none)
    Stats* stats;
    uint32_t L, n_tx, n_ty, pad;
};

// Work lists of (medium, tile) entries to relax in a launch. Launch k reads
// list[k % 2] with length len[k % 3], appends to list[(k + 1) % 2] /
// len[(k + 1) % 3] and clears len[(k + 2) % 3]; a medium's queued[p][tile]
// says whether the tile is in list p, so no tile is listed twice.
struct WorkLists {
    uint2* list[2];
    uint32_t* len;  // 3 counters
};

hipError_t launch_draw(uint8_t* pore, uint32_t* arr, uint32_t L, uint64_t pthr, uint32_t k0, uint32_t k1,
                       uint32_t source, uint32_t i0, uint32_t j0, Stats* stats, hipStream_t s);
// clear the list counters (before the media of a run are seeded)
hipError_t launch_reset_lists(const WorkLists& w, hipStream_t s);
// append medium m's source tiles to list 0
hipError_t launch_seed(const WorkLists& w, const Medium* media, uint32_t m, uint32_t n_tx, uint32_t source,
                       uint32_t i0, uint32_t j0, hipStream_t s);
hipError_t launch_relax(const Medium* media, const WorkLists& w, uint64_t k, uint32_t grid, hipStream_t s);
hipError_t launch_finish(uint32_t* arr, uint32_t L, Stats* stats, hipStream_t s);

}  // namespace perc
