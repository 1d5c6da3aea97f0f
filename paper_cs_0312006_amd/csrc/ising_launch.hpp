// Host-visible launch interface between the runtime (ising_runtime.cpp) and
// the kernels (ising_kernels.hip, ising_fused.hip, ising_batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

// The two colour planes of one lattice state (see ising_device.hpp).
struct Planes {
    uint8_t* p[2];  // plane c: L rows of H bytes
    uint32_t L;     // side
    uint32_t H;     // L / 2
    uint32_t Hw;    // H / 4 (meaningful when L % 8 == 0)
};

// Arguments of the fused one-pass sweep (ising_fused.hip).
struct FusedArgs {
    const uint32_t* src0;  // lattice of sweep t-1, colour planes 0 and 1
    const uint32_t* src1;
    uint32_t* dst0;        // lattice of sweep t
    uint32_t* dst1;
    uint32_t L, Hw, t, k0, k1;
    uint32_t n_tx;     // tiles across a plane row
    uint32_t n_tiles;  // tiles in the lattice (one wave each)
    int64_t* part;     // 2 int64 per tile: partial (B, M)
};

// Device-side state of a context's graph replays: the sweep index of the
// replay's first sweep and where its first (B, M) goes. The replay's last
// node advances both by the replay's sweeps; arrived counts its finished
// workgroups.
struct SweepHeader {
    uint32_t t;
    uint32_t arrived;
    int64_t* ser;
};
hipError_t launch_set_header(SweepHeader* hdr, uint32_t t, int64_t* ser, hipStream_t s);
// Sum each of g sweeps' n partial pairs (sweep k's at part + 2 k n) into
// hdr->ser + 2 k, then advance hdr by g sweeps.
hipError_t launch_reduce_group(const int64_t* part, uint32_t n, uint32_t g, SweepHeader* hdr, hipStream_t s);

// Sum of n per-tile (or per-block) partial (B, M) pairs into dst[0], dst[1].
struct PartialReduce {
    const int64_t* part;
    uint32_t n;
    int64_t* dst;
};

// Sum n partial (B, M) pairs into dst (one block of up to 1024 threads;
// every thread must call).
__device__ __forceinline__ void reduce_partials(const PartialReduce& red) {
    if (red.n == 0) return;
    __shared__ int64_t acc[2][16];
    int64_t b = 0, m = 0;
    uint32_t k = threadIdx.x;
    for (; k + 3 * blockDim.x < red.n; k += 4 * blockDim.x) {  // four loads in flight
        const int64_t b0 = red.part[2 * k], m0 = red.part[2 * k + 1];
        const int64_t b1 = red.part[2 * (k + blockDim.x)], m1 = red.part[2 * (k + blockDim.x) + 1];
        const int64_t b2 = red.part[2 * (k + 2 * blockDim.x)], m2 = red.part[2 * (k + 2 * blockDim.x) + 1];
        const int64_t b3 = red.part[2 * (k + 3 * blockDim.x)], m3 = red.part[2 * (k + 3 * blockDim.x) + 1];
        b += (b0 + b1) + (b2 + b3);
        m += (m0 + m1) + (m2 + m3);
    }
    for (; k < red.n; k += blockDim.x) {
        b += red.part[2 * k];
        m += red.part[2 * k + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        b += __shfl_xor(b, off, 64);
        m += __shfl_xor(m, off, 64);
    }
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    if (lane == 0) {
        acc[0][wv] = b;
        acc[1][wv] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sb = 0, sm = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
            sb += acc[0][w];
            sm += acc[1][w];
        }
        red.dst[0] = sb;
        red.dst[1] = sm;
    }
}

hipError_t launch_init(const Planes& pl, bool words, uint32_t k0, uint32_t k1, uint64_t pthr, hipStream_t s);
uint32_t two_pass_blocks(const Planes& pl, uint32_t cw);
hipError_t launch_two_pass(const Planes& pl, const AcceptTable& at, bool exact, uint32_t cw, uint32_t t,
                           uint32_t k0, uint32_t k1, int64_t* part, const PartialReduce& red, hipStream_t s,
                           const uint32_t* t_dev = nullptr);
hipError_t launch_generic_sweep(const Planes& pl, const AcceptTable& at, bool exact, uint32_t t, uint32_t k0,
                                uint32_t k1, int64_t* obs, hipStream_t s);
hipError_t launch_observe(const Planes& pl, int64_t* out, hipStream_t s);
hipError_t launch_zero(int64_t* p, uint64_t n, hipStream_t s);
bool fused_supported(uint32_t L, uint32_t cw, uint32_t rows);
uint32_t fused_tiles(uint32_t L, uint32_t cw, uint32_t rows);
hipError_t launch_fused(const FusedArgs& a, const AcceptTable& at, bool exact, uint32_t cw, uint32_t rows,
                        const PartialReduce& red, hipStream_t s);
hipError_t launch_reduce_partials(const PartialReduce& red, hipStream_t s);
// The fused sweep by full-row workgroups (ising_fused_rows.hip): one
// workgroup of L/8 / (64 cw) <= 16 waves per band of `rows` rows; a.n_tx is
// unused and a.part holds one (B, M) pair per band.
bool fused_rows_supported(uint32_t L, uint32_t cw, uint32_t rows);
uint32_t fused_rows_bands(uint32_t L, uint32_t rows);
hipError_t launch_fused_rows(const FusedArgs& a, const AcceptTable& at, uint32_t cw, uint32_t rows,
                             const PartialReduce& red, hipStream_t s);

// One lattice of a workgroup-resident batch (ising_batch.hip).
struct BatchItem {
    uint32_t* p0;       // colour planes, updated in place
    uint32_t* p1;
    uint32_t* q0;       // the other buffer's planes (stepped fused plan: ping-pong)
    uint32_t* q1;
    int64_t* series;    // 2 int64 per sweep, for sweeps t0 .. t0+n-1
    uint32_t L, Hw, cw, t0, n, k0, k1, exact;
    uint32_t bits;      // resident batch: 1 / 2 / 3 = bit-packed in LDS (see bits_mode), 0 = not
    uint32_t pad;
    AcceptTable table;
};

struct BatchHeader {
    uint32_t count;  // items in this launch
    uint32_t head;   // work-queue position, 0 at launch
};

// Lattices whose two planes fit in this many bytes run from LDS in the
// resident batch kernel (256 x 256 sites).
constexpr uint32_t kBatchLdsBytes = 65536;
// Lattices whose two planes fit in this many bytes at one bit per site run
// bit-packed from LDS in the resident batch kernel (sides up to 1072).
constexpr uint32_t kBatchBitsLdsBytes = 147456;

// Bit-packed update of a lattice's acceptance table: when the threshold
// depends only on the number m of disagreeing neighbours (h = 0), with
// m = 2, 3, 4 always accepted (1: J >= 0) or m = 0, 1, 2 always accepted
// (2: J < 0), two class compares per site; otherwise (3) one compare per
// (spin, m) class that is neither always nor never accepted.
uint32_t bits_mode(const AcceptTable& at);
// Whether an L x L lattice fits the bit-packed LDS area.
bool bits_fit(uint32_t L);
// Whether a side-L lattice fits the resident kernel's local memory as bytes.
bool bytes_fit(uint32_t L);

hipError_t launch_batch(const BatchItem* items, const uint32_t* order, BatchHeader* hdr, uint32_t grid,
                        hipStream_t s);
// One workgroup runs every sweep of the lattice `it` describes (passed by
// value: nothing to stage).
hipError_t launch_batch_one(const BatchItem& it, hipStream_t s);
// Copy `bytes` (a multiple of 4) from pinned host memory to device memory
// with a kernel on stream s: it starts as soon as the stream's earlier work
// ends, where a copy-engine transfer waiting on another stream's event
// started hundreds of microseconds later.
hipError_t launch_stage_copy(void* dst, const void* host_src, size_t bytes, hipStream_t s);
uint32_t batch_block_threads();
hipError_t batch_occupancy(int* blocks_per_cu);

// Stepped multi-lattice passes (ising_multi.hip).
struct MultiHeader {
    uint32_t n_items;        // items in the work list
    uint32_t total_vblocks;  // virtual blocks (fused walk: tiles) over all items
    uint32_t s_base;         // sweep base; the graph's first node adds G to it
    uint32_t rows;           // fused walk: rows per tile (8, 16 or 32)
    int64_t* part;           // (B, M) of every virtual block for each sweep of a replay (sweep-major)
};
constexpr uint32_t kMultiChunksPerThread = 4;
uint32_t multi_vblocks(uint32_t L, uint32_t cw);
hipError_t launch_multi_graph_body(const BatchItem* items, const uint32_t* vb_start, MultiHeader* hdr,
                                   uint32_t sweeps_per_replay, uint32_t grid, hipStream_t s);
// The last node of a stepped replay (either walk): item k's series entries
// for the replay's sweeps = the sums of hdr->part over its virtual blocks
// vb_start[k] .. vb_start[k + 1] - 1.
hipError_t launch_multi_reduce(const BatchItem* items, const uint32_t* vb_start, const MultiHeader* hdr,
                               uint32_t sweeps_per_replay, uint32_t grid, hipStream_t s);

// Stepped multi-lattice sweeps with the fused walk (ising_multi_fused.hip):
// one launch per sweep over the tiles (hdr->rows rows by 128 words) of
// every item, each lattice ping-ponging between p and q; vb_start[k] is item
// k's first tile. Sides must satisfy L % 16 == 0. Each tile writes its
// (B, M) to hdr->part (G x total tiles pairs, sweep-major), and the replay's
// last node sums them per item into the series.
bool multi_fused_supported(uint32_t L);
// Tiles of a side-L lattice at `rows` rows per tile: n_tx columns of up to
// 128 words (the last may be narrower) by n_ty row bands. When the last
// column is at most 32 lanes (64 words) wide, `pack` of its row bands share
// one wave (pack * prow <= 64), so that a narrow lattice does not leave
// most lanes of its waves idle; its bands are prow rows high (rows, or 16
// when rows does not divide L), n_typ of them. Tile order: the full
// columns' tiles (column-fastest), then the last column's packed tiles;
// with pack == 1, column-fastest over all columns.
struct MfLayout {
    uint32_t n_tx, n_ty, pack, prow, n_typ, tiles;
};
__host__ __device__ inline MfLayout mf_layout(uint32_t L, uint32_t rows) {
    MfLayout o;
    const uint32_t Hw = L / 8u;
    o.n_tx = (Hw + 127u) / 128u;
    o.n_ty = (L + rows - 1u) / rows;
    o.pack = 1u;
    o.prow = rows;
    o.n_typ = o.n_ty;
    const uint32_t last_lanes = (Hw - (o.n_tx - 1u) * 128u) / 2u;
    if (last_lanes <= 32u) {
        const uint32_t pr = L % rows == 0u ? rows : 16u;  // sides are multiples of 16
        const uint32_t nb = L / pr;
        uint32_t pk = 64u / last_lanes < 64u / pr ? 64u / last_lanes : 64u / pr;
        if (pk > nb) pk = nb;
        if (pk > 1u) {
            o.pack = pk;
            o.prow = pr;
            o.n_typ = nb;
        }
    }
    o.tiles = (o.n_tx - 1u) * o.n_ty + (o.n_typ + o.pack - 1u) / o.pack;
    return o;
}
uint32_t multi_fused_tiles(uint32_t L, uint32_t rows);
// Waves of the fused walk resident at once on a GPU with `cus` compute units.
uint32_t multi_fused_wave_slots(uint32_t cus);
hipError_t launch_multi_fused_graph_body(const BatchItem* items, const uint32_t* tile_start, MultiHeader* hdr,
                                         uint32_t sweeps_per_replay, uint32_t grid, hipStream_t s);

// Creutz demon dynamics (ising_creutz.hip): dm holds the demon planes, in
// the spin planes' layout. A sweep is two in-place passes; the word path
// (L % 8 == 0) writes the finished sweep's (B, M) partials into part
// (creutz_blocks() pairs) and reduces `red` first.
uint32_t creutz_blocks(const Planes& pl);
hipError_t launch_creutz_sweep(const Planes& pl, const Planes& dm, bool reverse, int64_t* part,
                               const PartialReduce& red, hipStream_t s);
hipError_t launch_creutz_sweep_sites(const Planes& pl, const Planes& dm, bool reverse, hipStream_t s);
hipError_t launch_demon_sum(const uint8_t* d, uint64_t n, int64_t* out, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s);
hipError_t launch_bytes_to_canonical(const Planes& pl, uint8_t* out, hipStream_t s);
hipError_t launch_bytes_from_canonical(const Planes& pl, const uint8_t* in, hipStream_t s);
hipError_t launch_to_canonical(const Planes& pl, int8_t* out, hipStream_t s);
hipError_t launch_from_canonical(const Planes& pl, const int8_t* in, hipStream_t s);

}  // namespace ising
