// Workgroup-resident sweeps for many independent lattices in one launch.
//
// Each workgroup takes the next lattice from a device work queue (the host
// orders the queue by work, largest first) and runs all of that lattice's
// sweeps itself: colour 0 of sweep t, a workgroup barrier, colour 1, a
// barrier, then the sweep's (B, M) (Section 2.2's consecutive black and
// white passes). Lattices stay in their own colour planes and are updated
// in place; small ones live in the L1/L2 of the workgroup's CU for the whole
// run. The grid is sized to the resident capacity of the chip, so the kernel
// is persistent: no workgroup waits on another.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr uint32_t kBatchThreads = 512;

template <int CW, bool OBS, bool EXACT, typename PT>
__device__ __forceinline__ void colour_pass(const LdsTable& lt, const BatchItem& it, PT p0, PT p1, uint32_t c,
                                            uint32_t t, uint32_t& sad, uint32_t& ups) {
    PT own = c ? p1 : p0;
    PT oth = c ? p0 : p1;
    const uint32_t L = it.L, Hw = it.Hw;
    const uint32_t per_row = Hw / CW;
    const uint32_t total = L * per_row;
    for (uint32_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const uint32_t i = idx / per_row;
        const uint32_t wc = (idx - i * per_row) * CW;
        const uint32_t iu = i == 0 ? L - 1 : i - 1;
        const uint32_t id = i + 1 == L ? 0 : i + 1;
        const uint32_t p = (i + c) & 1u;
        const size_t row = (size_t)i * Hw;
        uint32_t W[CW], U[CW], D[CW], O[CW];
#pragma unroll
        for (int w = 0; w < CW; ++w) {
            W[w] = own[row + wc + w];
            U[w] = oth[(size_t)iu * Hw + wc + w];
            D[w] = oth[(size_t)id * Hw + wc + w];
            O[w] = oth[row + wc + w];
        }
        const uint32_t ew = p ? (wc + CW == Hw ? 0u : wc + CW) : (wc == 0 ? Hw - 1 : wc - 1);
        const uint32_t E = oth[row + ew];
#pragma unroll
        for (int w = 0; w < CW; ++w) {
            const uint32_t nxt = (w + 1 < CW) ? O[(w + 1 < CW) ? w + 1 : 0] : E;
            const uint32_t prv = (w > 0) ? O[(w > 0) ? w - 1 : 0] : E;
            const uint32_t S = shifted(O[w], nxt, prv, p);
            const uint32_t n = U[w] + D[w] + O[w] + S;
            const uint4 r = philox((uint32_t)(row + wc + w), t, c, 0u, it.k0, it.k1);
            const uint32_t Wn = W[w] ^ flip_mask<EXACT>(lt, W[w], n, r);
            own[row + wc + w] = Wn;
            if (OBS) {
                sad = sad_misaligned(Wn, n, sad);
                ups += __builtin_popcount(Wn) + __builtin_popcount(O[w]);
            }
        }
    }
}

// Per-wave (sad, ups) partials of the last kFlush sweeps live in LDS and are
// summed into the series every kFlush sweeps, so no sweep waits on a global
// store before its barrier.
constexpr uint32_t kFlush = 64;
constexpr uint32_t kMaxWaves = kBatchThreads / 64;

template <int CW, bool EXACT, typename PT>
__device__ __forceinline__ void run_lattice(const LdsTable& lt, const BatchItem& it, PT p0, PT p1,
                                            uint32_t (*part)[kMaxWaves][2]) {
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t nwaves = blockDim.x >> 6;
    const uint32_t total = it.L * (it.Hw / CW);  // colour-1 chunks of the lattice
    const int64_t words = (int64_t)total * CW;   // colour-1 words of the lattice
    auto flush = [&](uint32_t first, uint32_t count) {
        // thread k < count sums sweep first + k over the waves
        if (threadIdx.x < count) {
            const uint32_t slot = (first + threadIdx.x) % kFlush;
            int64_t ss = 0, su = 0;
            for (uint32_t w = 0; w < nwaves; ++w) {
                ss += part[slot][w][0];
                su += part[slot][w][1];
            }
            it.series[2 * (first + threadIdx.x)] = 16 * words - 2 * ss;
            it.series[2 * (first + threadIdx.x) + 1] = 2 * su - 8 * words;
        }
    };
    for (uint32_t s = 0; s < it.n; ++s) {
        const uint32_t t = it.t0 + s;
        uint32_t sad = 0, ups = 0;
        colour_pass<CW, false, EXACT>(lt, it, p0, p1, 0u, t, sad, ups);
        __syncthreads();
        colour_pass<CW, true, EXACT>(lt, it, p0, p1, 1u, t, sad, ups);
        // 32-bit wave sums (a thread covers at most a few hundred words per
        // pass here, far from overflow); sweep totals are formed in 64 bits
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sad += __shfl_xor(sad, off, 64);
            ups += __shfl_xor(ups, off, 64);
        }
        if (lane == 0) {
            part[s % kFlush][wv][0] = sad;
            part[s % kFlush][wv][1] = ups;
        }
        // separates colour 1 of sweep s from colour 0 of sweep s+1, and makes
        // the partials visible to the flush
        __syncthreads();
        if ((s + 1) % kFlush == 0) flush(s + 1 - kFlush, kFlush);
    }
    const uint32_t rem = it.n % kFlush;
    if (rem) flush(it.n - rem, rem);
}

}  // namespace

// Run all sweeps of one lattice with its planes at p0/p1 (global memory or
// this workgroup's LDS copy).
template <bool EXACT, typename PT>
__device__ __forceinline__ void run_any(const LdsTable& lt, const BatchItem& it, PT p0, PT p1,
                                        uint32_t (*red)[kMaxWaves][2]) {
    if (it.cw == 4) run_lattice<4, EXACT>(lt, it, p0, p1, red);
    else if (it.cw == 2) run_lattice<2, EXACT>(lt, it, p0, p1, red);
    else run_lattice<1, EXACT>(lt, it, p0, p1, red);
}

__global__ void __launch_bounds__(kBatchThreads) k_batch(const BatchItem* __restrict__ items,
                                                         const uint32_t* __restrict__ order, BatchHeader* hdr) {
    __shared__ LdsTable lt;
    __shared__ uint32_t s_slot;
    __shared__ uint32_t red[kFlush][kMaxWaves][2];
    // lattices of at most kBatchLdsBytes run from this LDS copy
    __shared__ uint32_t lat[kBatchLdsBytes / 4];
    const uint32_t count = hdr->count;
    for (;;) {
        if (threadIdx.x == 0) s_slot = atomicAdd(&hdr->head, 1u);
        __syncthreads();
        const uint32_t slot = s_slot;
        if (slot >= count) break;
        const BatchItem& it = items[order[slot]];
        load_table(lt, it.table);
        __syncthreads();
        const uint32_t plane_words = it.L * it.Hw;
        if (2u * plane_words * 4u <= kBatchLdsBytes && it.n > 0) {
            uint32_t* l0 = lat;
            uint32_t* l1 = lat + plane_words;
            const global_u32* g0 = as_global(it.p0);
            const global_u32* g1 = as_global(it.p1);
            for (uint32_t k = threadIdx.x; k < plane_words; k += blockDim.x) {
                l0[k] = g0[k];
                l1[k] = g1[k];
            }
            __syncthreads();
            if (it.exact) run_any<true>(lt, it, l0, l1, red);
            else run_any<false>(lt, it, l0, l1, red);
            __syncthreads();
            global_u32* g0w = as_global(it.p0);
            global_u32* g1w = as_global(it.p1);
            for (uint32_t k = threadIdx.x; k < plane_words; k += blockDim.x) {
                g0w[k] = l0[k];
                g1w[k] = l1[k];
            }
        } else {
            if (it.exact) run_any<true>(lt, it, as_global(it.p0), as_global(it.p1), red);
            else run_any<false>(lt, it, as_global(it.p0), as_global(it.p1), red);
        }
        // everyone has read s_slot and the table before they are replaced
        __syncthreads();
    }
}

uint32_t batch_block_threads() { return kBatchThreads; }

hipError_t batch_occupancy(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch, (int)kBatchThreads, 0);
}

hipError_t launch_batch(const BatchItem* items, const uint32_t* order, BatchHeader* hdr, uint32_t grid,
                        hipStream_t s) {
    if (grid == 0) return hipSuccess;
    k_batch<<<grid, kBatchThreads, 0, s>>>(items, order, hdr);
    return hipGetLastError();
}

}  // namespace ising
