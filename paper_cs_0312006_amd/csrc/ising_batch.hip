// Workgroup-resident sweeps for many independent lattices in one launch.
//
// Each workgroup takes the next lattice from a device work queue (the host
// orders the queue by work, largest first) and runs all of that lattice's
// sweeps itself: colour 0 of sweep t, a workgroup barrier, colour 1, a
// barrier, then the sweep's (B, M) (Section 2.2's consecutive black and
// white passes). The grid is sized to the resident capacity of the chip, so
// the kernel is persistent: no workgroup waits on another.
//
// Where a lattice lives while it is swept:
//   - lattices whose two colour planes fit this workgroup's LDS at one bit
//     per site (sides up to 1072) are converted to bits, swept there for all
//     their sweeps and converted back (the bit-packed path below): h = 0
//     lattices whenever the host asks for it, h != 0 lattices when they do
//     not fit as bytes;
//   - other lattices of at most 64 KiB are copied to LDS as bytes;
//   - the rest are swept in place in global memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_bits.hpp"
#include "ising_device.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr uint32_t kBatchThreads = 1024;

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

// The bit layout and the word update are those of ising_bits.hpp.

// Colour pass c of sweep t over the bit planes at lat (plane c at c * L * Wr).
template <bool OBS, bool GENERAL>
__device__ __forceinline__ void bits_pass(uint32_t* __restrict__ lat, const BitsLattice& bl, uint32_t c,
                                          uint32_t t, uint32_t k0, uint32_t k1, uint32_t& mis, uint32_t& ups) {
    const uint32_t L = bl.L, Wr = bl.Wr, Hw = bl.Hw;
    uint32_t* own_p = lat + c * L * Wr;
    const uint32_t* oth_p = lat + (1u - c) * L * Wr;
    const uint32_t rs = blockDim.x / Wr;  // rows per step
    const uint32_t tid = threadIdx.x;
    if (tid >= rs * Wr) return;
    const uint32_t k = tid % Wr;
    const bool last = k + 1 == Wr;
    const uint32_t valid = last ? bl.last_valid : 0xffffffffu;
    const uint32_t top = last ? bl.hb : 31u;
    const uint32_t kn = last ? 0u : k + 1;       // next word of the row (wrapping)
    const uint32_t kp = k == 0 ? Wr - 1 : k - 1;  // previous word of the row (wrapping)
    const uint32_t top_p = k == 0 ? bl.hb : 31u;  // last valid bit of the previous word
    // row i's word offset, and its first quad, stepped rather than multiplied
    uint32_t i = tid / Wr;
    uint32_t ro = i * Wr, q0 = i * Hw + 8u * k;
    const uint32_t ro_step = rs * Wr, q_step = rs * Hw, wrap = L * Wr;
    for (; i < L; i += rs, ro += ro_step, q0 += q_step) {
        const uint32_t rou = i == 0 ? wrap - Wr : ro - Wr;
        const uint32_t rod = i + 1 == L ? 0u : ro + Wr;
        const uint32_t own = own_p[ro + k];
        const uint32_t U = oth_p[rou + k];
        const uint32_t D = oth_p[rod + k];
        const uint32_t O = oth_p[ro + k];
        const uint32_t On = oth_p[ro + kn];
        const uint32_t Op = oth_p[ro + kp];
        const uint32_t S = bits_same_row(O, On, Op, top, top_p, valid, (i + c) & 1u);
        const uint32_t reject = bits_reject<GENERAL>(bl, own, U, D, O, S, q0, t, c, k0, k1);
        const uint32_t nw = own ^ (valid & ~reject);
        own_p[ro + k] = nw;
        if (OBS) {
            // bonds of this colour-1 word, all final now, that disagree (bits
            // past the row's end are zero in every operand)
            mis += __builtin_popcount(nw ^ U) + __builtin_popcount(nw ^ D) + __builtin_popcount(nw ^ O) +
                   __builtin_popcount(nw ^ S);
        }
        ups += __builtin_popcount(nw);
    }
}

// Convert plane bytes (0 / 1) of global memory to bit words in LDS, or back.
__device__ __forceinline__ void bits_load(uint32_t* __restrict__ lat, const BatchItem& it, uint32_t Wr) {
    const uint32_t L = it.L, Hw = it.Hw;
    const uint32_t words = L * Wr;
    for (uint32_t w = threadIdx.x; w < 2u * words; w += blockDim.x) {
        const uint32_t c = w >= words ? 1u : 0u;
        const uint32_t r = w - c * words;
        const uint32_t i = r / Wr, k = r - i * Wr;
        const global_u32* g = as_global(c ? it.p1 : it.p0) + (size_t)i * Hw + 8u * k;
        uint32_t v = 0;
        for (uint32_t j = 0; j < 8u && 8u * k + j < Hw; ++j) {
            // bytes b0..b3 (0 / 1) -> bits 24..27, then to bits 4 j .. 4 j + 3
            v |= ((g[j] * 0x01020408u) >> 24) << (4u * j);
        }
        lat[w] = v;
    }
}

__device__ __forceinline__ void bits_store(const uint32_t* __restrict__ lat, const BatchItem& it, uint32_t Wr) {
    const uint32_t L = it.L, Hw = it.Hw;
    const uint32_t words = L * Wr;
    for (uint32_t w = threadIdx.x; w < 2u * words; w += blockDim.x) {
        const uint32_t c = w >= words ? 1u : 0u;
        const uint32_t r = w - c * words;
        const uint32_t i = r / Wr, k = r - i * Wr;
        global_u32* g = as_global(c ? it.p1 : it.p0) + (size_t)i * Hw + 8u * k;
        const uint32_t v = lat[w];
        for (uint32_t j = 0; j < 8u && 8u * k + j < Hw; ++j) {
            // 4 bits -> bytes 0..3 (bit b to bit 8 b, then keep bit 0 of each byte)
            g[j] = (((v >> (4u * j)) & 0xfu) * 0x00204081u) & 0x01010101u;
        }
    }
}

__device__ __forceinline__ BitsLattice bits_setup(const BatchItem& it) {
    return bits_lattice(it.table, it.L, it.Hw, it.bits);
}

// All sweeps of one bit-packed lattice (already in LDS at lat).
template <bool GENERAL>
__device__ void run_bits(uint32_t* __restrict__ lat, const BatchItem& it, uint32_t (*part)[kMaxWaves][2]) {
    const BitsLattice bl = bits_setup(it);
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t nwaves = blockDim.x >> 6;
    const int64_t N = (int64_t)it.L * it.L;
    auto flush = [&](uint32_t first, uint32_t count) {
        if (threadIdx.x < count) {
            const uint32_t slot = (first + threadIdx.x) % kFlush;
            int64_t sm = 0, su = 0;
            for (uint32_t w = 0; w < nwaves; ++w) {
                sm += part[slot][w][0];
                su += part[slot][w][1];
            }
            // every bond joins colour 0 to colour 1 and was counted once
            it.series[2 * (first + threadIdx.x)] = 2 * N - 2 * sm;
            it.series[2 * (first + threadIdx.x) + 1] = 2 * su - N;
        }
    };
    for (uint32_t s = 0; s < it.n; ++s) {
        const uint32_t t = it.t0 + s;
        uint32_t mis = 0, ups = 0;
        bits_pass<false, GENERAL>(lat, bl, 0u, t, it.k0, it.k1, mis, ups);
        __syncthreads();
        bits_pass<true, GENERAL>(lat, bl, 1u, t, it.k0, it.k1, mis, ups);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            mis += __shfl_xor(mis, off, 64);
            ups += __shfl_xor(ups, off, 64);
        }
        if (lane == 0) {
            part[s % kFlush][wv][0] = mis;
            part[s % kFlush][wv][1] = ups;
        }
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

// Every sweep of one lattice, by the whole workgroup: bit-packed in LDS,
// as bytes in LDS, or in global memory (see the resident plan's notes).
__device__ __forceinline__ void batch_one(const BatchItem& it, LdsTable& lt, uint32_t* lat,
                                          uint32_t (*red)[kMaxWaves][2]) {
    load_table(lt, it.table);
    __syncthreads();
    const uint32_t plane_words = it.L * it.Hw;
    const uint32_t bit_words = it.L * ((it.Hw + 7u) / 8u);
    if (it.bits && 2u * bit_words * 4u <= kBatchBitsLdsBytes && it.n > 0) {
        bits_load(lat, it, (it.Hw + 7u) / 8u);
        __syncthreads();
        if (it.bits == 3u) run_bits<true>(lat, it, red);
        else run_bits<false>(lat, it, red);
        __syncthreads();
        bits_store(lat, it, (it.Hw + 7u) / 8u);
    } else if (2u * plane_words * 4u <= kBatchLdsBytes && it.n > 0) {
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
}

__global__ void __launch_bounds__(kBatchThreads) k_batch(const BatchItem* __restrict__ items,
                                                         const uint32_t* __restrict__ order, BatchHeader* hdr) {
    __shared__ LdsTable lt;
    __shared__ uint32_t s_slot;
    __shared__ uint32_t red[kFlush][kMaxWaves][2];
    // the LDS copy of the lattice being swept (bytes or bits)
    __shared__ uint32_t lat[kBatchBitsLdsBytes / 4];
    const uint32_t count = hdr->count;
    for (;;) {
        if (threadIdx.x == 0) s_slot = atomicAdd(&hdr->head, 1u);
        __syncthreads();
        // the same for every thread: keep it (and the item's fields) scalar
        const uint32_t slot = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_slot);
        if (slot >= count) break;
        batch_one(items[order[slot]], lt, lat, red);
        // everyone has read s_slot and the table before they are replaced
        __syncthreads();
    }
}

// One lattice whose descriptor is the kernel argument: the resident plan of
// a single context, with no descriptor staging, work queue or idle
// workgroups.
__global__ void __launch_bounds__(kBatchThreads) k_batch_one(const BatchItem it) {
    __shared__ LdsTable lt;
    __shared__ uint32_t red[kFlush][kMaxWaves][2];
    __shared__ uint32_t lat[kBatchBitsLdsBytes / 4];
    batch_one(it, lt, lat, red);
}

uint32_t bits_mode(const AcceptTable& at) {
    const uint64_t one = (uint64_t)1 << 32;
    auto thr = [&](uint32_t code) { return ((uint64_t)at.thr_hi[code] << 32) | at.thr_lo[code]; };
    uint64_t T[5];
    for (uint32_t m = 0; m < 5; ++m) {
        T[m] = thr(8u + (4u - m));    // up spin, 4 - m up neighbours
        if (thr(m) != T[m]) return 3;  // down spin, m up neighbours
    }
    if (T[2] != one) return 3;
    if (T[3] == one && T[4] == one) return 1;
    if (T[0] == one && T[1] == one) return 2;
    return 3;
}

bool bits_fit(uint32_t L) {
    if (L % 8u != 0u) return false;
    const uint64_t wr = (L / 8u + 7u) / 8u;
    return 2ull * L * wr * 4ull <= kBatchBitsLdsBytes;
}

bool bytes_fit(uint32_t L) {
    const uint64_t plane_words = (uint64_t)L * (L / 8u);
    return 2ull * plane_words * 4ull <= kBatchLdsBytes;
}

uint32_t batch_block_threads() { return kBatchThreads; }

hipError_t batch_occupancy(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch, (int)kBatchThreads, 0);
}

// Word copy from pinned host memory (read over the bus) to device memory.
__global__ void __launch_bounds__(256) k_stage_copy(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                                    uint32_t words) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < words; k += gridDim.x * blockDim.x) dst[k] = src[k];
}

hipError_t launch_stage_copy(void* dst, const void* host_src, size_t bytes, hipStream_t s) {
    const uint32_t words = (uint32_t)(bytes / 4u);
    if (words == 0) return hipSuccess;
    const uint32_t blocks = min((words + 255u) / 256u, 64u);
    k_stage_copy<<<blocks, 256, 0, s>>>(static_cast<uint32_t*>(dst), static_cast<const uint32_t*>(host_src), words);
    return hipGetLastError();
}

hipError_t launch_batch_one(const BatchItem& it, hipStream_t s) {
    k_batch_one<<<1, kBatchThreads, 0, s>>>(it);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchItem* items, const uint32_t* order, BatchHeader* hdr, uint32_t grid,
                        hipStream_t s) {
    if (grid == 0) return hipSuccess;
    k_batch<<<grid, kBatchThreads, 0, s>>>(items, order, hdr);
    return hipGetLastError();
}

}  // namespace ising
