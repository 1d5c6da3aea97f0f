// Stepped multi-lattice sweeps, one pass per colour: one launch per colour
// pass covers the chunks of every lattice in a work list, so each lattice,
// small or large, is spread over the whole GPU (the resident batch kernel
// gives each lattice one workgroup instead). Used by the stepped batch plan
// when some side is not a multiple of 16 (otherwise the one-pass walk of
// ising_multi_fused.hip runs).
//
// Work list: items (BatchItem, as for the resident kernel) and, per item,
// the first of its virtual blocks; a launch strides over all virtual
// blocks. A graph of G sweeps (2 G passes) is captured once; its first node
// advances the sweep base by G, so replaying it ceil(n / G) times runs n
// sweeps with no host work between replays. Items with fewer sweeps than
// the others simply skip the passes beyond their count. Each virtual block
// writes its (B, M) partial of a sweep, and the replay's last node sums them
// per item into the series.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr uint32_t kMultiThreads = 256;

template <int CW>
__device__ __forceinline__ void multi_chunk(const LdsTable& lt, const BatchItem& it, uint32_t c, uint32_t t,
                                            uint32_t idx, bool obs, bool exact, uint32_t& sad, uint32_t& ups) {
    global_u32* own = as_global(c ? it.p1 : it.p0);
    const global_u32* oth = as_global(c ? it.p0 : it.p1);
    const uint32_t L = it.L, Hw = it.Hw;
    const uint32_t per_row = Hw / CW;
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
        const uint32_t f = exact ? flip_mask<true>(lt, W[w], n, r) : flip_mask<false>(lt, W[w], n, r);
        const uint32_t Wn = W[w] ^ f;
        own[row + wc + w] = Wn;
        if (obs) {
            sad = sad_misaligned(Wn, n, sad);
            ups += __builtin_popcount(Wn) + __builtin_popcount(O[w]);
        }
    }
}

}  // namespace

__global__ void __launch_bounds__(kMultiThreads) k_multi_advance(MultiHeader* hdr, uint32_t g) {
    if (threadIdx.x == 0 && blockIdx.x == 0) hdr->s_base += g;
}

// Colour pass c of sweep s_base + s for every item with that sweep pending.
__global__ void __launch_bounds__(kMultiThreads) k_multi_pass(const BatchItem* __restrict__ items,
                                                              const uint32_t* __restrict__ vb_start,
                                                              const MultiHeader* __restrict__ hdr, uint32_t s,
                                                              uint32_t c) {
    __shared__ LdsTable lt;
    __shared__ int64_t acc[2][kMultiThreads / 64];
    const uint32_t n_items = hdr->n_items, total = hdr->total_vblocks;
    const uint32_t sweep = hdr->s_base + s;
    for (uint32_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
        uint32_t lo = 0, hi = n_items;  // last item whose first virtual block is <= vb
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (vb_start[mid] <= vb) lo = mid;
            else hi = mid;
        }
        const BatchItem& it = items[lo];
        if (sweep >= it.n) continue;  // uniform over the block
        __syncthreads();              // previous virtual block is done with lt and acc
        load_table(lt, it.table);
        __syncthreads();
        const uint32_t t = it.t0 + sweep;
        const uint32_t local = vb - vb_start[lo];
        const uint32_t total_chunks = it.L * (it.Hw / it.cw);
        const uint32_t first = local * kMultiThreads * kMultiChunksPerThread;
        uint32_t sad = 0, ups = 0, nw = 0;
        for (uint32_t k = 0; k < kMultiChunksPerThread; ++k) {
            const uint32_t idx = first + k * kMultiThreads + threadIdx.x;
            if (idx >= total_chunks) break;
            if (it.cw == 4) multi_chunk<4>(lt, it, c, t, idx, c == 1, it.exact != 0, sad, ups);
            else if (it.cw == 2) multi_chunk<2>(lt, it, c, t, idx, c == 1, it.exact != 0, sad, ups);
            else multi_chunk<1>(lt, it, c, t, idx, c == 1, it.exact != 0, sad, ups);
            nw += it.cw;
        }
        if (c == 1) {
            int64_t b = 16 * (int64_t)nw - 2 * (int64_t)sad;
            int64_t m = 2 * (int64_t)ups - 8 * (int64_t)nw;
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
                for (uint32_t w = 0; w < kMultiThreads / 64; ++w) {
                    sb += acc[0][w];
                    sm += acc[1][w];
                }
                // this block's partial; the replay's last node sums them
                int64_t* p = hdr->part + 2ull * ((uint64_t)s * total + vb);
                p[0] = sb;
                p[1] = sm;
            }
        }
    }
}

uint32_t multi_vblocks(uint32_t L, uint32_t cw) {
    const uint64_t chunks = (uint64_t)L * (L / 8u / cw);
    const uint64_t per = (uint64_t)kMultiThreads * kMultiChunksPerThread;
    return (uint32_t)((chunks + per - 1) / per);
}

hipError_t launch_multi_graph_body(const BatchItem* items, const uint32_t* vb_start, MultiHeader* hdr,
                                   uint32_t sweeps_per_replay, uint32_t grid, hipStream_t s) {
    k_multi_advance<<<1, 64, 0, s>>>(hdr, sweeps_per_replay);
    for (uint32_t k = 0; k < sweeps_per_replay; ++k) {
        k_multi_pass<<<grid, kMultiThreads, 0, s>>>(items, vb_start, hdr, k, 0u);
        k_multi_pass<<<grid, kMultiThreads, 0, s>>>(items, vb_start, hdr, k, 1u);
    }
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    return launch_multi_reduce(items, vb_start, hdr, sweeps_per_replay, grid, s);
}

}  // namespace ising
