// HIP kernels of the gfx950 site-percolation engine (Section 2.3 of Tomov
// et al. 2003): porosity draw, then invasion of the medium from the source.
//
// The paper's GPU program spreads the cluster by one pass over the whole
// lattice per invasion step, so a medium whose cluster needs D steps costs
// D full passes. Here the arrival pass of every site (its breadth-first
// distance from the source through pores) is computed directly by
// relaxation, arrival = min(arrival, 1 + min over the four neighbours), in
// 64 x 64 tiles held in LDS: a workgroup relaxes its tile to a local fixed
// point (many steps per HBM round trip), and a tile is revisited only when
// a neighbouring tile changed the sites on their shared edge. Launch k
// admits arrival values up to 32 (k + 1) only (larger improvements wait in
// their tile, which stays queued), so the front is swept roughly in
// breadth-first order and tiles are seldom recomputed. Values only ever
// decrease and every read value is an upper bound of the true distance, so
// the unique fixed point, reached when no tile is queued, is exact
// whatever the timing of concurrent reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "perc_launch.hpp"

namespace perc {

namespace {

constexpr uint32_t kSide = kTile + 2;          // tile plus one-site halo
constexpr uint32_t kMaxIters = 1u << 14;       // per visit; a tile still changing is queued again
#ifndef PERC_BOUND_STEP
#define PERC_BOUND_STEP 32
#endif
constexpr uint32_t kBoundStep = PERC_BOUND_STEP;  // arrival passes admitted per launch

// LDS accesses of the relaxation: other waves update neighbouring rows
// concurrently, so reads and writes are relaxed atomics (plain ds_read /
// ds_write on the hardware) and may see either value.
__device__ __forceinline__ uint32_t lds_ld(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// New arrival of a site from its current value and its four neighbours
// (solid neighbours hold 0xffffffff, unreached ones kUnreached, and both
// give kUnreached + 1 > any reachable value). Improvements beyond this
// launch's bound are left for a later launch and flagged as pending.
__device__ __forceinline__ uint32_t relax1(uint32_t cur, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                           uint32_t bound, bool& pend) {
    uint32_t m = min(min(a, b), min(c, d));
    m = min(m, kUnreached) + 1u;
    if (m < cur) {
        if (m <= bound) return m;
        pend = true;
    }
    return cur;
}

__device__ __forceinline__ void push(const WorkLists& w, uint32_t* queued, uint32_t par, uint32_t lout, uint32_t m,
                                     uint32_t tile) {
    if (atomicExch(&queued[tile], 1u) == 0u) {
        const uint32_t pos = atomicAdd(&w.len[lout], 1u);
        w.list[par][pos] = make_uint2(m, tile);
    }
}

}  // namespace

// Porosity draw and initial arrival: one Philox call per group of four
// row-major sites. Counts pores into st->pores.
__global__ void __launch_bounds__(kThreads) k_perc_draw(uint8_t* pore, uint32_t* arr, uint32_t L, uint64_t N,
                                                        uint64_t pthr, uint32_t k0, uint32_t k1, uint32_t source,
                                                        uint32_t i0, uint32_t j0, Stats* st) {
    const uint64_t groups = (N + 3) / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t cnt = 0;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < groups; g += stride) {
        const uint4 r = ising::philox((uint32_t)g, 0u, 0u, 2u, k0, k1);
        const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b) {
            const uint64_t ord = 4 * g + b;
            if (ord >= N) break;
            const uint32_t p = (uint64_t)u[b] < pthr ? 1u : 0u;
            const uint32_t i = (uint32_t)(ord / L), j = (uint32_t)(ord - (uint64_t)i * L);
            const bool src = source == 0u ? i == 0u : (i == i0 && j == j0);
            pore[ord] = (uint8_t)p;
            arr[ord] = p ? (src ? 0u : kUnreached) : kSolid;
            cnt += p;
        }
    }
    const uint32_t s = ising::wave_sum_u32(cnt);
    if ((threadIdx.x & 63u) == 0u && s) atomicAdd(&st->pores, (unsigned long long)s);
}

__global__ void k_perc_reset(WorkLists w) {
    if (threadIdx.x < 3) w.len[threadIdx.x] = 0u;
}

// Medium m's source tiles, appended to work list 0.
__global__ void __launch_bounds__(kThreads) k_perc_seed(WorkLists w, const Medium* media, uint32_t m, uint32_t n_tx,
                                                        uint32_t source, uint32_t i0, uint32_t j0) {
    uint32_t* q = media[m].queued[0];
    if (source == 0u) {
        for (uint32_t t = threadIdx.x; t < n_tx; t += blockDim.x) {
            q[t] = 1u;
            w.list[0][atomicAdd(&w.len[0], 1u)] = make_uint2(m, t);
        }
    } else if (threadIdx.x == 0) {
        const uint32_t t = (i0 / kTile) * n_tx + j0 / kTile;
        q[t] = 1u;
        w.list[0][atomicAdd(&w.len[0], 1u)] = make_uint2(m, t);
    }
}

// One relaxation launch (number k of the run): relax every listed tile to
// its local fixed point, write back what changed, queue the neighbours
// whose shared edge changed.
__global__ void __launch_bounds__(kThreads) k_perc_relax(const Medium* __restrict__ media, WorkLists w, uint32_t pin,
                                                         uint32_t lin, uint32_t lout, uint32_t lclr, uint32_t bound) {
    __shared__ uint32_t d[kSide * kSide];
    if (blockIdx.x == 0 && threadIdx.x == 0) w.len[lclr] = 0u;
    const uint32_t n = w.len[lin];
    const uint32_t x = threadIdx.x & (kTile - 1);
    const uint32_t y0 = (threadIdx.x / kTile) * kStrip;
    // row phase: row hr, sites hx0 .. hx0 + 15 (a wave covers 64 rows of
    // one column segment; the 66-word row pitch spreads them over banks)
    const uint32_t hr = threadIdx.x & (kTile - 1);
    const uint32_t hx0 = (threadIdx.x / kTile) * kStrip;
    for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
        const uint2 ent = w.list[pin][e];
        // the entry is the same for the whole workgroup: keep it scalar
        const uint32_t m = (uint32_t)__builtin_amdgcn_readfirstlane((int)ent.x);
        const uint32_t tile = (uint32_t)__builtin_amdgcn_readfirstlane((int)ent.y);
        const Medium& md = media[m];
        uint32_t* const arr = md.arr;
        const uint32_t L = md.L, n_tx = md.n_tx, n_ty = md.n_ty;
        uint32_t* q_in = pin ? md.queued[1] : md.queued[0];
        const uint32_t ty = tile / n_tx, tx = tile - ty * n_tx;
        const int64_t gi0 = (int64_t)ty * kTile - 1, gj0 = (int64_t)tx * kTile - 1;  // halo origin
        if (threadIdx.x == 0) q_in[tile] = 0u;
        for (uint32_t k = threadIdx.x; k < kSide * kSide; k += blockDim.x) {
            const uint32_t yy = k / kSide, xx = k - yy * kSide;
            const int64_t gi = gi0 + yy, gj = gj0 + xx;
            uint32_t v = kSolid;
            if (gi >= 0 && gj >= 0 && gi < (int64_t)L && gj < (int64_t)L) v = arr[(size_t)gi * L + (size_t)gj];
            d[k] = v;
        }
        __syncthreads();
        uint32_t orig[kStrip];
#pragma unroll
        for (uint32_t r = 0; r < kStrip; ++r) orig[r] = d[(y0 + r + 1) * kSide + x + 1];
        uint32_t* col = d + x + 1;  // this thread's column; row yy at col[yy * kSide]
        uint32_t iters = 0;
        int go;
        bool pend;
        do {
            bool ch = false;
            pend = false;
            {
                // column strip: LDS rows y0 .. y0 + 17 of column x, own sites
                // 1 .. 16; all reads issued first, the chain then runs in
                // registers, top to bottom and back
                uint32_t c[kStrip + 2], lf[kStrip], rt[kStrip], o[kStrip];
#pragma unroll
                for (uint32_t r = 0; r < kStrip + 2; ++r) c[r] = lds_ld(col + (y0 + r) * kSide);
#pragma unroll
                for (uint32_t r = 0; r < kStrip; ++r) {
                    lf[r] = lds_ld(col + (y0 + 1 + r) * kSide - 1);
                    rt[r] = lds_ld(col + (y0 + 1 + r) * kSide + 1);
                    o[r] = c[r + 1];
                }
#pragma unroll
                for (uint32_t r = 1; r <= kStrip; ++r)
                    if (c[r] != kSolid) c[r] = relax1(c[r], c[r - 1], c[r + 1], lf[r - 1], rt[r - 1], bound, pend);
#pragma unroll
                for (uint32_t r = kStrip; r >= 1; --r)
                    if (c[r] != kSolid) c[r] = relax1(c[r], c[r - 1], c[r + 1], lf[r - 1], rt[r - 1], bound, pend);
#pragma unroll
                for (uint32_t r = 0; r < kStrip; ++r) {
                    if (c[r + 1] != o[r]) {
                        lds_st(col + (y0 + 1 + r) * kSide, c[r + 1]);
                        ch = true;
                    }
                }
            }
            // each site has one writer per phase: its column owner above,
            // its row owner below, so a site's value never goes up
            __syncthreads();
            {
                // row segment: LDS columns hx0 .. hx0 + 17 of row hr + 1, own
                // sites 1 .. 16, left to right and back
                uint32_t* row = d + (hr + 1) * kSide + hx0;
                uint32_t c[kStrip + 2], up[kStrip], dn[kStrip], o[kStrip];
#pragma unroll
                for (uint32_t k = 0; k < kStrip + 2; ++k) c[k] = lds_ld(row + k);
#pragma unroll
                for (uint32_t k = 0; k < kStrip; ++k) {
                    up[k] = lds_ld(row + k + 1 - kSide);
                    dn[k] = lds_ld(row + k + 1 + kSide);
                    o[k] = c[k + 1];
                }
#pragma unroll
                for (uint32_t k = 1; k <= kStrip; ++k)
                    if (c[k] != kSolid) c[k] = relax1(c[k], c[k - 1], c[k + 1], up[k - 1], dn[k - 1], bound, pend);
#pragma unroll
                for (uint32_t k = kStrip; k >= 1; --k)
                    if (c[k] != kSolid) c[k] = relax1(c[k], c[k - 1], c[k + 1], up[k - 1], dn[k - 1], bound, pend);
#pragma unroll
                for (uint32_t k = 0; k < kStrip; ++k) {
                    if (c[k + 1] != o[k]) {
                        lds_st(row + k + 1, c[k + 1]);
                        ch = true;
                    }
                }
            }
            ++iters;
            go = __syncthreads_or(ch);
        } while (go && iters < kMaxIters);
        // pending improvements of the last (unchanging) iteration: revisit
        // the tile in the next launch, whose bound is higher
        const int later = __syncthreads_or(pend);
        if (threadIdx.x == 0) {
            atomicAdd(&md.stats->visits, 1ull);
            atomicAdd(&md.stats->iterations, (unsigned long long)iters);
        }
        bool top = false, bot = false, lft = false, rgt = false;
#pragma unroll
        for (uint32_t r = 0; r < kStrip; ++r) {
            const uint32_t v = d[(y0 + r + 1) * kSide + x + 1];
            if (v != orig[r]) {
                // sites beyond the lattice are solid and never change
                arr[(size_t)(gi0 + 1 + y0 + r) * L + (size_t)(gj0 + 1 + x)] = v;
                top |= (y0 + r) == 0u;
                bot |= (y0 + r) == kTile - 1;
                lft |= x == 0u;
                rgt |= x == kTile - 1;
            }
        }
        top = __syncthreads_or(top);
        bot = __syncthreads_or(bot);
        lft = __syncthreads_or(lft);
        rgt = __syncthreads_or(rgt);
        if (threadIdx.x == 0) {
            const uint32_t par = pin ^ 1u;
            uint32_t* q_out = par ? md.queued[1] : md.queued[0];
            if (top && ty > 0) push(w, q_out, par, lout, m, tile - n_tx);
            if (bot && ty + 1 < n_ty) push(w, q_out, par, lout, m, tile + n_tx);
            if (lft && tx > 0) push(w, q_out, par, lout, m, tile - 1);
            if (rgt && tx + 1 < n_tx) push(w, q_out, par, lout, m, tile + 1);
            if (go || later) push(w, q_out, par, lout, m, tile);  // not yet at its fixed point
        }
    }
}

// Final pass: unreached pores become -1; count the cluster, its largest
// arrival and which lattice edges it touches.
__global__ void __launch_bounds__(kThreads) k_perc_finish(uint32_t* arr, uint32_t L, uint64_t N, Stats* st) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t cnt = 0, mx = 0, edges = 0;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < N; k += stride) {
        const uint32_t v = arr[k];
        if (v == kUnreached) {
            arr[k] = kSolid;
        } else if (v != kSolid) {
            const uint32_t i = (uint32_t)(k / L), j = (uint32_t)(k - (uint64_t)i * L);
            ++cnt;
            mx = max(mx, v);
            edges |= (i == 0u ? 1u : 0u) | (i == L - 1 ? 2u : 0u) | (j == 0u ? 4u : 0u) | (j == L - 1 ? 8u : 0u);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        mx = max(mx, (uint32_t)__shfl_xor(mx, off, 64));
        edges |= (uint32_t)__shfl_xor(edges, off, 64);
    }
    if ((threadIdx.x & 63u) == 0u) {
        if (cnt) atomicAdd(&st->invaded, (unsigned long long)cnt);
        if (mx) atomicMax(&st->max_arrival, mx);
        if (edges) atomicOr(&st->edges, edges);
    }
}

static uint32_t grid_for(uint64_t n) {
    const uint64_t b = (n + kThreads - 1) / kThreads;
    return (uint32_t)(b > 8192 ? 8192 : (b ? b : 1));
}

hipError_t launch_draw(uint8_t* pore, uint32_t* arr, uint32_t L, uint64_t pthr, uint32_t k0, uint32_t k1,
                       uint32_t source, uint32_t i0, uint32_t j0, Stats* stats, hipStream_t s) {
    const uint64_t N = (uint64_t)L * L;
    k_perc_draw<<<grid_for((N + 3) / 4), kThreads, 0, s>>>(pore, arr, L, N, pthr, k0, k1, source, i0, j0, stats);
    return hipGetLastError();
}

hipError_t launch_reset_lists(const WorkLists& w, hipStream_t s) {
    k_perc_reset<<<1, 64, 0, s>>>(w);
    return hipGetLastError();
}

hipError_t launch_seed(const WorkLists& w, const Medium* media, uint32_t m, uint32_t n_tx, uint32_t source,
                       uint32_t i0, uint32_t j0, hipStream_t s) {
    k_perc_seed<<<1, kThreads, 0, s>>>(w, media, m, n_tx, source, i0, j0);
    return hipGetLastError();
}

hipError_t launch_relax(const Medium* media, const WorkLists& w, uint64_t k, uint32_t grid, hipStream_t s) {
    // arrival passes accepted in launch k: up to (k + 1) * kBoundStep, so the
    // invasion front is swept in order, a band per launch, and tiles are
    // rarely revisited with a better value
    const uint64_t b = (k + 1) * (uint64_t)kBoundStep;
    const uint32_t bound = b >= kUnreached ? kUnreached - 1 : (uint32_t)b;
    k_perc_relax<<<grid, kThreads, 0, s>>>(media, w, (uint32_t)(k % 2), (uint32_t)(k % 3), (uint32_t)((k + 1) % 3),
                                           (uint32_t)((k + 2) % 3), bound);
    return hipGetLastError();
}

hipError_t launch_finish(uint32_t* arr, uint32_t L, Stats* stats, hipStream_t s) {
    const uint64_t N = (uint64_t)L * L;
    k_perc_finish<<<grid_for(N), kThreads, 0, s>>>(arr, L, N, stats);
    return hipGetLastError();
}

}  // namespace perc
