// HIP kernels of the gfx950 site-percolation engine (Section 2.3 of Tomov
// et al. 2003): porosity draw, then invasion of the medium from the source.
//
// The paper's GPU program spreads the cluster by one pass over the whole
// lattice per invasion step, so a medium whose cluster needs D steps costs
// D full passes. Here the arrival pass of every site (its breadth-first
// distance from the source through pores) is computed tile by tile: one
// wave owns a 64 x 64 tile, lane r holding tile row r as 64 arrival values
// and as 64-bit masks, and brings the tile to its fixed point (arrival =
// min(arrival, 1 + min over the four neighbours) for every pore) by
// breadth-first levels over the masks, a handful of bit operations per row
// and level; a tile is revisited only when a neighbouring tile changed the
// sites on their shared edge. Launch k admits arrival values up to 32 (k + 1)
// only (a tile with sites one level beyond stays queued), so the front is
// swept roughly in breadth-first order and tiles are seldom revisited.
// Values only ever decrease and every read value is an upper bound of the
// true distance, so the unique fixed point, reached when no tile is queued,
// is exact whatever the timing of concurrent reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "perc_launch.hpp"

namespace perc {

namespace {

constexpr uint32_t kBoundStep = 32;  // arrival passes admitted per launch (32 beat 64, 128 and 256)
#ifndef PERC_MAX_LEVELS
#define PERC_MAX_LEVELS 64
#endif
// Breadth-first levels per tile visit: a launch lasts as long as its
// longest visit, so a visit that would run longer stops and resumes in the
// next launch.
constexpr uint32_t kMaxLevels = PERC_MAX_LEVELS;

// DPP controls (GFX9): whole-wave shift by one lane.
constexpr int kDppWaveShl1 = 0x130;  // lane l reads lane l+1
constexpr int kDppWaveShr1 = 0x138;  // lane l reads lane l-1

// Row mask of the tile row above (lane l gets lane l-1's; lane 0 gets `edge`)
// and below (lane l gets lane l+1's; lane 63 gets `edge`).
__device__ __forceinline__ uint64_t mask_from_above(uint64_t v, uint64_t edge) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)edge, (int)(uint32_t)v, kDppWaveShr1,
                                                              0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(edge >> 32), (int)(uint32_t)(v >> 32),
                                                              kDppWaveShr1, 0xf, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t mask_from_below(uint64_t v, uint64_t edge) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)edge, (int)(uint32_t)v, kDppWaveShl1,
                                                              0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(edge >> 32), (int)(uint32_t)(v >> 32),
                                                              kDppWaveShl1, 0xf, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

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

// One relaxation launch (number k of the run, admitting arrival values up
// to `bound`, the previous launch's bound being `lo`): a wave per listed
// tile.
//
// A visit takes the tile's halo (the sites just outside its four sides) as
// sources and computes breadth-first levels from the lowest level d0 at
// which anything can change: lo, or a halo value h below it that would
// lower the site next to it (h + 1 less than that site's value). Every
// stored value is the fixed point of an earlier visit for levels up to lo
// and halo values only decrease, so below d0 nothing changes and the pores
// with stored values up to d0 are sources too. From d0, A holds the pores
// reached by level d; level d + 1 adds the pores next to A or to a halo
// site of value at most d. A stored value above d0 came from sources no
// closer than today's, so the levels reach that site at or below it: it is
// written only where the level is lower. Levels where nothing is added
// jump to the next halo value. At `bound` the visit stops; a pore that
// level bound + 1 would reach keeps the tile queued for the next launch.
__global__ void __launch_bounds__(kRelaxThreads) k_perc_relax(const Medium* __restrict__ media, WorkLists w,
                                                              uint32_t pin, uint32_t lin, uint32_t lout,
                                                              uint32_t lclr, uint32_t lo, uint32_t bound) {
    __shared__ uint32_t vs[kTile][kTile + 1];  // the stored values of the tile being visited
    if (blockIdx.x == 0 && threadIdx.x == 0) w.len[lclr] = 0u;
    const uint32_t n = w.len[lin];
    const uint32_t r = threadIdx.x;  // the tile row of this lane
    for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
        const uint2 ent = w.list[pin][e];
        // the entry is the same for the whole wave: keep it scalar
        const uint32_t m = (uint32_t)__builtin_amdgcn_readfirstlane((int)ent.x);
        const uint32_t tile = (uint32_t)__builtin_amdgcn_readfirstlane((int)ent.y);
        const Medium& md = media[m];
        ising::global_u32* const arr = ising::as_global(md.arr);
        const uint32_t L = md.L, n_tx = md.n_tx, n_ty = md.n_ty;
        uint32_t* q_in = pin ? md.queued[1] : md.queued[0];
        const uint32_t ty = tile / n_tx, tx = tile - ty * n_tx;
        const uint32_t i0 = ty * kTile, j0 = tx * kTile;
        if (r == 0) q_in[tile] = 0u;
        // rows and columns of the tile inside the lattice; every address
        // below is clamped into the lattice, and a value read for a site
        // outside it is turned into solid (OR with all ones, so that every
        // load's result is used and all of them are issued together)
        const uint32_t nrow = min(kTile, L - i0), ncol = min(kTile, L - j0);
        const bool row_in = r < nrow, col_in = r < ncol;  // lane r as a row, and as a column
        const uint32_t gi = i0 + (row_in ? r : nrow - 1);
        ising::global_u32* const rowp = arr + (size_t)gi * L + j0;
        const uint32_t out_row = row_in ? 0u : kSolid;
        // the tile's stored values into LDS row by row, lane r taking
        // column r (each load reads 64 consecutive words), then each lane's
        // row back out of LDS; the padded row keeps both directions free of
        // bank conflicts. The copy stays for the levels, which read it where
        // a site is reached, to skip values that do not drop.
        const uint32_t jc = j0 + (col_in ? r : ncol - 1);  // lane r's column, clamped
        const uint32_t out_col = col_in ? 0u : kSolid;
#pragma unroll 16
        for (uint32_t rr = 0; rr < kTile; ++rr)
            vs[rr][r] = arr[(size_t)(i0 + min(rr, nrow - 1)) * L + jc] | (rr < nrow ? out_col : kSolid);
        __builtin_amdgcn_wave_barrier();
        uint32_t v[kTile];
#pragma unroll
        for (uint32_t c = 0; c < kTile; ++c) v[c] = vs[r][c];
        const bool has_top = i0 > 0, has_bot = i0 + kTile < L, has_lft = j0 > 0, has_rgt = j0 + kTile < L;
        const uint32_t top = arr[(size_t)(has_top ? i0 - 1 : i0) * L + jc] | (has_top ? out_col : kSolid);
        const uint32_t bot = arr[(size_t)(has_bot ? i0 + kTile : i0) * L + jc] | (has_bot ? out_col : kSolid);
        const uint32_t first = vs[0][r], last = vs[nrow - 1][r];  // tile row 0 and the last, column r
        const uint32_t lft = rowp[has_lft ? -1 : 0] | (has_lft ? out_row : kSolid);
        const uint32_t rgt = rowp[has_rgt ? (int)kTile : 0] | (has_rgt ? out_row : kSolid);
        // the row's pores
        uint64_t P = 0;
#pragma unroll
        for (uint32_t c = 0; c < kTile; ++c) P |= (uint64_t)(v[c] != kSolid) << c;
        // the lowest level at which the halo lowers a site next to it
        // (solid and unreached sites are >= kUnreached and lower nothing)
        uint32_t d0 = lo;
        if (top < kUnreached && first != kSolid && top + 1u < first) d0 = min(d0, top);
        if (bot < kUnreached && last != kSolid && bot + 1u < last) d0 = min(d0, bot);
        if (lft < kUnreached && v[0] != kSolid && lft + 1u < v[0]) d0 = min(d0, lft);
        if (rgt < kUnreached && v[kTile - 1] != kSolid && rgt + 1u < v[kTile - 1]) d0 = min(d0, rgt);
        d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_min_u32(d0));
        d0 = min(d0, md.resume[tile]);  // where an earlier visit stopped short
        uint64_t A = 0, F = 0;  // F: pores with a stored value above d0
#pragma unroll
        for (uint32_t c = 0; c < kTile; ++c) {
            A |= (uint64_t)(v[c] <= d0) << c;
            F |= (uint64_t)(v[c] > d0 && v[c] < kUnreached) << c;
        }
        // halo sites at or below level d, as tile-row bits
        auto halo = [&](uint32_t d) {
            const uint64_t T = __ballot(top <= d), B = __ballot(bot <= d);
            uint64_t h = (lft <= d ? 1ull : 0ull) | (rgt <= d ? 1ull << (kTile - 1) : 0ull);
            if (r == 0) h |= T;
            if (r == nrow - 1) h |= B;
            return h;
        };
        auto grow = [&](uint64_t a, uint32_t d) {
            return a | (a << 1) | (a >> 1) | mask_from_above(a, 0) | mask_from_below(a, 0) | halo(d);
        };
        uint64_t W = 0;
        uint32_t levels = 0;
        const uint32_t stop = bound - d0 > kMaxLevels ? d0 + kMaxLevels : bound;
        uint32_t d = d0;
        while (d < stop) {
            const uint64_t nw = grow(A, d) & P & ~A;
            uint64_t x = nw & ~F;  // unreached until now: always written
            W |= x;
            while (x) {
                const uint32_t c = (uint32_t)__builtin_ctzll(x);
                x &= x - 1;
                rowp[c] = d + 1u;
            }
            x = nw & F;
            while (x) {
                const uint32_t c = (uint32_t)__builtin_ctzll(x);
                x &= x - 1;
                if (vs[r][c] > d + 1u) {
                    rowp[c] = d + 1u;
                    W |= 1ull << c;
                }
            }
            A |= nw;
            ++levels;
            ++d;
            if (!wave_any(nw != 0)) {
                // nothing added: the next level that can add a site is a
                // halo value at or above d
                uint32_t nx = bound;
                nx = min(nx, top >= d ? top : kSolid);
                nx = min(nx, bot >= d ? bot : kSolid);
                nx = min(nx, lft >= d ? lft : kSolid);
                nx = min(nx, rgt >= d ? rgt : kSolid);
                d = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_min_u32(nx));
            }
        }
        // stopped short of bound: the values are the fixed point up to d,
        // and the tile's next visit starts there; otherwise, pores that
        // level bound + 1 would reach keep the tile queued
        const bool short_stop = d < bound;
        if (r == 0 && (short_stop || md.resume[tile] != kSolid)) md.resume[tile] = short_stop ? d : kSolid;
        const bool later = short_stop || wave_any((grow(A, bound) & P & ~A) != 0);
        if (r == 0) {
            atomicAdd(&md.stats->visits, 1ull);
            atomicAdd(&md.stats->iterations, (unsigned long long)levels);
        }
        const bool top_ch = wave_any(r == 0 && W != 0);
        const bool bot_ch = wave_any(r == kTile - 1 && W != 0);
        const bool lft_ch = wave_any((W & 1u) != 0);
        const bool rgt_ch = wave_any(((W >> (kTile - 1)) & 1u) != 0);
        if (r == 0) {
            const uint32_t par = pin ^ 1u;
            uint32_t* q_out = par ? md.queued[1] : md.queued[0];
            if (top_ch && ty > 0) push(w, q_out, par, lout, m, tile - n_tx);
            if (bot_ch && ty + 1 < n_ty) push(w, q_out, par, lout, m, tile + n_tx);
            if (lft_ch && tx > 0) push(w, q_out, par, lout, m, tile - 1);
            if (rgt_ch && tx + 1 < n_tx) push(w, q_out, par, lout, m, tile + 1);
            if (later) push(w, q_out, par, lout, m, tile);
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
    auto cap = [](uint64_t b) { return b >= kUnreached ? kUnreached - 1 : (uint32_t)b; };
    const uint32_t bound = cap((k + 1) * (uint64_t)kBoundStep), lo = cap(k * (uint64_t)kBoundStep);
    k_perc_relax<<<grid, kRelaxThreads, 0, s>>>(media, w, (uint32_t)(k % 2), (uint32_t)(k % 3),
                                                (uint32_t)((k + 1) % 3), (uint32_t)((k + 2) % 3), lo, bound);
    return hipGetLastError();
}

hipError_t launch_finish(uint32_t* arr, uint32_t L, Stats* stats, hipStream_t s) {
    const uint64_t N = (uint64_t)L * L;
    k_perc_finish<<<grid_for(N), kThreads, 0, s>>>(arr, L, N, stats);
    return hipGetLastError();
}

}  // namespace perc
