// Stepped multi-lattice sweeps with the fused one-pass walk: one launch per
// sweep covers the tiles of every lattice in a work list, so each lattice,
// small or large, is spread over the whole GPU and crosses HBM once per
// sweep (2 bytes per site update, against 3 for a pass per colour).
//
// Each lattice ping-pongs between its two buffers: sweep s of a call reads
// buffer s & 1 of the item (p = the current lattice, q = the other one) and
// writes the other. A wave walks one tile of up to 32 rows (8 or 16 when a
// call has too few tiles to fill the GPU) by 128 words of a plane row (two
// words per lane), exactly as the single-lattice fused kernel does, with
// three differences:
//   - tiles at a lattice's right and bottom edges may be narrower and
//     shorter: lanes past the lattice's last word shadow its last lane
//     (their loads stay in range, nothing of theirs is stored or counted),
//     and that lane takes its right neighbour from the edge word;
//   - a lattice's last column, when at most 32 lanes wide, packs several of
//     its row bands into one wave (see mf_tile_packed and mf_layout);
//   - each tile writes its (B, M) to a partial slot of its own, and the last
//     node of a replay sums them per lattice into the series (no atomics: a
//     lattice of thousands of tiles would serialise them on one address).
// The draws are keyed by (seed, sweep, colour, site) as everywhere else, so
// the result is the same as any other schedule of the same sweeps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_fused_core.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr uint32_t kMfThreads = 256;
constexpr int kMfCW = 2;  // words per lane
constexpr uint32_t kMfTileWords = 64u * kMfCW;

__device__ __forceinline__ uint32_t wrap_row_m(int i, uint32_t L) {
    return (uint32_t)(i < 0 ? i + (int)L : (i >= (int)L ? i - (int)L : i));
}

// Partial (B, M) of one tile of item `it` for its sweep `s` of this call.
__device__ __forceinline__ void mf_tile(const LdsTable& lt, const BatchItem& it, uint32_t tx, uint32_t ty,
                                        uint32_t rows, uint32_t s, int64_t& b_out, int64_t& m_out) {
    constexpr int CW = kMfCW;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t L = it.L, Hw = it.Hw, k0 = it.k0, k1 = it.k1;
    const uint32_t t = it.t0 + s;
    const uint32_t X0 = tx * kMfTileWords;
    const uint32_t wds = min(kMfTileWords, Hw - X0);  // words of the lattice in this tile
    const uint32_t la = wds / CW - 1u;                 // last lane holding lattice words
    const bool active = lane <= la;
    const bool is_last = lane == la;
    const uint32_t x = X0 + min(lane, la) * CW;
    const int r0 = (int)(ty * rows);
    const int R = (int)min(rows, L - ty * rows);  // a multiple of 8 (L % 16 == 0, rows in {8, 16, 32})
    const uint32_t xl = X0 == 0 ? Hw - 1 : X0 - 1;
    const uint32_t xr = X0 + wds == Hw ? 0u : X0 + wds;
    const bool odd = (s & 1u) != 0u;
    const uint32_t* __restrict__ s0 = odd ? it.q0 : it.p0;
    const uint32_t* __restrict__ s1 = odd ? it.q1 : it.p1;
    uint32_t* __restrict__ d0 = odd ? it.p0 : it.q0;
    uint32_t* __restrict__ d1 = odd ? it.p1 : it.q1;

    auto row_ptr = [&](const uint32_t* base, int i) { return base + (size_t)wrap_row_m(i, L) * Hw; };

    // old colour-1 word just outside the tile for the colour-0 update of row
    // r0 + 1 + lane, and the new colour-0 word just outside it for row
    // r0 + lane (see the single-lattice kernel)
    uint32_t edge_c1 = 0;
    if (lane < (uint32_t)R) {
        const int j = r0 + 1 + (int)lane;
        const uint32_t rj = wrap_row_m(j, L);
        edge_c1 = row_ptr(s1, j)[(rj & 1u) ? xr : xl];
    }
    uint32_t edge_c0 = 0;
    if (lane < (uint32_t)R) {
        const int i = r0 + (int)lane;
        const uint32_t ri = wrap_row_m(i, L);
        const uint32_t xe = (ri & 1u) ? xl : xr;
        const uint32_t pe = ri & 1u;
        const uint32_t xn = pe ? (xe + 1 == Hw ? 0u : xe + 1) : (xe == 0 ? Hw - 1 : xe - 1);
        const uint32_t own = row_ptr(s0, i)[xe];
        const uint32_t up = row_ptr(s1, i - 1)[xe];
        const uint32_t dn = row_ptr(s1, i + 1)[xe];
        const uint32_t same = row_ptr(s1, i)[xe];
        const uint32_t nbw = row_ptr(s1, i)[xn];
        const uint32_t S = pe ? __builtin_amdgcn_alignbyte(nbw, same, 1) : __builtin_amdgcn_alignbyte(same, nbw, 3);
        const uint32_t n = up + dn + same + S;
        const uint4 r = philox(ri * Hw + xe, t, 0u, 0u, k0, k1);
        edge_c0 = accept_word(lt, (own << 3) + n, r);
    }

    uint32_t sad = 0, ups = 0, ups8 = 0, dummy = 0;
    const uint32_t xb = x * 4u;
    Row<CW> xw;
#pragma unroll
    for (int w = 0; w < CW; ++w) xw.v[w] = x + (uint32_t)w;
    const __amdgpu_buffer_rsrc_t rs0 = plane_rsrc(s0), rs1 = plane_rsrc(s1);
    const __amdgpu_buffer_rsrc_t rd0 = plane_rsrc(d0), rd1 = plane_rsrc(d1);
    auto rword = [&](int i) { return wrap_row_m(i, L) * Hw; };
    auto rbyte = [&](int i) { return rword(i) * 4u; };
    Row<CW> c1[4], c0o[2], c0n[4];
    const Row<CW> c1m2 = ld<CW>(rs1, xb, rbyte(r0 - 2));
    const Row<CW> c1m1 = ld<CW>(rs1, xb, rbyte(r0 - 1));
    c1[0] = ld<CW>(rs1, xb, rbyte(r0));
    c1[1] = ld<CW>(rs1, xb, rbyte(r0 + 1));
    c1[2] = ld<CW>(rs1, xb, rbyte(r0 + 2));
    const Row<CW> c0om1 = ld<CW>(rs0, xb, rbyte(r0 - 1));
    c0o[0] = ld<CW>(rs0, xb, rbyte(r0));
    c0o[1] = ld<CW>(rs0, xb, rbyte(r0 + 1));
    const uint32_t eR = row_ptr(s1, r0 - 1)[xr];
    const uint32_t eL = row_ptr(s1, r0)[xl];
    c0n[0] = update_row<CW, 1, false, true>(lt, c0om1, c1m2, c1[0], c1m1, eR, xw, rword(r0 - 1), t, 0u, k0,
                                                   k1, dummy, is_last);
    c0n[1] = update_row<CW, 0, false, true>(lt, c0o[0], c1m1, c1[1], c1[0], eL, xw, rword(r0), t, 0u, k0,
                                                   k1, dummy, is_last);
    if (active) st<CW>(rd0, xb + rbyte(r0), c0n[1]);

#pragma unroll 1
    for (int k = 0; k < R; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = r0 + k + u;
            c1[(u + 3) & 3] = ld<CW>(rs1, xb, rbyte(i + 3));
            c0o[u & 1] = ld<CW>(rs0, xb, rbyte(i + 2));
            const uint32_t e1 = (uint32_t)__builtin_amdgcn_readlane((int)edge_c1, k + u);
            const uint32_t e0 = (uint32_t)__builtin_amdgcn_readlane((int)edge_c0, k + u);
            const uint32_t m1 = rword(i + 1);
            const uint32_t m0 = rword(i);
            Row<CW> c1n;
            if ((u & 1) == 0) {
                c0n[(u + 2) & 3] =
                    update_row<CW, 1, false, true>(lt, c0o[(u + 1) & 1], c1[u & 3], c1[(u + 2) & 3],
                                                          c1[(u + 1) & 3], e1, xw, m1, t, 0u, k0, k1, dummy, is_last);
                c1n = update_row<CW, 1, true, true>(lt, c1[u & 3], c0n[u & 3], c0n[(u + 2) & 3],
                                                           c0n[(u + 1) & 3], e0, xw, m0, t, 1u, k0, k1, sad, is_last);
            } else {
                c0n[(u + 2) & 3] =
                    update_row<CW, 0, false, true>(lt, c0o[(u + 1) & 1], c1[u & 3], c1[(u + 2) & 3],
                                                          c1[(u + 1) & 3], e1, xw, m1, t, 0u, k0, k1, dummy, is_last);
                c1n = update_row<CW, 0, true, true>(lt, c1[u & 3], c0n[u & 3], c0n[(u + 2) & 3],
                                                           c0n[(u + 1) & 3], e0, xw, m0, t, 1u, k0, k1, sad, is_last);
            }
            if (active) {
                if (k + u + 1 < R) st<CW>(rd0, xb + rbyte(i + 1), c0n[(u + 2) & 3]);
                st<CW>(rd1, xb + rbyte(i), c1n);
            }
#pragma unroll
            for (int w = 0; w < CW; ++w) ups8 += c1n.v[w] + c0n[(u + 1) & 3].v[w];
            __builtin_amdgcn_sched_barrier(0);
        }
        ups = __builtin_amdgcn_sad_u8(ups8, 0u, ups);
        ups8 = 0;
    }

    // partials of the lanes that hold lattice words: B = 16 * words - 2 *
    // sad, M = 2 * ups - 8 * words
    const int64_t words = active ? (int64_t)R * CW : 0;
    int64_t b = active ? 16 * words - 2 * (int64_t)sad : 0;
    int64_t m = active ? 2 * (int64_t)ups - 8 * words : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        b += __shfl_xor(b, off, 64);
        m += __shfl_xor(m, off, 64);
    }
    b_out = b;
    m_out = m;
}

// Partial (B, M) of a packed tile: `bands` row bands ty0, ty0 + 1, ... (of
// `rows` rows each) of the last column tx of item `it`, which is at most 32
// lanes wide. Band b
// takes lanes b S .. b S + S - 1 (S lanes per band); lanes past the last
// band shadow band 0's last lane (in-range loads, nothing stored or
// counted). Every band has `rows` rows (rows divides L), so all bands walk
// in step; each lane addresses its band's rows through its own offsets. The
// edge words of band b's rows are computed by lanes b rows .. b rows +
// rows - 1 and fetched with a lane permute.
__device__ __forceinline__ void mf_tile_packed(const LdsTable& lt, const BatchItem& it, uint32_t tx, uint32_t ty0,
                                               uint32_t bands, uint32_t rows, uint32_t s, int64_t& b_out,
                                               int64_t& m_out) {
    constexpr int CW = kMfCW;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t L = it.L, Hw = it.Hw, k0 = it.k0, k1 = it.k1;
    const uint32_t t = it.t0 + s;
    const uint32_t X0 = tx * kMfTileWords;
    const uint32_t S = (Hw - X0) / CW;  // lanes per band (<= 32)
    const uint32_t band = lane / S;
    const bool active = band < bands;
    const uint32_t bl = active ? band : 0u;
    const uint32_t sl = active ? lane - band * S : S - 1u;
    const bool is_first = sl == 0u;
    const bool is_last = sl == S - 1u;
    const uint32_t x = X0 + sl * CW;
    const int R = (int)rows;
    const int rb = (int)((ty0 + bl) * rows);  // first row of this lane's band
    const uint32_t xl = X0 == 0 ? Hw - 1 : X0 - 1;
    const uint32_t xr = 0u;  // right of the last column: word 0 (periodic)
    const bool odd = (s & 1u) != 0u;
    const uint32_t* __restrict__ s0 = odd ? it.q0 : it.p0;
    const uint32_t* __restrict__ s1 = odd ? it.q1 : it.p1;
    uint32_t* __restrict__ d0 = odd ? it.p0 : it.q0;
    uint32_t* __restrict__ d1 = odd ? it.p1 : it.q1;

    auto row_ptr = [&](const uint32_t* base, int i) { return base + (size_t)wrap_row_m(i, L) * Hw; };

    // edge words: lane j < bands * rows holds those of row j % rows of band
    // j / rows (the same words as the single-band tile's lanes hold)
    uint32_t edge_c1 = 0, edge_c0 = 0;
    if (lane < bands * rows) {
        const uint32_t eb = lane / rows;
        const int row0 = (int)((ty0 + eb) * rows + (lane - eb * rows));
        {
            const int j = row0 + 1;
            const uint32_t rj = wrap_row_m(j, L);
            edge_c1 = row_ptr(s1, j)[(rj & 1u) ? xr : xl];
        }
        const int i = row0;
        const uint32_t ri = wrap_row_m(i, L);
        const uint32_t xe = (ri & 1u) ? xl : xr;
        const uint32_t pe = ri & 1u;
        const uint32_t xn = pe ? (xe + 1 == Hw ? 0u : xe + 1) : (xe == 0 ? Hw - 1 : xe - 1);
        const uint32_t own = row_ptr(s0, i)[xe];
        const uint32_t up = row_ptr(s1, i - 1)[xe];
        const uint32_t dn = row_ptr(s1, i + 1)[xe];
        const uint32_t same = row_ptr(s1, i)[xe];
        const uint32_t nbw = row_ptr(s1, i)[xn];
        const uint32_t S4 = pe ? __builtin_amdgcn_alignbyte(nbw, same, 1) : __builtin_amdgcn_alignbyte(same, nbw, 3);
        const uint32_t n = up + dn + same + S4;
        const uint4 r = philox(ri * Hw + xe, t, 0u, 0u, k0, k1);
        edge_c0 = accept_word(lt, (own << 3) + n, r);
    }

    uint32_t sad = 0, ups = 0, ups8 = 0, dummy = 0;
    const uint32_t xb = x * 4u;
    Row<CW> xw;
#pragma unroll
    for (int w = 0; w < CW; ++w) xw.v[w] = x + (uint32_t)w;
    const __amdgpu_buffer_rsrc_t rs0 = plane_rsrc(s0), rs1 = plane_rsrc(s1);
    const __amdgpu_buffer_rsrc_t rd0 = plane_rsrc(d0), rd1 = plane_rsrc(d1);
    // byte offset of this lane's word in row rb + d, and the Philox row term
    auto vrow = [&](int d) { return xb + wrap_row_m(rb + d, L) * Hw * 4u; };
    auto m0of = [&](uint32_t vo) { return (vo - xb) >> 2; };  // row word offset of this lane's band
    Row<CW> c1[4], c0o[2], c0n[4];
    uint32_t vo[4];  // offsets of rows i .. i + 3 (ring, slot (i - rb) & 3)
    const uint32_t vm2 = vrow(-2), vm1 = vrow(-1);
    vo[0] = vrow(0);
    vo[1] = vrow(1);
    vo[2] = vrow(2);
    const Row<CW> c1m2 = ld<CW>(rs1, vm2, 0u);
    const Row<CW> c1m1 = ld<CW>(rs1, vm1, 0u);
    c1[0] = ld<CW>(rs1, vo[0], 0u);
    c1[1] = ld<CW>(rs1, vo[1], 0u);
    c1[2] = ld<CW>(rs1, vo[2], 0u);
    const Row<CW> c0om1 = ld<CW>(rs0, vm1, 0u);
    c0o[0] = ld<CW>(rs0, vo[0], 0u);
    c0o[1] = ld<CW>(rs0, vo[1], 0u);
    const uint32_t eR = row_ptr(s1, rb - 1)[xr];
    const uint32_t eL = row_ptr(s1, rb)[xl];
    c0n[0] = update_row<CW, 1, false, true, true>(lt, c0om1, c1m2, c1[0], c1m1, eR, xw, m0of(vm1), t, 0u, k0,
                                                         k1, dummy, is_last, is_first);
    c0n[1] = update_row<CW, 0, false, true, true>(lt, c0o[0], c1m1, c1[1], c1[0], eL, xw, m0of(vo[0]), t, 0u,
                                                         k0, k1, dummy, is_last, is_first);
    if (active) st<CW>(rd0, vo[0], c0n[1]);

    const int eb0 = (int)(bl * rows) * 4;  // byte index of this band's first edge lane
#pragma unroll 1
    for (int k = 0; k < R; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = k + u;  // row rb + i
            vo[(u + 3) & 3] = vrow(i + 3);
            c1[(u + 3) & 3] = ld<CW>(rs1, vo[(u + 3) & 3], 0u);
            c0o[u & 1] = ld<CW>(rs0, vo[(u + 2) & 3], 0u);
            const uint32_t e1 = (uint32_t)__builtin_amdgcn_ds_bpermute(eb0 + 4 * i, (int)edge_c1);
            const uint32_t e0 = (uint32_t)__builtin_amdgcn_ds_bpermute(eb0 + 4 * i, (int)edge_c0);
            const uint32_t m1 = m0of(vo[(u + 1) & 3]);
            const uint32_t m0 = m0of(vo[u & 3]);
            Row<CW> c1n;
            if ((u & 1) == 0) {
                c0n[(u + 2) & 3] = update_row<CW, 1, false, true, true>(
                    lt, c0o[(u + 1) & 1], c1[u & 3], c1[(u + 2) & 3], c1[(u + 1) & 3], e1, xw, m1, t, 0u, k0, k1,
                    dummy, is_last, is_first);
                c1n = update_row<CW, 1, true, true, true>(lt, c1[u & 3], c0n[u & 3], c0n[(u + 2) & 3],
                                                                 c0n[(u + 1) & 3], e0, xw, m0, t, 1u, k0, k1, sad,
                                                                 is_last, is_first);
            } else {
                c0n[(u + 2) & 3] = update_row<CW, 0, false, true, true>(
                    lt, c0o[(u + 1) & 1], c1[u & 3], c1[(u + 2) & 3], c1[(u + 1) & 3], e1, xw, m1, t, 0u, k0, k1,
                    dummy, is_last, is_first);
                c1n = update_row<CW, 0, true, true, true>(lt, c1[u & 3], c0n[u & 3], c0n[(u + 2) & 3],
                                                                 c0n[(u + 1) & 3], e0, xw, m0, t, 1u, k0, k1, sad,
                                                                 is_last, is_first);
            }
            if (active) {
                if (i + 1 < R) st<CW>(rd0, vo[(u + 1) & 3], c0n[(u + 2) & 3]);
                st<CW>(rd1, vo[u & 3], c1n);
            }
#pragma unroll
            for (int w = 0; w < CW; ++w) ups8 += c1n.v[w] + c0n[(u + 1) & 3].v[w];
            __builtin_amdgcn_sched_barrier(0);
        }
        ups = __builtin_amdgcn_sad_u8(ups8, 0u, ups);
        ups8 = 0;
    }

    const int64_t words = active ? (int64_t)R * CW : 0;
    int64_t b = active ? 16 * words - 2 * (int64_t)sad : 0;
    int64_t m = active ? 2 * (int64_t)ups - 8 * words : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        b += __shfl_xor(b, off, 64);
        m += __shfl_xor(m, off, 64);
    }
    b_out = b;
    m_out = m;
}

}  // namespace

// Sweep hdr->s_base + s of every item with that sweep pending. Waves take
// virtual tiles (tile_start[k] = item k's first) in a grid-stride loop.
__global__ void __launch_bounds__(kMfThreads) k_multi_fused(const BatchItem* __restrict__ items,
                                                            const uint32_t* __restrict__ tile_start,
                                                            const MultiHeader* __restrict__ hdr, uint32_t s) {
    __shared__ LdsTable lt[kMfThreads / 64];
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t n_items = hdr->n_items, total = hdr->total_vblocks;
    const uint32_t sweep = hdr->s_base + s;
    const uint32_t rows = hdr->rows;
    int64_t* __restrict__ part = hdr->part + 2ull * s * total;
    const uint32_t waves = gridDim.x * (kMfThreads / 64);
    for (uint32_t g0 = blockIdx.x * (kMfThreads / 64) + wv; g0 < total; g0 += waves) {
        const uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)g0);
        uint32_t lo = 0, hi = n_items;  // last item whose first tile is <= g
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tile_start[mid] <= g) lo = mid;
            else hi = mid;
        }
        const BatchItem& it = items[lo];
        if (sweep >= it.n) continue;  // this lattice is done: the whole wave skips
        // this wave's copy of the item's acceptance table
        if (lane < 16) lt[wv].tm[lane] = mad_entry(lane, it.table.thr_lo[lane], it.table.thr_hi[lane]);
        __builtin_amdgcn_wave_barrier();
        const MfLayout lay = mf_layout(it.L, rows);
        const uint32_t tile = g - tile_start[lo];
        const uint32_t full = (lay.n_tx - 1u) * lay.n_ty;  // tiles of the full columns when packing
        int64_t b, m;
        if (lay.pack > 1u && tile >= full) {
            const uint32_t ty0 = (tile - full) * lay.pack;
            const uint32_t bands = min(lay.pack, lay.n_typ - ty0);
            mf_tile_packed(lt[wv], it, lay.n_tx - 1u, ty0, bands, lay.prow, sweep, b, m);
        } else {
            const uint32_t cols = lay.pack > 1u ? lay.n_tx - 1u : lay.n_tx;
            const uint32_t tx = tile % cols, ty = tile / cols;
            mf_tile(lt[wv], it, tx, ty, rows, sweep, b, m);
        }
        if (lane == 0) {
            part[2ull * g] = b;
            part[2ull * g + 1] = m;
        }
        // the next tile's table must not overwrite this one while lanes read it
        __builtin_amdgcn_wave_barrier();
    }
}

// Sum the partials (one per tile or virtual block) of each item's sweeps of
// this replay into its series: one wave per (item, sweep of the replay),
// grid-stride.
__global__ void __launch_bounds__(256) k_multi_reduce(const BatchItem* __restrict__ items,
                                                            const uint32_t* __restrict__ tile_start,
                                                            const MultiHeader* __restrict__ hdr, uint32_t g_sweeps) {
    const uint32_t n_items = hdr->n_items, total = hdr->total_vblocks, s_base = hdr->s_base;
    const int64_t* __restrict__ part = hdr->part;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t waves = gridDim.x * (blockDim.x / 64u);
    const uint32_t pairs = n_items * g_sweeps;
    for (uint32_t q = blockIdx.x * (blockDim.x / 64u) + (threadIdx.x >> 6); q < pairs; q += waves) {
        const uint32_t k = q / g_sweeps, j = q - k * g_sweeps;
        const BatchItem& it = items[k];
        const uint32_t sweep = s_base + j;
        if (sweep >= it.n) continue;
        const int64_t* __restrict__ pj = part + 2ull * j * total;
        int64_t b = 0, m = 0;
        for (uint32_t g = tile_start[k] + lane; g < tile_start[k + 1]; g += 64u) {
            b += pj[2ull * g];
            m += pj[2ull * g + 1];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            b += __shfl_xor(b, off, 64);
            m += __shfl_xor(m, off, 64);
        }
        if (lane == 0) {
            it.series[2ull * sweep] = b;
            it.series[2ull * sweep + 1] = m;
        }
    }
}

bool multi_fused_supported(uint32_t L) { return L % 16u == 0u && L >= 16u; }

uint32_t multi_fused_tiles(uint32_t L, uint32_t rows) { return mf_layout(L, rows).tiles; }

uint32_t multi_fused_wave_slots(uint32_t cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_multi_fused, (int)kMfThreads, 0) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return cus * (uint32_t)per_cu * (kMfThreads / 64);
}

hipError_t launch_multi_reduce(const BatchItem* items, const uint32_t* vb_start, const MultiHeader* hdr,
                               uint32_t sweeps_per_replay, uint32_t grid, hipStream_t s) {
    k_multi_reduce<<<grid, 256, 0, s>>>(items, vb_start, hdr, sweeps_per_replay);
    return hipGetLastError();
}

__global__ void __launch_bounds__(64) k_multi_fused_advance(MultiHeader* hdr, uint32_t g) {
    if (threadIdx.x == 0 && blockIdx.x == 0) hdr->s_base += g;
}

hipError_t launch_multi_fused_graph_body(const BatchItem* items, const uint32_t* tile_start, MultiHeader* hdr,
                                         uint32_t sweeps_per_replay, uint32_t grid, hipStream_t s) {
    k_multi_fused_advance<<<1, 64, 0, s>>>(hdr, sweeps_per_replay);
    for (uint32_t k = 0; k < sweeps_per_replay; ++k)
        k_multi_fused<<<grid, kMfThreads, 0, s>>>(items, tile_start, hdr, k);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    return launch_multi_reduce(items, tile_start, hdr, sweeps_per_replay, grid, s);
}

}  // namespace ising
