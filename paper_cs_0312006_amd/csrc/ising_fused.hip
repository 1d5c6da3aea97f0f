// Fused one-pass sweep: both colours of sweep t in one launch, reading the
// lattice of sweep t-1 from `src` and writing sweep t to `dst` (ping-pong),
// so the lattice crosses HBM once per sweep (2 bytes per site update).
//
// Work unit: one wave owns a tile of R rows by 64*CW words of a plane row
// (lane l holds words X0 + l*CW .. X0 + l*CW + CW-1). It walks down the
// tile computing, at row i, colour 0 of row i+1 and then colour 1 of row i,
// which needs the new colour 0 of rows i-1, i, i+1 (Section 2.2's order:
// all of colour 0, then all of colour 1; sites of one colour are
// independent, so any order within a colour gives the same lattice).
//   - Same-row neighbours across lanes come from the adjacent lane (DPP
//     wave shift). Across the tile's left/right edge, old colour-1 words are
//     read from memory; the new colour-0 word just outside the tile is
//     recomputed up front, one row per lane (two registers for a tile of
//     128 rows).
//   - Above and below the tile, the new colour-0 rows r0-1 and r0+R are
//     recomputed (two extra row updates per tile).
// Recomputed sites use the same counter-based draws as their owners, so the
// result is bit-identical to any other schedule of the same sweep.
//
// Row traffic goes through buffer resources: a plane is one raw buffer, the
// lane's byte offset within a row is fixed for the whole tile and the row's
// byte offset is a scalar, so loads and stores cost no vector instructions
// for addressing (a plane is at most 2^31 bytes).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_fused_core.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

__device__ __forceinline__ uint32_t xcd_block_f(uint32_t nblocks) {
    const uint32_t b = blockIdx.x;
    if ((nblocks & 7u) != 0u) return b;
    return (b & 7u) * (nblocks >> 3) + (b >> 3);
}

}  // namespace

// At least four waves per SIMD (at most 128 VGPRs): the 32768^2 sweep's
// tiles then fill the GPU in whole rounds of 1024 blocks.
template <int CW, int R>
__global__ void __launch_bounds__(256, 4) k_fused(FusedArgs a, AcceptTable at, PartialReduce red) {
    __shared__ LdsTable lt;
    load_table(lt, at);
    __syncthreads();
    const uint32_t lblock = xcd_block_f(gridDim.x);
    if (lblock == 0) reduce_partials(red);

    const uint32_t lane = threadIdx.x & 63u;
    // the tile is wave-uniform: keep it (and all row arithmetic) scalar
    const uint32_t tile = (uint32_t)__builtin_amdgcn_readfirstlane((int)(lblock * 4u + (threadIdx.x >> 6)));
    if (tile >= a.n_tiles) return;  // whole wave
    const uint32_t L = a.L, Hw = a.Hw, t = a.t, k0 = a.k0, k1 = a.k1;
    const uint32_t tx = tile % a.n_tx, ty = tile / a.n_tx;
    const uint32_t X0 = tx * 64u * CW;
    const uint32_t x = X0 + lane * CW;
    const int r0 = (int)(ty * R);
    const uint32_t xl = X0 == 0 ? Hw - 1 : X0 - 1;
    const uint32_t xr = X0 + 64u * CW == Hw ? 0u : X0 + 64u * CW;
    const uint32_t* __restrict__ s0 = a.src0;
    const uint32_t* __restrict__ s1 = a.src1;
    uint32_t* __restrict__ d0 = a.dst0;
    uint32_t* __restrict__ d1 = a.dst1;

    auto row_ptr = [&](const uint32_t* base, int i) { return base + (size_t)wrap_row(i, L) * Hw; };

    // Edge words of the 64 rows from r0 + base (lane l holds row r0 + base +
    // l's; a tile of 128 rows keeps two such registers of each):
    //   edge_c1: the old colour-1 word just outside the tile that the
    //     colour-0 update of row j = r0 + base + 1 + l needs: right of the
    //     tile for odd j, left for even j;
    //   edge_c0: the new colour-0 word just outside the tile for row
    //     i = r0 + base + l: the right neighbour word for even i (its byte 0
    //     is needed), the left one for odd i (its byte 3).
    auto edges = [&](int base, uint32_t& edge_c1, uint32_t& edge_c0) {
        edge_c1 = 0;
        edge_c0 = 0;
        if (lane < (uint32_t)(R - base)) {
            const int j = r0 + base + 1 + (int)lane;
            const uint32_t rj = wrap_row(j, L);
            edge_c1 = row_ptr(s1, j)[(rj & 1u) ? xr : xl];
            const int i = r0 + base + (int)lane;
            const uint32_t ri = wrap_row(i, L);
            const uint32_t xe = (ri & 1u) ? xl : xr;
            const uint32_t pe = ri & 1u;  // same-row side for colour 0 at row i
            const uint32_t xn = pe ? (xe + 1 == Hw ? 0u : xe + 1) : (xe == 0 ? Hw - 1 : xe - 1);
            const uint32_t own = row_ptr(s0, i)[xe];
            const uint32_t up = row_ptr(s1, i - 1)[xe];
            const uint32_t dn = row_ptr(s1, i + 1)[xe];
            const uint32_t same = row_ptr(s1, i)[xe];
            const uint32_t nbw = row_ptr(s1, i)[xn];
            const uint32_t S =
                pe ? __builtin_amdgcn_alignbyte(nbw, same, 1) : __builtin_amdgcn_alignbyte(same, nbw, 3);
            const uint32_t n = up + dn + same + S;
            const uint4 r = philox(ri * Hw + xe, t, 0u, 0u, k0, k1);
            edge_c0 = accept_word(lt, (own << 3) + n, r);
        }
    };
    uint32_t e1_lo, e0_lo, e1_hi = 0, e0_hi = 0;
    edges(0, e1_lo, e0_lo);
    if (R > 64) edges(64, e1_hi, e0_hi);

    uint32_t sad = 0, ups = 0, ups8 = 0, dummy = 0;
    const uint32_t xb = x * 4u;  // lane's byte offset within a row
    Row<CW> xw;                  // lane's word indices within a row
#pragma unroll
    for (int w = 0; w < CW; ++w) xw.v[w] = x + (uint32_t)w;
    const __amdgpu_buffer_rsrc_t rs0 = plane_rsrc(s0), rs1 = plane_rsrc(s1);
    const __amdgpu_buffer_rsrc_t rd0 = plane_rsrc(d0), rd1 = plane_rsrc(d1);
    // word offset of row i (wrapped) and its byte offset
    auto rword = [&](int i) { return wrap_row(i, L) * Hw; };
    auto rbyte = [&](int i) { return rword(i) * 4u; };
    // Ring buffers, indexed by compile-time slots in a loop unrolled by 4,
    // so that a prefetched row is never copied between registers (a copy
    // would force a wait on the load):
    //   c1[(row - r0) & 3]      old colour-1 rows
    //   c0o[(row - r0) & 1]     old colour-0 rows
    //   c0n[(row - r0 + 1) & 3] new colour-0 rows
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
    // new colour-0 rows r0-1 (odd: same-row side P = 1) and r0 (even: P = 0)
    c0n[0] = update_row<CW, 1, false>(lt, c0om1, c1m2, c1[0], c1m1, eR, xw, rword(r0 - 1), t, 0u, k0, k1,
                                             dummy);
    c0n[1] = update_row<CW, 0, false>(lt, c0o[0], c1m1, c1[1], c1[0], eL, xw, rword(r0), t, 0u, k0, k1,
                                             dummy);
    st<CW>(rd0, xb + rbyte(r0), c0n[1]);

#pragma unroll 1
    for (int k = 0; k < R; k += 4) {
        const uint32_t edge_c1 = (R > 64 && k >= 64) ? e1_hi : e1_lo;
        const uint32_t edge_c0 = (R > 64 && k >= 64) ? e0_hi : e0_lo;
        // the four steps of k, each with compile-time ring slots (a generic
        // lambda instantiated per step: the unroller is not relied on)
        auto step = [&](auto uc) {
            constexpr int u = decltype(uc)::value;
            const int i = r0 + k + u;
            // prefetch old colour-1 row i+3 and old colour-0 row i+2 into the
            // slots of rows i-1 and i, which this step no longer reads
            c1[(u + 3) & 3] = ld<CW>(rs1, xb, rbyte(i + 3));
            c0o[u & 1] = ld<CW>(rs0, xb, rbyte(i + 2));
            const uint32_t e1 = (uint32_t)__builtin_amdgcn_readlane((int)edge_c1, (k + u) & 63);
            const uint32_t e0 = (uint32_t)__builtin_amdgcn_readlane((int)edge_c0, (k + u) & 63);
            const uint32_t m1 = rword(i + 1);
            const uint32_t m0 = rword(i);
            constexpr int P = (u & 1) == 0 ? 1 : 0;  // i even: both updates have same-row side P = 1
            c0n[(u + 2) & 3] = update_row<CW, P, false>(lt, c0o[(u + 1) & 1], c1[u & 3], c1[(u + 2) & 3],
                                                        c1[(u + 1) & 3], e1, xw, m1, t, 0u, k0, k1, dummy);
            const Row<CW> c1n = update_row<CW, P, true>(lt, c1[u & 3], c0n[u & 3], c0n[(u + 2) & 3],
                                                        c0n[(u + 1) & 3], e0, xw, m0, t, 1u, k0, k1, sad);
            if (k + u + 1 < R) st<CW>(rd0, xb + rbyte(i + 1), c0n[(u + 2) & 3]);
            st<CW>(rd1, xb + rbyte(i), c1n);
            // up spins of both new rows, byte-wise (at most 8 CW <= 32 per
            // byte over the four steps of k)
#pragma unroll
            for (int w = 0; w < CW; ++w) ups8 += c1n.v[w] + c0n[(u + 1) & 3].v[w];
            // keep the next step's use of this step's prefetch after this
            // step's work, so the load has a whole step to arrive
            __builtin_amdgcn_sched_barrier(0);
        };
        step(Step<0>{});
        step(Step<1>{});
        step(Step<2>{});
        step(Step<3>{});
        ups = __builtin_amdgcn_sad_u8(ups8, 0u, ups);
        ups8 = 0;
    }

    // per-wave partials: B = 16 * words - 2 * sad, M = 2 * ups - 8 * words
    const int64_t words = (int64_t)R * CW;
    int64_t b = 16 * words - 2 * (int64_t)sad;
    int64_t m = 2 * (int64_t)ups - 8 * words;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        b += __shfl_xor(b, off, 64);
        m += __shfl_xor(m, off, 64);
    }
    if (lane == 0) {
        a.part[2 * tile] = b;
        a.part[2 * tile + 1] = m;
    }
}

// Stand-alone reduction of one sweep's partials (after the last sweep of a call).
__global__ void __launch_bounds__(256) k_reduce_partials(PartialReduce red) { reduce_partials(red); }

template <int CW, int R>
static void launch_fused_t(const FusedArgs& a, const AcceptTable& at, const PartialReduce& red, hipStream_t s) {
    const uint32_t blocks = (a.n_tiles + 3u) / 4u;
    k_fused<CW, R><<<blocks, 256, 0, s>>>(a, at, red);
}

bool fused_supported(uint32_t L, uint32_t cw, uint32_t rows) {
    if (L % 8u != 0u) return false;
    const uint32_t Hw = L / 8u;
    if (cw != 1 && cw != 2 && cw != 4) return false;
    if (rows != 4 && rows != 8 && rows != 16 && rows != 32 && rows != 64 && rows != 128) return false;
    return Hw % (64u * cw) == 0u && L % rows == 0u && L >= 4u;
}

uint32_t fused_tiles(uint32_t L, uint32_t cw, uint32_t rows) {
    return (L / 8u / (64u * cw)) * (L / rows);
}

// Every threshold in [0, 2^32] takes the same path (accept_word), so the
// table's exact flag needs no separate kernel.
hipError_t launch_fused(const FusedArgs& a, const AcceptTable& at, bool /*exact*/, uint32_t cw, uint32_t rows,
                        const PartialReduce& red, hipStream_t s) {
#define ISING_FUSED_CASE(CWv, Rv)                  \
    if (cw == CWv && rows == Rv) {                 \
        launch_fused_t<CWv, Rv>(a, at, red, s);    \
        return hipGetLastError();                  \
    }
    ISING_FUSED_CASE(1, 4) ISING_FUSED_CASE(1, 8) ISING_FUSED_CASE(1, 16) ISING_FUSED_CASE(1, 32)
    ISING_FUSED_CASE(1, 64) ISING_FUSED_CASE(2, 4) ISING_FUSED_CASE(2, 8) ISING_FUSED_CASE(2, 16)
    ISING_FUSED_CASE(2, 32) ISING_FUSED_CASE(2, 64) ISING_FUSED_CASE(4, 4) ISING_FUSED_CASE(4, 8)
    ISING_FUSED_CASE(4, 16) ISING_FUSED_CASE(4, 32) ISING_FUSED_CASE(4, 64) ISING_FUSED_CASE(1, 128)
    ISING_FUSED_CASE(2, 128) ISING_FUSED_CASE(4, 128)
#undef ISING_FUSED_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_reduce_partials(const PartialReduce& red, hipStream_t s) {
    if (red.n == 0) return hipSuccess;
    k_reduce_partials<<<1, 256, 0, s>>>(red);
    return hipGetLastError();
}

}  // namespace ising
