// Fused one-pass Creutz sweep: both colours of a sweep in one launch,
// reading spins and demons of the previous sweep from `src` buffers and
// writing the new ones to `dst` buffers (ping-pong), so spins and demons
// cross HBM once per sweep (4 bytes per site update, against 5 for the
// in-place two-pass form).
//
// The walk is the one of the fused Metropolis sweep: a wave owns R rows by
// 64*CW words of a plane row and, going down, updates colour 0 of row i+1
// and then colour 1 of row i; same-row neighbours across lanes come by DPP,
// the new colour-0 word just outside the tile is recomputed up front for
// all R rows (one row per lane), and the colour-0 rows just above and below
// the tile are recomputed. A recomputed site reads the old demon of that
// site, as its owner does, so both compute the same move; only the owner
// writes it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_creutz.hpp"
#include "ising_device.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr int kShl1 = 0x130;  // lane l reads lane l+1
constexpr int kShr1 = 0x138;  // lane l reads lane l-1

__device__ __forceinline__ uint32_t right_of(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, kShl1, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t left_of(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, kShr1, 0xf, 0xf, false);
}

template <int CW>
struct Words {
    uint32_t v[CW];
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Row words are loaded and stored nontemporally: a sweep touches every word
// of the spin and demon planes once each way, and the four 1 GiB planes of
// a 32768^2 lattice dwarf the caches (measured 7% faster at that size than
// plain loads and stores, bit-identical).
template <int CW>
__device__ __forceinline__ Words<CW> load(const uint32_t* __restrict__ p) {
    Words<CW> r;
    if constexpr (CW == 4) {
        const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
        r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
    } else if constexpr (CW == 2) {
        const u32x2 x = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
        r.v[0] = x.x; r.v[1] = x.y;
    } else {
        r.v[0] = __builtin_nontemporal_load(p);
    }
    return r;
}

template <int CW>
__device__ __forceinline__ void store(uint32_t* __restrict__ p, const Words<CW>& r) {
    if constexpr (CW == 4) {
        const u32x4 x = {r.v[0], r.v[1], r.v[2], r.v[3]};
        __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(p));
    } else if constexpr (CW == 2) {
        const u32x2 x = {r.v[0], r.v[1]};
        __builtin_nontemporal_store(x, reinterpret_cast<u32x2*>(p));
    } else {
        __builtin_nontemporal_store(r.v[0], p);
    }
}

// Creutz update of one lane's CW words of a plane row: own spins, old
// demons `dem`, the other colour's rows above, below and alongside, and the
// word just outside the tile on the same-row side (right for P == 1, left
// for P == 0). New demons go to `dem_out`.
template <int CW, int P, bool OBS>
__device__ __forceinline__ Words<CW> creutz_row(const Words<CW>& own, const Words<CW>& dem, const Words<CW>& up,
                                                const Words<CW>& dn, const Words<CW>& same, uint32_t edge,
                                                Words<CW>& dem_out, uint32_t& sad) {
    const uint32_t nb = P ? right_of(same.v[0], edge) : left_of(same.v[CW - 1], edge);
    Words<CW> out;
#pragma unroll
    for (int w = 0; w < CW; ++w) {
        uint32_t S;
        if (P) {
            const uint32_t nxt = (w + 1 < CW) ? same.v[(w + 1 < CW) ? w + 1 : 0] : nb;
            S = __builtin_amdgcn_alignbyte(nxt, same.v[w], 1);
        } else {
            const uint32_t prv = (w > 0) ? same.v[(w > 0) ? w - 1 : 0] : nb;
            S = __builtin_amdgcn_alignbyte(same.v[w], prv, 3);
        }
        const uint32_t n = up.v[w] + dn.v[w] + same.v[w] + S;
        creutz_word(own.v[w], n, dem.v[w], out.v[w], dem_out.v[w]);
        if (OBS) sad = sad_misaligned(out.v[w], n, sad);
    }
    return out;
}

template <int CW>
__device__ __forceinline__ uint32_t popcnt(const Words<CW>& r) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < CW; ++w) s += __builtin_popcount(r.v[w]);
    return s;
}

__device__ __forceinline__ uint32_t wrapped(int i, uint32_t L) {
    return (uint32_t)(i < 0 ? i + (int)L : (i >= (int)L ? i - (int)L : i));
}

}  // namespace

template <int CW, int R>
__global__ void __launch_bounds__(256) k_creutz_fused(CreutzFusedArgs a, PartialReduce red) {
    const uint32_t lblock = xcd_block(gridDim.x);
    if (lblock == 0) reduce_partials(red);

    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t tile = (uint32_t)__builtin_amdgcn_readfirstlane((int)(lblock * 4u + (threadIdx.x >> 6)));
    if (tile >= a.n_tiles) return;  // whole wave
    const uint32_t L = a.L, Hw = a.Hw;
    const uint32_t tx = tile % a.n_tx, ty = tile / a.n_tx;
    const uint32_t X0 = tx * 64u * CW;
    const uint32_t x = X0 + lane * CW;
    const int r0 = (int)(ty * R);
    const uint32_t xl = X0 == 0 ? Hw - 1 : X0 - 1;
    const uint32_t xr = X0 + 64u * CW == Hw ? 0u : X0 + 64u * CW;
    const uint32_t* __restrict__ s0 = a.src0;
    const uint32_t* __restrict__ s1 = a.src1;
    const uint32_t* __restrict__ e0 = a.dsrc0;
    const uint32_t* __restrict__ e1 = a.dsrc1;

    auto at = [&](const uint32_t* base, int i) { return base + (size_t)wrapped(i, L) * Hw; };
    auto out = [&](uint32_t* base, int i) { return base + (size_t)wrapped(i, L) * Hw; };

    // old colour-1 word just outside the tile for the colour-0 update of
    // row j = r0 + 1 + lane (right of the tile for odd j, left for even j)
    uint32_t edge_c1 = 0;
    if (lane < (uint32_t)R) {
        const int j = r0 + 1 + (int)lane;
        edge_c1 = at(s1, j)[(wrapped(j, L) & 1u) ? xr : xl];
    }
    // new colour-0 word just outside the tile for row i = r0 + lane
    uint32_t edge_c0 = 0;
    if (lane < (uint32_t)R) {
        const int i = r0 + (int)lane;
        const uint32_t ri = wrapped(i, L);
        const uint32_t xe = (ri & 1u) ? xl : xr;
        const uint32_t pe = ri & 1u;
        const uint32_t xn = pe ? (xe + 1 == Hw ? 0u : xe + 1) : (xe == 0 ? Hw - 1 : xe - 1);
        const uint32_t same = at(s1, i)[xe];
        const uint32_t nbw = at(s1, i)[xn];
        const uint32_t S = pe ? __builtin_amdgcn_alignbyte(nbw, same, 1) : __builtin_amdgcn_alignbyte(same, nbw, 3);
        const uint32_t n = at(s1, i - 1)[xe] + at(s1, i + 1)[xe] + same + S;
        uint32_t dnew;
        creutz_word(at(s0, i)[xe], n, at(e0, i)[xe], edge_c0, dnew);
    }

    uint32_t sad = 0, ups = 0, dummy = 0;
    // ring buffers with compile-time slots (loop unrolled by 4):
    //   c1[(row - r0) & 3]  old colour-1 spins     c0o[(row - r0) & 1]  old colour-0 spins
    //   c0n[(row - r0 + 1) & 3]  new colour-0 spins
    //   m0[(row - r0) & 1]  old colour-0 demons    m1[(row - r0) & 1]   old colour-1 demons
    Words<CW> c1[4], c0o[2], c0n[4], m0[2], m1[2], dout;
    const Words<CW> c1m2 = load<CW>(at(s1, r0 - 2) + x);
    const Words<CW> c1m1 = load<CW>(at(s1, r0 - 1) + x);
    c1[0] = load<CW>(at(s1, r0) + x);
    c1[1] = load<CW>(at(s1, r0 + 1) + x);
    c1[2] = load<CW>(at(s1, r0 + 2) + x);
    const Words<CW> c0om1 = load<CW>(at(s0, r0 - 1) + x);
    c0o[0] = load<CW>(at(s0, r0) + x);
    c0o[1] = load<CW>(at(s0, r0 + 1) + x);
    const Words<CW> m0m1 = load<CW>(at(e0, r0 - 1) + x);
    const Words<CW> m0r0 = load<CW>(at(e0, r0) + x);
    m0[1] = load<CW>(at(e0, r0 + 1) + x);
    m1[0] = load<CW>(at(e1, r0) + x);
    const uint32_t eR = at(s1, r0 - 1)[xr];
    const uint32_t eL = at(s1, r0)[xl];
    // new colour-0 rows r0-1 (odd relative parity: P = 1) and r0 (P = 0);
    // row r0-1 belongs to the tile above, row r0 is stored here
    c0n[0] = creutz_row<CW, 1, false>(c0om1, m0m1, c1m2, c1[0], c1m1, eR, dout, dummy);
    c0n[1] = creutz_row<CW, 0, false>(c0o[0], m0r0, c1m1, c1[1], c1[0], eL, dout, dummy);
    store<CW>(out(a.dst0, r0) + x, c0n[1]);
    store<CW>(out(a.ddst0, r0) + x, dout);

#pragma unroll 1
    for (int k = 0; k < R; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = r0 + k + u;
            // prefetch for the next step into slots this step no longer reads
            c1[(u + 3) & 3] = load<CW>(at(s1, i + 3) + x);
            c0o[u & 1] = load<CW>(at(s0, i + 2) + x);
            m0[u & 1] = load<CW>(at(e0, i + 2) + x);
            m1[(u + 1) & 1] = load<CW>(at(e1, i + 1) + x);
            const uint32_t g1 = (uint32_t)__builtin_amdgcn_readlane((int)edge_c1, k + u);
            const uint32_t g0 = (uint32_t)__builtin_amdgcn_readlane((int)edge_c0, k + u);
            Words<CW> c1n, d0n, d1n;
            if ((u & 1) == 0) {  // i even relative to r0, so even: P = 1 for both updates
                c0n[(u + 2) & 3] = creutz_row<CW, 1, false>(c0o[(u + 1) & 1], m0[(u + 1) & 1], c1[u & 3],
                                                            c1[(u + 2) & 3], c1[(u + 1) & 3], g1, d0n, dummy);
                c1n = creutz_row<CW, 1, true>(c1[u & 3], m1[u & 1], c0n[u & 3], c0n[(u + 2) & 3], c0n[(u + 1) & 3],
                                              g0, d1n, sad);
            } else {
                c0n[(u + 2) & 3] = creutz_row<CW, 0, false>(c0o[(u + 1) & 1], m0[(u + 1) & 1], c1[u & 3],
                                                            c1[(u + 2) & 3], c1[(u + 1) & 3], g1, d0n, dummy);
                c1n = creutz_row<CW, 0, true>(c1[u & 3], m1[u & 1], c0n[u & 3], c0n[(u + 2) & 3], c0n[(u + 1) & 3],
                                              g0, d1n, sad);
            }
            if (k + u + 1 < R) {
                store<CW>(out(a.dst0, i + 1) + x, c0n[(u + 2) & 3]);
                store<CW>(out(a.ddst0, i + 1) + x, d0n);
            }
            store<CW>(out(a.dst1, i) + x, c1n);
            store<CW>(out(a.ddst1, i) + x, d1n);
            ups += popcnt<CW>(c1n) + popcnt<CW>(c0n[(u + 1) & 3]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // per-wave partials: B = 16 * words - 2 * sad, M = 2 * ups - 8 * words
    const int64_t words = (int64_t)R * CW;
    int64_t b = wave_sum_i64(16 * words - 2 * (int64_t)sad);
    int64_t m = wave_sum_i64(2 * (int64_t)ups - 8 * words);
    if (lane == 0) {
        a.part[2 * tile] = b;
        a.part[2 * tile + 1] = m;
    }
}

template <int CW, int R>
static void launch_cf(const CreutzFusedArgs& a, const PartialReduce& red, hipStream_t s) {
    k_creutz_fused<CW, R><<<(a.n_tiles + 3u) / 4u, 256, 0, s>>>(a, red);
}

hipError_t launch_creutz_fused(const CreutzFusedArgs& a, uint32_t cw, uint32_t rows, const PartialReduce& red,
                               hipStream_t s) {
#define ISING_CF_CASE(CWv, Rv)                 \
    if (cw == CWv && rows == Rv) {             \
        launch_cf<CWv, Rv>(a, red, s);         \
        return hipGetLastError();              \
    }
    ISING_CF_CASE(1, 8) ISING_CF_CASE(1, 16) ISING_CF_CASE(1, 32) ISING_CF_CASE(1, 64)
    ISING_CF_CASE(2, 8) ISING_CF_CASE(2, 16) ISING_CF_CASE(2, 32) ISING_CF_CASE(2, 64)
    ISING_CF_CASE(4, 8) ISING_CF_CASE(4, 16) ISING_CF_CASE(4, 32) ISING_CF_CASE(4, 64)
#undef ISING_CF_CASE
    return hipErrorInvalidValue;
}

}  // namespace ising
