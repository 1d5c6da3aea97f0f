// Device pieces of the fused one-pass walk, shared by the single-lattice
// kernel (ising_fused.hip) and the multi-lattice stepped kernel
// (ising_multi_fused.hip): row loads and stores through buffer resources,
// the DPP lane shifts, and the update of one lane's words of a plane row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {
namespace {

// DPP controls (GFX9): whole-wave shift by one lane.
constexpr int kDppWaveShl1 = 0x130;  // lane l reads lane l+1
constexpr int kDppWaveShr1 = 0x138;  // lane l reads lane l-1

// lane l gets v of lane l+1; lane 63 gets `edge`.
__device__ __forceinline__ uint32_t from_right(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, kDppWaveShl1, 0xf, 0xf, false);
}
// lane l gets v of lane l-1; lane 0 gets `edge`.
__device__ __forceinline__ uint32_t from_left(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, kDppWaveShr1, 0xf, 0xf, false);
}

// A compile-time step index for the generic lambdas that stand for the
// four unrolled steps of a tile walk.
template <int N>
struct Step {
    static constexpr int value = N;
};

template <int CW>
struct Row {
    uint32_t v[CW];
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Raw buffer over a whole plane; word 3 is the gfx9 resource format for
// untyped 32-bit data.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const uint32_t* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(p), 0, -1, 0x00020000);
}

// Cache policy of the row loads and stores: nontemporal (the NT bit of
// gfx950's buffer instructions). A sweep reads every row once and writes it
// once, and the planes of any lattice this walk streams are far larger than
// the caches; with the hint the 32768^2 sweep measured 2-5% faster (wave
// tiles and full rows), the stepped batch walk unchanged.
constexpr int kRowCachePolicy = 2;

// CW words at byte offset xb (lane) + soff (row, uniform) of a plane.
template <int CW>
__device__ __forceinline__ Row<CW> ld(__amdgpu_buffer_rsrc_t rs, uint32_t xb, uint32_t soff) {
    Row<CW> r;
    if constexpr (CW == 4) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, xb, soff, kRowCachePolicy);
        r.v[0] = v.x; r.v[1] = v.y; r.v[2] = v.z; r.v[3] = v.w;
    } else if constexpr (CW == 2) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, xb, soff, kRowCachePolicy);
        r.v[0] = v.x; r.v[1] = v.y;
    } else {
        r.v[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, xb, soff, kRowCachePolicy);
    }
    return r;
}

// CW words to byte offset off of a plane. The whole offset is in the vector
// operand and the scalar offset is the constant 0: a store wider than 64
// bits reads part of its data registers after issue, and with a register in
// the scalar offset field the compiler does not keep the next instructions
// from overwriting them (seen on gfx950 as wrong words in the last lanes of
// each group of 16); with a constant there it does.
template <int CW>
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t rs, uint32_t off, const Row<CW>& r) {
    if constexpr (CW == 4) {
        const u32x4 v = {r.v[0], r.v[1], r.v[2], r.v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, kRowCachePolicy);
    } else if constexpr (CW == 2) {
        const u32x2 v = {r.v[0], r.v[1]};
        __builtin_amdgcn_raw_buffer_store_b64(v, rs, off, 0, kRowCachePolicy);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(r.v[0], rs, off, 0, kRowCachePolicy);
    }
}

// accept_word in two parts: the four LDS table entries of a word's sites,
// read as soon as the word's codes are known, and the new spins from them
// and the word's draws. update_row reads the entries before the word's
// Philox call, so the LDS latency is spent behind the 37 Philox operations
// rather than right before the entries' use.
struct AcceptEntries {
    uint64_t e0, e1, e2, e3;
};

__device__ __forceinline__ AcceptEntries accept_entries(const LdsTable& lt, uint32_t code) {
    const uint64_t* tm = reinterpret_cast<const uint64_t*>(lt.tm);
    return {lds_at(tm, byte0_x8(code)), lds_at(tm, __builtin_amdgcn_ubfe(code, 5, 11)),
            lds_at(tm, __builtin_amdgcn_ubfe(code, 13, 11)), lds_at(tm, code >> 21)};
}

__device__ __forceinline__ uint32_t accept_from(const AcceptEntries& e, uint4 r) {
    const uint32_t d0 = mad_hi(r.x, e.e0), d1 = mad_hi(r.y, e.e1), d2 = mad_hi(r.z, e.e2), d3 = mad_hi(r.w, e.e3);
    const uint32_t w01 = __builtin_amdgcn_perm(d1, d0, 0x0c0c0400u);
    const uint32_t w23 = __builtin_amdgcn_perm(d3, d2, 0x04000c0cu);
    return (w01 | w23) & 0x01010101u;
}

// Update one lane's CW words of a plane row. P = (i + c) & 1 selects the
// same-row neighbour side; `edge` is the word just outside the tile on that
// side (right for P == 1, left for P == 0) of the `same` row. Word w's draw
// counter is q = rowoff + xw[w] (rowoff: the row's word offset, wave-uniform
// unless PACKED; xw[w] = xw[0] + w), so the first Philox product M0 * q is
// one multiply-add per word: M0 * xw[0] + M0 * (rowoff + w), the second
// term on the scalar unit.
//
// RAGGED: the tile may end before lane 63; `is_last` marks the last lane
// that holds words of the lattice, whose right neighbour is then `edge`
// rather than the next lane's word. PACKED: the wave holds several row
// bands side by side; `is_first` marks a band's first lane, whose left
// neighbour is then `edge` rather than the previous lane's word, and `edge`
// is per lane (its band's).
template <int CW, int P, bool OBS, bool RAGGED = false, bool PACKED = false>
__device__ __forceinline__ Row<CW> update_row(const LdsTable& lt, const Row<CW>& own, const Row<CW>& up,
                                              const Row<CW>& dn, const Row<CW>& same, uint32_t edge,
                                              const Row<CW>& xw, uint32_t rowoff, uint32_t t, uint32_t c,
                                              uint32_t k0, uint32_t k1, uint32_t& sad,
                                              bool is_last = false, bool is_first = false) {
    uint32_t nb = P ? from_right(same.v[0], edge) : from_left(same.v[CW - 1], edge);
    if (RAGGED && P && is_last) nb = edge;
    if (PACKED && !P && is_first) nb = edge;
    Row<CW> out;
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
        const uint32_t n = (up.v[w] + dn.v[w] + S) + same.v[w];  // up neighbours per byte
        const uint32_t code = (own.v[w] << 3) + n;                 // 8 s + n per byte
        uint64_t p0;
        if (PACKED)  // rows differ between the wave's bands: q per lane
            p0 = mul_u64(rowoff + xw.v[w], kPhiloxM0);
        else  // xw[w] = xw[0] + w: the word's offset joins the uniform part
            p0 = mad_u64_uniform(xw.v[0], kPhiloxM0, (uint64_t)kPhiloxM0 * (rowoff + (uint32_t)w));
        const AcceptEntries ent = accept_entries(lt, code);
        __builtin_amdgcn_sched_barrier(0);  // the LDS reads stay ahead of the Philox call
        const uint4 r = philox_p0(p0, t, c, 0u, k0, k1);
        const uint32_t Wn = accept_from(ent, r);
        out.v[w] = Wn;
        if (OBS) sad = sad_misaligned(Wn, n, sad);
    }
    return out;
}

__device__ __forceinline__ uint32_t wrap_row(int i, uint32_t L) {
    return (uint32_t)(i < 0 ? i + (int)L : (i >= (int)L ? i - (int)L : i));
}

}  // namespace
}  // namespace ising
