// Device building blocks of the gfx950 checkerboard Metropolis engine.
//
// Lattice storage ("colour planes"): the sites of colour c = (i + j) & 1 of
// row i are stored contiguously in plane c, row i, at byte m = j >> 1, so a
// row of a plane holds H = L/2 bytes and plane c's byte (i, m) is the site
// j = 2m + ((i + c) & 1). This is the two-lattice layout Section 5 of the
// paper proposes to remove the checkerboard branch. Each byte is 1 for an up
// spin and 0 for a down spin, so four sites pack into a 32-bit word and
// neighbour counts are byte-wise sums (SWAR), never exceeding 4.
//
// Neighbours of plane-c byte (i, m), with p = (i + c) & 1, all in plane 1-c:
// (i-1, m), (i+1, m), (i, m) and (i, m-1) if p == 0 or (i, m+1) if p == 1,
// indices taken modulo L rows and H bytes.
//
// Draw keying (fixed by the public header): site ordinal ord = i*H + m within
// its colour, Philox counter (ord >> 2, t, c, d). When H % 4 == 0 a 32-bit
// word of a plane row is exactly one Philox call: q = i*(H/4) + word, and
// output word b belongs to byte b.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Consecutive logical blocks land on the same XCD (blocks are dealt
// round-robin over the 8 XCDs), so neighbouring rows share an L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t nblocks) {
    const uint32_t b = blockIdx.x;
    if ((nblocks & 7u) != 0u) return b;
    return (b & 7u) * (nblocks >> 3) + (b >> 3);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// a ^ b ^ c in one gfx950 VALU op (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon et al., SC 2011) of counter (x0, c1, c2, c3) and key
// (k0, k1), given the first round's product p0 = M0 * x0 (64-bit). Only x0
// varies across lanes in this engine; c1..c3 and the key are wave-uniform,
// so the uniform halves of the first rounds stay on the scalar unit and the
// vector cost is about 37 ops per call: each later round is two 32x32->64
// multiplies (v_mad_u64_u32) and two three-way XORs. Callers whose x0 is a
// uniform part plus a lane part pass p0 = M0 * lane + M0 * uniform, one
// multiply-add (x0 < 2^32 without wrap, so the two products agree).
__device__ __forceinline__ uint4 philox_p0(uint64_t p0_first, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
    uint32_t x0 = 0, x1 = c1, x2 = c2, x3 = c3;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = r == 0 ? p0_first : (uint64_t)kPhiloxM0 * x0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * x2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), hi1 = (uint32_t)(p1 >> 32);
        // the round keys are wave-uniform: keep them in scalar registers (the
        // compiler otherwise copies them into vector registers in long loops)
        const uint32_t rk0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k0);
        const uint32_t rk1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k1);
        uint32_t y0, y2;
        if (r < 2) {  // at least one operand of each XOR is uniform
            y0 = hi1 ^ x1 ^ rk0;
            y2 = hi0 ^ x3 ^ rk1;
        } else if (r == 2) {  // x3 is still uniform here
            y0 = xor3(hi1, x1, rk0);
            y2 = hi0 ^ x3 ^ rk1;
        } else {
            y0 = xor3(hi1, x1, rk0);
            y2 = xor3(hi0, x3, rk1);
        }
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return make_uint4(x0, x1, x2, x3);
}

// m * x + a (64-bit) in one v_mad_u64_u32: x and m in vector registers, a
// wave-uniform (scalar registers). Written out because the compiler would
// otherwise merge M0 * x + M0 * r into M0 * (x + r) with a 64-bit sum, a
// 64 x 32-bit product of three instructions and a move.
__device__ __forceinline__ uint64_t mad_u64_uniform(uint32_t x, uint32_t m, uint64_t a) {
    uint64_t d, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(carry) : "v"(x), "v"(m), "s"(a));
    return d;
}

// m * x (64-bit) in one v_mad_u64_u32, for the same reason.
__device__ __forceinline__ uint64_t mul_u64(uint32_t x, uint32_t m) {
    uint64_t d, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(d), "=s"(carry) : "v"(x), "v"(m));
    return d;
}

// Philox4x32-10 of counter (q, c1, c2, c3) and key (k0, k1).
__device__ __forceinline__ uint4 philox(uint32_t q, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
    return philox_p0((uint64_t)kPhiloxM0 * q, c1, c2, c3, k0, k1);
}

// Acceptance tables, indexed by code = 8*s + n (s = spin bit, n = number of
// up neighbours, 0..4). thr_m1[code] = thr - 1 (accept iff u <= thr_m1),
// valid when no threshold is 0; thr_lo/thr_hi hold the full thr in [0, 2^32]
// for the exact path (accept iff u < thr) used when some threshold is 0.
struct AcceptTable {
    uint32_t thr_m1[16];
    uint32_t thr_lo[16];
    uint32_t thr_hi[16];
};

// LDS copy of the table. t32 is read at byte offset 4*code, t64 and tm at
// 8*code. tm[code] = (2^32 - thr mod 2^32, X): for a draw u, the high word
// of u + (X 2^32 + lo) is X + [u >= thr] when thr >= 1 and X when thr = 0.
// X = 1 - s for thr >= 1 and X = s for thr = 0, so bit 0 of that high word
// is the site's new spin bit in every case (thr = 2^32: lo = 0, a certain
// flip; thr = 0: lo = 0, never a flip).
struct LdsTable {
    uint32_t t32[16];
    uint2 t64[16];
    uint2 tm[16];
};

__device__ __forceinline__ uint2 mad_entry(uint32_t code, uint32_t thr_lo, uint32_t thr_hi) {
    const uint32_t s = code >> 3;
    const bool never = thr_lo == 0u && thr_hi == 0u;
    return make_uint2(0u - thr_lo, never ? s : 1u - s);
}

__device__ __forceinline__ void load_table(LdsTable& lt, const AcceptTable& at) {
    const uint32_t tid = threadIdx.x;
    if (tid < 16) {
        lt.t32[tid] = at.thr_m1[tid];
        lt.t64[tid] = make_uint2(at.thr_lo[tid], at.thr_hi[tid]);
        lt.tm[tid] = mad_entry(tid, at.thr_lo[tid], at.thr_hi[tid]);
    }
}

template <typename T>
__device__ __forceinline__ T lds_at(const T* base, uint32_t byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Flip mask of one word of four sites: byte b is 1 when site b's move is
// accepted. code4 holds 4 * (8 s + n) per byte (s the spin bit, n the number
// of up neighbours) and r the four draws of the word's Philox call.
template <bool EXACT>
__device__ __forceinline__ uint32_t flip_mask_code(const LdsTable& lt, uint32_t code4, uint4 r) {
    if (!EXACT) {
        const uint32_t a0 = lds_at(lt.t32, code4 & 0xffu);
        const uint32_t a1 = lds_at(lt.t32, (code4 >> 8) & 0xffu);
        const uint32_t a2 = lds_at(lt.t32, (code4 >> 16) & 0xffu);
        const uint32_t a3 = lds_at(lt.t32, code4 >> 24);
        const uint32_t f0 = r.x <= a0 ? 0x00000001u : 0u;
        const uint32_t f1 = r.y <= a1 ? 0x00000100u : 0u;
        const uint32_t f2 = r.z <= a2 ? 0x00010000u : 0u;
        const uint32_t f3 = r.w <= a3 ? 0x01000000u : 0u;
        return (f0 | f1) | (f2 | f3);
    } else {
        const uint32_t code8 = code4 << 1;  // per byte: 8 * (8 s + n) <= 96
        const uint2 a0 = lds_at(lt.t64, code8 & 0xffu);
        const uint2 a1 = lds_at(lt.t64, (code8 >> 8) & 0xffu);
        const uint2 a2 = lds_at(lt.t64, (code8 >> 16) & 0xffu);
        const uint2 a3 = lds_at(lt.t64, code8 >> 24);
        auto lt64 = [](uint32_t u, uint2 a) {
            return (uint64_t)u < (((uint64_t)a.y << 32) | a.x);
        };
        const uint32_t f0 = lt64(r.x, a0) ? 0x00000001u : 0u;
        const uint32_t f1 = lt64(r.y, a1) ? 0x00000100u : 0u;
        const uint32_t f2 = lt64(r.z, a2) ? 0x00010000u : 0u;
        const uint32_t f3 = lt64(r.w, a3) ? 0x01000000u : 0u;
        return (f0 | f1) | (f2 | f3);
    }
}

// 8 * (byte 0 of c) in one op: a shift that reads byte 0 of its operand.
__device__ __forceinline__ uint32_t byte0_x8(uint32_t c) {
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r)
        : "v"(c));
    return r;
}

// High word of u + e (u a 32-bit draw, e a 64-bit table entry) in one
// v_mad_u64_u32 (u times the inline constant 1, plus e). Written out because
// the compiler otherwise forms the sum with two or more instructions.
__device__ __forceinline__ uint32_t mad_hi(uint32_t u, uint64_t e) {
    uint64_t d, carry;
    asm("v_mad_u64_u32 %0, %1, %2, 1, %3" : "=v"(d), "=s"(carry) : "v"(u), "v"(e));
    return (uint32_t)(d >> 32);
}

// New spins of one word of four sites. code holds 8 s + n per byte (s the
// spin bit, n the number of up neighbours; at most 12, so bits 5..7 of every
// byte are 0 and a field of 11 bits starting 3 below a byte is 8 times that
// byte), r the four draws of the word's Philox call. One LDS read of the
// site's tm entry and one 64-bit multiply-add give the new spin bit (see
// LdsTable), for any thresholds in [0, 2^32]; two byte permutes and one
// three-input logic op assemble the word.
__device__ __forceinline__ uint32_t accept_word(const LdsTable& lt, uint32_t code, uint4 r) {
    const uint64_t e0 = lds_at(reinterpret_cast<const uint64_t*>(lt.tm), byte0_x8(code));
    const uint64_t e1 = lds_at(reinterpret_cast<const uint64_t*>(lt.tm), __builtin_amdgcn_ubfe(code, 5, 11));
    const uint64_t e2 = lds_at(reinterpret_cast<const uint64_t*>(lt.tm), __builtin_amdgcn_ubfe(code, 13, 11));
    const uint64_t e3 = lds_at(reinterpret_cast<const uint64_t*>(lt.tm), code >> 21);
    const uint32_t d0 = mad_hi(r.x, e0), d1 = mad_hi(r.y, e1), d2 = mad_hi(r.z, e2), d3 = mad_hi(r.w, e3);
    // byte b of the result = byte 0 of d_b (bit 1 of it may be set: masked)
    const uint32_t w01 = __builtin_amdgcn_perm(d1, d0, 0x0c0c0400u);
    const uint32_t w23 = __builtin_amdgcn_perm(d3, d2, 0x04000c0cu);
    return (w01 | w23) & 0x01010101u;
}

// The same from the spin bits W and the up-neighbour counts n.
template <bool EXACT>
__device__ __forceinline__ uint32_t flip_mask(const LdsTable& lt, uint32_t W, uint32_t n, uint4 r) {
    return flip_mask_code<EXACT>(lt, (W << 5) | (n << 2), r);
}

// Same-row neighbour word: bytes m+1..m+4 (p == 1) or m-1..m+2 (p == 0) of
// the other plane, from the word O at m..m+3 and the word after / before it.
__device__ __forceinline__ uint32_t shifted(uint32_t O, uint32_t O_next, uint32_t O_prev, uint32_t p) {
    return p ? __builtin_amdgcn_alignbyte(O_next, O, 1) : __builtin_amdgcn_alignbyte(O, O_prev, 3);
}

// Observable partial sums of one updated colour-1 word (new spins Wn, up
// counts n of its colour-0 neighbours). Each lattice edge joins colour 0 to
// colour 1, so the bond sum is sum over colour-1 sites of s * (sum of
// neighbours) = sum over those sites of (2 a - 4), a = neighbours aligned
// with the site = 4 - |4 s - n|. Per word: B = 16 - 2 * sum_b |4 s_b - n_b|,
// one v_sad_u8.
__device__ __forceinline__ uint32_t sad_misaligned(uint32_t Wn, uint32_t n, uint32_t acc) {
    return __builtin_amdgcn_sad_u8(Wn << 2, n, acc);
}

// The same from n4 = 4 n per byte; adds 4 * sum_b |4 s_b - n_b|.
__device__ __forceinline__ uint32_t sad_misaligned4(uint32_t Wn, uint32_t n4, uint32_t acc) {
    return __builtin_amdgcn_sad_u8(Wn << 4, n4, acc);
}

// Pointers read from descriptors in memory are generic; naming the global
// address space lets the compiler use global (not flat) loads and stores.
typedef __attribute__((address_space(1))) uint32_t global_u32;
__device__ __forceinline__ global_u32* as_global(uint32_t* p) { return (global_u32*)p; }

}  // namespace ising
