// Bit-packed Metropolis update of one 32-site word, shared by the kernels
// that keep lattices at one bit per site (the resident batch and the
// band-resident single lattice).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

// Plane c of an L x L lattice is kept as L rows of Wr =
// ceil(Hw / 8) 32-bit words; bit 4 j + b of word k of row i is the site of
// byte m = 32 k + 4 j + b of the plane row (quad 8 k + j, Philox output b),
// so a word holds the four draws of eight consecutive Philox calls. Bits
// past the H = 4 Hw sites of a row are zero and stay zero.
//
// For h = 0 the acceptance threshold of a site depends only on the number m
// of its neighbours that disagree with it (Delta E = 2 J (4 - 2 m) when it
// flips), so a word's update is bitwise: the four disagreement masks give
// the masks of the classes m = 0, 1 (J > 0) or m = 3, 4 (J < 0) whose
// threshold is below one, each site's draw is compared with both class
// thresholds (bit by bit, shifted into two masks of failed compares), and a
// site flips unless it is in such a class and its compare failed. The draws and thresholds
// are those of the byte kernels, so the results are the same bit for bit.
//
// For h != 0 the threshold depends on the site's spin s as well: the class
// is (s, m), ten of them, with threshold thr(code 8 s + n), n = s ? 4 - m :
// m up neighbours. A bit-sliced count of the four disagreement masks gives
// the five masks "exactly m disagree"; per class that is never accepted
// (threshold 0) its sites are rejected outright, per class that is always
// accepted (threshold 2^32) nothing is done, and per remaining class its
// sites' draws are compared with its threshold as above.

// acc = 2 acc + (r > thr_m1): the borrow of thr_m1 - r shifted in, two VALU
// operations (the compiler's own form of this takes three).
__device__ __forceinline__ uint32_t shift_in_reject(uint32_t acc, uint32_t r, uint32_t thr_m1) {
    uint32_t diff;
    asm("v_sub_co_u32 %1, vcc, %3, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc"
        : "+v"(acc), "=&v"(diff)
        : "v"(r), "s"(thr_m1)
        : "vcc");
    return acc;
}

// One word's worth of the two threshold compares: bit 4 j + b of *ra (*rb)
// is set when draw b of quad j fails class A's (B's) threshold.
__device__ __forceinline__ void bits_compares(uint32_t q0, uint32_t t, uint32_t c, uint32_t k0, uint32_t k1,
                                              uint32_t thra_m1, uint32_t thrb_m1, uint32_t& ra, uint32_t& rb) {
    uint32_t a = 0, b = 0;
#pragma unroll
    for (int j = 7; j >= 0; --j) {
        const uint4 r = philox(q0 + (uint32_t)j, t, c, 0u, k0, k1);
        // highest bit first: after 32 steps bit 4 j + b holds site (j, b)
        a = shift_in_reject(a, r.w, thra_m1);
        b = shift_in_reject(b, r.w, thrb_m1);
        a = shift_in_reject(a, r.z, thra_m1);
        b = shift_in_reject(b, r.z, thrb_m1);
        a = shift_in_reject(a, r.y, thra_m1);
        b = shift_in_reject(b, r.y, thrb_m1);
        a = shift_in_reject(a, r.x, thra_m1);
        b = shift_in_reject(b, r.x, thrb_m1);
    }
    ra = a;
    rb = b;
}

struct BitsLattice {
    uint32_t L, Hw, Wr;
    uint32_t hb;        // index of the last valid bit of a row's last word
    uint32_t last_valid;  // valid-bit mask of a row's last word
    uint32_t thra_m1, thrb_m1;  // class thresholds minus one (when not never)
    bool never_a, never_b;
    bool ferro;         // classes A, B are m = 1, 0 (else m = 3, 4)
    // general classes (h != 0): class (s, m) is entry 5 s + m
    uint32_t cls_m1[10];    // threshold minus one, for the compared classes
    uint32_t cls_kind[10];  // kClassAlways, kClassNever or kClassCompare
};

constexpr uint32_t kClassAlways = 0, kClassNever = 1, kClassCompare = 2;

// Rejection mask of one class over the 32 draws of a word (bit 4 j + b set
// when draw b of quad j is at or above the class threshold).
__device__ __forceinline__ uint32_t class_rejects(const uint4 (&r)[8], uint32_t thr_m1) {
    uint32_t acc = 0;
#pragma unroll
    for (int j = 7; j >= 0; --j) {
        acc = shift_in_reject(acc, r[j].w, thr_m1);
        acc = shift_in_reject(acc, r[j].z, thr_m1);
        acc = shift_in_reject(acc, r[j].y, thr_m1);
        acc = shift_in_reject(acc, r[j].x, thr_m1);
    }
    return acc;
}

// Sites of a word that keep their spin, for the general (s, m) classes.
__device__ __forceinline__ uint32_t general_rejects(const BitsLattice& bl, uint32_t own, uint32_t a, uint32_t b,
                                                    uint32_t d, uint32_t e, uint32_t q0, uint32_t t, uint32_t c,
                                                    uint32_t k0, uint32_t k1) {
    uint4 r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = philox(q0 + (uint32_t)j, t, c, 0u, k0, k1);
    // bit-sliced m = a + b + d + e: ones, twos and fours planes
    const uint32_t x = a ^ b, y = a & b, z = d ^ e, w = d & e;
    const uint32_t ones = x ^ z, cz = x & z;
    const uint32_t twos = y ^ w ^ cz;
    const uint32_t fours = (y & w) | (cz & (y ^ w));
    const uint32_t exactly[5] = {~(ones | twos | fours), ones & ~twos, twos & ~ones, ones & twos, fours};
    uint32_t reject = 0;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
        const uint32_t sm = sp ? own : ~own;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const uint32_t kind = bl.cls_kind[5 * sp + m];
            if (kind == kClassNever) reject |= sm & exactly[m];
            else if (kind == kClassCompare) reject |= sm & exactly[m] & class_rejects(r, bl.cls_m1[5 * sp + m]);
        }
    }
    return reject;
}

// Same-row neighbours (in the other plane) of the 32 sites of a word: O is
// the other plane's word at the same position, On / Op the next and previous
// words of that row (wrapping), top / top_p the last valid bit of this word
// and of the previous one, valid the valid-bit mask of this word, odd the
// parity of row + colour: the neighbour of site m is m + 1 when it is odd,
// else m - 1.
__device__ __forceinline__ uint32_t bits_same_row(uint32_t O, uint32_t On, uint32_t Op, uint32_t top, uint32_t top_p,
                                                  uint32_t valid, uint32_t odd) {
    const uint32_t s_up = (O >> 1) | ((On & 1u) << top);
    const uint32_t s_dn = ((O << 1) | ((Op >> top_p) & 1u)) & valid;
    return odd ? s_up : s_dn;
}

// Sites of the word `own` (colour c, first quad q0, sweep t) whose proposal
// is rejected, given its four neighbour words U, D, O and S.
template <bool GENERAL>
__device__ __forceinline__ uint32_t bits_reject(const BitsLattice& bl, uint32_t own, uint32_t U, uint32_t D,
                                                uint32_t O, uint32_t S, uint32_t q0, uint32_t t, uint32_t c,
                                                uint32_t k0, uint32_t k1) {
    // disagreement masks
    const uint32_t a = own ^ U, b = own ^ D, d = own ^ O, e = own ^ S;
    if (GENERAL) return general_rejects(bl, own, a, b, d, e, q0, t, c, k0, k1);
    uint32_t ra, rb;
    bits_compares(q0, t, c, k0, k1, bl.thra_m1, bl.thrb_m1, ra, rb);
    if (bl.never_a) ra = 0xffffffffu;
    if (bl.never_b) rb = 0xffffffffu;
    // the two classes
    const uint32_t odd = a ^ b ^ d ^ e;
    const uint32_t pair = (a & b) | (d & e);
    uint32_t ea, eb;
    if (bl.ferro) {
        ea = odd & ~pair;       // exactly one disagrees
        eb = ~(a | b | d | e);  // none
    } else {
        ea = odd & pair;        // exactly three
        eb = a & b & d & e;     // all four
    }
    return (ea & ra) | (eb & rb);
}

// Class thresholds of a bit-packed lattice from its acceptance table (code
// 8 s + n; an up spin with n up neighbours has m = 4 - n disagreeing); mode
// 1 or 2 is the two-class h = 0 update, 3 the general (s, m) classes.
__host__ __device__ inline BitsLattice bits_lattice(const AcceptTable& table, uint32_t L, uint32_t Hw,
                                                   uint32_t mode) {
    BitsLattice bl;
    bl.L = L;
    bl.Hw = Hw;
    bl.Wr = (Hw + 7u) / 8u;
    const uint32_t H = 4u * Hw;
    bl.hb = (H - 1u) & 31u;
    bl.last_valid = bl.hb == 31u ? 0xffffffffu : ((1u << (bl.hb + 1u)) - 1u);
    bl.ferro = mode == 1u;  // (mode 3: the general classes below)
    const uint32_t ma = bl.ferro ? 1u : 3u, mb = bl.ferro ? 0u : 4u;
    auto thr64 = [&](uint32_t m) {
        const uint32_t code = 8u + (4u - m);
        return ((uint64_t)table.thr_hi[code] << 32) | table.thr_lo[code];
    };
    const uint64_t ta = thr64(ma), tb = thr64(mb);
    bl.never_a = ta == 0;
    bl.never_b = tb == 0;
    bl.thra_m1 = ta == 0 ? 0u : (uint32_t)(ta - 1);
    bl.thrb_m1 = tb == 0 ? 0u : (uint32_t)(tb - 1);
#pragma unroll
    for (uint32_t sp = 0; sp < 2; ++sp) {
#pragma unroll
        for (uint32_t m = 0; m < 5; ++m) {
            const uint32_t code = 8u * sp + (sp ? 4u - m : m);
            const uint64_t thr = ((uint64_t)table.thr_hi[code] << 32) | table.thr_lo[code];
            bl.cls_kind[5 * sp + m] = thr == 0 ? kClassNever : (thr >> 32) ? kClassAlways : kClassCompare;
            bl.cls_m1[5 * sp + m] = thr == 0 ? 0u : (uint32_t)(thr - 1);
        }
    }
    return bl;
}

}  // namespace ising
