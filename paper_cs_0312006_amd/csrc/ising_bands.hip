// Band-resident sweeps of one lattice too large for a workgroup's LDS but
// small enough for the LDS of the whole chip (Section 2.2's consecutive
// black and white passes, every one of them kept on chip).
//
// The L rows are split into G bands, band g holding rows [g L / G,
// (g + 1) L / G), one workgroup per band, all resident at once (a
// cooperative launch). A workgroup converts its band of both colour planes
// to bits in LDS (the layout and word update of ising_bits.hpp), runs every
// half-sweep of the launch there and converts the band back at the end, so
// the lattice crosses HBM once per launch rather than once per sweep. A
// wave sweeps its rows in chunks of 64 words, a word per lane.
//
// A band's first and last rows need the rows just outside it, which belong
// to the bands above and below. After each half-sweep the wave that updated
// a band's first (last) row stores each of its words to an edge slot in
// global memory as one 64-bit agent-scope atomic holding the word and a tag,
// the number of the half-sweep (counted across launches from `base`); before
// a half-sweep the wave that updates a first (last) row reads the upper
// (lower) band's slot until every word carries the previous half-sweep's
// tag. A word and its tag travel in one atomic, so no fence orders them:
// the slots are the only memory bands share during a launch, and agent-scope
// atomics reach every XCD without writing back or invalidating the L2 (the
// fences an agent-scope flag would need cost about 40 ns per workgroup,
// serialised over the chip). Only these two waves of a workgroup wait on
// another workgroup; the rest wait only at the workgroup barrier that ends
// each half-sweep. Edge slots alternate between two buffers by half-sweep
// parity: a band cannot publish half-sweep tau + 1 over the slot of tau - 1
// before its neighbour has published tau, which that neighbour does only
// after reading tau - 1.
// The lattice is updated in place: a band's rows in HBM are read by its
// neighbours at their first half-sweep and written back only after the
// band's last one, which waits on both neighbours' second to last.
//
// Tags grow across launches, so slots are cleared only when the 32-bit tag
// would wrap. Every wait gives up after a bounded number of polls, marks
// *err and lets every later wait of the launch fall through, so a launch
// always ends.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "ising_bands.hpp"
#include "ising_bits.hpp"
#include "ising_fused_core.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr uint32_t kBandMaxWaves = 16;
// Polls of an edge word (each a read of its coherent copy and a short sleep)
// before a wait gives up: several seconds.
constexpr uint32_t kBandMaxPolls = 1u << 24;

__device__ __forceinline__ void put_word(uint64_t* p, uint32_t tag, uint32_t w) {
    __hip_atomic_store(p, ((uint64_t)tag << 32) | w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The word at p once its tag is `tag` (the whole wave waits until every
// lane's word has it).
__device__ __forceinline__ uint32_t take_word(const uint64_t* p, uint32_t tag, uint32_t* err) {
    uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t polls = 0;
    while (__ballot((uint32_t)(v >> 32) != tag)) {
        if ((++polls & 255u) == 0u) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (polls >= kBandMaxPolls) {
                __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return (uint32_t)v;
}

// Bit word k of row i of a byte plane (bit 4 j + b is byte b of quad 8 k + j).
__device__ __forceinline__ uint32_t bits_of_bytes(const uint32_t* plane, uint32_t i, uint32_t k, uint32_t Hw) {
    const uint32_t* q = plane + (size_t)i * Hw + 8u * k;
    uint32_t v = 0;
    for (uint32_t j = 0; j < 8u && 8u * k + j < Hw; ++j) v |= ((q[j] * 0x01020408u) >> 24) << (4u * j);
    return v;
}

__device__ __forceinline__ void bytes_of_bits(uint32_t* plane, uint32_t i, uint32_t k, uint32_t Hw, uint32_t v) {
    uint32_t* q = plane + (size_t)i * Hw + 8u * k;
    for (uint32_t j = 0; j < 8u && 8u * k + j < Hw; ++j) q[j] = (((v >> (4u * j)) & 0xfu) * 0x00204081u) & 0x01010101u;
}

// CH: chunks of 64 words a row (Wr <= 64 CH).
template <bool GENERAL, int CH>
__global__ __launch_bounds__(1024) void k_bands(BandArgs a) {
    extern __shared__ uint32_t lat[];  // [plane][band row][Wr]
    __shared__ uint32_t red[kBandMaxWaves][2];
    const BitsLattice& bl = a.bl;
    const uint32_t G = gridDim.x, g = blockIdx.x;
    const uint32_t L = a.L, Hw = a.Hw, Wr = a.Wr;
    const uint32_t r0 = (uint32_t)((uint64_t)g * L / G);
    const uint32_t H = (uint32_t)((uint64_t)(g + 1u) * L / G) - r0;
    const uint32_t P = H * Wr;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t gu = g == 0 ? G - 1u : g - 1u, gd = g + 1u == G ? 0u : g + 1u;

    for (uint32_t w = threadIdx.x; w < 2u * P; w += blockDim.x) {
        const uint32_t c = w >= P ? 1u : 0u, rw = w - c * P, r = rw / Wr;
        lat[w] = bits_of_bytes(c ? a.p1 : a.p0, r0 + r, rw - r * Wr, Hw);
    }
    __syncthreads();

    // per chunk of 64 words, the lane's word and what its update needs
    uint32_t kw[CH], valid[CH], top[CH], kn[CH], kp[CH], top_p[CH], kc[CH];
    bool active[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const uint32_t k = 64u * (uint32_t)ch + lane;
        const bool lastw = k + 1u == Wr;
        kw[ch] = k;
        active[ch] = k < Wr;
        valid[ch] = lastw ? bl.last_valid : 0xffffffffu;
        top[ch] = lastw ? bl.hb : 31u;
        kn[ch] = lastw ? 0u : k + 1u;
        kp[ch] = k == 0 ? Wr - 1u : k - 1u;
        top_p[ch] = k == 0 ? bl.hb : 31u;
        kc[ch] = k < Wr ? k : Wr - 1u;  // lanes past the row poll its last word
    }
    // rows of this wave: r = wv (mod nw), the band's edge rows first
    const uint32_t nrows = H > wv ? (H - 1u - wv) / nw + 1u : 0u;
    const bool owns_last = (H - 1u) % nw == wv;
    const size_t slot_words = (size_t)G * 2u * Wr;
    const uint32_t summer = nw > 1u ? 64u : 0u;  // a thread off the first wave's edge row
    uint32_t mis = 0, ups = 0;

    for (uint32_t tau = 0; tau < 2u * a.n; ++tau) {
        const uint32_t c = tau & 1u, t = a.t0 + (tau >> 1);
        uint32_t* own_p = lat + c * P;
        const uint32_t* oth_p = lat + (1u - c) * P;
        const uint32_t* oth_g = c ? a.p0 : a.p1;  // the other plane in HBM (first half-sweep)
        const uint64_t* in_slot = a.pub + (size_t)((tau - 1u) & 1u) * slot_words;
        uint64_t* out_slot = a.pub + (size_t)(tau & 1u) * slot_words;
        const uint32_t tag_in = a.base + tau, tag_out = a.base + tau + 1u;
        for (uint32_t j = 0; j < nrows; ++j) {
            uint32_t r;
            if (owns_last && wv != 0u) r = j == 0 ? H - 1u : wv + (j - 1u) * nw;
            else if (owns_last && H > 1u) r = j == 0 ? 0u : j == 1u ? H - 1u : (j - 1u) * nw;
            else r = wv + j * nw;
            const uint32_t i = r0 + r;
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) {
                const uint32_t k = kw[ch];
                uint32_t U = 0, D = 0;
                if (r == 0) {
                    if (tau == 0) {
                        if (active[ch]) U = bits_of_bytes(oth_g, i == 0 ? L - 1u : i - 1u, k, Hw);
                    } else {
                        U = take_word(in_slot + (2u * gu + 1u) * Wr + kc[ch], tag_in, a.err);
                    }
                } else if (active[ch]) {
                    U = oth_p[(r - 1u) * Wr + k];
                }
                if (r == H - 1u) {
                    if (tau == 0) {
                        if (active[ch]) D = bits_of_bytes(oth_g, i + 1u == L ? 0u : i + 1u, k, Hw);
                    } else {
                        D = take_word(in_slot + 2u * gd * Wr + kc[ch], tag_in, a.err);
                    }
                } else if (active[ch]) {
                    D = oth_p[(r + 1u) * Wr + k];
                }
                if (active[ch]) {
                    const uint32_t own = own_p[r * Wr + k];
                    const uint32_t O = oth_p[r * Wr + k], On = oth_p[r * Wr + kn[ch]], Op = oth_p[r * Wr + kp[ch]];
                    const uint32_t S = bits_same_row(O, On, Op, top[ch], top_p[ch], valid[ch], (i + c) & 1u);
                    const uint32_t reject = bits_reject<GENERAL>(bl, own, U, D, O, S, i * Hw + 8u * k, t, c, a.k0, a.k1);
                    const uint32_t nwd = own ^ (valid[ch] & ~reject);
                    own_p[r * Wr + k] = nwd;
                    if (r == 0) put_word(out_slot + 2u * g * Wr + k, tag_out, nwd);
                    if (r == H - 1u) put_word(out_slot + (2u * g + 1u) * Wr + k, tag_out, nwd);
                    if (c) {
                        // bonds of this colour-1 word, all final now, that disagree
                        mis += __builtin_popcount(nwd ^ U) + __builtin_popcount(nwd ^ D) +
                               __builtin_popcount(nwd ^ O) + __builtin_popcount(nwd ^ S);
                    }
                    ups += __builtin_popcount(nwd);
                }
            }
        }
        if (c) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                mis += __shfl_xor(mis, off, 64);
                ups += __shfl_xor(ups, off, 64);
            }
            if (lane == 0) {
                red[wv][0] = mis;
                red[wv][1] = ups;
            }
            mis = 0;
            ups = 0;
        }
        __syncthreads();
        if (c && threadIdx.x == summer) {
            int64_t sm = 0, su = 0;
            for (uint32_t w = 0; w < nw; ++w) {
                sm += red[w][0];
                su += red[w][1];
            }
            // the band's colour-1 sites own 2 H L bonds, each counted once
            const int64_t HL = (int64_t)H * L;
            int64_t* p = a.part + 2u * ((size_t)(tau >> 1) * G + g);
            p[0] = 2 * HL - 2 * sm;
            p[1] = 2 * su - HL;
        }
    }

    for (uint32_t w = threadIdx.x; w < 2u * P; w += blockDim.x) {
        const uint32_t c = w >= P ? 1u : 0u, rw = w - c * P, r = rw / Wr;
        bytes_of_bits(c ? a.p1 : a.p0, r0 + r, rw - r * Wr, Hw, lat[w]);
    }
}

// Byte-resident bands. Sides whose plane rows are 64 CW words (CW = 1, 2,
// 4 or 8: L = 512, 1024, 2048, 4096) can keep their bands as the byte words
// of the HBM planes (eight times the LDS of bits), a wave a row and CW words
// a lane, updated with the fused kernels' word update (update_row: a table
// read and one multiply-add a site, against two threshold compares a site
// in the bit layout). Edge rows still travel as tagged bit words, so slots,
// tags, waits and the in-place protocol are those of k_bands.

// The bits of a lane's CW byte words in the bit layout of ising_bits.hpp
// (site b of quad q is bit 4 (q mod 8) + b of bit word q / 8), OR-ed over
// the 8 / CW lanes that share a bit word: every lane of such a group ends
// with the group's whole word.
template <int CW>
__device__ __forceinline__ uint32_t bit_word_of(const Row<CW>& r, uint32_t x) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < CW; ++j) v |= ((r.v[j] * 0x01020408u) >> 24) << (4u * ((x + (uint32_t)j) & 7u));
#pragma unroll
    for (int off = 1; off < 8 / CW; off <<= 1) v |= (uint32_t)__shfl_xor((int)v, off, 64);
    return v;
}

// A lane's CW byte words (quads x .. x + CW - 1) from the bit word holding them.
template <int CW>
__device__ __forceinline__ Row<CW> bytes_of_bit_word(uint32_t v, uint32_t x) {
    Row<CW> r;
#pragma unroll
    for (int j = 0; j < CW; ++j)
        r.v[j] = (((v >> (4u * ((x + (uint32_t)j) & 7u))) & 0xfu) * 0x00204081u) & 0x01010101u;
    return r;
}

template <int CW>
__device__ __forceinline__ Row<CW> words_at(const uint32_t* p) {
    Row<CW> r;
#pragma unroll
    for (int j = 0; j < CW; ++j) r.v[j] = p[j];
    return r;
}

// In LDS a band row is stored lane-major: word j of lane l (row word CW l +
// j) at j 64 + l, so the 64 lanes reading their word j touch 64
// consecutive words (row-major, CW words a lane apart, 8 lanes hit each
// bank when CW = 8).
template <int CW>
__device__ __forceinline__ uint32_t lds_slot(uint32_t col) {
    return (col % (uint32_t)CW) * 64u + col / (uint32_t)CW;
}

template <int CW>
__device__ __forceinline__ Row<CW> lds_words(const uint32_t* row, uint32_t lane) {
    Row<CW> r;
#pragma unroll
    for (int j = 0; j < CW; ++j) r.v[j] = row[(uint32_t)j * 64u + lane];
    return r;
}

template <int CW>
__global__ __launch_bounds__(1024) void k_bands_bytes(BandArgs a) {
    extern __shared__ uint32_t lat[];  // [plane][band row][Hw]
    __shared__ LdsTable lt;
    __shared__ uint32_t red[kBandMaxWaves][2];
    load_table(lt, a.at);
    const uint32_t G = gridDim.x, g = blockIdx.x;
    const uint32_t L = a.L, Hw = a.Hw, Wr = a.Wr;  // Hw = 64 CW, Wr = Hw / 8
    const uint32_t r0 = (uint32_t)((uint64_t)g * L / G);
    const uint32_t H = (uint32_t)((uint64_t)(g + 1u) * L / G) - r0;
    const uint32_t P = H * Hw;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t gu = g == 0 ? G - 1u : g - 1u, gd = g + 1u == G ? 0u : g + 1u;

    // the band's rows of both planes are contiguous in HBM
    for (uint32_t w = threadIdx.x; w < 2u * P; w += blockDim.x) {
        const uint32_t c = w >= P ? 1u : 0u, rw = w - c * P, r = rw / Hw;
        lat[c * P + r * Hw + lds_slot<CW>(rw - r * Hw)] = (c ? a.p1 : a.p0)[(size_t)r0 * Hw + rw];
    }
    __syncthreads();

    const uint32_t x = lane * (uint32_t)CW;  // the lane's first word of a row
    const uint32_t kb = x / 8u;              // and the bit word of an edge row holding it
    const bool publisher = (lane & (8u / (uint32_t)CW - 1u)) == 0u;
    Row<CW> xw;  // the lane's word indices within a row
#pragma unroll
    for (int j = 0; j < CW; ++j) xw.v[j] = x + (uint32_t)j;
    // rows of this wave: r = wv (mod nw), the band's edge rows first
    const uint32_t nrows = H > wv ? (H - 1u - wv) / nw + 1u : 0u;
    const bool owns_last = (H - 1u) % nw == wv;
    const size_t slot_words = (size_t)G * 2u * Wr;
    const uint32_t summer = nw > 1u ? 64u : 0u;  // a thread off the first wave's edge row
    uint32_t sad = 0, ups = 0;

    for (uint32_t tau = 0; tau < 2u * a.n; ++tau) {
        const uint32_t c = tau & 1u, t = a.t0 + (tau >> 1);
        uint32_t* own_p = lat + c * P;
        const uint32_t* oth_p = lat + (1u - c) * P;
        const uint32_t* oth_g = c ? a.p0 : a.p1;  // the other plane in HBM (first half-sweep)
        const uint64_t* in_slot = a.pub + (size_t)((tau - 1u) & 1u) * slot_words;
        uint64_t* out_slot = a.pub + (size_t)(tau & 1u) * slot_words;
        const uint32_t tag_in = a.base + tau, tag_out = a.base + tau + 1u;
        uint32_t ups8 = 0;
        for (uint32_t j = 0; j < nrows; ++j) {
            uint32_t r;
            if (owns_last && wv != 0u) r = j == 0 ? H - 1u : wv + (j - 1u) * nw;
            else if (owns_last && H > 1u) r = j == 0 ? 0u : j == 1u ? H - 1u : (j - 1u) * nw;
            else r = wv + j * nw;
            const uint32_t i = r0 + r;
            const Row<CW> own = lds_words<CW>(own_p + r * Hw, lane);
            const Row<CW> same = lds_words<CW>(oth_p + r * Hw, lane);
            Row<CW> up, dn;
            if (r == 0) {
                if (tau == 0) up = words_at<CW>(oth_g + (size_t)(i == 0 ? L - 1u : i - 1u) * Hw + x);
                else up = bytes_of_bit_word<CW>(take_word(in_slot + (2u * gu + 1u) * Wr + kb, tag_in, a.err), x);
            } else {
                up = lds_words<CW>(oth_p + (r - 1u) * Hw, lane);
            }
            if (r == H - 1u) {
                if (tau == 0) dn = words_at<CW>(oth_g + (size_t)(i + 1u == L ? 0u : i + 1u) * Hw + x);
                else dn = bytes_of_bit_word<CW>(take_word(in_slot + 2u * gd * Wr + kb, tag_in, a.err), x);
            } else {
                dn = lds_words<CW>(oth_p + (r + 1u) * Hw, lane);
            }
            // a wave holds a whole row: the word past either end of it is the
            // row's other end (periodic)
            Row<CW> nwr;
            if ((i + c) & 1u) {
                const uint32_t edge = (uint32_t)__builtin_amdgcn_readlane((int)same.v[0], 0);
                nwr = c ? update_row<CW, 1, true>(lt, own, up, dn, same, edge, xw, i * Hw, t, 1u, a.k0, a.k1, sad)
                        : update_row<CW, 1, false>(lt, own, up, dn, same, edge, xw, i * Hw, t, 0u, a.k0, a.k1, sad);
            } else {
                const uint32_t edge = (uint32_t)__builtin_amdgcn_readlane((int)same.v[CW - 1], 63);
                nwr = c ? update_row<CW, 0, true>(lt, own, up, dn, same, edge, xw, i * Hw, t, 1u, a.k0, a.k1, sad)
                        : update_row<CW, 0, false>(lt, own, up, dn, same, edge, xw, i * Hw, t, 0u, a.k0, a.k1, sad);
            }
#pragma unroll
            for (int w = 0; w < CW; ++w) {
                own_p[r * Hw + (uint32_t)w * 64u + lane] = nwr.v[w];
                ups8 += nwr.v[w];  // at most 255 words a lane a half-sweep (checked at launch)
            }
            if (r == 0 || r == H - 1u) {
                const uint32_t bw = bit_word_of<CW>(nwr, x);
                if (publisher && r == 0) put_word(out_slot + 2u * g * Wr + kb, tag_out, bw);
                if (publisher && r == H - 1u) put_word(out_slot + (2u * g + 1u) * Wr + kb, tag_out, bw);
            }
        }
        ups = __builtin_amdgcn_sad_u8(ups8, 0u, ups);
        if (c) {
            uint32_t ms = sad, us = ups;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                ms += __shfl_xor(ms, off, 64);
                us += __shfl_xor(us, off, 64);
            }
            if (lane == 0) {
                red[wv][0] = ms;
                red[wv][1] = us;
            }
            sad = 0;
            ups = 0;
        }
        __syncthreads();
        if (c && threadIdx.x == summer) {
            int64_t sm = 0, su = 0;
            for (uint32_t w = 0; w < nw; ++w) {
                sm += red[w][0];
                su += red[w][1];
            }
            // B = 16 (colour-1 words) - 2 (their misaligned bonds); M = 2 ups - sites
            const int64_t HL = (int64_t)H * L;
            int64_t* p = a.part + 2u * ((size_t)(tau >> 1) * G + g);
            p[0] = 2 * HL - 2 * sm;
            p[1] = 2 * su - HL;
        }
    }

    for (uint32_t w = threadIdx.x; w < 2u * P; w += blockDim.x) {
        const uint32_t c = w >= P ? 1u : 0u, rw = w - c * P, r = rw / Hw;
        (c ? a.p1 : a.p0)[(size_t)r0 * Hw + rw] = lat[c * P + r * Hw + lds_slot<CW>(rw - r * Hw)];
    }
}

// Dynamic LDS beyond the default 64 KiB has to be allowed per kernel.
hipError_t allow_lds(const void* kernel, uint32_t bytes) {
    if (bytes <= 65536u) return hipSuccess;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

__global__ __launch_bounds__(256) void k_bands_clear(uint64_t* pub, size_t words) {
    for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (size_t)gridDim.x * blockDim.x)
        pub[w] = 0;
}

__global__ __launch_bounds__(256) void k_bands_reduce(const int64_t* part, uint32_t G, int64_t* ser) {
    const uint32_t s = blockIdx.x;
    reduce_partials(PartialReduce{part + 2ull * s * G, G, ser + 2ull * s});
}

template <bool GENERAL>
const void* bands_kernel_t(uint32_t chunks) {
    switch (chunks) {
        case 1: return reinterpret_cast<const void*>(&k_bands<GENERAL, 1>);
        case 2: return reinterpret_cast<const void*>(&k_bands<GENERAL, 2>);
        case 3: return reinterpret_cast<const void*>(&k_bands<GENERAL, 3>);
        default: return reinterpret_cast<const void*>(&k_bands<GENERAL, 4>);
    }
}

const void* bands_kernel(bool general, uint32_t Wr) {
    const uint32_t chunks = (Wr + 63u) / 64u;
    return general ? bands_kernel_t<true>(chunks) : bands_kernel_t<false>(chunks);
}

}  // namespace

uint32_t bands_capacity(uint32_t threads, uint32_t lds_bytes, bool general, uint32_t Wr) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (Wr == 0 || Wr > kBandMaxWr) return 0;
    const void* k = bands_kernel(general, Wr);
    if (allow_lds(k, lds_bytes) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, (int)threads, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return (uint32_t)(per > 0 ? per : 0) * (uint32_t)cus;
}

namespace {

const void* bands_bytes_kernel(uint32_t cw) {
    switch (cw) {
        case 1: return reinterpret_cast<const void*>(&k_bands_bytes<1>);
        case 2: return reinterpret_cast<const void*>(&k_bands_bytes<2>);
        case 4: return reinterpret_cast<const void*>(&k_bands_bytes<4>);
        default: return reinterpret_cast<const void*>(&k_bands_bytes<8>);
    }
}

// Bytes a byte-resident band holds in LDS (both planes).
uint32_t band_bytes_lds(uint32_t L, uint32_t G) { return 2u * ((L + G - 1u) / G) * (L / 8u) * 4u; }

// Whether the bands of a launch are kept as bytes: plane rows of 64 CW
// words, the two planes of a band within the workgroup's LDS, and every
// band resident. Measured per sweep at the default band heights (one band
// a compute unit), bytes against bits: 3.1 against 4.5 us at 512, 3.1
// against 4.1 at 1024, 4.8 against 7.3 at 2048 (h != 0); at 4096 (eight
// words a lane) 9.4 against 11.9 for h != 0 but 9.4 against 8.4 for the two
// h = 0 classes, which keep bits there.
bool bands_as_bytes(uint32_t L, uint32_t G, uint32_t threads, bool general) {
    if (L % 8u != 0u || (L / 8u) % 64u != 0u) return false;
    const uint32_t cw = L / 8u / 64u;
    if (cw != 1u && cw != 2u && cw != 4u && !(cw == 8u && general)) return false;
    // a lane sums the up spins of its new words bytewise over a half-sweep:
    // at most 255 words a lane
    const uint32_t rows = (L + G - 1u) / G, waves = threads / 64u;
    if (waves == 0 || (rows + waves - 1u) / waves * cw > 255u) return false;
    const uint32_t lds = band_bytes_lds(L, G);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    static std::mutex mu;
    static std::map<std::tuple<int, uint32_t, uint32_t, uint32_t>, uint32_t> cap;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(dev, cw, threads, lds);
    auto it = cap.find(key);
    if (it == cap.end()) {
        int cus = 0, per = 0;
        const void* k = bands_bytes_kernel(cw);
        uint32_t n = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            allow_lds(k, lds) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, (int)threads, lds) == hipSuccess)
            n = (uint32_t)(per > 0 ? per : 0) * (uint32_t)cus;
        (void)hipGetLastError();
        it = cap.emplace(key, n).first;
    }
    return it->second >= G;
}

}  // namespace

hipError_t launch_bands(const BandArgs& a, uint32_t G, uint32_t threads, hipStream_t s) {
    if (G < 2u || G > a.L || a.Wr == 0 || a.Wr > kBandMaxWr || a.n == 0 || threads % 64u != 0 || threads == 0 ||
        threads > 64u * kBandMaxWaves)
        return hipErrorInvalidValue;
    BandArgs arg = a;
    void* args[] = {&arg};
    if (a.Hw == a.L / 8u && a.Wr * 8u == a.Hw && bands_as_bytes(a.L, G, threads, a.general != 0)) {
        const uint32_t lds = band_bytes_lds(a.L, G);
        const void* k = bands_bytes_kernel(a.Hw / 64u);
        const hipError_t e = allow_lds(k, lds);
        if (e != hipSuccess) return e;
        return hipLaunchCooperativeKernel(k, dim3(G), dim3(threads), args, lds, s);
    }
    const uint32_t lds = band_lds_bytes(a.L, G, a.Wr);
    const void* k = bands_kernel(a.general != 0, a.Wr);
    const hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(k, dim3(G), dim3(threads), args, lds, s);
}

hipError_t launch_bands_clear(uint64_t* pub, size_t words, hipStream_t s) {
    if (words == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_bands_clear, dim3((uint32_t)blocks), dim3(256), 0, s, pub, words);
    return hipGetLastError();
}

hipError_t launch_bands_reduce(const int64_t* part, uint32_t G, uint32_t n, int64_t* ser, hipStream_t s) {
    if (n == 0 || G == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bands_reduce, dim3(n), dim3(256), 0, s, part, G, ser);
    return hipGetLastError();
}

}  // namespace ising
