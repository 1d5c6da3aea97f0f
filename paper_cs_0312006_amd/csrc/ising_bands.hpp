// Band-resident sweeps of one lattice: the lattice is split into G bands of
// whole rows, one workgroup per band, each band kept at one bit per site in
// its workgroup's LDS for every sweep of a launch; neighbouring bands trade
// their edge rows through global memory after every half-sweep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_bits.hpp"

namespace ising {

struct BandArgs {
    uint32_t* p0;       // byte colour planes of the lattice, read at the start
    uint32_t* p1;       // and written back at the end (in place)
    uint32_t L, Hw, Wr;  // side, quads and bit words per plane row
    uint32_t t0, n;     // first sweep, sweeps (n >= 1)
    uint32_t k0, k1;    // Philox key
    uint64_t* pub;      // edge rows: [2 slots][G][top, bottom][Wr] tagged words
    uint32_t base;      // tag of the last half-sweep published before this launch
    int64_t* part;      // [n][G] (B, M) partial pairs of each band
    uint32_t* err;      // set when a wait for a neighbour gives up
    uint32_t general;   // 1: the (s, m) classes (h != 0), 0: the two h = 0 classes
    BitsLattice bl;
    AcceptTable at;     // the acceptance table (byte-resident bands)
};

// A wave sweeps a band row in chunks of 64 words (a word per lane); rows of
// up to 256 words (sides up to 16384), and every band holds at least one
// row.
constexpr uint32_t kBandMaxWr = 256;
// Tagged edge-row words a band launch uses (64-bit: tag << 32 | bit word).
inline size_t band_pub_words(uint32_t G, uint32_t Wr) { return (size_t)2 * G * 2 * Wr; }
inline uint32_t band_lds_bytes(uint32_t L, uint32_t G, uint32_t Wr) { return 2u * ((L + G - 1u) / G) * Wr * 4u; }

// Workgroups of `threads` threads that can be resident at once for bands of
// lds_bytes each and rows of Wr words (0 on error).
uint32_t bands_capacity(uint32_t threads, uint32_t lds_bytes, bool general, uint32_t Wr);
// One cooperative launch of G band workgroups of `threads` threads. Sides
// 512, 1024 and 2048, and 4096 with h != 0, keep their bands as bytes when
// those fit (the fused kernels' word update), every other side as bits.
hipError_t launch_bands(const BandArgs& a, uint32_t G, uint32_t threads, hipStream_t s);
// Zero `words` tagged edge words (before tags restart from 0).
hipError_t launch_bands_clear(uint64_t* pub, size_t words, hipStream_t s);
// Sum each sweep's G band partials into ser (2 int64 per sweep, n sweeps).
hipError_t launch_bands_reduce(const int64_t* part, uint32_t G, uint32_t n, int64_t* ser, hipStream_t s);

}  // namespace ising
