// Creutz demon rule (the random-number-free dynamics Section 2.2 of Tomov
// et al. cites), shared by the in-place and fused Creutz kernels. Every
// site carries a demon energy d in units of 4J (zero field), 0 <= d <= 255.
// A site flips iff its demon can pay for the move: e = dE / 4J = s n / 2 in
// {-2..2} (n the sum of the four neighbour spins), flip iff e <= d and
// d - e <= 255, then d -= e.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_launch.hpp"

namespace ising {

// Demon update of four sites at once. W: spin bytes (0/1), n: up-neighbour
// counts (0..4), D: demon bytes. With g = e + 2 = (s ? n : 4 - n) in 0..4,
// y = d + 258 - g lies in [254, 513] and the move is allowed iff
// 256 <= y <= 511, in which case the new demon is y - 256. Even and odd
// bytes are handled in 16-bit lanes so y never borrows across sites.
__device__ __forceinline__ void creutz_word(uint32_t W, uint32_t n, uint32_t D, uint32_t& Wn, uint32_t& Dn) {
    const uint32_t sm = W * 0xffu;
    const uint32_t g = (n & sm) | ((0x04040404u - n) & ~sm);
    const uint32_t ye = (D & 0x00ff00ffu) + 0x01020102u - (g & 0x00ff00ffu);
    const uint32_t yo = ((D >> 8) & 0x00ff00ffu) + 0x01020102u - ((g >> 8) & 0x00ff00ffu);
    const uint32_t fe = (ye >> 8) & ~(ye >> 9) & 0x00010001u;
    const uint32_t fo = (yo >> 8) & ~(yo >> 9) & 0x00010001u;
    const uint32_t f = fe | (fo << 8);
    const uint32_t fm = f * 0xffu;
    const uint32_t y = (ye & 0x00ff00ffu) | ((yo & 0x00ff00ffu) << 8);
    Wn = W ^ f;
    Dn = (y & fm) | (D & ~fm);
}


// Fused Creutz sweep (ising_creutz_fused.hip): spins and demons of the
// previous sweep in src / dsrc (colour planes), the new ones to dst / ddst;
// tiles and partials as for the fused Metropolis sweep.
struct CreutzFusedArgs {
    const uint32_t* src0;
    const uint32_t* src1;
    const uint32_t* dsrc0;
    const uint32_t* dsrc1;
    uint32_t* dst0;
    uint32_t* dst1;
    uint32_t* ddst0;
    uint32_t* ddst1;
    uint32_t L, Hw, n_tx, n_tiles;
    int64_t* part;
};

hipError_t launch_creutz_fused(const CreutzFusedArgs& a, uint32_t cw, uint32_t rows, const PartialReduce& red,
                               hipStream_t s);

}  // namespace ising
