// Fused one-pass sweep by full-row workgroups: both colours of sweep t in
// one launch, reading the lattice of sweep t-1 from `src` and writing sweep
// t to `dst` (ping-pong), 2 bytes per site update over HBM, like k_fused.
//
// Work unit: a workgroup of NW waves owns a band of R whole rows; wave w
// holds words w*64*CW .. (w+1)*64*CW - 1 of every plane row of the band
// (NW * 64 * CW = L/8 words, at most 16 waves). Every wave walks down the
// band as k_fused's waves walk their tiles: at row i, colour 0 of row i+1,
// then colour 1 of row i (Section 2.2's order; sites of one colour are
// independent). The words just outside a wave's columns belong to its left
// and right neighbours in the same workgroup (periodic: wave NW-1 and wave
// 0 are neighbours), which publish them in LDS:
//   - at step i (row i), after its colour-0 update of row i+1, every wave
//     writes the first and last words of its new colour-0 row i+1 and of its
//     old colour-1 row i+2 (already in its ring of prefetched rows);
//   - one barrier per step; at step i+1 every wave reads, on the same-row
//     side of the updates, the neighbour's old colour-1 word of row i+2 (for
//     colour 0 of row i+2) and its new colour-0 word of row i+1 (for colour
//     1 of row i+1).
// So nothing outside the band's rows is read or recomputed except the two
// halo rows above and below the band (the colour-0 rows r0-1 and r0+R, as
// in k_fused), and no row is read by scattered single-word loads. The
// slots alternate between two LDS buffers: a buffer is rewritten one step
// after it was read, behind the barrier of that step.
//
// Draws are the counter-based Philox words of the sites, so the result is
// bit-identical to every other schedule of the same sweep.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_fused_core.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr uint32_t kRowsMaxWaves = 16;

// Wait for this wave's LDS writes, then the workgroup barrier; LDS only, so
// the row loads in flight stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace

template <int CW, int R>
__global__ void __launch_bounds__(1024, 4) k_fused_rows(FusedArgs a, AcceptTable at, PartialReduce red) {
    __shared__ LdsTable lt;
    // published edge words: [buffer][wave][c0 first, c0 last, c1 first, c1 last]
    __shared__ uint32_t pub[2][kRowsMaxWaves][4];
    __shared__ int64_t wpart[kRowsMaxWaves][2];
    load_table(lt, at);
    const uint32_t band = xcd_block(gridDim.x);
    if (band == 0) reduce_partials(red);  // every thread of the workgroup takes part
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t wl = w == 0 ? nw - 1u : w - 1u;  // left and right neighbour waves
    const uint32_t wr = w + 1u == nw ? 0u : w + 1u;
    const uint32_t L = a.L, Hw = a.Hw, t = a.t, k0 = a.k0, k1 = a.k1;
    const uint32_t x = w * 64u * CW + lane * CW;
    const int r0 = (int)(band * R);
    const uint32_t* __restrict__ s0 = a.src0;
    const uint32_t* __restrict__ s1 = a.src1;
    uint32_t* __restrict__ d0 = a.dst0;
    uint32_t* __restrict__ d1 = a.dst1;

    uint32_t sad = 0, ups = 0, ups8 = 0, dummy = 0;
    const uint32_t xb = x * 4u;  // lane's byte offset within a row
    Row<CW> xw;                  // lane's word indices within a row
#pragma unroll
    for (int v = 0; v < CW; ++v) xw.v[v] = x + (uint32_t)v;
    const __amdgpu_buffer_rsrc_t rs0 = plane_rsrc(s0), rs1 = plane_rsrc(s1);
    const __amdgpu_buffer_rsrc_t rd0 = plane_rsrc(d0), rd1 = plane_rsrc(d1);
    auto rword = [&](int i) { return wrap_row(i, L) * Hw; };
    auto rbyte = [&](int i) { return rword(i) * 4u; };
    // first / last words of a row: written by lanes 0 and 63
    auto publish = [&](uint32_t buf, const Row<CW>& c0new, const Row<CW>& c1old) {
        if (lane == 0u) {
            pub[buf][w][0] = c0new.v[0];
            pub[buf][w][2] = c1old.v[0];
        } else if (lane == 63u) {
            pub[buf][w][1] = c0new.v[CW - 1];
            pub[buf][w][3] = c1old.v[CW - 1];
        }
    };
    // the word just outside this wave's columns on same-row side P (1: the
    // right neighbour's first word, 0: the left neighbour's last word) of a
    // published row: f = 0 for the new colour-0 row, 2 for the old colour-1 row
    auto edge = [&](uint32_t buf, int P, uint32_t f) { return P ? pub[buf][wr][f] : pub[buf][wl][f + 1]; };

    // Ring buffers as in k_fused:
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
    // the old colour-1 rows r0-1 and r0 for the band's first colour-0 rows
    publish(1u, c1m1, c1[0]);
    lds_barrier();
    // new colour-0 rows r0-1 (odd: same-row side P = 1) and r0 (even: P = 0);
    // in buffer 1, "c0" holds old colour-1 row r0-1 and "c1" old colour-1 row r0
    const uint32_t eR = pub[1][wr][0];
    const uint32_t eL = pub[1][wl][3];
    c0n[0] = update_row<CW, 1, false>(lt, c0om1, c1m2, c1[0], c1m1, eR, xw, rword(r0 - 1), t, 0u, k0, k1, dummy);
    c0n[1] = update_row<CW, 0, false>(lt, c0o[0], c1m1, c1[1], c1[0], eL, xw, rword(r0), t, 0u, k0, k1, dummy);
    st<CW>(rd0, xb + rbyte(r0), c0n[1]);
    // buffer 0: new colour-0 row r0 and old colour-1 row r0+1, for step r0
    publish(0u, c0n[1], c1[1]);
    lds_barrier();

#pragma unroll 1
    for (int k = 0; k < R; k += 4) {
        // the four steps of k, each with compile-time ring slots and LDS
        // buffer (buffer u & 1 holds what step u reads)
        auto step = [&](auto uc) {
            constexpr int u = decltype(uc)::value;
            constexpr uint32_t rd = u & 1, wrb = rd ^ 1u;
            const int i = r0 + k + u;
            // prefetch old colour-1 row i+3 and old colour-0 row i+2 into the
            // slots of rows i-1 and i, which this step no longer reads
            c1[(u + 3) & 3] = ld<CW>(rs1, xb, rbyte(i + 3));
            c0o[u & 1] = ld<CW>(rs0, xb, rbyte(i + 2));
            // issued here, a whole step before their use (the scheduler would
            // otherwise sink them to the middle of the step)
            __builtin_amdgcn_sched_barrier(0);
            constexpr int P = (u & 1) == 0 ? 1 : 0;  // i even: both updates have same-row side P = 1
            const uint32_t e1 = edge(rd, P, 2u);  // old colour-1 row i+1
            const uint32_t e0 = edge(rd, P, 0u);  // new colour-0 row i
            const uint32_t m1 = rword(i + 1);
            const uint32_t m0 = rword(i);
            c0n[(u + 2) & 3] = update_row<CW, P, false>(lt, c0o[(u + 1) & 1], c1[u & 3], c1[(u + 2) & 3],
                                                        c1[(u + 1) & 3], e1, xw, m1, t, 0u, k0, k1, dummy);
            // for step i+1: new colour-0 row i+1, old colour-1 row i+2
            publish(wrb, c0n[(u + 2) & 3], c1[(u + 2) & 3]);
            const Row<CW> c1n = update_row<CW, P, true>(lt, c1[u & 3], c0n[u & 3], c0n[(u + 2) & 3],
                                                        c0n[(u + 1) & 3], e0, xw, m0, t, 1u, k0, k1, sad);
            if (k + u + 1 < R) st<CW>(rd0, xb + rbyte(i + 1), c0n[(u + 2) & 3]);
            st<CW>(rd1, xb + rbyte(i), c1n);
#pragma unroll
            for (int v = 0; v < CW; ++v) ups8 += c1n.v[v] + c0n[(u + 1) & 3].v[v];
            lds_barrier();
            __builtin_amdgcn_sched_barrier(0);
        };
        step(Step<0>{});
        step(Step<1>{});
        step(Step<2>{});
        step(Step<3>{});
        ups = __builtin_amdgcn_sad_u8(ups8, 0u, ups);
        ups8 = 0;
    }

    // partials of the band: B = 16 * words - 2 * sad, M = 2 * ups - 8 * words
    // per wave, summed over the workgroup
    const int64_t words = (int64_t)R * CW;
    int64_t b = 16 * words - 2 * (int64_t)sad;
    int64_t m = 2 * (int64_t)ups - 8 * words;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        b += __shfl_xor(b, off, 64);
        m += __shfl_xor(m, off, 64);
    }
    if (lane == 0) {
        wpart[w][0] = b;
        wpart[w][1] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sb = 0, sm = 0;
        for (uint32_t v = 0; v < nw; ++v) {
            sb += wpart[v][0];
            sm += wpart[v][1];
        }
        a.part[2 * band] = sb;
        a.part[2 * band + 1] = sm;
    }
}

template <int CW, int R>
static void launch_rows_t(const FusedArgs& a, const AcceptTable& at, const PartialReduce& red, hipStream_t s) {
    const uint32_t nw = a.Hw / (64u * CW);
    k_fused_rows<CW, R><<<a.L / R, 64u * nw, 0, s>>>(a, at, red);
}

bool fused_rows_supported(uint32_t L, uint32_t cw, uint32_t rows) {
    if (L % 8u != 0u) return false;
    const uint32_t Hw = L / 8u;
    if (cw != 1 && cw != 2 && cw != 4) return false;
    if (rows != 8 && rows != 16 && rows != 32 && rows != 64 && rows != 128) return false;
    if (Hw % (64u * cw) != 0u) return false;
    const uint32_t nw = Hw / (64u * cw);
    return nw >= 1u && nw <= kRowsMaxWaves && L % rows == 0u;
}

uint32_t fused_rows_bands(uint32_t L, uint32_t rows) { return L / rows; }

hipError_t launch_fused_rows(const FusedArgs& a, const AcceptTable& at, uint32_t cw, uint32_t rows,
                             const PartialReduce& red, hipStream_t s) {
#define ISING_ROWS_CASE(CWv, Rv)                   \
    if (cw == CWv && rows == Rv) {                 \
        launch_rows_t<CWv, Rv>(a, at, red, s);     \
        return hipGetLastError();                  \
    }
    ISING_ROWS_CASE(1, 8) ISING_ROWS_CASE(1, 16) ISING_ROWS_CASE(1, 32) ISING_ROWS_CASE(1, 64)
    ISING_ROWS_CASE(1, 128) ISING_ROWS_CASE(2, 8) ISING_ROWS_CASE(2, 16) ISING_ROWS_CASE(2, 32)
    ISING_ROWS_CASE(2, 64) ISING_ROWS_CASE(2, 128) ISING_ROWS_CASE(4, 8) ISING_ROWS_CASE(4, 16)
    ISING_ROWS_CASE(4, 32) ISING_ROWS_CASE(4, 64) ISING_ROWS_CASE(4, 128)
#undef ISING_ROWS_CASE
    return hipErrorInvalidValue;
}

}  // namespace ising
