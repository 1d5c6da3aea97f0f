// HIP kernels of the gfx950 checkerboard Metropolis engine (Section 2.2 of
// Tomov et al. 2003: checkerboard colouring, Metropolis decision with the
// Boltzmann ratio; the layout and keying are described in ising_device.hpp).
//
// Every kernel is integer-only: the acceptance test is an unsigned compare
// against a host-built threshold table, so the GPU and any CPU evaluation of
// the same rule agree bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_launch.hpp"

namespace ising {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

// Block-wide sum of two int64 values, added atomically to out[0], out[1].
__device__ __forceinline__ void block_add2(int64_t a, int64_t b, int64_t* out) {
    __shared__ int64_t part[2][16];
    a = wave_sum_i64(a);
    b = wave_sum_i64(b);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wave] = a;
        part[1][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sa = 0, sb = 0;
        const uint32_t nw = (blockDim.x + 63u) >> 6;
        for (uint32_t w = 0; w < nw; ++w) {
            sa += part[0][w];
            sb += part[1][w];
        }
        atomicAdd(reinterpret_cast<unsigned long long*>(&out[0]), (unsigned long long)sa);
        atomicAdd(reinterpret_cast<unsigned long long*>(&out[1]), (unsigned long long)sb);
    }
}

// ---------------------------------------------------------------------------
// Initial state (Section 2.2): up iff draw(t=0, c, d=1) < pthr.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_init_words(Planes pl, uint32_t c, uint32_t k0, uint32_t k1,
                                                    uint64_t pthr) {
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t words = pl.L * pl.Hw;
    if (idx >= words) return;
    const uint4 r = philox(idx, 0u, c, 1u, k0, k1);  // q = i*Hw + w = idx
    uint32_t v = 0;
    v |= (uint64_t)r.x < pthr ? 0x00000001u : 0u;
    v |= (uint64_t)r.y < pthr ? 0x00000100u : 0u;
    v |= (uint64_t)r.z < pthr ? 0x00010000u : 0u;
    v |= (uint64_t)r.w < pthr ? 0x01000000u : 0u;
    reinterpret_cast<uint32_t*>(pl.p[c])[idx] = v;
}

// Any even L: one thread per site of colour c, its own Philox call.
__global__ void __launch_bounds__(256) k_init_sites(Planes pl, uint32_t c, uint32_t k0, uint32_t k1,
                                                    uint64_t pthr) {
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;  // ord = i*H + m
    const uint32_t sites = pl.L * pl.H;
    if (idx >= sites) return;
    const uint4 r = philox(idx >> 2, 0u, c, 1u, k0, k1);
    const uint32_t sel = idx & 3u;
    const uint32_t u = sel == 0 ? r.x : sel == 1 ? r.y : sel == 2 ? r.z : r.w;
    pl.p[c][idx] = (uint64_t)u < pthr ? 1u : 0u;
}

// ---------------------------------------------------------------------------
// Two-pass sweep: one launch per colour, in place. Thread = CW consecutive
// words of one plane row. Neighbour words come straight from memory (L2).
// ---------------------------------------------------------------------------
template <int CW>
struct Chunk {
    uint32_t v[CW];
};

template <int CW>
__device__ __forceinline__ Chunk<CW> load_chunk(const uint32_t* p) {
    Chunk<CW> c;
    if constexpr (CW == 4) {
        const uint4 x = *reinterpret_cast<const uint4*>(p);
        c.v[0] = x.x; c.v[1] = x.y; c.v[2] = x.z; c.v[3] = x.w;
    } else if constexpr (CW == 2) {
        const uint2 x = *reinterpret_cast<const uint2*>(p);
        c.v[0] = x.x; c.v[1] = x.y;
    } else {
#pragma unroll
        for (int w = 0; w < CW; ++w) c.v[w] = p[w];
    }
    return c;
}

template <int CW>
__device__ __forceinline__ void store_chunk(uint32_t* p, const Chunk<CW>& c) {
    if constexpr (CW == 4) {
        *reinterpret_cast<uint4*>(p) = make_uint4(c.v[0], c.v[1], c.v[2], c.v[3]);
    } else if constexpr (CW == 2) {
        *reinterpret_cast<uint2*>(p) = make_uint2(c.v[0], c.v[1]);
    } else {
#pragma unroll
        for (int w = 0; w < CW; ++w) p[w] = c.v[w];
    }
}

// Update the CW words of plane c at row i starting at word wc, in place.
// Accumulates the colour-1 observable partials when OBS.
template <int CW, bool OBS, bool EXACT>
__device__ __forceinline__ void update_chunk_inplace(const LdsTable& lt, uint32_t* own, const uint32_t* oth,
                                                     uint32_t L, uint32_t Hw, uint32_t i, uint32_t wc,
                                                     uint32_t c, uint32_t t, uint32_t k0, uint32_t k1,
                                                     uint32_t& sad, uint32_t& ups) {
    const uint32_t iu = i == 0 ? L - 1 : i - 1;
    const uint32_t id = i + 1 == L ? 0 : i + 1;
    const uint32_t p = (i + c) & 1u;
    const size_t row = (size_t)i * Hw;
    const Chunk<CW> W = load_chunk<CW>(own + row + wc);
    const Chunk<CW> U = load_chunk<CW>(oth + (size_t)iu * Hw + wc);
    const Chunk<CW> D = load_chunk<CW>(oth + (size_t)id * Hw + wc);
    const Chunk<CW> O = load_chunk<CW>(oth + row + wc);
    // the one word outside the chunk that the same-row shift needs
    const uint32_t ew = p ? (wc + CW == Hw ? 0u : wc + CW) : (wc == 0 ? Hw - 1 : wc - 1);
    const uint32_t E = oth[row + ew];
    Chunk<CW> out;
#pragma unroll
    for (int w = 0; w < CW; ++w) {
        const uint32_t nxt = (w + 1 < CW) ? O.v[w + 1 < CW ? w + 1 : w] : E;
        const uint32_t prv = (w > 0) ? O.v[w > 0 ? w - 1 : 0] : E;
        const uint32_t S = shifted(O.v[w], nxt, prv, p);
        const uint32_t n = U.v[w] + D.v[w] + O.v[w] + S;
        const uint4 r = philox((uint32_t)(row + wc + w), t, c, 0u, k0, k1);
        const uint32_t Wn = W.v[w] ^ flip_mask<EXACT>(lt, W.v[w], n, r);
        out.v[w] = Wn;
        if (OBS) {
            sad = sad_misaligned(Wn, n, sad);
            ups += __builtin_popcount(Wn) + __builtin_popcount(O.v[w]);
        }
    }
    store_chunk<CW>(own + row + wc, out);
}

// Colour-c pass. Grid-stride over (row, chunk); colour 1 leaves one partial
// (B, M) per block in part[]; colour 0 first folds the previous sweep's
// partials (if any) into that sweep's series slot.
template <int CW, bool OBS, bool EXACT>
__global__ void __launch_bounds__(256) k_two_pass(Planes pl, AcceptTable at, uint32_t c, uint32_t t_off,
                                                  uint32_t k0, uint32_t k1, int64_t* part, PartialReduce red,
                                                  const uint32_t* t_dev) {
    const uint32_t t = t_dev ? *t_dev + t_off : t_off;  // graph replays read the sweep index from memory
    __shared__ LdsTable lt;
    load_table(lt, at);
    __syncthreads();
    if (!OBS && blockIdx.x == 0) reduce_partials(red);
    const uint32_t chunks_per_row = pl.Hw / CW;
    const uint32_t total = pl.L * chunks_per_row;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t sad = 0, ups = 0, nw = 0;
    for (uint32_t idx = xcd_block(gridDim.x) * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const uint32_t i = idx / chunks_per_row;
        const uint32_t wc = (idx - i * chunks_per_row) * CW;
        update_chunk_inplace<CW, OBS, EXACT>(lt, reinterpret_cast<uint32_t*>(pl.p[c]),
                                             reinterpret_cast<const uint32_t*>(pl.p[c ^ 1u]), pl.L, pl.Hw, i,
                                             wc, c, t, k0, k1, sad, ups);
        nw += CW;
    }
    if (OBS) {
        // B = 16 * words - 2 * sum(sad); M = 2 * ups - 4 * 2 * words
        int64_t b = 16 * (int64_t)nw - 2 * (int64_t)sad;
        int64_t m = 2 * (int64_t)ups - 8 * (int64_t)nw;
        b = wave_sum_i64(b);
        m = wave_sum_i64(m);
        __shared__ int64_t acc[2][4];
        const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
        if (lane == 0) {
            acc[0][wave] = b;
            acc[1][wave] = m;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            part[2 * blockIdx.x] = acc[0][0] + acc[0][1] + acc[0][2] + acc[0][3];
            part[2 * blockIdx.x + 1] = acc[1][0] + acc[1][1] + acc[1][2] + acc[1][3];
        }
    }
}

// ---------------------------------------------------------------------------
// Generic path (any even L): one thread per site of colour c, in place.
// ---------------------------------------------------------------------------
template <bool EXACT>
__global__ void __launch_bounds__(256) k_half_sites(Planes pl, AcceptTable at, uint32_t c, uint32_t t,
                                                    uint32_t k0, uint32_t k1) {
    __shared__ LdsTable lt;
    load_table(lt, at);
    __syncthreads();
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;  // ord = i*H + m
    const uint32_t H = pl.H, L = pl.L;
    if (idx >= L * H) return;
    const uint32_t i = idx / H, m = idx - i * H;
    const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
    const uint32_t p = (i + c) & 1u;
    const uint8_t* oth = pl.p[c ^ 1u];
    const uint32_t m2 = p ? (m + 1 == H ? 0 : m + 1) : (m == 0 ? H - 1 : m - 1);
    const uint32_t n = oth[(size_t)iu * H + m] + oth[(size_t)id * H + m] + oth[(size_t)i * H + m] +
                       oth[(size_t)i * H + m2];
    const uint32_t s = pl.p[c][idx];
    const uint4 r = philox(idx >> 2, t, c, 0u, k0, k1);
    const uint32_t sel = idx & 3u;
    const uint32_t u = sel == 0 ? r.x : sel == 1 ? r.y : sel == 2 ? r.z : r.w;
    const uint32_t code = 8u * s + n;
    bool acc;
    if (EXACT) {
        acc = (uint64_t)u < (((uint64_t)lt.t64[code].y << 32) | lt.t64[code].x);
    } else {
        acc = u <= lt.t32[code];
    }
    if (acc) pl.p[c][idx] = (uint8_t)(s ^ 1u);
}

// ---------------------------------------------------------------------------
// Observables of the current state (any even L): B over colour-1 sites, M
// over both planes. Grid-stride with a bounded grid, one atomic pair per
// block. out[0], out[1] must be zero beforehand.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_observe(Planes pl, int64_t* out) {
    const uint32_t H = pl.H, L = pl.L;
    const uint32_t stride = gridDim.x * blockDim.x;
    int64_t b = 0, m = 0;
    if ((L & 7u) == 0u) {
        // word path: 4 sites at a time, B = 16 - 2 * sad per colour-1 word
        const uint32_t Hw = pl.Hw;
        const uint32_t* p0 = reinterpret_cast<const uint32_t*>(pl.p[0]);
        const uint32_t* p1 = reinterpret_cast<const uint32_t*>(pl.p[1]);
        uint32_t sad = 0, ups = 0, nw = 0;
        for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < L * Hw; idx += stride) {
            const uint32_t i = idx / Hw, w = idx - i * Hw;
            const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
            const uint32_t p = (i + 1u) & 1u;
            const uint32_t O = p0[(size_t)i * Hw + w];
            const uint32_t E = p0[(size_t)i * Hw + (p ? (w + 1 == Hw ? 0 : w + 1) : (w == 0 ? Hw - 1 : w - 1))];
            const uint32_t n = p0[(size_t)iu * Hw + w] + p0[(size_t)id * Hw + w] + O + shifted(O, E, E, p);
            const uint32_t W = p1[idx];
            sad = sad_misaligned(W, n, sad);
            ups += __builtin_popcount(W) + __builtin_popcount(O);
            ++nw;
            if (nw == 1u << 20) {  // keep the 32-bit partials far from overflow
                b += 16 * (int64_t)nw - 2 * (int64_t)sad;
                m += 2 * (int64_t)ups - 8 * (int64_t)nw;
                sad = ups = nw = 0;
            }
        }
        b += 16 * (int64_t)nw - 2 * (int64_t)sad;
        m += 2 * (int64_t)ups - 8 * (int64_t)nw;
    } else {
        for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < L * H; idx += stride) {
            const uint32_t i = idx / H, mm = idx - i * H;
            const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
            const uint32_t p = (i + 1u) & 1u;
            const uint8_t* o = pl.p[0];
            const uint32_t m2 = p ? (mm + 1 == H ? 0 : mm + 1) : (mm == 0 ? H - 1 : mm - 1);
            const int n = o[(size_t)iu * H + mm] + o[(size_t)id * H + mm] + o[(size_t)i * H + mm] +
                          o[(size_t)i * H + m2];
            const int s1 = pl.p[1][idx] ? 1 : -1;
            b += (int64_t)(s1 * (2 * n - 4));
            m += (int64_t)s1 + (pl.p[0][idx] ? 1 : -1);
        }
    }
    block_add2(b, m, out);
}

// ---------------------------------------------------------------------------
// Layout conversion between planes and canonical row-major int8 +1 / -1.
// ---------------------------------------------------------------------------
// Grid-stride over the L*L sites (a 65536^2 lattice has 2^32 sites, more
// than one launch can give a thread each).
__global__ void __launch_bounds__(256) k_to_canonical(Planes pl, int8_t* out) {
    const size_t N = (size_t)pl.L * pl.L, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) {
        const uint32_t i = (uint32_t)(idx / pl.L), j = (uint32_t)(idx - (size_t)i * pl.L);
        const uint32_t c = (i + j) & 1u;
        out[idx] = pl.p[c][(size_t)i * pl.H + (j >> 1)] ? (int8_t)1 : (int8_t)-1;
    }
}

__global__ void __launch_bounds__(256) k_from_canonical(Planes pl, const int8_t* in) {
    const size_t N = (size_t)pl.L * pl.L, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) {
        const uint32_t i = (uint32_t)(idx / pl.L), j = (uint32_t)(idx - (size_t)i * pl.L);
        const uint32_t c = (i + j) & 1u;
        pl.p[c][(size_t)i * pl.H + (j >> 1)] = in[idx] > 0 ? 1u : 0u;
    }
}

// Fill n int64 with zero (a kernel, not a memset, so it can sit in a graph).
__global__ void __launch_bounds__(256) k_zero_i64(int64_t* p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) p[idx] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
static inline uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

hipError_t launch_init(const Planes& pl, bool words, uint32_t k0, uint32_t k1, uint64_t pthr,
                       hipStream_t s) {
    for (uint32_t c = 0; c < 2; ++c) {
        if (words) {
            k_init_words<<<blocks_for((uint64_t)pl.L * pl.Hw, 256), 256, 0, s>>>(pl, c, k0, k1, pthr);
        } else {
            k_init_sites<<<blocks_for((uint64_t)pl.L * pl.H, 256), 256, 0, s>>>(pl, c, k0, k1, pthr);
        }
    }
    return hipGetLastError();
}

uint32_t two_pass_blocks(const Planes& pl, uint32_t cw) {
    const uint64_t total = (uint64_t)pl.L * (pl.Hw / cw);
    uint32_t nb = blocks_for(total, 256);
    return nb > 4096u ? 4096u : nb;
}

template <int CW, bool EXACT>
static void two_pass_sweep(const Planes& pl, const AcceptTable& at, uint32_t t, uint32_t k0, uint32_t k1,
                           int64_t* part, const PartialReduce& red, hipStream_t s, const uint32_t* t_dev) {
    const uint32_t nb = two_pass_blocks(pl, CW);
    k_two_pass<CW, false, EXACT><<<nb, 256, 0, s>>>(pl, at, 0u, t, k0, k1, part, red, t_dev);
    k_two_pass<CW, true, EXACT><<<nb, 256, 0, s>>>(pl, at, 1u, t, k0, k1, part, PartialReduce{nullptr, 0, nullptr},
                                                   t_dev);
}

hipError_t launch_two_pass(const Planes& pl, const AcceptTable& at, bool exact, uint32_t cw, uint32_t t,
                           uint32_t k0, uint32_t k1, int64_t* part, const PartialReduce& red, hipStream_t s,
                           const uint32_t* t_dev) {
    switch (cw * 2 + (exact ? 1 : 0)) {
        case 2: two_pass_sweep<1, false>(pl, at, t, k0, k1, part, red, s, t_dev); break;
        case 3: two_pass_sweep<1, true>(pl, at, t, k0, k1, part, red, s, t_dev); break;
        case 4: two_pass_sweep<2, false>(pl, at, t, k0, k1, part, red, s, t_dev); break;
        case 5: two_pass_sweep<2, true>(pl, at, t, k0, k1, part, red, s, t_dev); break;
        case 8: two_pass_sweep<4, false>(pl, at, t, k0, k1, part, red, s, t_dev); break;
        case 9: two_pass_sweep<4, true>(pl, at, t, k0, k1, part, red, s, t_dev); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Graph replays of the two-pass plan: the sweep index and series slot of
// a replay live in a device header the replay's last node advances.
__global__ void __launch_bounds__(64) k_set_header(SweepHeader* hdr, uint32_t t, int64_t* ser) {
    if (threadIdx.x == 0) {
        hdr->t = t;
        hdr->arrived = 0;
        hdr->ser = ser;
    }
}

// Block k sums sweep k's partials into its series slot. A block has read
// the header before its thread 0 arrives (the slot's address feeds the
// store that precedes the arrival), so the last block to arrive may advance
// the header for the next replay and re-arm the count.
__global__ void __launch_bounds__(256) k_reduce_group(const int64_t* part, uint32_t n, SweepHeader* hdr) {
    const uint32_t k = blockIdx.x;
    reduce_partials(PartialReduce{part + 2ull * k * n, n, hdr->ser + 2ull * k});
    if (threadIdx.x == 0 && atomicAdd(&hdr->arrived, 1u) == gridDim.x - 1u) {
        hdr->arrived = 0;
        hdr->t += gridDim.x;
        hdr->ser += 2ull * gridDim.x;
    }
}

hipError_t launch_set_header(SweepHeader* hdr, uint32_t t, int64_t* ser, hipStream_t s) {
    k_set_header<<<1, 64, 0, s>>>(hdr, t, ser);
    return hipGetLastError();
}

hipError_t launch_reduce_group(const int64_t* part, uint32_t n, uint32_t g, SweepHeader* hdr, hipStream_t s) {
    if (n == 0) return hipErrorInvalidValue;  // every block must store, then arrive
    k_reduce_group<<<g, 256, 0, s>>>(part, n, hdr);
    return hipGetLastError();
}

hipError_t launch_generic_sweep(const Planes& pl, const AcceptTable& at, bool exact, uint32_t t, uint32_t k0,
                                uint32_t k1, int64_t* obs, hipStream_t s) {
    const uint32_t nb = blocks_for((uint64_t)pl.L * pl.H, 256);
    for (uint32_t c = 0; c < 2; ++c) {
        if (exact)
            k_half_sites<true><<<nb, 256, 0, s>>>(pl, at, c, t, k0, k1);
        else
            k_half_sites<false><<<nb, 256, 0, s>>>(pl, at, c, t, k0, k1);
    }
    k_observe<<<nb > 2048u ? 2048u : nb, 256, 0, s>>>(pl, obs);
    return hipGetLastError();
}

hipError_t launch_observe(const Planes& pl, int64_t* out, hipStream_t s) {
    k_zero_i64<<<1, 64, 0, s>>>(out, 2);
    const uint32_t nb = blocks_for((uint64_t)pl.L * pl.H, 256);
    k_observe<<<nb > 2048u ? 2048u : nb, 256, 0, s>>>(pl, out);
    return hipGetLastError();
}

hipError_t launch_zero(int64_t* p, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t nb = blocks_for(n, 256);
    k_zero_i64<<<nb > 4096u ? 4096u : (nb ? nb : 1u), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_to_canonical(const Planes& pl, int8_t* out, hipStream_t s) {
    const uint32_t nb = blocks_for((uint64_t)pl.L * pl.L, 256);
    k_to_canonical<<<nb > 65536u ? 65536u : nb, 256, 0, s>>>(pl, out);
    return hipGetLastError();
}

hipError_t launch_from_canonical(const Planes& pl, const int8_t* in, hipStream_t s) {
    const uint32_t nb = blocks_for((uint64_t)pl.L * pl.L, 256);
    k_from_canonical<<<nb > 65536u ? 65536u : nb, 256, 0, s>>>(pl, in);
    return hipGetLastError();
}

}  // namespace ising
