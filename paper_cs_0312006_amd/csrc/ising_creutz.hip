// Creutz's deterministic checkerboard dynamics, the random-number-free
// alternative that Section 2.2 of Tomov et al. cites. Every site carries a
// demon energy d in units of 4J (zero field), 0 <= d <= 255, stored in
// demon planes laid out like the spin planes. A pass over colour c flips a
// site iff its demon can pay for the move: e = dE / 4J = s n / 2 (n the sum
// of the four neighbour spins, so e in {-2..2}); flip iff e <= d and
// d - e <= 255, then d -= e. Each pass is its own inverse, so the reversed
// sweep (colour 1, then colour 0) undoes a sweep exactly, and spin energy
// plus 4J times the demon total is conserved exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_creutz.hpp"
#include "ising_device.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

constexpr uint32_t kCreutzThreads = 256;

}  // namespace

// One pass over colour c, in place, four sites per word (L % 8 == 0). The
// second pass of a sweep (OBS) also sums the observables of the finished
// sweep into per-block partials: every bond joins the two colours, so the
// bond sum is taken over the sites of the colour just updated. The first
// pass's block 0 reduces the previous sweep's partials into its series slot.
template <bool OBS>
__global__ void __launch_bounds__(kCreutzThreads) k_creutz_words(Planes pl, Planes dm, uint32_t c, int64_t* part,
                                                                 PartialReduce red) {
    if (!OBS && blockIdx.x == 0) reduce_partials(red);
    const uint32_t L = pl.L, Hw = pl.Hw;
    global_u32* own = as_global(reinterpret_cast<uint32_t*>(pl.p[c]));
    const global_u32* oth = as_global(reinterpret_cast<uint32_t*>(pl.p[c ^ 1u]));
    global_u32* dem = as_global(reinterpret_cast<uint32_t*>(dm.p[c]));
    const uint32_t total = L * Hw, stride = gridDim.x * blockDim.x;
    uint32_t sad = 0, ups = 0, nw = 0;
    for (uint32_t idx = xcd_block(gridDim.x) * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const uint32_t i = idx / Hw, w = idx - i * Hw;
        const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
        const uint32_t p = (i + c) & 1u;
        const size_t row = (size_t)i * Hw;
        const uint32_t ew = p ? (w + 1 == Hw ? 0u : w + 1) : (w == 0 ? Hw - 1 : w - 1);
        const uint32_t O = oth[row + w], E = oth[row + ew];
        const uint32_t n = oth[(size_t)iu * Hw + w] + oth[(size_t)id * Hw + w] + O + shifted(O, E, E, p);
        uint32_t Wn, Dn;
        creutz_word(own[row + w], n, dem[row + w], Wn, Dn);
        own[row + w] = Wn;
        dem[row + w] = Dn;
        if (OBS) {
            sad = sad_misaligned(Wn, n, sad);
            ups += __builtin_popcount(Wn) + __builtin_popcount(O);
            nw += 1;
        }
    }
    if (OBS) {
        int64_t b = wave_sum_i64(16 * (int64_t)nw - 2 * (int64_t)sad);
        int64_t m = wave_sum_i64(2 * (int64_t)ups - 8 * (int64_t)nw);
        __shared__ int64_t acc[2][kCreutzThreads / 64];
        const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
        if (lane == 0) {
            acc[0][wave] = b;
            acc[1][wave] = m;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t sb = 0, sm = 0;
            for (uint32_t k = 0; k < kCreutzThreads / 64; ++k) {
                sb += acc[0][k];
                sm += acc[1][k];
            }
            part[2 * blockIdx.x] = sb;
            part[2 * blockIdx.x + 1] = sm;
        }
    }
}

// One pass over colour c, one thread per site (any even L), in place.
__global__ void __launch_bounds__(kCreutzThreads) k_creutz_sites(Planes pl, Planes dm, uint32_t c) {
    const uint32_t L = pl.L, H = pl.H;
    const uint32_t total = L * H, stride = gridDim.x * blockDim.x;
    const uint8_t* oth = pl.p[c ^ 1u];
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const uint32_t i = idx / H, m = idx - i * H;
        const uint32_t iu = i == 0 ? L - 1 : i - 1, id = i + 1 == L ? 0 : i + 1;
        const uint32_t p = (i + c) & 1u;
        const uint32_t m2 = p ? (m + 1 == H ? 0 : m + 1) : (m == 0 ? H - 1 : m - 1);
        const uint32_t n = oth[(size_t)iu * H + m] + oth[(size_t)id * H + m] + oth[(size_t)i * H + m] +
                           oth[(size_t)i * H + m2];
        uint32_t Wn, Dn;
        creutz_word(pl.p[c][idx], n, dm.p[c][idx], Wn, Dn);
        pl.p[c][idx] = (uint8_t)Wn;
        dm.p[c][idx] = (uint8_t)Dn;
    }
}

// Demon total (units of 4J): block sums added atomically to out[0], which
// the launcher clears first.
__global__ void __launch_bounds__(kCreutzThreads) k_demon_sum(const uint8_t* d, uint64_t n, int64_t* out) {
    uint64_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n4 = n / 4;
    const uint32_t* d4 = reinterpret_cast<const uint32_t*>(d);
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n4; k += stride)
        acc += __builtin_amdgcn_sad_u8(d4[k], 0u, 0u);
    for (uint64_t k = 4 * n4 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += stride) acc += d[k];
    const int64_t s = wave_sum_i64((int64_t)acc);
    if ((threadIdx.x & 63u) == 0) atomicAdd(reinterpret_cast<unsigned long long*>(out), (unsigned long long)s);
}

__global__ void __launch_bounds__(kCreutzThreads) k_fill_u8(uint8_t* p, uint64_t n, uint8_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

// Byte planes <-> canonical row-major bytes (demon values copied as is).
__global__ void __launch_bounds__(kCreutzThreads) k_bytes_to_canonical(Planes pl, uint8_t* out) {
    const uint64_t N = (uint64_t)pl.L * pl.L, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; idx < N; idx += stride) {
        const uint32_t i = (uint32_t)(idx / pl.L), j = (uint32_t)(idx - (uint64_t)i * pl.L);
        out[idx] = pl.p[(i + j) & 1u][(size_t)i * pl.H + (j >> 1)];
    }
}

__global__ void __launch_bounds__(kCreutzThreads) k_bytes_from_canonical(Planes pl, const uint8_t* in) {
    const uint64_t N = (uint64_t)pl.L * pl.L, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; idx < N; idx += stride) {
        const uint32_t i = (uint32_t)(idx / pl.L), j = (uint32_t)(idx - (uint64_t)i * pl.L);
        pl.p[(i + j) & 1u][(size_t)i * pl.H + (j >> 1)] = in[idx];
    }
}

static uint32_t grid_for(uint64_t n) {
    const uint64_t b = (n + kCreutzThreads - 1) / kCreutzThreads;
    return (uint32_t)(b > 4096 ? 4096 : (b ? b : 1));
}

uint32_t creutz_blocks(const Planes& pl) { return grid_for((uint64_t)pl.L * pl.Hw); }

hipError_t launch_creutz_sweep(const Planes& pl, const Planes& dm, bool reverse, int64_t* part,
                               const PartialReduce& red, hipStream_t s) {
    const uint32_t c0 = reverse ? 1u : 0u;
    const uint32_t nb = creutz_blocks(pl);
    k_creutz_words<false><<<nb, kCreutzThreads, 0, s>>>(pl, dm, c0, part, red);
    k_creutz_words<true><<<nb, kCreutzThreads, 0, s>>>(pl, dm, c0 ^ 1u, part, PartialReduce{nullptr, 0, nullptr});
    return hipGetLastError();
}

hipError_t launch_creutz_sweep_sites(const Planes& pl, const Planes& dm, bool reverse, hipStream_t s) {
    const uint32_t c0 = reverse ? 1u : 0u;
    const uint32_t nb = grid_for((uint64_t)pl.L * pl.H);
    k_creutz_sites<<<nb, kCreutzThreads, 0, s>>>(pl, dm, c0);
    k_creutz_sites<<<nb, kCreutzThreads, 0, s>>>(pl, dm, c0 ^ 1u);
    return hipGetLastError();
}

hipError_t launch_demon_sum(const uint8_t* d, uint64_t n, int64_t* out, hipStream_t s) {
    const hipError_t r = launch_zero(out, 1, s);
    if (r != hipSuccess) return r;
    k_demon_sum<<<grid_for(n / 4 + 1), kCreutzThreads, 0, s>>>(d, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s) {
    k_fill_u8<<<grid_for(n), kCreutzThreads, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_bytes_to_canonical(const Planes& pl, uint8_t* out, hipStream_t s) {
    k_bytes_to_canonical<<<grid_for((uint64_t)pl.L * pl.L), kCreutzThreads, 0, s>>>(pl, out);
    return hipGetLastError();
}

hipError_t launch_bytes_from_canonical(const Planes& pl, const uint8_t* in, hipStream_t s) {
    k_bytes_from_canonical<<<grid_for((uint64_t)pl.L * pl.L), kCreutzThreads, 0, s>>>(pl, in);
    return hipGetLastError();
}

}  // namespace ising
