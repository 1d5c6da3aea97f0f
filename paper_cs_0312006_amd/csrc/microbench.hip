// Vector-operation and host-transfer micro-benchmarks (include/microbench.h):
// the MI355X counterparts of the paper's GPU calibration (Table 2: one pass
// of a simple operation over float vectors; Table 5: whole-lattice and
// border-only transfers between host and GPU).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "microbench.h"

namespace {

constexpr uint32_t kThreads = 256;

template <uint32_t OP>
__device__ __forceinline__ float apply(float a, float c) {
    if constexpr (OP == MB_OP_COPY) return c;
    if constexpr (OP == MB_OP_ADD) return a + c;
    if constexpr (OP == MB_OP_SUB) return a - c;
    if constexpr (OP == MB_OP_MUL) return a * c;
    if constexpr (OP == MB_OP_DIV) return a / c;
    if constexpr (OP == MB_OP_SIN) return sinf(a);
    if constexpr (OP == MB_OP_COS) return cosf(a);
    if constexpr (OP == MB_OP_LOG) return logf(a);
    return expf(a);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Streaming pass over float4s (n4 of them), then the scalar tail. A block
// takes chunks of kUnroll * blockDim consecutive float4s (grid-stride over
// chunks): each thread issues all of its kUnroll loads of a chunk before the
// first store, and loads and stores are nontemporal (each line is touched
// once), so many bytes are in flight per wave.
constexpr int kUnroll = 4;

template <uint32_t OP>
__global__ void __launch_bounds__(kThreads) k_vec(float* __restrict__ a, const float* __restrict__ c, size_t n) {
    constexpr bool reads_a = OP != MB_OP_COPY;
    constexpr bool reads_c = OP <= MB_OP_DIV;
    const size_t n4 = n / 4;
    f32x4* a4 = reinterpret_cast<f32x4*>(a);
    const f32x4* c4 = reinterpret_cast<const f32x4*>(c);
    const size_t chunk = (size_t)blockDim.x * kUnroll;
    for (size_t base = blockIdx.x * chunk; base < n4; base += (size_t)gridDim.x * chunk) {
        f32x4 x[kUnroll], y[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const size_t k = base + (size_t)j * blockDim.x + threadIdx.x;
            x[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            y[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (k < n4) {
                if (reads_a) x[j] = __builtin_nontemporal_load(a4 + k);
                if (reads_c) y[j] = __builtin_nontemporal_load(c4 + k);
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const size_t k = base + (size_t)j * blockDim.x + threadIdx.x;
            if (k < n4) {
                f32x4 v;
                v.x = apply<OP>(x[j].x, y[j].x);
                v.y = apply<OP>(x[j].y, y[j].y);
                v.z = apply<OP>(x[j].z, y[j].z);
                v.w = apply<OP>(x[j].w, y[j].w);
                __builtin_nontemporal_store(v, a4 + k);
            }
        }
    }
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = 4 * n4 + blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += stride)
        a[k] = apply<OP>(reads_a ? a[k] : 0.f, reads_c ? c[k] : 0.f);
}

template <uint32_t OP>
hipError_t launch(float* a, const float* c, size_t n, hipStream_t s) {
    size_t blocks = (n / 4 + kThreads * kUnroll - 1) / (kThreads * kUnroll);
    if (blocks > 2048) blocks = 2048;  // eight workgroups per compute unit, grid-stride beyond
    if (blocks == 0) blocks = 1;
    k_vec<OP><<<(uint32_t)blocks, kThreads, 0, s>>>(a, c, n);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kThreads) k_philox(uint32_t* out, uint32_t n, uint32_t calls, uint32_t k0,
                                                     uint32_t k1) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= n) return;
    uint32_t acc = 0;
    for (uint32_t k = 0; k < calls; ++k) {
        const uint4 r = ising::philox(tid, k, 0u, 0u, k0, k1);
        acc ^= ising::xor3(r.x, r.y, r.z) ^ r.w;
    }
    out[tid] = acc;
}

}  // namespace

extern "C" {

int mb_philox(uint32_t* out, size_t n_threads, uint32_t calls_per_thread, uint64_t seed, void* stream) {
    if (!out || n_threads == 0 || n_threads > (size_t)1 << 31) return ISING_EINVAL;
    const uint32_t n = (uint32_t)n_threads;
    k_philox<<<(n + kThreads - 1) / kThreads, kThreads, 0, (hipStream_t)stream>>>(out, n, calls_per_thread,
                                                                                  (uint32_t)seed,
                                                                                  (uint32_t)(seed >> 32));
    if (hipGetLastError() != hipSuccess) return ISING_EDEVICE;
    return ISING_OK;
}


int mb_vector_op(uint32_t op, float* a, const float* c, size_t n, void* stream) {
    if (op > MB_OP_EXP || !a) return ISING_EINVAL;
    if (op <= MB_OP_DIV && !c) return ISING_EINVAL;
    if (((uintptr_t)a & 15u) || ((uintptr_t)c & 15u)) return ISING_EINVAL;
    if (n == 0) return ISING_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    switch (op) {
        case MB_OP_COPY: e = launch<MB_OP_COPY>(a, c, n, s); break;
        case MB_OP_ADD: e = launch<MB_OP_ADD>(a, c, n, s); break;
        case MB_OP_SUB: e = launch<MB_OP_SUB>(a, c, n, s); break;
        case MB_OP_MUL: e = launch<MB_OP_MUL>(a, c, n, s); break;
        case MB_OP_DIV: e = launch<MB_OP_DIV>(a, c, n, s); break;
        case MB_OP_SIN: e = launch<MB_OP_SIN>(a, c, n, s); break;
        case MB_OP_COS: e = launch<MB_OP_COS>(a, c, n, s); break;
        case MB_OP_LOG: e = launch<MB_OP_LOG>(a, c, n, s); break;
        default: e = launch<MB_OP_EXP>(a, c, n, s); break;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return ISING_EDEVICE;
    }
    return ISING_OK;
}

int mb_copy_lattice(void* dst, const void* src, uint32_t L, uint32_t elem, uint32_t direction, int border,
                    void* stream) {
    if (!dst || !src || L == 0 || elem == 0 || direction > MB_DEVICE_TO_HOST) return ISING_EINVAL;
    const hipMemcpyKind kind = direction == MB_HOST_TO_DEVICE ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
    hipStream_t s = (hipStream_t)stream;
    const size_t row = (size_t)L * elem;
    char* d = static_cast<char*>(dst);
    const char* c = static_cast<const char*>(src);
    hipError_t e = hipSuccess;
    if (!border || L <= 2) {
        e = hipMemcpyAsync(d, c, row * L, kind, s);
    } else {
        const size_t last = (size_t)(L - 1) * row;
        e = hipMemcpyAsync(d, c, row, kind, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d + last, c + last, row, kind, s);
        // columns 0 and L-1 of rows 1 .. L-2: pitched copies of one site per row
        if (e == hipSuccess) e = hipMemcpy2DAsync(d + row, row, c + row, row, elem, L - 2, kind, s);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(d + row + row - elem, row, c + row + row - elem, row, elem, L - 2, kind, s);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return ISING_EDEVICE;
    }
    return ISING_OK;
}

}  // extern "C"
