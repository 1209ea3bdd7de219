// Streaming probes of the HBM bandwidth this device sustains: a read-only
// reduction, a write-only fill and a copy, each over one caller buffer far
// larger than every cache level, 16 bytes per lane per access, grid-stride.
// They give the practical ceiling the step kernels are compared with (the
// nominal 8 TB/s of HBM3E is not reachable by any access pattern).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "mclbm.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// each lane reads UNR float4 per iteration with non-temporal loads; the sum
// is written per lane only if it equals a value the data never produces, so
// the loads are kept without adding write traffic
template <int UNR>
__global__ void __launch_bounds__(256) k_read(const f4* __restrict__ a, size_t n4, f4* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (UNR - 1) * stride < n4; i += UNR * stride) {
        f4 v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) v[u] = __builtin_nontemporal_load(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < UNR; ++u) acc += v[u];
    }
    for (; i < n4; i += stride) acc += __builtin_nontemporal_load(a + i);
    if (acc.x == -1.2345f) sink[threadIdx.x] = acc;
}

template <int UNR>
__global__ void __launch_bounds__(256) k_write(f4* __restrict__ a, size_t n4, float v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const f4 val = {v, v, v, v};
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (UNR - 1) * stride < n4; i += UNR * stride)
#pragma unroll
        for (int u = 0; u < UNR; ++u) __builtin_nontemporal_store(val, a + i + u * stride);
    for (; i < n4; i += stride) __builtin_nontemporal_store(val, a + i);
}

template <int UNR>
__global__ void __launch_bounds__(256) k_copy(const f4* __restrict__ a, f4* __restrict__ b, size_t n4) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (UNR - 1) * stride < n4; i += UNR * stride) {
        f4 v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) v[u] = __builtin_nontemporal_load(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < UNR; ++u) __builtin_nontemporal_store(v[u], b + i + u * stride);
    }
    for (; i < n4; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

}  // namespace

extern "C" int mclbm_hbm_probe(int32_t kind, void* a, void* b, size_t bytes, int32_t blocks_per_cu, int32_t iters,
                               void* stream, double* best_gbps) {
    if (!a || !best_gbps || bytes < 4096 || (bytes & 15) || iters < 1 || blocks_per_cu < 1 || kind < 0 ||
        kind > 2 || ((kind == 0 || kind == 2) && !b))
        return MCLBM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return MCLBM_EHIP;
    const size_t n4 = bytes / 16;
    const dim3 grid((unsigned)(ncu * blocks_per_cu)), block(256);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return MCLBM_EHIP;
    }
    double best = 0.0;
    int rc = MCLBM_OK;
    for (int it = 0; it < iters + 1 && rc == MCLBM_OK; ++it) {   // first pass untimed (warm-up)
        if (hipEventRecord(e0, st) != hipSuccess) { rc = MCLBM_EHIP; break; }
        if (kind == 0)
            hipLaunchKernelGGL(k_read<4>, grid, block, 0, st, (const f4*)a, n4, (f4*)b);
        else if (kind == 1)
            hipLaunchKernelGGL(k_write<4>, grid, block, 0, st, (f4*)a, n4, 1.0f);
        else
            hipLaunchKernelGGL(k_copy<4>, grid, block, 0, st, (const f4*)a, (f4*)b, n4);
        float ms = 0.f;
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = MCLBM_EHIP;
            break;
        }
        const double moved = (kind == 2 ? 2.0 : 1.0) * (double)(n4 * 16);
        if (it > 0 && ms > 0.f) best = std::max(best, moved / (ms * 1e-3) / 1e9);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best_gbps = best;
    return rc;
}
