// Renumbering of the fluid-only state after the geometry changes (particle
// deposition turns fluid nodes solid): the populations of every node that is
// still fluid move from its old fluid index to its new one, on the device.
//
// Arrays are chunked as in the step kernels: element (plane j, fluid node k)
// of an array with P planes at ((k >> 6) * P + j) * 64 + (k & 63).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace mclbm {

// dst(j, k) = src(j, from[k]) for every plane j, or 0 where from[k] < 0 (the
// unused lanes of the last chunk).  One thread per new fluid index k.
template <typename T>
__global__ void __launch_bounds__(256) k_remap(T* __restrict__ dst, const T* __restrict__ src, int P,
                                               const int* __restrict__ from, long long nnew) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnew) return;
    const int o = from[k];
    T* d = dst + ((size_t)(k >> 6) * (size_t)P) * 64u + (size_t)(k & 63);
    if (o < 0) {
        for (int j = 0; j < P; ++j) d[(size_t)j * 64u] = T(0);
        return;
    }
    const T* s = src + ((size_t)(o >> 6) * (size_t)P) * 64u + (size_t)(o & 63);
    for (int j = 0; j < P; ++j) d[(size_t)j * 64u] = s[(size_t)j * 64u];
}

hipError_t k_remap_planes(void* dst, const void* src, int planes, const int* from, long long nnew, int elem_bytes,
                          hipStream_t stream) {
    if (nnew <= 0 || planes <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nnew + 255) / 256));
    switch (elem_bytes) {
        case 8:
            hipLaunchKernelGGL(k_remap<uint64_t>, grid, dim3(256), 0, stream, (uint64_t*)dst, (const uint64_t*)src,
                               planes, from, nnew);
            break;
        case 4:
            hipLaunchKernelGGL(k_remap<uint32_t>, grid, dim3(256), 0, stream, (uint32_t*)dst, (const uint32_t*)src,
                               planes, from, nnew);
            break;
        case 2:
            hipLaunchKernelGGL(k_remap<uint16_t>, grid, dim3(256), 0, stream, (uint16_t*)dst, (const uint16_t*)src,
                               planes, from, nnew);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mclbm
