// HBM read-stream calibration: the practical read bandwidth of the device,
// against which the lag sum (a pure read stream of ring rows and Green
// spectra) is compared.  Every lane reads 16-byte words with non-temporal
// loads, as the lag sum does, and folds them into one word, stored once.
#include "rpot.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef unsigned nu4 __attribute__((ext_vector_type(4)));

template <int U>
__global__ __launch_bounds__(256) void k_read_stream(const nu4 *__restrict__ p, int64_t n16, uint32_t *sink) {
    uint32_t acc = 0;
    const int64_t stride = int64_t(gridDim.x) * 256 * U;
    for (int64_t i0 = int64_t(blockIdx.x) * 256 * U + threadIdx.x; i0 < n16; i0 += stride) {
        nu4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + int64_t(u) * 256;
            v[u] = i < n16 ? __builtin_nontemporal_load(p + i) : nu4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    sink[int64_t(blockIdx.x) * 256 + threadIdx.x] = acc;
}

}  // namespace

extern "C" {

rp_status rp_read_stream(const void *buf, size_t bytes, uint32_t *sink, int32_t grid, int32_t unroll,
                         void *hip_stream) {
    if (!buf || !sink || bytes < 16 || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(buf) % 16 != 0 ||
        grid < 1 || grid > (1 << 20))
        return RP_ERR_ARG;
    const nu4 *p = static_cast<const nu4 *>(buf);
    const int64_t n16 = int64_t(bytes / 16);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    switch (unroll) {
    case 1: hipLaunchKernelGGL(k_read_stream<1>, dim3(unsigned(grid)), dim3(256), 0, st, p, n16, sink); break;
    case 2: hipLaunchKernelGGL(k_read_stream<2>, dim3(unsigned(grid)), dim3(256), 0, st, p, n16, sink); break;
    case 4: hipLaunchKernelGGL(k_read_stream<4>, dim3(unsigned(grid)), dim3(256), 0, st, p, n16, sink); break;
    case 8: hipLaunchKernelGGL(k_read_stream<8>, dim3(unsigned(grid)), dim3(256), 0, st, p, n16, sink); break;
    default: return RP_ERR_ARG;
    }
    return hipGetLastError() == hipSuccess ? RP_OK : RP_ERR_DEVICE;
}

}  // extern "C"
