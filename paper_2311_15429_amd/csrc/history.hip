// Host tier of a split history: the copy kernel that moves real-space source
// snapshots between device staging buffers and rings in pinned host memory
// (the retained history of Sec. IV, kept off the device).  It runs on the
// plan's second stream beside the lag sum.
#include "rpot_internal.hpp"

#include <algorithm>

namespace rpot {

// One block row per job; each thread moves kTierU 16-byte words per pass,
// all loads before the stores.  Few blocks: the copies cross PCIe, so they
// are bound by the link and the requests in flight, not by compute units,
// and they run beside the lag sum, whose waves need the compute units.
constexpr int kTierU = 8;
constexpr int kTierBlocks = 16;

__global__ void __launch_bounds__(256) k_tier_copy(TierArgs a) {
    const TierJob &j = a.jobs[blockIdx.y];
    const int64_t step = *a.step;
    int64_t slot = 0;
    const int depth = j.src_depth > 0 ? j.src_depth : j.dst_depth;
    if (depth > 0) {
        slot = (int64_t(a.head[j.head_idx]) + j.shift) % depth;
        if (slot < 0) slot += depth;
    }
    const uint4 *src = j.src + (j.src_depth > 0 ? slot * j.n16 : 0);
    if (j.alt && step + j.shift <= 0) src = j.alt;
    uint4 *dst = j.dst + (j.dst_depth > 0 ? slot * j.n16 : 0);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x * kTierU;
    for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x * kTierU + threadIdx.x; i0 < j.n16; i0 += stride) {
        uint4 v[kTierU];
#pragma unroll
        for (int u = 0; u < kTierU; ++u) {
            const int64_t i = i0 + int64_t(u) * blockDim.x;
            if (i < j.n16) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < kTierU; ++u) {
            const int64_t i = i0 + int64_t(u) * blockDim.x;
            if (i < j.n16) dst[i] = v[u];
        }
    }
}

void launch_tier_copy(const TierArgs &a, hipStream_t st) {
    if (a.n_jobs <= 0) return;
    int64_t n16 = 0;
    for (int i = 0; i < a.n_jobs; ++i) n16 = std::max(n16, a.jobs[i].n16);
    const int64_t nb = std::min<int64_t>((n16 + 256 * kTierU - 1) / (256 * kTierU), kTierBlocks);
    if (nb == 0) return;
    hipLaunchKernelGGL(k_tier_copy, dim3(unsigned(nb), unsigned(a.n_jobs)), dim3(256), 0, st, a);
}

__global__ __launch_bounds__(256) void k_broadcast(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n16,
                                                   int64_t total) {
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256)
        dst[k] = src[k % n16];
}

void launch_broadcast(void *dst, const void *src, int64_t bytes, int32_t count, hipStream_t st) {
    const int64_t n16 = bytes / 16, total = n16 * count;
    if (total <= 0) return;
    const int64_t nb = std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_broadcast, dim3(unsigned(nb)), dim3(256), 0, st, static_cast<uint4 *>(dst),
                       static_cast<const uint4 *>(src), n16, total);
}

}  // namespace rpot
