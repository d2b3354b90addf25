// Lag-sum multiply-accumulate over the ring of source spectra, and the small
// helper kernels of the step path.
//
// For every target sub-domain s and frequency k (Eq. "retardation space-time
// sampled lorentz four vector potential" after the spatial FFT, Sec. IV):
//
//   acc_s,mu(k) = sum_n sum_{m = m_lo(s,n)}^{m_hi(s,n)} Ghat_{s,n,m}(k) dShat_n,mu(l - m, k)
//
// One thread owns one frequency k and the four components of every target in
// its group (up to 8), so a ring snapshot (n, l-m) that feeds several targets
// is read once.  Every byte of the Green spectra and of the ring window is read
// exactly once per launch and nothing is shared between blocks: the kernel is a
// pure HBM stream (about 0.8 flop per byte in FP32), with no LDS and no atomics.
// The (source, lag) schedule is uniform across the block and is read through
// the scalar cache.
#include "rpot_internal.hpp"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>

namespace rpot {

typedef float nf2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef double nd4 __attribute__((ext_vector_type(4)));
typedef unsigned nu4 __attribute__((ext_vector_type(4)));

template <typename T, int FMT>
struct RingLoad;

template <>
struct RingLoad<double, RING_F64> {
    __device__ static void get(const void *ring, int64_t idx, const float *, Cx<double> (&x)[4]) {
        const nd4 *p = reinterpret_cast<const nd4 *>(reinterpret_cast<const Cx<double> *>(ring) + idx);
        const nd4 a = __builtin_nontemporal_load(p);
        const nd4 b = __builtin_nontemporal_load(p + 1);
        x[0] = {a.x, a.y};
        x[1] = {a.z, a.w};
        x[2] = {b.x, b.y};
        x[3] = {b.z, b.w};
    }
};
template <>
struct RingLoad<float, RING_F32> {
    __device__ static void get(const void *ring, int64_t idx, const float *, Cx<float> (&x)[4]) {
        const nf4 *p = reinterpret_cast<const nf4 *>(reinterpret_cast<const Cx<float> *>(ring) + idx);
        const nf4 a = __builtin_nontemporal_load(p);
        const nf4 b = __builtin_nontemporal_load(p + 1);
        x[0] = {a.x, a.y};
        x[1] = {a.z, a.w};
        x[2] = {b.x, b.y};
        x[3] = {b.z, b.w};
    }
};
template <>
struct RingLoad<float, RING_F16> {
    __device__ static void get(const void *ring, int64_t idx, const float *sc, Cx<float> (&x)[4]) {
        const nu4 *p = reinterpret_cast<const nu4 *>(reinterpret_cast<const __half2 *>(ring) + idx);
        const nu4 v = __builtin_nontemporal_load(p);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            __half2 h;
            __builtin_memcpy(&h, &w[mu], 4);
            const float2 f = __half22float2(h);
            x[mu] = {f.x * sc[mu], f.y * sc[mu]};
        }
    }
};
template <>
struct RingLoad<float, RING_BF16> {
    __device__ static void get(const void *ring, int64_t idx, const float *sc, Cx<float> (&x)[4]) {
        const nu4 *p = reinterpret_cast<const nu4 *>(reinterpret_cast<const unsigned *>(ring) + idx);
        const nu4 v = __builtin_nontemporal_load(p);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            // bf16 -> fp32 is a 16-bit left shift of the bit pattern
            const float re = __uint_as_float(w[mu] << 16);
            const float im = __uint_as_float(w[mu] & 0xffff0000u);
            x[mu] = {re * sc[mu], im * sc[mu]};
        }
    }
};

__device__ __forceinline__ Cx<float> load_spec(const Cx<float> *p) {
    const nf2 v = __builtin_nontemporal_load(reinterpret_cast<const nf2 *>(p));
    return {v.x, v.y};
}
__device__ __forceinline__ Cx<double> load_spec(const Cx<double> *p) {
    const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2 *>(p));
    return {v.x, v.y};
}

// Everything one (source, lag) entry contributes to a thread: the ring
// snapshot of the source at that lag and the Green spectrum of every group
// member fed by it.
template <typename T, int TG>
struct EntryData {
    Cx<T> x[4];
    Cx<T> g[TG];
    uint32_t mask;
};

template <typename T, int FMT, int TG>
__device__ __forceinline__ void load_entry(const K2Args &a, const K2Entry &en, int64_t l, int64_t C, int64_t k,
                                           const Cx<T> *__restrict__ spec, EntryData<T, TG> &d) {
    const DomDev &dd = a.doms[en.src];
    int64_t slot = (l - en.m) % dd.depth;
    if (slot < 0) slot += dd.depth;
    float sc[4] = {1.f, 1.f, 1.f, 1.f};
    if (FMT == RING_F16 || FMT == RING_BF16) {
        const float *s = a.scales + dd.scale_off + slot * 4;
        sc[0] = s[0];
        sc[1] = s[1];
        sc[2] = s[2];
        sc[3] = s[3];
    }
    RingLoad<T, FMT>::get(a.ring, dd.ring_off + (slot * C + k) * 4, sc, d.x);
    d.mask = en.mask;
    const uint32_t cj = en.conj;
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        if (en.mask & (1u << t)) {
            d.g[t] = load_spec(spec + int64_t(en.spec[t]) * C);
            if (cj & (1u << t)) d.g[t].y = -d.g[t].y;
        }
    }
}

template <typename T, int TG>
__device__ __forceinline__ void mac_entry(const EntryData<T, TG> &d, Cx<T> (&acc)[TG][4]) {
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        if (d.mask & (1u << t)) {
            const Cx<T> gv = d.g[t];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                acc[t][mu].x = fma(gv.x, d.x[mu].x, acc[t][mu].x);
                acc[t][mu].x = fma(-gv.y, d.x[mu].y, acc[t][mu].x);
                acc[t][mu].y = fma(gv.x, d.x[mu].y, acc[t][mu].y);
                acc[t][mu].y = fma(gv.y, d.x[mu].x, acc[t][mu].y);
            }
        }
    }
}

// U entries are loaded before any of them is accumulated, so a wave keeps U
// entries' worth of loads in flight (the kernel is bound by memory-level
// parallelism, not by arithmetic).
template <typename T, int FMT, int TG, int U>
__global__ __launch_bounds__(256) void k_lagsum(K2Args a) {
    const K2Item item = a.items[blockIdx.x];
    const K2Group &g = a.groups[item.group];
    const int64_t C = g.C;
    const int64_t k = int64_t(item.k0) + threadIdx.x;
    if (k >= C) return;
    const int64_t l = *a.step;
    const Cx<T> *__restrict__ spec = reinterpret_cast<const Cx<T> *>(a.spectra) + g.spec_base + k;

    Cx<T> acc[TG][4];
#pragma unroll
    for (int t = 0; t < TG; ++t)
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) acc[t][mu] = {T(0), T(0)};

    int e = g.entry_begin;
    for (; e + U <= g.entry_end; e += U) {
        EntryData<T, TG> d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) load_entry<T, FMT, TG>(a, a.entries[e + u], l, C, k, spec, d[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) mac_entry<T, TG>(d[u], acc);
    }
    for (; e < g.entry_end; ++e) {
        EntryData<T, TG> d;
        load_entry<T, FMT, TG>(a, a.entries[e], l, C, k, spec, d);
        mac_entry<T, TG>(d, acc);
    }

    Cx<T> *__restrict__ out = reinterpret_cast<Cx<T> *>(a.acc);
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        if (t < g.n_members) {
            Cx<T> *o = out + a.doms[g.member[t]].acc_off + k * 4;
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) o[mu] = acc[t][mu];
        }
    }
}

template <typename T, int FMT, int TG>
static void launch_u(const K2Args &a, int unroll, hipStream_t st) {
    dim3 grid(a.n_items), block(256);
    switch (unroll) {
    case 1: hipLaunchKernelGGL((k_lagsum<T, FMT, TG, 1>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_lagsum<T, FMT, TG, 4>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((k_lagsum<T, FMT, TG, 2>), grid, block, 0, st, a); break;
    }
}

template <typename T, int FMT>
static void launch_tg(const K2Args &a, int tg, int unroll, hipStream_t st) {
    switch (tg) {
    case 1: launch_u<T, FMT, 1>(a, unroll, st); break;
    case 2: launch_u<T, FMT, 2>(a, unroll, st); break;
    case 4: launch_u<T, FMT, 4>(a, unroll, st); break;
    default: launch_u<T, FMT, 8>(a, unroll, st); break;
    }
}

void launch_lagsum(const K2Args &a, int prec64, int ring_fmt, int tg, int unroll, hipStream_t st) {
    if (a.n_items == 0) return;
    if (prec64) {
        launch_tg<double, RING_F64>(a, tg, unroll, st);
    } else if (ring_fmt == RING_F16) {
        launch_tg<float, RING_F16>(a, tg, unroll, st);
    } else if (ring_fmt == RING_BF16) {
        launch_tg<float, RING_BF16>(a, tg, unroll, st);
    } else {
        launch_tg<float, RING_F32>(a, tg, unroll, st);
    }
}

// ---------------------------------------------------------------------------
__global__ void k_ring_scale(ScaleArgs a) {
    const ScaleJob &j = a.jobs[blockIdx.x];
    const int mu = threadIdx.x & 3;
    const int lane = threadIdx.x >> 2;     // 64 threads: 16 per component
    float m = 0.f;
    for (int b = lane; b < j.nblk; b += 16) m = fmaxf(m, j.zmax[b * 4 + mu]);
    for (int o = 4; o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (lane == 0) {
        const double bound = j.npts * double(m);
        float s = 1.0f;
        if (bound > 0.0) {
            int e;
            frexp(bound, &e);              // bound <= 2^e
            s = ldexpf(1.0f, e - 15);      // |value| / s <= 2^15 < FP16 max
        }
        const int64_t slot = (*a.step) % j.depth;
        j.scales[slot * 4 + mu] = s;
    }
}

void launch_ring_scale(const ScaleArgs &a, hipStream_t st) {
    if (a.n_jobs == 0) return;
    hipLaunchKernelGGL(k_ring_scale, dim3(a.n_jobs), dim3(64), 0, st, a);
}

// acc[k][mu] += g[k] * s[k][mu]  (FP64; static potential)
__global__ void k_static_mac(Cx<double> *acc, const Cx<double> *g, const Cx<double> *s, int64_t C) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= C) return;
    const Cx<double> gv = g[k];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const Cx<double> x = s[k * 4 + mu];
        Cx<double> &o = acc[k * 4 + mu];
        o.x += gv.x * x.x - gv.y * x.y;
        o.y += gv.x * x.y + gv.y * x.x;
    }
}

void launch_static_mac(void *acc, const void *g, const void *s, int64_t C, hipStream_t st) {
    const int64_t nb = (C + 255) / 256;
    hipLaunchKernelGGL(k_static_mac, dim3(unsigned(nb)), dim3(256), 0, st, reinterpret_cast<Cx<double> *>(acc),
                       reinterpret_cast<const Cx<double> *>(g), reinterpret_cast<const Cx<double> *>(s), C);
}

template <typename D, typename S>
__global__ void k_convert(D *dst, const S *src, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = D(src[i]);
}

void launch_convert(void *dst, int dst64, const void *src, int src64, int64_t n, hipStream_t st) {
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
    if (nb == 0) return;
    if (dst64 && src64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(unsigned(nb)), dim3(256), 0, st,
                           (double *)dst, (const double *)src, n);
    else if (dst64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(unsigned(nb)), dim3(256), 0, st,
                           (double *)dst, (const float *)src, n);
    else if (src64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(unsigned(nb)), dim3(256), 0, st,
                           (float *)dst, (const double *)src, n);
    else
        hipLaunchKernelGGL((k_convert<float, float>), dim3(unsigned(nb)), dim3(256), 0, st,
                           (float *)dst, (const float *)src, n);
}

__global__ void k_fill_zero(uint4 *p, int64_t n16) {
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = z;
}

void launch_fill_zero(void *dst, size_t bytes, hipStream_t st) {
    // bytes is a multiple of 16 (every workspace region is 256-byte aligned and padded)
    const int64_t n16 = int64_t(bytes / 16);
    if (n16 == 0) return;
    const int64_t nb = std::min<int64_t>((n16 + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_zero, dim3(unsigned(nb)), dim3(256), 0, st, reinterpret_cast<uint4 *>(dst), n16);
}

__global__ void k_advance_step(int64_t *step) {
    if (threadIdx.x == 0) *step += 1;
}

void launch_advance_step(int64_t *step, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(64), 0, st, step);
}

}  // namespace rpot
