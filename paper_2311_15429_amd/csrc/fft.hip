// LDS-staged mixed-radix (4, 2, 3) FFT passes for gfx950.
//
// The 3-D transforms of the method (Sec. IV: a 3-D FFT of every time slice of
// the zero-padded sources, and the inverse on the target domain) are split into
// one pass per axis.  A pass block stages a tile of whole lines in LDS, runs a
// self-sorting (Stockham) FFT over all of them in place, and writes back; the
// tile is read and written along the contiguous direction of global memory.
// Zero padding is pruned on input (only n_in points are read) and the crop on
// output (only n_out points are written).  Intermediate 3-D arrays keep the
// four components interleaved ([..][4]) so every pass moves 32/64-byte runs.
//
// Spectra index frequencies as k = (y Hz + z) Px + x (x fastest): the lag sum
// is pointwise in k, and this order lets the x passes, the only ones that
// touch spectra, move whole lines of Px frequencies as contiguous runs.
// Lines are staged in LDS at an odd row stride, so lanes that walk across
// lines do not share a bank.  FP32 passes of the usual lengths are compiled
// for their length (constant radix plan and index arithmetic); the others use
// the run-time kernel.  FP16/BF16 ring rows are written two components per
// lane, as one 8-byte store.
#include "rpot_internal.hpp"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>

namespace rpot {

template <typename T>
struct Lds;
template <>
struct Lds<float> {
    static constexpr int E = 4096;   // complex elements staged per block (32 KiB)
};
template <>
struct Lds<double> {
    static constexpr int E = 2048;   // 32 KiB
};

// Global reads of a tile go in chunks of kLoadChunk per thread: all loads of
// a chunk are issued before the first is used, so a wave keeps that many in
// flight instead of one (the passes are bound by the requests in flight).
constexpr int kLoadChunk = 8;

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
// multiply by sgn * i
template <typename T>
__device__ __forceinline__ Cx<T> mul_i(Cx<T> a, int sgn) {
    return sgn > 0 ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}

// Radix-R butterfly in place (after the twiddles), R = 2, 3 or 4; dir is the
// sign of the exponent.
template <typename T, int R>
__device__ __forceinline__ void butterfly(Cx<T> (&v)[R], int dir) {
    if constexpr (R == 4) {
        const Cx<T> t0 = cadd(v[0], v[2]);
        const Cx<T> t1 = csub(v[0], v[2]);
        const Cx<T> t2 = cadd(v[1], v[3]);
        const Cx<T> t3 = mul_i(csub(v[1], v[3]), dir);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    } else if constexpr (R == 2) {
        const Cx<T> t0 = v[0];
        v[0] = cadd(t0, v[1]);
        v[1] = csub(t0, v[1]);
    } else {
        static_assert(R == 3, "radix 2, 3 or 4");
        const T s3 = T(0.86602540378443864676372317075294);
        const Cx<T> s = cadd(v[1], v[2]);
        const Cx<T> d = csub(v[1], v[2]);
        const Cx<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
        const Cx<T> e = mul_i(Cx<T>{s3 * d.x, s3 * d.y}, dir);
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, e);
        v[2] = csub(m, e);
    }
}

// n / D: by the constant D when D > 0, else by the run-time divisor fd.
template <int D>
__device__ __forceinline__ int divc(int n, const FastDiv &fd) {
    if constexpr (D > 0) return int(unsigned(n) / unsigned(D));
    else return fd.div(n);
}

// Row stride (complex elements) of the lines staged in LDS: odd for lines of
// 8 points or more, so that lanes walking across lines (same point, next line)
// fall in different banks instead of all in one.
__host__ __device__ constexpr int lds_stride(int P) { return P >= 8 ? (P | 1) : P; }
// Staged elements per block for a tile of E elements: room for the padding
// (L <= E / 8 lines when P >= 8).
__host__ __device__ constexpr int lds_room(int E) { return E + E / 8; }

// One Stockham stage of radix R over the L lines in LDS: butterfly b of line
// li reads x[i + r nq] (i = b mod nq, r < R), multiplies by the twiddles
// w^(r k) (k = i mod p, p the product of the earlier radices), transforms,
// and writes x[(i - k) R + k + r p].  Each butterfly's indices are computed
// once, for the read and the write.  With NQ, PP, TWS, NBF > 0 the stage
// constants are compile-time (the transform length is fixed), else the
// run-time values nq, p, tws, nbf are used.
template <typename T, int NT, int BMAX, int R, int NQ = 0, int PP = 0, int TWS = 0, int NBF = 0>
__device__ __forceinline__ void lds_stage(Cx<T> *buf, int S, int nbf_rt, int nq_rt, int p_rt, int tws_rt,
                                          FastDiv dq, FastDiv dp, int dir, const Cx<T> *tw) {
    const int tid = threadIdx.x;
    const int nq = NQ ? NQ : nq_rt;
    const int p = PP ? PP : p_rt;
    const int tws = TWS ? TWS : tws_rt;
    const int nbf = NBF ? NBF : nbf_rt;
    Cx<T> v[BMAX][R];
    int wpos[BMAX];
#pragma unroll
    for (int it = 0; it < BMAX; ++it) {
        const int b = tid + it * NT;
        wpos[it] = -1;
        if ((NBF > 0 && NBF % NT == 0) || b < nbf) {
            const int li = divc<NQ>(b, dq);
            const int i = b - li * nq;
            const int q = divc<PP>(i, dp);
            const int k = i - q * p;
            const Cx<T> *row = buf + li * S;
            wpos[it] = li * S + q * p * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = row[i + r * nq];
            if (PP != 1 && k != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    Cx<T> w = tw[r * k * tws];
                    w.y = dir > 0 ? -w.y : w.y;
                    v[it][r] = cmul(v[it][r], w);
                }
            }
            butterfly<T, R>(v[it], dir);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < BMAX; ++it) {
        if (wpos[it] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[wpos[it] + r * p] = v[it][r];
        }
    }
    __syncthreads();
}

// In-place FFT of L lines of length P held in LDS (row-major, row stride S).
// dir = -1: sum_j x_j exp(-2 pi i jk/P);  dir = +1: exp(+2 pi i jk/P).
// The twiddles tw come from LDS; every division by a stage constant is a
// multiply-high (RadixPlan::dq, dp).
template <typename T, int NT, int BMAX>
__device__ void lds_fft(Cx<T> *buf, int P, int S, int L, int dir, const Cx<T> *tw, const RadixPlan &rp) {
    int p = 1;
    for (int st = 0; st < rp.n; ++st) {
        const int R = rp.r[st];
        const int nq = P / R;
        const int nbf = L * nq;
        if (R == 4) lds_stage<T, NT, BMAX, 4>(buf, S, nbf, nq, p, rp.tws[st], rp.dq[st], rp.dp[st], dir, tw);
        else if (R == 2) lds_stage<T, NT, BMAX, 2>(buf, S, nbf, nq, p, rp.tws[st], rp.dq[st], rp.dp[st], dir, tw);
        else lds_stage<T, NT, BMAX, 3>(buf, S, nbf, nq, p, rp.tws[st], rp.dq[st], rp.dp[st], dir, tw);
        p *= R;
    }
}

// The same transform for a length P fixed at compile time (L lines): the
// radix plan (4s, then a 2, then 3s, as make_radix) unrolls into stages whose
// index arithmetic is by constants.
struct RadixList {
    int n;
    int r[16];
};
__host__ __device__ constexpr RadixList radix_list(int P) {
    RadixList l{};
    int m = P;
    while (m % 4 == 0) { l.r[l.n++] = 4; m /= 4; }
    while (m % 2 == 0) { l.r[l.n++] = 2; m /= 2; }
    while (m % 3 == 0) { l.r[l.n++] = 3; m /= 3; }
    return l;
}
__host__ __device__ constexpr int radix_prod(int P, int st) {
    const RadixList l = radix_list(P);
    int p = 1;
    for (int i = 0; i < st; ++i) p *= l.r[i];
    return p;
}

template <typename T, int NT, int P, int L, int ST = 0>
__device__ __forceinline__ void lds_fft_s(Cx<T> *buf, int dir, const Cx<T> *tw) {
    constexpr RadixList rl = radix_list(P);
    if constexpr (ST < rl.n) {
        constexpr int R = rl.r[ST];
        constexpr int PP = radix_prod(P, ST);
        constexpr int NQ = P / R;
        constexpr int NBF = L * NQ;
        constexpr int TWS = P / (PP * R);
        constexpr int BM = (NBF + NT - 1) / NT;
        const FastDiv none;
        lds_stage<T, NT, BM, R, NQ, PP, TWS, NBF>(buf, lds_stride(P), NBF, NQ, PP, TWS, none, none, dir, tw);
        lds_fft_s<T, NT, P, L, ST + 1>(buf, dir, tw);
    }
}

// ---------------------------------------------------------------------------
// Output conversion for the generic pass.
template <typename T, int FMT>
struct Store;
template <typename T>
struct Store<T, RING_F64> {
    __device__ static void put(void *base, int64_t idx, Cx<T> v, float) {
        reinterpret_cast<Cx<double> *>(base)[idx] = Cx<double>{double(v.x), double(v.y)};
    }
};
template <typename T>
struct Store<T, RING_F32> {
    __device__ static void put(void *base, int64_t idx, Cx<T> v, float) {
        reinterpret_cast<Cx<float> *>(base)[idx] = Cx<float>{float(v.x), float(v.y)};
    }
};
template <typename T>
struct Store<T, RING_F16> {
    __device__ static void put(void *base, int64_t idx, Cx<T> v, float inv_scale) {
        reinterpret_cast<__half2 *>(base)[idx] =
            __halves2half2(__float2half_rn(float(v.x) * inv_scale), __float2half_rn(float(v.y) * inv_scale));
    }
};
template <typename T>
struct Store<T, RING_BF16> {
    __device__ static void put(void *base, int64_t idx, Cx<T> v, float inv_scale) {
        __hip_bfloat162 r;
        r.x = __float2bfloat16(float(v.x) * inv_scale);
        r.y = __float2bfloat16(float(v.y) * inv_scale);
        reinterpret_cast<__hip_bfloat162 *>(base)[idx] = r;
    }
};

// Hardware dispatches consecutive blocks round-robin over the 8 XCDs, each
// with its own L2.  This bijection gives every XCD a contiguous range of
// block indices, so neighbouring tiles, which share the cache lines at their
// edges, are fetched through one L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int x = b % kNumXcd, i = b / kNumXcd;
    const int q = n / kNumXcd, r = n % kNumXcd;
    return x * q + min(x, r) + i;
}

// Lines per block of a line pass with a compile-time length P: whole groups
// of four lines (every grouped order fits).
__host__ __device__ constexpr int static_lines(int E, int P) { return (E / P) & ~3; }

// PS > 0: the transform length is the compile-time PS (the launcher sets
// L = static_lines(E, PS)); PS = 0: run-time length and lines per block.
// One scaled FP16 / BF16 complex value as its 32-bit pattern (re low, im high).
template <int FMT>
__device__ __forceinline__ uint32_t pack_half2(float x, float y, float s) {
    if constexpr (FMT == RING_F16) {
        const __half2 h = __halves2half2(__float2half_rn(x * s), __float2half_rn(y * s));
        uint32_t u;
        __builtin_memcpy(&u, &h, 4);
        return u;
    } else {
        __hip_bfloat162 h;
        h.x = __float2bfloat16(x * s);
        h.y = __float2bfloat16(y * s);
        uint32_t u;
        __builtin_memcpy(&u, &h, 4);
        return u;
    }
}

template <typename T, int FMT, int E, int PS = 0>
__global__ __launch_bounds__(kFftThreads) void k_line_pass(LinePass a) {
    constexpr int NT = kFftThreads;
    constexpr int BMAX = (E / 2 + NT - 1) / NT;
    constexpr int LS = PS ? static_lines(E, PS) : 0;
    static_assert(PS == 0 || LS >= 4, "fixed-length pass needs four lines per block");
    constexpr int NB = PS ? LS * lds_stride(PS) : lds_room(E);
    constexpr int NTW = PS ? PS : kMaxFft;
    static_assert((NB + NTW) * sizeof(Cx<T>) <= 64 * 1024, "line-pass LDS above 64 KiB");
    __shared__ Cx<T> buf[NB];
    __shared__ Cx<T> twl[NTW];
    const LineJob &job = a.jobs[blockIdx.y];
    const int P = PS ? PS : a.P;
    const int L = PS ? LS : a.L;
    const int S = lds_stride(P);
    const int line0 = xcd_block(int(blockIdx.x), int(gridDim.x)) * L;
    const int nl = min(L, a.lines - line0);
    const Cx<T> *__restrict__ in = reinterpret_cast<const Cx<T> *>(job.in);
    for (int i = threadIdx.x; i < P; i += NT) twl[i] = reinterpret_cast<const Cx<T> *>(a.tw)[i];

    const bool jfast_in = (a.in_j == 1);
    const int LP = L * P;
    for (int e0 = threadIdx.x; e0 < LP; e0 += NT * kLoadChunk) {
        Cx<T> v[kLoadChunk];
        int o[kLoadChunk];
#pragma unroll
        for (int u = 0; u < kLoadChunk; ++u) {
            const int e = e0 + u * NT;
            int li, j;
            if (a.in_group > 0) {
                const int sh = a.in_group >> 1;   // groups of 1, 2 or 4 lines
                const int t = e >> sh;
                const int r = divc<PS>(t, a.dP);
                j = t - r * P;
                li = (r << sh) + (e & (a.in_group - 1));
            } else if (jfast_in) {
                li = divc<PS>(e, a.dP);
                j = e - li * P;
            } else {
                j = divc<LS>(e, a.dL);
                li = e - j * L;
            }
            o[u] = li * S + j;
            v[u] = {T(0), T(0)};
            if (e < LP && li < nl && j < a.n_in) {
                const int line = line0 + li;
                const int outer = a.dinner.div(line);
                const int inner = line - outer * a.n_inner;
                v[u] = in[outer * a.in_outer + inner * a.in_inner + int64_t(j) * a.in_j];
            }
        }
#pragma unroll
        for (int u = 0; u < kLoadChunk; ++u)
            if (e0 + u * NT < LP) buf[o[u]] = v[u];
    }
    __syncthreads();
    if constexpr (PS > 0) lds_fft_s<T, NT, PS, LS>(buf, a.dir, twl);
    else lds_fft<T, NT, BMAX>(buf, P, S, L, a.dir, twl, a.rp);

    void *obase = job.out;
    const float *qs = job.qscale;
    if (job.head) {
        const int64_t slot = *job.head;
        constexpr int esz = (FMT == RING_F64) ? 16 : ((FMT == RING_F32) ? 8 : 4);
        obase = reinterpret_cast<char *>(obase) + slot * job.slot_stride * esz;
        if (qs) qs += slot * 4;
    }
    // the snapshot's four component scales, inverted once (powers of two: exact)
    float iq0 = 1.0f, iq1 = 1.0f, iq2 = 1.0f, iq3 = 1.0f;
    if (FMT == RING_F16 || FMT == RING_BF16) {
        iq0 = 1.0f / qs[0];
        iq1 = 1.0f / qs[1];
        iq2 = 1.0f / qs[2];
        iq3 = 1.0f / qs[3];
    }
    const bool jfast_out = (a.out_j == 1);
    const int nout = a.n_out;
    if constexpr (FMT == RING_F16 || FMT == RING_BF16) {
        if (job.tile_stride && a.tile_comp == 4 && a.out_group == 4) {
            // ring rows [k][c] of 4-byte values: each lane converts the
            // components c0, c0 + 1 (c0 = 0 or 2) of one frequency and writes
            // them as one 8-byte store.  Blocks start on whole groups of four
            // lines (L is a multiple of 4), so line li0 carries component c0.
            for (int e = threadIdx.x; e < L * nout / 2; e += NT) {
                const int cp = e & 1;
                const int t = e >> 1;
                const int r = a.dnout.div(t);
                const int j = t - r * nout;
                const int li0 = r * 4 + cp * 2;
                if (li0 >= nl) continue;
                const int line = line0 + li0;
                const int outer = a.dinner.div(line);
                const int inner = line - outer * a.n_inner;
                const uint32_t u = uint32_t(outer * a.out_outer + inner * a.out_inner + int64_t(j) * a.out_j);
                const uint32_t kk = u >> 2;
                const int64_t idx = int64_t(kk / kTile) * job.tile_stride + int64_t((kk % kTile) * 4 + (u & 3));
                const Cx<T> v0 = buf[li0 * S + j];
                const Cx<T> v1 = buf[(li0 + 1) * S + j];
                const uint2 w = {pack_half2<FMT>(float(v0.x), float(v0.y), cp ? iq2 : iq0),
                                 pack_half2<FMT>(float(v1.x), float(v1.y), cp ? iq3 : iq1)};
                *reinterpret_cast<uint2 *>(reinterpret_cast<char *>(obase) + idx * 4) = w;
            }
            return;
        }
    }
    for (int e = threadIdx.x; e < L * nout; e += NT) {
        int li, j;
        if (a.out_group > 0) {
            const int sh = a.out_group >> 1;   // groups of 1, 2 or 4 lines
            const int t = e >> sh;
            const int r = a.dnout.div(t);
            j = t - r * nout;
            li = (r << sh) + (e & (a.out_group - 1));
        } else if (jfast_out) {
            li = a.dnout.div(e);
            j = e - li * nout;
        } else {
            j = divc<LS>(e, a.dL);
            li = e - j * L;
        }
        if (li < nl) {
            const int line = line0 + li;
            const int outer = a.dinner.div(line);
            const int inner = line - outer * a.n_inner;
            // the component is the fastest batch index (inner mod 4)
            const int comp = inner & 3;
            const float inv_scale = comp == 0 ? iq0 : (comp == 1 ? iq1 : (comp == 2 ? iq2 : iq3));
            int64_t idx = outer * a.out_outer + inner * a.out_inner + int64_t(j) * a.out_j;
            if (job.tile_stride) {
                // tile_comp is 1 or 4; one job's indices stay below 2^31
                const uint32_t u = uint32_t(idx);
                const uint32_t kk = a.tile_comp == 4 ? (u >> 2) : u;
                const uint32_t c = u - kk * uint32_t(a.tile_comp);
                const uint32_t kt = kk % kTile;
                // within a tile row: FP32 ring [c/2][k][c%2], FP64 ring [c][k],
                // FP16/BF16 ring [k][c] (one 16-byte lane load of every ring
                // row then covers a contiguous run); one component: [k]
                uint32_t w = kt;
                if (a.tile_comp == 4) {
                    if (FMT == RING_F32) w = (c >> 1) * (2 * kTile) + kt * 2 + (c & 1);
                    else if (FMT == RING_F64) w = c * kTile + kt;
                    else w = kt * 4 + c;
                }
                idx = int64_t(kk / kTile) * job.tile_stride + int64_t(w);
            }
            Store<T, FMT>::put(obase, idx, buf[li * S + j], inv_scale);
        }
    }
}

// Stage divisors of a radix plan (host).
static void fill_stage_divisors(RadixPlan &rp, int P) {
    int p = 1;
    for (int st = 0; st < rp.n; ++st) {
        rp.dq[st] = FastDiv(uint32_t(P / rp.r[st]));
        rp.dp[st] = FastDiv(uint32_t(p));
        rp.tws[st] = P / (p * rp.r[st]);
        p *= rp.r[st];
    }
}

template <typename T, int FMT>
static void launch_line_e(const LinePass &a, dim3 grid, int E, hipStream_t st) {
    // E is the staged element count of the T path (the FP64 path stages half)
    switch (E) {
    case Lds<T>::E / 2: hipLaunchKernelGGL((k_line_pass<T, FMT, Lds<T>::E / 2>), grid, dim3(kFftThreads), 0, st, a); break;
    case Lds<T>::E * 3 / 2:
        hipLaunchKernelGGL((k_line_pass<T, FMT, Lds<T>::E * 3 / 2>), grid, dim3(kFftThreads), 0, st, a);
        break;
    default: hipLaunchKernelGGL((k_line_pass<T, FMT, Lds<T>::E>), grid, dim3(kFftThreads), 0, st, a); break;
    }
}

// FP32 passes at the 2048 and 4096 tiles have a compile-time kernel for these
// transform lengths (the pads of the usual grids); other lengths, FP64 and the
// 6144 tile use the run-time kernel.
template <int FMT, int E, int P0, int... Ps>
static bool launch_line_static(const LinePass &a, dim3 grid, hipStream_t st) {
    if (a.P == P0) {
        hipLaunchKernelGGL((k_line_pass<float, FMT, E, P0>), grid, dim3(kFftThreads), 0, st, a);
        return true;
    }
    if constexpr (sizeof...(Ps) > 0) return launch_line_static<FMT, E, Ps...>(a, grid, st);
    else return false;
}
template <int FMT>
static bool launch_line_static_any(const LinePass &a, int E, dim3 grid, hipStream_t st) {
    if (E == Lds<float>::E) return launch_line_static<FMT, Lds<float>::E, 32, 48, 64, 96, 108, 128, 256>(a, grid, st);
    return launch_line_static<FMT, Lds<float>::E / 2, 32, 48, 64, 96, 108, 128, 256>(a, grid, st);
}
static bool has_static_len(int P) {
    for (int q : {32, 48, 64, 96, 108, 128, 256})
        if (P == q) return true;
    return false;
}

int line_pass_elems(int lds_elems, int prec64) {
    const int base = prec64 ? Lds<double>::E : Lds<float>::E;
    // default: the 16 KiB tile in FP32 (measured fastest on the 128^3 pads),
    // the 32 KiB tile in FP64
    if (lds_elems == 0) lds_elems = prec64 ? 4096 : 2048;
    if (lds_elems == 2048) return base / 2;
    if (lds_elems == 6144) return base * 3 / 2;
    return base;
}

void launch_line_pass(const LinePass &a0, int prec64, hipStream_t st) {
    if (!prec64 && a0.reg && launch_line_reg(a0, st)) return;
    LinePass a = a0;
    const int E = line_pass_elems(a.lds_elems, prec64);
    const bool fixed = !prec64 && (E == Lds<float>::E / 2 || E == Lds<float>::E) && a.out_fmt != RING_F64 &&
                       has_static_len(a.P);
    // grouped orders (groups of 1, 2 or 4 lines) need whole groups of lines in a block
    int G = std::max(std::max(a.in_group, a.out_group), 1);
    while (G > 1 && E / a.P < G) G /= 2;
    a.in_group = std::min(a.in_group, G);
    a.out_group = std::min(a.out_group, G);
    const int L = fixed ? static_lines(E, a.P) : E / a.P - (E / a.P) % G;
    a.L = L;
    a.dL = FastDiv(uint32_t(L));
    a.dP = FastDiv(uint32_t(a.P));
    a.dinner = FastDiv(uint32_t(a.n_inner));
    a.dnout = FastDiv(uint32_t(std::max(a.n_out, 1)));
    fill_stage_divisors(a.rp, a.P);
    dim3 grid((a.lines + L - 1) / L, a.n_jobs);
    if (prec64) {
        if (a.out_fmt == RING_F64) launch_line_e<double, RING_F64>(a, grid, E, st);
        else launch_line_e<double, RING_F32>(a, grid, E, st);
    } else if (fixed) {
        switch (a.out_fmt) {
        case RING_F16: launch_line_static_any<RING_F16>(a, E, grid, st); break;
        case RING_BF16: launch_line_static_any<RING_BF16>(a, E, grid, st); break;
        default: launch_line_static_any<RING_F32>(a, E, grid, st);
        }
    } else {
        switch (a.out_fmt) {
        case RING_F64: launch_line_e<float, RING_F64>(a, grid, E, st); break;
        case RING_F16: launch_line_e<float, RING_F16>(a, grid, E, st); break;
        case RING_BF16: launch_line_e<float, RING_BF16>(a, grid, E, st); break;
        default: launch_line_e<float, RING_F32>(a, grid, E, st);
        }
    }
}

// ---------------------------------------------------------------------------
// Complex lines per block of the z passes: a multiple of 4 (the four
// components of a position pair).
template <typename T>
__host__ __device__ constexpr int zfwd_lpb(int P) { return (Lds<T>::E / P) & ~3; }

// Sampled Green's function of one lag (modes 1 and 2 of ZFwd), FP64.
__device__ __forceinline__ int kernel_disp(int q, int P, int Ns, int Nn, bool &valid) {
    if (q < Ns) return q;
    if (q > P - Nn) return q - P;
    valid = false;
    return 0;
}

__device__ __forceinline__ double green_value(const ZFwd &a, const ZFwdJob &job, int qx, int qy, int qz) {
    bool valid = true;
    const int dx = kernel_disp(qx, a.Px, job.Ns[0], job.Nn[0], valid);
    const int dy = kernel_disp(qy, a.Py, job.Ns[1], job.Nn[1], valid);
    const int dz = kernel_disp(qz, a.Pz, job.Ns[2], job.Nn[2], valid);
    if (!valid) return 0.0;
    if (job.self && dx == 0 && dy == 0 && dz == 0) {
        if (a.mode == 2) return a.w_static * a.scale;
        return (job.m == 0 ? a.w_self0 : (job.m == 1 ? a.w_self1 : 0.0)) * a.scale;
    }
    const double X = job.off[0] + a.h * dx;
    const double Y = job.off[1] + a.h * dy;
    const double Z = job.off[2] + a.h * dz;
    const double R = sqrt(X * X + Y * Y + Z * Z);
    const double h3 = a.h * a.h * a.h;
    if (a.mode == 2) return h3 / R * a.scale;
    // T(m dt - R/c) with T(x) = max(0, 1 - |x|/dt), in units of dt
    const double x = double(job.m) - R * a.inv_cdt;
    const double tv = 1.0 - fabs(x);
    return tv > 0.0 ? h3 * tv / R * a.scale : 0.0;
}

// Two real lines of the SAME component are packed into one complex line
// (neighbouring (x, y) positions for sources, neighbouring y for the Green's
// function), so the rounding crosstalk of the packing never mixes the large
// scalar-potential source into the much smaller vector-potential ones.
// PS > 0: the z length is the compile-time PS (sources only, mode 0).
template <typename T, int PS = 0>
__global__ __launch_bounds__(kFftThreads) void k_zfwd(ZFwd a) {
    constexpr int E = Lds<T>::E;
    constexpr int NT = kFftThreads;
    constexpr int BMAX = (E / 2 + NT - 1) / NT;
    constexpr int LS = PS ? zfwd_lpb<T>(PS) : 0;
    constexpr int HS = PS ? PS / 2 + 1 : 0;
    constexpr int NB = PS ? LS * lds_stride(PS) : lds_room(E);
    constexpr int NTW = PS ? PS : kMaxFft;
    __shared__ Cx<T> buf[NB];
    __shared__ Cx<T> twl[NTW];
    __shared__ float red[4][NT / 64];
    const ZFwdJob &job = a.jobs[blockIdx.y];
    const int P = PS ? PS : a.Pz;
    const int L = PS ? LS : zfwd_lpb<T>(P);
    const int RS = lds_stride(P);   // LDS row stride
    for (int i = threadIdx.x; i < P; i += NT) twl[i] = reinterpret_cast<const Cx<T> *>(a.tw)[i];
    const int line0 = blockIdx.x * L;
    const int npos = a.Nx * a.Ny;
    const int nlines = (a.mode == 0) ? 4 * ((npos + 1) / 2) : a.Px * (a.Py / 2);
    const int nl = min(L, nlines - line0);

    float mx[4] = {0.f, 0.f, 0.f, 0.f};
    if (a.mode == 0) {
        // complex line c = pair * 4 + mu holds positions 2 pair (re) and 2 pair + 1 (im)
        const int64_t npts = int64_t(npos) * a.Nz;
        const T *__restrict__ S = reinterpret_cast<const T *>(job.src);
        if (job.src_head) {
            // a real-space history ring: the snapshot src_lag steps before the newest
            int h = (*job.src_head - job.src_lag) % job.src_depth;
            if (h < 0) h += job.src_depth;
            S += int64_t(h) * 4 * npts;
        }
        const T *__restrict__ S0 = reinterpret_cast<const T *>(job.s0);
        T *__restrict__ St = nullptr;
        if (job.store)
            St = reinterpret_cast<T *>(job.store) + (job.store_head ? int64_t(*job.store_head) * 4 * npts : 0);
        const int LP = L * P;
        for (int e0 = threadIdx.x; e0 < LP; e0 += NT * kLoadChunk) {
            // position a (real part) and b = a + 1 (imaginary part) of each element
            T sa[kLoadChunk], sb[kLoadChunk], qa[kLoadChunk], qb[kLoadChunk];
            int64_t oa[kLoadChunk];
            bool va[kLoadChunk], vb[kLoadChunk];
#pragma unroll
            for (int u = 0; u < kLoadChunk; ++u) {
                const int e = e0 + u * NT;
                const int li = divc<PS>(e, a.dP);
                const int z = e - li * P;
                const int c = line0 + li;
                const int pa = (c >> 2) * 2;
                va[u] = e < LP && li < nl && z < a.Nz;
                vb[u] = va[u] && pa + 1 < npos;
                oa[u] = (c & 3) * npts + int64_t(pa) * a.Nz + z;
                sa[u] = sb[u] = qa[u] = qb[u] = T(0);
                if (va[u]) {
                    sa[u] = S[oa[u]];
                    if (S0) qa[u] = S0[oa[u]];
                }
                if (vb[u]) {
                    sb[u] = S[oa[u] + a.Nz];
                    if (S0) qb[u] = S0[oa[u] + a.Nz];
                }
            }
#pragma unroll
            for (int u = 0; u < kLoadChunk; ++u) {
                const int e = e0 + u * NT;
                if (e >= LP) continue;
                const int li = divc<PS>(e, a.dP);
                const int z = e - li * P;
                Cx<T> v = {T(0), T(0)};
                if (va[u]) {
                    if (St) St[oa[u]] = sa[u];
                    v.x = sa[u] - qa[u];
                    if (vb[u]) {
                        if (St) St[oa[u] + a.Nz] = sb[u];
                        v.y = sb[u] - qb[u];
                    }
                    const int mu = (line0 + li) & 3;
                    mx[mu] = fmaxf(mx[mu], fmaxf(fabsf(float(v.x)), fabsf(float(v.y))));
                }
                buf[li * RS + z] = v;
            }
        }
    } else {
        for (int e = threadIdx.x; e < L * P; e += NT) {
            const int li = divc<PS>(e, a.dP);
            const int z = e - li * P;
            Cx<T> v = {T(0), T(0)};
            if (li < nl) {
                const int line = line0 + li;
                const int qx = a.dPy2.div(line);
                const int qy = 2 * (line - qx * (a.Py / 2));
                v.x = T(green_value(a, job, qx, qy, z));
                v.y = T(green_value(a, job, qx, qy + 1, z));
            }
            buf[li * RS + z] = v;
        }
    }
    if (a.mode == 0 && job.zmax) {
        for (int c = 0; c < 4; ++c) {
            float v = mx[c];
            for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
            if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
        }
    }
    __syncthreads();
    if (a.mode == 0 && job.zmax && threadIdx.x < 4) {
        float v = 0.f;
        for (int w = 0; w < NT / 64; ++w) v = fmaxf(v, red[threadIdx.x][w]);
        job.zmax[blockIdx.x * 4 + threadIdx.x] = v;
    }
    if constexpr (PS > 0) lds_fft_s<T, NT, PS, LS>(buf, -1, twl);
    else lds_fft<T, NT, BMAX>(buf, P, RS, L, -1, twl, a.rp);

    // unpack: X_re = (Z_k + conj Z_-k)/2,  X_im = (Z_k - conj Z_-k)/(2i)
    const int Hz = a.Hz;
    Cx<T> *__restrict__ out = reinterpret_cast<Cx<T> *>(job.out);
    if (a.mode == 0) {
        const int pos0 = (line0 >> 2) * 2;
        const int np = min(2 * ((nl + 3) >> 2), npos - pos0);
        for (int e = threadIdx.x; e < np * Hz * 4; e += NT) {
            const int mu = e & 3;
            const int pl = divc<HS>(e >> 2, a.dHz);
            const int k = (e >> 2) - pl * Hz;
            const int li = (pl >> 1) * 4 + mu;
            const Cx<T> zk = buf[li * RS + k];
            const Cx<T> zm = buf[li * RS + (k == 0 ? 0 : P - k)];
            Cx<T> r;
            if ((pl & 1) == 0) r = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            else r = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
            out[(int64_t(pos0 + pl) * Hz + k) * 4 + mu] = r;
        }
    } else {
        for (int e = threadIdx.x; e < 2 * nl * Hz; e += NT) {
            const int rl = divc<HS>(e, a.dHz);
            const int k = e - rl * Hz;
            const int li = rl >> 1;
            const Cx<T> zk = buf[li * RS + k];
            const Cx<T> zm = buf[li * RS + (k == 0 ? 0 : P - k)];
            Cx<T> r;
            if ((rl & 1) == 0) r = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            else r = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
            out[int64_t(2 * line0 + rl) * Hz + k] = r;
        }
    }
}

int zfwd_lines_per_block(int Pz, int prec64) {
    return prec64 ? zfwd_lpb<double>(Pz) : zfwd_lpb<float>(Pz);
}

static_assert(sizeof(ZFwd) <= 4096, "z-pass kernel arguments above 4 KiB");

// FP32 forward z pass of the sources with a compile-time length, for the
// same lengths as the line passes.
template <int P0, int... Ps>
static bool launch_zfwd_static(const ZFwd &a, dim3 grid, hipStream_t st) {
    if (a.Pz == P0) {
        hipLaunchKernelGGL((k_zfwd<float, P0>), grid, dim3(kFftThreads), 0, st, a);
        return true;
    }
    if constexpr (sizeof...(Ps) > 0) return launch_zfwd_static<Ps...>(a, grid, st);
    else return false;
}

void launch_zfwd(const ZFwd &a0, int prec64, hipStream_t st) {
    if (!prec64 && a0.reg && launch_zfwd_reg(a0, st)) return;
    ZFwd a = a0;
    a.dP = FastDiv(uint32_t(a.Pz));
    a.dHz = FastDiv(uint32_t(a.Hz));
    a.dPy2 = FastDiv(uint32_t(std::max(a.Py / 2, 1)));
    fill_stage_divisors(a.rp, a.Pz);
    const int L = zfwd_lines_per_block(a.Pz, prec64);
    const int nlines = (a.mode == 0) ? 4 * ((a.Nx * a.Ny + 1) / 2) : a.Px * (a.Py / 2);
    dim3 grid((nlines + L - 1) / L, a.n_jobs);
    if (prec64) hipLaunchKernelGGL(k_zfwd<double>, grid, dim3(kFftThreads), 0, st, a);
    else if (a.mode != 0 || !launch_zfwd_static<32, 48, 64, 96, 108, 128, 256>(a, grid, st))
        hipLaunchKernelGGL(k_zfwd<float>, grid, dim3(kFftThreads), 0, st, a);
}

// ---------------------------------------------------------------------------
// Complex-to-real z pass with crop and static add.  Complex line
// c = pair * 4 + mu carries positions 2 pair (real part) and 2 pair + 1
// (imaginary part) of component mu.
// PS > 0: the z length is the compile-time PS.
template <typename T, int PS = 0>
__global__ __launch_bounds__(kFftThreads) void k_zinv(ZInv a) {
    constexpr int E = Lds<T>::E;
    constexpr int NT = kFftThreads;
    constexpr int BMAX = (E / 2 + NT - 1) / NT;
    constexpr int LS = PS ? zfwd_lpb<T>(PS) : 0;
    constexpr int HS = PS ? PS / 2 + 1 : 0;
    constexpr int NB = PS ? LS * lds_stride(PS) : lds_room(E);
    constexpr int NTW = PS ? PS : kMaxFft;
    __shared__ Cx<T> buf[NB];
    __shared__ Cx<T> twl[NTW];
    const ZInvJob &job = a.jobs[blockIdx.y];
    const int P = PS ? PS : a.Pz;
    const int Hz = PS ? HS : a.Hz;
    for (int i = threadIdx.x; i < P; i += NT) twl[i] = reinterpret_cast<const Cx<T> *>(a.tw)[i];
    const int L = PS ? LS : zfwd_lpb<T>(P);
    const int S = lds_stride(P);
    const int line0 = blockIdx.x * L;
    const int npos = a.Nx * a.Ny;
    const int nlines = 4 * ((npos + 1) / 2);
    const int nl = min(L, nlines - line0);
    const Cx<T> *__restrict__ in = reinterpret_cast<const Cx<T> *>(job.in);
    const int pos0 = (line0 >> 2) * 2;

    // Z_k = X_a(k) + i X_b(k) and Z_{P-k} = conj X_a(k) + i conj X_b(k)
    const int nin = (L / 4) * Hz * 4;
    for (int e0 = threadIdx.x; e0 < nin; e0 += NT * kLoadChunk) {
        Cx<T> xa[kLoadChunk], xb[kLoadChunk];
#pragma unroll
        for (int u = 0; u < kLoadChunk; ++u) {
            const int e = e0 + u * NT;
            const int mu = e & 3;
            const int ppl = divc<HS>(e >> 2, a.dHz);
            const int k = (e >> 2) - ppl * Hz;
            const int li = ppl * 4 + mu;
            const int pa = pos0 + 2 * ppl;
            xa[u] = xb[u] = Cx<T>{T(0), T(0)};
            if (e < nin && li < nl) {
                xa[u] = in[(int64_t(pa) * Hz + k) * 4 + mu];
                if (pa + 1 < npos) xb[u] = in[(int64_t(pa + 1) * Hz + k) * 4 + mu];
            }
        }
#pragma unroll
        for (int u = 0; u < kLoadChunk; ++u) {
            const int e = e0 + u * NT;
            if (e >= nin) continue;
            const int mu = e & 3;
            const int ppl = divc<HS>(e >> 2, a.dHz);
            const int k = (e >> 2) - ppl * Hz;
            const int li = ppl * 4 + mu;
            if (k == 0 || 2 * k == P) {
                buf[li * S + k] = Cx<T>{xa[u].x, xb[u].x};
            } else {
                buf[li * S + k] = Cx<T>{xa[u].x - xb[u].y, xa[u].y + xb[u].x};
                buf[li * S + (P - k)] = Cx<T>{xa[u].x + xb[u].y, xb[u].x - xa[u].y};
            }
        }
    }
    __syncthreads();
    if constexpr (PS > 0) lds_fft_s<T, NT, PS, LS>(buf, +1, twl);
    else lds_fft<T, NT, BMAX>(buf, P, S, L, +1, twl, a.rp);

    T *__restrict__ out = reinterpret_cast<T *>(job.out);
    const T *__restrict__ add = reinterpret_cast<const T *>(job.add);
    const int np = min(2 * ((nl + 3) >> 2), npos - pos0);
    const int64_t npts = int64_t(npos) * a.Nz;
    // np is the block's position count: at most 2 (L / 4); a short block
    // (the last one) divides by its own count
    const int nout = 4 * np * a.Nz;
    const bool full = np == 2 * (L >> 2);
    for (int e0 = threadIdx.x; e0 < nout; e0 += NT * kLoadChunk) {
        T ad[kLoadChunk];
        int64_t o[kLoadChunk];
        int bi[kLoadChunk];
        bool odd[kLoadChunk];
#pragma unroll
        for (int u = 0; u < kLoadChunk; ++u) {
            const int e = e0 + u * NT;
            const int r = a.dNz.div(e);
            const int z = e - r * a.Nz;
            const int mu = full ? a.dnp.div(r) : r / np;
            const int pl = r - mu * np;
            bi[u] = ((pl >> 1) * 4 + mu) * S + z;
            odd[u] = (pl & 1) != 0;
            o[u] = mu * npts + int64_t(pos0 + pl) * a.Nz + z;
            ad[u] = (add && e < nout) ? add[o[u]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kLoadChunk; ++u) {
            if (e0 + u * NT >= nout) continue;
            const Cx<T> v = buf[bi[u]];
            T val = odd[u] ? v.y : v.x;
            if (add) val += ad[u];
            out[o[u]] = val;
        }
    }
}

// FP32 inverse z pass with a compile-time length (the line-pass lengths).
template <int P0, int... Ps>
static bool launch_zinv_static(const ZInv &a, dim3 grid, hipStream_t st) {
    if (a.Pz == P0) {
        hipLaunchKernelGGL((k_zinv<float, P0>), grid, dim3(kFftThreads), 0, st, a);
        return true;
    }
    if constexpr (sizeof...(Ps) > 0) return launch_zinv_static<Ps...>(a, grid, st);
    else return false;
}

void launch_zinv(const ZInv &a0, int prec64, hipStream_t st) {
    if (!prec64 && a0.reg && launch_zinv_reg(a0, st)) return;
    ZInv a = a0;
    const int L = zfwd_lines_per_block(a.Pz, prec64);
    a.dHz = FastDiv(uint32_t(a.Hz));
    a.dNz = FastDiv(uint32_t(a.Nz));
    a.dnp = FastDiv(uint32_t(std::max(2 * (L >> 2), 1)));
    fill_stage_divisors(a.rp, a.Pz);
    const int nlines = 4 * ((a.Nx * a.Ny + 1) / 2);
    dim3 grid((nlines + L - 1) / L, a.n_jobs);
    if (prec64) hipLaunchKernelGGL(k_zinv<double>, grid, dim3(kFftThreads), 0, st, a);
    else if (!launch_zinv_static<32, 48, 64, 96, 108, 128, 256>(a, grid, st))
        hipLaunchKernelGGL(k_zinv<float>, grid, dim3(kFftThreads), 0, st, a);
}

}  // namespace rpot
