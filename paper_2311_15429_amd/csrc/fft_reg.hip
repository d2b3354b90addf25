// Register-resident line passes of the 3-D transforms (FP32, fixed lengths).
//
// The y and x passes of the padded 3-D FFTs (Sec. IV: one 3-D FFT per time
// slice of the zero-padded sources, and the inverse on the target domain) run
// many independent lines of one length P.  Here a line is split as
// P = T x E over T threads of E points each:
//
//   x[t + T n],  t < T, n < E          (thread t holds its E points)
//   X[k1 + E k2] = sum_t w_T^(t k2) [ w_P^(t k1) sum_n x[t + T n] w_E^(n k1) ]
//
// Stage 1 is an E-point DFT in registers per thread, then the twiddle
// w_P^(t k1) (table in LDS, index t k1 < P); one exchange through LDS; stage 2
// is E / T DFTs of T points per thread.  The small DFTs are mixed-radix
// (4, 2, 3) codelets unrolled at compile time, their twiddles compile-time
// constants.  Compared with a staged radix-by-radix transform this keeps one
// LDS round trip per pass and no per-butterfly index arithmetic; the passes
// were bound by instruction issue, not by HBM.
//
// Global loads and stores go straight from and to registers.  Which thread
// holds which (line, t) is chosen separately for the loads and the stores, so
// that consecutive lanes touch consecutive addresses: lines fastest when
// neighbouring lines are adjacent in memory, else groups of G lines
// interleaved with t (G = 1, 2, 4, the element order of the pass).
#include "rpot_internal.hpp"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace rpot {

namespace {

using Cf = Cx<float>;

constexpr double kPiD = 3.14159265358979323846264338327950288;

// sin and cos for |x| <= pi by their Taylor series (compile time)
constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / double((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / double((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}

// cos and sin of 2 pi j / N, j < N, rounded to FP32
template <int N>
struct UnitRoots {
    float c[N], s[N];
    constexpr UnitRoots() : c(), s() {
        for (int j = 0; j < N; ++j) {
            double a = 2.0 * kPiD * double(j) / double(N);
            if (a > kPiD) a -= 2.0 * kPiD;
            c[j] = float(taylor_cos(a));
            s[j] = float(taylor_sin(a));
        }
    }
};
template <int N>
constexpr UnitRoots<N> kRoots{};

// v * exp(DIR 2 pi i e / N); e is a constant once the codelets are unrolled,
// so the branches and the table reads fold away
template <int N, int DIR>
__device__ __forceinline__ Cf twid(Cf v, int e) {
    e %= N;
    if (e == 0) return v;
    if (2 * e == N) return Cf{-v.x, -v.y};
    if (4 * e == N) return DIR > 0 ? Cf{-v.y, v.x} : Cf{v.y, -v.x};
    if (4 * e == 3 * N) return DIR > 0 ? Cf{v.y, -v.x} : Cf{-v.y, v.x};
    const float c = kRoots<N>.c[e], s = float(DIR) * kRoots<N>.s[e];
    return Cf{v.x * c - v.y * s, v.x * s + v.y * c};
}

__device__ __forceinline__ Cf add(Cf a, Cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ Cf sub(Cf a, Cf b) { return {a.x - b.x, a.y - b.y}; }
// a * (DIR i)
template <int DIR>
__device__ __forceinline__ Cf rot(Cf a) {
    return DIR > 0 ? Cf{-a.y, a.x} : Cf{a.y, -a.x};
}

// X[k] = sum_n x[n] exp(DIR 2 pi i n k / N), natural order in and out.
// Composite N = R M (R = 4, else 2, else 3) by decimation in time:
// X[k + M q] = sum_r w_R^(r q) [ w_N^(r k) DFT_M(x[R m + r])[k] ].
template <int N, int DIR>
__device__ __forceinline__ void dft(const Cf (&x)[N], Cf (&X)[N]) {
    if constexpr (N == 1) {
        X[0] = x[0];
    } else if constexpr (N == 2) {
        X[0] = add(x[0], x[1]);
        X[1] = sub(x[0], x[1]);
    } else if constexpr (N == 3) {
        const float h = 0.86602540378443864676f;   // sin(2 pi / 3)
        const Cf s = add(x[1], x[2]);
        const Cf d = sub(x[1], x[2]);
        const Cf m = {x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y};
        const Cf e = rot<DIR>(Cf{h * d.x, h * d.y});
        X[0] = add(x[0], s);
        X[1] = add(m, e);
        X[2] = sub(m, e);
    } else if constexpr (N == 4) {
        const Cf a = add(x[0], x[2]), b = sub(x[0], x[2]);
        const Cf c = add(x[1], x[3]), d = rot<DIR>(sub(x[1], x[3]));
        X[0] = add(a, c);
        X[2] = sub(a, c);
        X[1] = add(b, d);
        X[3] = sub(b, d);
    } else {
        constexpr int R = (N % 4 == 0) ? 4 : ((N % 2 == 0) ? 2 : 3);
        constexpr int M = N / R;
        Cf A[R][M];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            Cf s[M];
#pragma unroll
            for (int m = 0; m < M; ++m) s[m] = x[R * m + r];
            dft<M, DIR>(s, A[r]);
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {
            Cf u[R], U[R];
#pragma unroll
            for (int r = 0; r < R; ++r) u[r] = twid<N, DIR>(A[r][k], r * k);
            dft<R, DIR>(u, U);
#pragma unroll
            for (int q = 0; q < R; ++q) X[k + M * q] = U[q];
        }
    }
}

// Zero-padded input (forward passes, x[n] = 0 for n >= N / 2): the first
// layer of a decimation in frequency needs no butterflies,
// X[2k] = DFT_{N/2}(x)[k], X[2k + 1] = DFT_{N/2}(x w_N^n)[k].
template <int N, int DIR>
__device__ __forceinline__ void dft_half_in(const Cf (&x)[N], Cf (&X)[N]) {
    constexpr int H = N / 2;
    Cf a[H], b[H], A[H], B[H];
#pragma unroll
    for (int n = 0; n < H; ++n) {
        a[n] = x[n];
        b[n] = twid<N, DIR>(x[n], n);
    }
    dft<H, DIR>(a, A);
    dft<H, DIR>(b, B);
#pragma unroll
    for (int k = 0; k < H; ++k) {
        X[2 * k] = A[k];
        X[2 * k + 1] = B[k];
    }
}

// Cropped output (inverse passes, only X[k] for k < N / 2 are kept): the last
// layer of a decimation in time computes its first half only,
// X[k] = DFT_{N/2}(x[2m])[k] + w_N^k DFT_{N/2}(x[2m + 1])[k].
template <int N, int DIR>
__device__ __forceinline__ void dft_half_out(const Cf (&x)[N], Cf (&X)[N]) {
    constexpr int H = N / 2;
    Cf a[H], b[H], A[H], B[H];
#pragma unroll
    for (int m = 0; m < H; ++m) {
        a[m] = x[2 * m];
        b[m] = x[2 * m + 1];
    }
    dft<H, DIR>(a, A);
    dft<H, DIR>(b, B);
#pragma unroll
    for (int k = 0; k < H; ++k) X[k] = add(A[k], twid<N, DIR>(B[k], k));
}

// (line in block, t) of thread tid: lg < 0 lines fastest; lg = 0, 1, 2
// groups of 2^lg lines fastest, then t, then the groups
template <int T, int L>
__device__ __forceinline__ void line_thread(int tid, int lg, int &li, int &t) {
    constexpr int lgT = __builtin_ctz(T);
    if (lg < 0) {
        li = tid & (L - 1);
        t = tid / L;
    } else {
        t = (tid >> lg) & (T - 1);
        li = ((tid >> (lg + lgT)) << lg) | (tid & ((1 << lg) - 1));
    }
}

constexpr int kNumXcd = 8;
// blocks of one XCD get a contiguous range of tiles (consecutive blocks are
// dispatched round-robin over the 8 XCDs, each with its own L2)
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b % kNumXcd, i = b / kNumXcd;
    const int q = n / kNumXcd, r = n % kNumXcd;
    return x * q + min(x, r) + i;
}

template <int FMT>
__device__ __forceinline__ uint32_t half2_bits(Cf v, float s) {
    if constexpr (FMT == RING_F16) {
        const __half2 h = __halves2half2(__float2half_rn(v.x * s), __float2half_rn(v.y * s));
        uint32_t u;
        __builtin_memcpy(&u, &h, 4);
        return u;
    } else {
        __hip_bfloat162 h;
        h.x = __float2bfloat16(v.x * s);
        h.y = __float2bfloat16(v.y * s);
        uint32_t u;
        __builtin_memcpy(&u, &h, 4);
        return u;
    }
}

// 16-bit integer pair (re low, im high) of a value already scaled to
// [-32767, 32767] (rounded to nearest, clamped)
__device__ __forceinline__ uint32_t i16_bits(float re, float im) {
    const int a = int(rintf(fminf(fmaxf(re, -32767.f), 32767.f)));
    const int b = int(rintf(fminf(fmaxf(im, -32767.f), 32767.f)));
    return (uint32_t(a) & 0xffffu) | (uint32_t(b) << 16);
}

constexpr int kRsrcWord3 = 0x00020000;   // gfx9-family buffer descriptor word 3
constexpr uint32_t kOutOfRange = 0x80000000u;   // beyond every input: the load returns 0

// Per-pass constants the launcher derives from the LinePass.
struct RegArgs {
    int lg_in, lg_out;     // thread orders of the loads and stores (line_thread)
    int in_bytes;          // extent of one job's input (buffer loads, bounds-checked)
};

// Lags m = 0 .. add_lags - 1 of a target's own sources, added to the
// accumulated spectrum values of one x-line (frequencies k = yz P + x of
// component c, x = t + T n) as the inverse x pass reads them: the terms the
// separate additions of a blocked step would add (Eq. "retardation space-time
// sampled lorentz four vector potential": lag m reads the sources of step
// l - m).  Storage is tile-major, so a line of a length that does not divide
// the tile may continue in the next tile (x >= xb).
template <int P, int T, int AF>
__device__ __forceinline__ void add_own_lags(const LineJob &job, int yz, int c, int t, Cf (&v)[P / T]) {
    constexpr int E = P / T;
    constexpr bool ONE_TILE = (kTile % P) == 0;
    const uint32_t kk0 = uint32_t(yz) * uint32_t(P);
    const int64_t tile0 = kk0 / kTile;
    const int off0 = int(kk0 % kTile);
    const int xb = kTile - off0;   // first x of the line in the next tile
    const int64_t w = job.add_w, depth = job.add_depth;
    // the self pair's spectra are real: rows of kTile floats at the start of
    // each row's place (2 kTile floats apart)
    const float *spec = reinterpret_cast<const float *>(job.add_spec);
    int slot = *job.add_head;
    for (int m = 0; m < job.add_lags; ++m) {
        const float *g0 = spec + (tile0 * w + m) * (2 * kTile) + off0 + t;
        const float *g1 = spec + ((tile0 + 1) * w + m) * (2 * kTile) + (off0 - kTile) + t;
        const int64_t row0 = (tile0 * depth + slot) * (4 * kTile), row1 = ((tile0 + 1) * depth + slot) * (4 * kTile);
        if constexpr (AF == RING_F32) {
            // rows [c/2][k][c%2] of complex FP32 values
            const Cf *ring = reinterpret_cast<const Cf *>(job.add_ring) + (c >> 1) * (2 * kTile) + (c & 1);
            const Cf *r0 = ring + row0 + 2 * (off0 + t), *r1 = ring + row1 + 2 * (off0 - kTile + t);
#pragma unroll
            for (int n = 0; n < E; ++n) {
                const bool hi = !ONE_TILE && t + T * n >= xb;
                const float g = (hi ? g1 : g0)[T * n];
                const Cf r = (hi ? r1 : r0)[2 * T * n];
                v[n] = Cf{v[n].x + g * r.x, v[n].y + g * r.y};
            }
        } else {
            // rows [k][c] of 4-byte values: FP16 / BF16 pairs times the
            // snapshot's scale, or 16-bit integers times the tile's scale
            const uint32_t *ring = reinterpret_cast<const uint32_t *>(job.add_ring) + c;
            const uint32_t *r0 = ring + row0 + 4 * (off0 + t), *r1 = ring + row1 + 4 * (off0 - kTile + t);
            float s0, s1;
            if constexpr (AF == RING_I16) {
                s0 = job.add_scales[(tile0 * depth + slot) * 4 + c];
                s1 = (!ONE_TILE && xb < P) ? job.add_scales[((tile0 + 1) * depth + slot) * 4 + c] : 0.f;
            } else {
                s0 = s1 = job.add_scales[int64_t(slot) * 4 + c];
            }
#pragma unroll
            for (int n = 0; n < E; ++n) {
                const bool hi = !ONE_TILE && t + T * n >= xb;
                const float g = (hi ? g1 : g0)[T * n];
                const uint32_t u = (hi ? r1 : r0)[4 * T * n];
                const float s = hi ? s1 : s0;
                Cf r;
                if constexpr (AF == RING_F16) {
                    __half2 h;
                    __builtin_memcpy(&h, &u, 4);
                    const float2 f = __half22float2(h);
                    r = Cf{f.x * s, f.y * s};
                } else if constexpr (AF == RING_BF16) {
                    r = Cf{__uint_as_float(u << 16) * s, __uint_as_float(u & 0xffff0000u) * s};
                } else {
                    r = Cf{float(int(u << 16) >> 16) * s, float(int(u) >> 16) * s};
                }
                v[n] = Cf{v[n].x + g * r.x, v[n].y + g * r.y};
            }
        }
        slot = slot == 0 ? int(depth) - 1 : slot - 1;
    }
}

// One pass over a.lines lines of length P (T threads per line, L = 256 / T
// lines per block).  FMT: output format (FP32 complex, or scaled FP16/BF16
// ring rows).  DIR: sign of the exponent.  HALF: the pass's zero padding
// (forward: n_in <= P / 2) or crop (inverse: n_out <= P / 2) is pruned from
// the DFTs at compile time.  AF != 0 (inverse x pass of a blocked lag-sum
// step): the step's own-source lags are added to the input (add_own_lags).
template <int P, int T, int FMT, int DIR, bool HALF, int AF = 0>
__global__ __launch_bounds__(256) void k_line_reg(LinePass a, RegArgs ra) {
    constexpr int E = P / T;
    constexpr int L = 256 / T;
    // odd LDS row stride; P + 3 rather than P + 1 spreads the exchange writes
    // of lines grouped by four (the inverse x pass: the four components of a
    // frequency on neighbouring lanes) over twice as many banks (length 96:
    // 1.5 instead of 4.4 conflict cycles per LDS instruction), at the same
    // blocks per CU
    constexpr int RS = P + 3;
    constexpr bool HALF_IN = HALF && DIR < 0, HALF_OUT = HALF && DIR > 0;
    static_assert(E % T == 0 && L % 4 == 0 && E % 2 == 0 && T % 2 == 0, "line split P = T x E");
    __shared__ Cf buf[L * RS];
    __shared__ Cf twl[P];
    const LineJob &job = a.jobs[blockIdx.y];
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += 256) twl[i] = reinterpret_cast<const Cf *>(a.tw)[i];
    const int line0 = xcd_tile(int(blockIdx.x), int(gridDim.x)) * L;

    // stage 1: loads, E-point DFT, twiddles, into LDS as row[k1 T + t]
    {
        int li, t;
        line_thread<T, L>(tid, ra.lg_in, li, t);
        const int line = line0 + li;
        // element j = t + T n of the line sits at byte offset lane_off + n step;
        // loads past n_in (or of a line past the last) read 0 by the bounds check
        int nv = 0;
        uint32_t lane_off = 0;
        if (line < a.lines) {
            const int outer = a.dinner.div(line);
            const int inner = line - outer * a.n_inner;
            lane_off = uint32_t((outer * a.in_outer + inner * a.in_inner + int64_t(t) * a.in_j) * 8);
            nv = (a.n_in - t + T - 1) / T;
        }
        const uint32_t step = uint32_t(int64_t(T) * a.in_j * 8);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(job.in), (short)0, ra.in_bytes, kRsrcWord3);
        constexpr int NL = HALF_IN ? E / 2 : E;
        Cf v[E];
#pragma unroll
        for (int n = 0; n < NL; ++n) {
            const uint32_t off = n < nv ? lane_off + uint32_t(n) * step : kOutOfRange;
            // the whole 8-byte value is reinterpreted at once (no per-element
            // casts of the vector)
            v[n] = __builtin_bit_cast(Cf, __builtin_amdgcn_raw_buffer_load_b64(rs, int(off), 0, 0));
        }
#pragma unroll
        for (int n = NL; n < E; ++n) v[n] = Cf{0.f, 0.f};
        if constexpr (AF != 0) {
            if (line < a.lines && job.add_lags > 0) add_own_lags<P, T, AF>(job, line >> 2, line & 3, t, v);
        }
        Cf X[E];
        if constexpr (HALF_IN) dft_half_in<E, DIR>(v, X);
        else dft<E, DIR>(v, X);
        __syncthreads();   // twiddle table
        Cf *row = buf + li * RS;
        row[t] = X[0];
#pragma unroll
        for (int k1 = 1; k1 < E; ++k1) {
            Cf w = twl[t * k1];
            if (DIR > 0) w.y = -w.y;
            row[k1 * T + t] = Cf{X[k1].x * w.x - X[k1].y * w.y, X[k1].x * w.y + X[k1].y * w.x};
        }
    }
    __syncthreads();

    // stage 2: E / T DFTs of T points per thread, stores
    int li, t;
    line_thread<T, L>(tid, ra.lg_out, li, t);
    const int line = line0 + li;
    const bool live = line < a.lines;
    const int outer = live ? a.dinner.div(line) : 0;
    const int inner = live ? line - outer * a.n_inner : 0;
    char *obase = reinterpret_cast<char *>(job.out);
    const float *qs = job.qscale;
    constexpr int esz = (FMT == RING_F32) ? 8 : 4;
    int32_t slot = 0;
    if (job.head) {
        slot = *job.head;
        obase += int64_t(slot) * job.slot_stride * esz;
        if (qs && FMT != RING_I16) qs += int64_t(slot) * 4;
    }
    float iq = 1.0f;
    if (FMT == RING_F16 || FMT == RING_BF16)
        if (live) iq = 1.0f / qs[inner & 3];   // scales are powers of two: exact
    const int64_t lbase = outer * a.out_outer + inner * a.out_inner;
    // tiled output of a length that divides the tile: the whole line is one
    // run of one ring row, out_j = 4 (four components per frequency)
    constexpr bool LINE_IN_TILE = (kTile % P) == 0;
    char *lrow = nullptr;
    if (LINE_IN_TILE && job.tile_stride) {
        const uint32_t kk0 = uint32_t(lbase) >> 2, c = uint32_t(lbase) & 3u, kt0 = kk0 % kTile;
        const int64_t w0 = (FMT == RING_F32) ? int64_t((c >> 1) * (2 * kTile) + kt0 * 2 + (c & 1u)) : int64_t(kt0 * 4 + c);
        lrow = obase + (int64_t(kk0 / kTile) * job.tile_stride + w0) * esz;
    }
    constexpr int kstep = (FMT == RING_F32) ? 2 : 4;   // ring-row elements between frequencies
    const Cf *row = buf + li * RS;
    constexpr int NO = HALF_OUT ? T / 2 : T;
    Cf Zs[E / T][NO];
#pragma unroll
    for (int i = 0; i < E / T; ++i) {
        const int k1 = t + T * i;
        Cf z[T], Z[T];
#pragma unroll
        for (int s = 0; s < T; ++s) z[s] = row[k1 * T + s];
        if constexpr (HALF_OUT) dft_half_out<T, DIR>(z, Z);
        else dft<T, DIR>(z, Z);
#pragma unroll
        for (int k2 = 0; k2 < NO; ++k2) Zs[i][k2] = Z[k2];
    }

    if constexpr (FMT == RING_I16) {
        // Block floating point, fused: a block's lines (L / 4 x-lines of four
        // components, the spectrum's x-fastest order) cover whole tiles of kTile
        // frequencies, so the largest |Re|, |Im| per (tile, component) is
        // reduced here, in LDS; then each value is scaled to 16 bits and
        // written, and each (tile, component) scale once.
        constexpr int NT = (L / 4) * P / kTile;
        static_assert((L / 4) * P % kTile == 0, "a block must cover whole tiles");
        __shared__ uint32_t tmax[NT][4];
        const uint32_t kk0 = uint32_t(lbase) >> 2, c = uint32_t(lbase) & 3u;
        const int tb = int(uint32_t(line0 / 4) * uint32_t(P) / kTile);   // the block's first tile
        const int off = int(kk0 % kTile);                                 // the line's first frequency in its tile
        const int tl0 = int(kk0 / kTile) - tb;                            // the line's first tile in the block
        float m0 = 0.f, m1 = 0.f;
#pragma unroll
        for (int i = 0; i < E / T; ++i)
#pragma unroll
            for (int k2 = 0; k2 < NO; ++k2) {
                const int k = t + T * i + E * k2;
                const float v = fmaxf(fabsf(Zs[i][k2].x), fabsf(Zs[i][k2].y));
                if (off + k < kTile) m0 = fmaxf(m0, v);
                else m1 = fmaxf(m1, v);
            }
        // the table is cleared before any thread adds to it
        if (tid < NT * 4) tmax[tid >> 2][tid & 3] = 0u;
        __syncthreads();
        if (live) {
            // non-negative floats order like their bit patterns
            atomicMax(&tmax[tl0][c], __float_as_uint(m0));
            if (tl0 + 1 < NT && m1 > 0.f) atomicMax(&tmax[tl0 + 1][c], __float_as_uint(m1));
        }
        __syncthreads();
        const int64_t depth = job.tile_stride / (int64_t(kTile) * 4);
        if (tid < NT * 4) {
            const int tg = tb + (tid >> 2);
            if (int64_t(tg) * kTile < int64_t(a.lines / 4) * P)
                job.qscale[(int64_t(tg) * depth + slot) * 4 + (tid & 3)] = __uint_as_float(tmax[tid >> 2][tid & 3]) / 32767.f;
        }
        if (!live) return;
        const float mx0 = __uint_as_float(tmax[tl0][c]);
        const float mx1 = tl0 + 1 < NT ? __uint_as_float(tmax[tl0 + 1][c]) : 0.f;
        const float inv0 = mx0 > 0.f ? 32767.f / mx0 : 0.f, inv1 = mx1 > 0.f ? 32767.f / mx1 : 0.f;
#pragma unroll
        for (int i = 0; i < E / T; ++i)
#pragma unroll
            for (int k2 = 0; k2 < NO; ++k2) {
                const int k = t + T * i + E * k2;
                if (k >= a.n_out) continue;
                const float s = off + k < kTile ? inv0 : inv1;
                const uint32_t bits = i16_bits(Zs[i][k2].x * s, Zs[i][k2].y * s);
                if (LINE_IN_TILE) {
                    reinterpret_cast<uint32_t *>(lrow)[int64_t(k) * kstep] = bits;
                } else {
                    const uint32_t kk = kk0 + uint32_t(k), kt = kk % kTile;
                    reinterpret_cast<uint32_t *>(obase)[int64_t(kk / kTile) * job.tile_stride + kt * 4 + c] = bits;
                }
            }
        return;
    }

    if (!live) return;
#pragma unroll
    for (int i = 0; i < E / T; ++i) {
        const int k1 = t + T * i;
#pragma unroll
        for (int k2 = 0; k2 < NO; ++k2) {
            const int k = k1 + E * k2;
            if (k >= a.n_out) continue;
            if (LINE_IN_TILE && job.tile_stride) {
                if constexpr (FMT == RING_F32) reinterpret_cast<Cf *>(lrow)[int64_t(k) * kstep] = Zs[i][k2];
                else reinterpret_cast<uint32_t *>(lrow)[int64_t(k) * kstep] = half2_bits<FMT>(Zs[i][k2], iq);
                continue;
            }
            int64_t idx = lbase + int64_t(k) * a.out_j;
            if (job.tile_stride) {
                // ring rows of kTile frequencies x 4 components: [c/2][k][c%2]
                // (FP32) or [k][c] (FP16/BF16); one job's indices stay below 2^31
                const uint32_t u = uint32_t(idx);
                const uint32_t kk = u >> 2, c = u & 3u, kt = kk % kTile;
                const uint32_t w = (FMT == RING_F32) ? (c >> 1) * (2 * kTile) + kt * 2 + (c & 1u) : kt * 4 + c;
                idx = int64_t(kk / kTile) * job.tile_stride + int64_t(w);
            }
            if constexpr (FMT == RING_F32) reinterpret_cast<Cf *>(obase)[idx] = Zs[i][k2];
            else reinterpret_cast<uint32_t *>(obase)[idx] = half2_bits<FMT>(Zs[i][k2], iq);
        }
    }
}

template <int P, int T, int FMT, bool HALF>
void launch_reg_dir(const LinePass &a, const RegArgs &ra, dim3 grid, hipStream_t st) {
    if (a.dir > 0) hipLaunchKernelGGL((k_line_reg<P, T, FMT, +1, HALF>), grid, dim3(256), 0, st, a, ra);
    else hipLaunchKernelGGL((k_line_reg<P, T, FMT, -1, HALF>), grid, dim3(256), 0, st, a, ra);
}

template <int P, int T, int AF>
void launch_reg_add(const LinePass &a, const RegArgs &ra, dim3 grid, hipStream_t st) {
    if (2 * a.n_out <= P) hipLaunchKernelGGL((k_line_reg<P, T, RING_F32, +1, true, AF>), grid, dim3(256), 0, st, a, ra);
    else hipLaunchKernelGGL((k_line_reg<P, T, RING_F32, +1, false, AF>), grid, dim3(256), 0, st, a, ra);
}

template <int P, int T>
void launch_reg_fmt(const LinePass &a, const RegArgs &ra, hipStream_t st) {
    constexpr int L = 256 / T;
    const dim3 grid((a.lines + L - 1) / L, a.n_jobs);
    const bool half = a.dir < 0 ? 2 * a.n_in <= P : 2 * a.n_out <= P;
    if (a.add_fmt != 0) {
        switch (a.add_fmt) {
        case RING_F16: launch_reg_add<P, T, RING_F16>(a, ra, grid, st); break;
        case RING_BF16: launch_reg_add<P, T, RING_BF16>(a, ra, grid, st); break;
        case RING_I16: launch_reg_add<P, T, RING_I16>(a, ra, grid, st); break;
        default: launch_reg_add<P, T, RING_F32>(a, ra, grid, st);
        }
        return;
    }
    switch (a.out_fmt) {
    case RING_F16:
        if (half) launch_reg_dir<P, T, RING_F16, true>(a, ra, grid, st);
        else launch_reg_dir<P, T, RING_F16, false>(a, ra, grid, st);
        break;
    case RING_BF16:
        if (half) launch_reg_dir<P, T, RING_BF16, true>(a, ra, grid, st);
        else launch_reg_dir<P, T, RING_BF16, false>(a, ra, grid, st);
        break;
    case RING_I16:
        if (half) launch_reg_dir<P, T, RING_I16, true>(a, ra, grid, st);
        else launch_reg_dir<P, T, RING_I16, false>(a, ra, grid, st);
        break;
    default:
        if (half) launch_reg_dir<P, T, RING_F32, true>(a, ra, grid, st);
        else launch_reg_dir<P, T, RING_F32, false>(a, ra, grid, st);
    }
}

// byte extent of one job's input: the largest element index + 1
int64_t input_extent(const LinePass &a) {
    const int64_t n_outer = (a.lines + a.n_inner - 1) / a.n_inner;
    return ((n_outer - 1) * a.in_outer + int64_t(a.n_inner - 1) * a.in_inner + int64_t(a.n_in - 1) * a.in_j + 1) * 8;
}

// ---------------------------------------------------------------------------
// z passes in registers.  A complex line c = pair * 4 + mu carries grid
// positions a = 2 pair (real part) and b = a + 1 (imaginary part) of
// component mu; the two real lines sit next to each other in memory, so a
// line's Nz + Nz real values are one contiguous run.  Loads and stores move
// those runs in 16-byte vectors (Nz a multiple of 4 T): vector j of thread t
// holds z = 4 (t + T j) .. + 3, so each load instruction of a line's T threads
// reads 16 T contiguous bytes.  The transform itself is the line passes'
// two-stage split, with LDS rows between the contiguous and the strided
// orders and for the real-to-complex unpack, which pairs k with P - k.

// Forward: dS = S - S0 (and a copy of S into a real-space ring), R2C along z,
// output [Nx][Ny][Hz][4].
template <int P, int T>
__global__ __launch_bounds__(256) void k_zfwd_reg(ZFwd a) {
    constexpr int E = P / T, L = 256 / T, RS = P + 1, HZ = P / 2 + 1;
    __shared__ Cf buf[L * RS];
    __shared__ Cf twl[P];
    const ZFwdJob &job = a.jobs[blockIdx.y];
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += 256) twl[i] = reinterpret_cast<const Cf *>(a.tw)[i];
    const int line0 = blockIdx.x * L;
    const int npos = a.Nx * a.Ny, Nz = a.Nz;
    const int nlines = 4 * ((npos + 1) / 2);
    const int64_t npts = int64_t(npos) * Nz;
    // contiguous loads: vector j of thread t of line li covers z = 4 (t + T j) .. + 3
    {
        const int t = tid & (T - 1), li = tid / T, c = line0 + li;
        Cf *row = buf + li * RS;
        if (c < nlines) {
            const int mu = c & 3, pa = (c >> 2) * 2;
            const bool hb = pa + 1 < npos;
            const float *S = reinterpret_cast<const float *>(job.src);
            if (job.src_head) {
                int h = (*job.src_head - job.src_lag) % job.src_depth;
                if (h < 0) h += job.src_depth;
                S += int64_t(h) * 4 * npts;
            }
            const float *S0 = reinterpret_cast<const float *>(job.s0);
            float *St = nullptr;
            if (job.store)
                St = reinterpret_cast<float *>(job.store) + (job.store_head ? int64_t(*job.store_head) * 4 * npts : 0);
            const int64_t oa = mu * npts + int64_t(pa) * Nz;
            for (int q = 4 * t; q < Nz; q += 4 * T) {
                const float4 sa = *reinterpret_cast<const float4 *>(S + oa + q);
                const float4 sb = hb ? *reinterpret_cast<const float4 *>(S + oa + Nz + q) : float4{0.f, 0.f, 0.f, 0.f};
                float4 qa = {0.f, 0.f, 0.f, 0.f}, qb = {0.f, 0.f, 0.f, 0.f};
                if (S0) {
                    qa = *reinterpret_cast<const float4 *>(S0 + oa + q);
                    if (hb) qb = *reinterpret_cast<const float4 *>(S0 + oa + Nz + q);
                }
                if (St) {
                    *reinterpret_cast<float4 *>(St + oa + q) = sa;
                    if (hb) *reinterpret_cast<float4 *>(St + oa + Nz + q) = sb;
                }
                const int z = q;
                row[z + 0] = Cf{sa.x - qa.x, sb.x - qb.x};
                row[z + 1] = Cf{sa.y - qa.y, sb.y - qb.y};
                row[z + 2] = Cf{sa.z - qa.z, sb.z - qb.z};
                row[z + 3] = Cf{sa.w - qa.w, sb.w - qb.w};
            }
        } else {
            for (int z = t; z < Nz; z += T) row[z] = Cf{0.f, 0.f};
        }
        // zero padding up to P / 2 (the strided read takes n < E / 2)
        for (int z = Nz + t; z < P / 2; z += T) row[z] = Cf{0.f, 0.f};
    }
    __syncthreads();
    const int t = tid & (T - 1), li = tid / T;
    Cf *row = buf + li * RS;
    {
        Cf v[E], X[E];
#pragma unroll
        for (int n = 0; n < E / 2; ++n) v[n] = row[t + T * n];
#pragma unroll
        for (int n = E / 2; n < E; ++n) v[n] = Cf{0.f, 0.f};
        dft_half_in<E, -1>(v, X);
        __syncthreads();
        row[t] = X[0];
#pragma unroll
        for (int k1 = 1; k1 < E; ++k1) {
            const Cf w = twl[t * k1];
            row[k1 * T + t] = Cf{X[k1].x * w.x - X[k1].y * w.y, X[k1].x * w.y + X[k1].y * w.x};
        }
    }
    __syncthreads();
    {
        Cf Zs[E / T][T];
#pragma unroll
        for (int i = 0; i < E / T; ++i) {
            const int k1 = t + T * i;
            Cf z[T];
#pragma unroll
            for (int s = 0; s < T; ++s) z[s] = row[k1 * T + s];
            dft<T, -1>(z, Zs[i]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E / T; ++i)
#pragma unroll
            for (int k2 = 0; k2 < T; ++k2) row[t + T * i + E * k2] = Zs[i][k2];
    }
    __syncthreads();
    // unpack: X_a(k) = (Z_k + conj Z_-k) / 2, X_b(k) = (Z_k - conj Z_-k) / (2i)
    Cf *__restrict__ out = reinterpret_cast<Cf *>(job.out);
    const int nl = min(L, nlines - line0);
    const int pos0 = (line0 >> 2) * 2;
    const int np = min(2 * ((nl + 3) >> 2), npos - pos0);
    for (int e = tid; e < np * HZ * 4; e += 256) {
        const int mu = e & 3;
        const int pl = (e >> 2) / HZ;
        const int k = (e >> 2) - pl * HZ;
        const int lq = (pl >> 1) * 4 + mu;
        const Cf zk = buf[lq * RS + k];
        const Cf zm = buf[lq * RS + (k == 0 ? 0 : P - k)];
        Cf r;
        if ((pl & 1) == 0) r = {0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
        else r = {0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x)};
        out[(int64_t(pos0 + pl) * HZ + k) * 4 + mu] = r;
    }
}

// Inverse: C2R along z of [Nx][Ny][Hz][4], crop to z < Nz, + add, output
// out[mu][x][y][z].
template <int P, int T>
__global__ __launch_bounds__(256) void k_zinv_reg(ZInv a) {
    constexpr int E = P / T, L = 256 / T, RS = P + 1, HZ = P / 2 + 1;
    __shared__ Cf buf[L * RS];
    __shared__ Cf twl[P];
    const ZInvJob &job = a.jobs[blockIdx.y];
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += 256) twl[i] = reinterpret_cast<const Cf *>(a.tw)[i];
    const int line0 = blockIdx.x * L;
    const int npos = a.Nx * a.Ny, Nz = a.Nz;
    const int nlines = 4 * ((npos + 1) / 2);
    const int64_t npts = int64_t(npos) * Nz;
    const int nl = min(L, nlines - line0);
    const int pos0 = (line0 >> 2) * 2;
    const Cf *__restrict__ in = reinterpret_cast<const Cf *>(job.in);
    // Z_k = X_a(k) + i X_b(k), Z_{P-k} = conj X_a(k) + i conj X_b(k); lines
    // past the last read zeros
    for (int e = tid; e < (L / 4) * HZ * 4; e += 256) {
        const int mu = e & 3;
        const int ppl = (e >> 2) / HZ;
        const int k = (e >> 2) - ppl * HZ;
        const int li = ppl * 4 + mu;
        const int pa = pos0 + 2 * ppl;
        Cf xa = {0.f, 0.f}, xb = {0.f, 0.f};
        if (li < nl) {
            xa = in[(int64_t(pa) * HZ + k) * 4 + mu];
            if (pa + 1 < npos) xb = in[(int64_t(pa + 1) * HZ + k) * 4 + mu];
        }
        if (k == 0 || 2 * k == P) {
            buf[li * RS + k] = Cf{xa.x, xb.x};
        } else {
            buf[li * RS + k] = Cf{xa.x - xb.y, xa.y + xb.x};
            buf[li * RS + (P - k)] = Cf{xa.x + xb.y, xb.x - xa.y};
        }
    }
    __syncthreads();
    const int t = tid & (T - 1), li = tid / T;
    Cf *row = buf + li * RS;
    {
        Cf v[E], X[E];
#pragma unroll
        for (int n = 0; n < E; ++n) v[n] = row[t + T * n];
        dft<E, +1>(v, X);
        __syncthreads();
        row[t] = X[0];
#pragma unroll
        for (int k1 = 1; k1 < E; ++k1) {
            const Cf w = twl[t * k1];
            row[k1 * T + t] = Cf{X[k1].x * w.x + X[k1].y * w.y, X[k1].y * w.x - X[k1].x * w.y};
        }
    }
    __syncthreads();
    {
        Cf Zs[E / T][T];
#pragma unroll
        for (int i = 0; i < E / T; ++i) {
            const int k1 = t + T * i;
            Cf z[T];
#pragma unroll
            for (int s = 0; s < T; ++s) z[s] = row[k1 * T + s];
            dft_half_out<T, +1>(z, Zs[i]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E / T; ++i)
#pragma unroll
            for (int k2 = 0; k2 < T / 2; ++k2) row[t + T * i + E * k2] = Zs[i][k2];
    }
    __syncthreads();
    // contiguous stores: vector j of thread t covers z = 4 (t + T j) .. + 3 of both positions
    const int c = line0 + li;
    if (c >= nlines) return;
    const int mu = c & 3, pa = (c >> 2) * 2;
    const bool hb = pa + 1 < npos;
    float *__restrict__ out = reinterpret_cast<float *>(job.out);
    const float *__restrict__ add = reinterpret_cast<const float *>(job.add);
    const int64_t oa = mu * npts + int64_t(pa) * Nz;
    for (int q = 4 * t; q < Nz; q += 4 * T) {
        const int z = q;
        const Cf v0 = row[z], v1 = row[z + 1], v2 = row[z + 2], v3 = row[z + 3];
        float4 ra = {v0.x, v1.x, v2.x, v3.x}, rb = {v0.y, v1.y, v2.y, v3.y};
        if (add) {
            const float4 da = *reinterpret_cast<const float4 *>(add + oa + q);
            ra = float4{ra.x + da.x, ra.y + da.y, ra.z + da.z, ra.w + da.w};
            if (hb) {
                const float4 db = *reinterpret_cast<const float4 *>(add + oa + Nz + q);
                rb = float4{rb.x + db.x, rb.y + db.y, rb.z + db.z, rb.w + db.w};
            }
        }
        *reinterpret_cast<float4 *>(out + oa + q) = ra;
        if (hb) *reinterpret_cast<float4 *>(out + oa + Nz + q) = rb;
    }
}

template <int P, int T>
void launch_zfwd_reg_p(const ZFwd &a, hipStream_t st) {
    const int nlines = 4 * ((a.Nx * a.Ny + 1) / 2);
    hipLaunchKernelGGL((k_zfwd_reg<P, T>), dim3((nlines + 256 / T - 1) / (256 / T), a.n_jobs), dim3(256), 0, st, a);
}
template <int P, int T>
void launch_zinv_reg_p(const ZInv &a, hipStream_t st) {
    const int nlines = 4 * ((a.Nx * a.Ny + 1) / 2);
    hipLaunchKernelGGL((k_zinv_reg<P, T>), dim3((nlines + 256 / T - 1) / (256 / T), a.n_jobs), dim3(256), 0, st, a);
}

// T threads per z line of length P (the line passes' split).  Lengths 48
// and 96 (E = 12, 24 points per thread) measured no faster than the staged
// pass (config 5: 80 / 74 us against 83 / 75 us per step), so they keep it.
int z_threads(int P) {
    switch (P) {
    case 32: return 4;
    case 64: case 128: case 192: return 8;
    case 256: return 16;
    default: return 0;
    }
}

// ---------------------------------------------------------------------------
// Plane passes: the z and y transforms of one x slice and one component in one
// block, so the z-transformed array between them never goes to HBM.  Forward:
// the Ny x Nz real sources dS = S - S0 of slice (x, mu) in, the P x Hz values
// of the y pass out ([Nx][P][Hz][4]).  Inverse: those values in, the cropped
// real potentials out.  Two neighbouring y rows form one complex z line (real
// and imaginary part; unpacked by pairing k with P - k).  Both transforms are
// the line passes' two-stage split.  One LDS buffer of Hz rows of P + 1 values
// holds, in turn, the z lines (one row per pair of y rows), the y lines (one
// row per z frequency, entries along y) and their exchanges.  The four
// components of a slice are consecutive tiles of one XCD, so the 8-byte
// accesses to the interleaved [..][4] array of the four blocks meet in its L2.
struct PlaneJob {
    const float *src;          // forward: S [4][Nx][Ny][Nz]; with src_head a ring of such arrays
    const float *s0;           // forward: S0 (or null)
    const int32_t *src_head;   // forward: read slot (*src_head - src_lag) mod src_depth
    float *store;              // forward: copy of S into slot *store_head of this ring (or null)
    const int32_t *store_head;
    int32_t src_depth, src_lag;
    Cf *yout;                  // forward: [Nx][P][Hz][4]
    float *zmax;               // forward: largest |Re|, |Im| of dS per (x, component), [Nx][4], or null
    const Cf *yin;             // inverse: [Nx][P][Hz][4]
    float *out;                // inverse: [4][Nx][Ny][Nz]
    const float *add;          // inverse: added to the output (same layout), or null
};

struct PlanePass {
    int Nx, Ny, Nz;
    const void *tw;            // exp(-2 pi i j / P), j < P
    int n_jobs;
    PlaneJob jobs[kMaxJobs];
};
static_assert(sizeof(PlanePass) <= 4096, "plane-pass kernel arguments above 4 KiB");

// Thread roles: the lanes of a wave take consecutive lines with one t (line
// fastest), so that with the odd row stride a wave's 8-byte LDS accesses fall
// in distinct banks in both stages of a transform (the t-fastest order puts
// lines 1 and t 1 on the same bank).  z lines: groups of 32 (at most P / 4 are
// used); y lines: groups of 256 / T, as many rounds as Hz needs.
template <int P, int T>
__global__ __launch_bounds__(256) void k_zy_fwd(PlanePass a) {
    constexpr int NT = 256, E = P / T, RS = P + 1, HZ = P / 2 + 1, LPI = NT / T, H = P / 2, ZL = 32;
    constexpr int NV = ((P / 4) * (H / 4) + NT - 1) / NT;   // (row pair, z quad) items per thread
    constexpr int NU = ((P / 4) * HZ + NT - 1) / NT;        // unpacked (row pair, kz) per thread
    static_assert(P / 4 <= ZL && ZL * T <= NT, "the z rows of a slice exceed one round of threads");
    __shared__ Cf buf[HZ * RS];
    __shared__ Cf twl[P];
    __shared__ float red[NT / 64];
    const PlaneJob &job = a.jobs[blockIdx.y];
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += NT) twl[i] = reinterpret_cast<const Cf *>(a.tw)[i];
    const int tile = xcd_tile(int(blockIdx.x), int(gridDim.x));
    const int x = tile >> 2, mu = tile & 3;
    const int Nx = a.Nx, Ny = a.Ny, Nz = a.Nz, NZL = (Ny + 1) / 2;
    const int64_t npts = int64_t(Nx) * Ny * Nz;
    const int64_t slab = (int64_t(mu) * Nx + x) * Ny * Nz;
    float mx = 0.f;   // largest |dS| of the slab (scaled 16-bit float rings)
    // dS = S - S0 of rows y = 2p (real parts) and 2p + 1 (imaginary parts)
    // into z row p, four z at a time (16-byte vectors, Nz % 4 == 0); a missing
    // odd last row reads as zeros
    {
        const float *S = job.src;
        if (job.src_head) {
            int h = (*job.src_head - job.src_lag) % job.src_depth;
            if (h < 0) h += job.src_depth;
            S += int64_t(h) * 4 * npts;
        }
        float *St = job.store ? job.store + (job.store_head ? int64_t(*job.store_head) * 4 * npts : 0) : nullptr;
        const float *S0 = job.s0;
        const int nzq = Nz / 4, nv = NZL * nzq;
        float4 va[NV], vb[NV], qa[NV], qb[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int e = tid + NT * j;
            va[j] = vb[j] = qa[j] = qb[j] = float4{0.f, 0.f, 0.f, 0.f};
            if (e < nv) {
                const int p = e / nzq;
                const int64_t o = slab + int64_t(2 * p) * Nz + 4 * (e - p * nzq);
                const bool hb = 2 * p + 1 < Ny;
                va[j] = *reinterpret_cast<const float4 *>(S + o);
                if (hb) vb[j] = *reinterpret_cast<const float4 *>(S + o + Nz);
                if (S0) {
                    qa[j] = *reinterpret_cast<const float4 *>(S0 + o);
                    if (hb) qb[j] = *reinterpret_cast<const float4 *>(S0 + o + Nz);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int e = tid + NT * j;
            if (e < nv) {
                const int p = e / nzq, z = 4 * (e - p * nzq);
                const int64_t o = slab + int64_t(2 * p) * Nz + z;
                if (St) {
                    *reinterpret_cast<float4 *>(St + o) = va[j];
                    if (2 * p + 1 < Ny) *reinterpret_cast<float4 *>(St + o + Nz) = vb[j];
                }
                Cf *r = buf + p * RS + z;
                const Cf d0 = {va[j].x - qa[j].x, vb[j].x - qb[j].x}, d1 = {va[j].y - qa[j].y, vb[j].y - qb[j].y};
                const Cf d2 = {va[j].z - qa[j].z, vb[j].z - qb[j].z}, d3 = {va[j].w - qa[j].w, vb[j].w - qb[j].w};
                r[0] = d0;
                r[1] = d1;
                r[2] = d2;
                r[3] = d3;
                mx = fmaxf(mx, fmaxf(fmaxf(fabsf(d0.x), fabsf(d0.y)), fmaxf(fabsf(d1.x), fabsf(d1.y))));
                mx = fmaxf(mx, fmaxf(fmaxf(fabsf(d2.x), fabsf(d2.y)), fmaxf(fabsf(d3.x), fabsf(d3.y))));
            }
        }
        if (job.zmax) {
            for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
            if ((tid & 63) == 0) red[tid >> 6] = mx;
        }
        // zeros: z in [Nz, P / 2) of every row
        const int nzero = H - Nz;
        for (int e = tid; e < NZL * nzero; e += NT) {
            const int p = e / nzero;
            buf[p * RS + Nz + e - p * nzero] = Cf{0.f, 0.f};
        }
    }
    __syncthreads();
    if (job.zmax && tid == 0) {
        float m = red[0];
        for (int w = 1; w < NT / 64; ++w) m = fmaxf(m, red[w]);
        job.zmax[x * 4 + mu] = m;
    }
    // z transforms (input z < P / 2), natural order back into the rows
    {
        const int li = tid % ZL, t = tid / ZL;
        const bool act = t < T && li < NZL;
        Cf *row = buf + li * RS;
        Cf X[E];
        if (act) {
            Cf v[E];
#pragma unroll
            for (int n = 0; n < E / 2; ++n) v[n] = row[t + T * n];
#pragma unroll
            for (int n = E / 2; n < E; ++n) v[n] = Cf{0.f, 0.f};
            dft_half_in<E, -1>(v, X);
        }
        __syncthreads();
        if (act) {
            row[t] = X[0];
#pragma unroll
            for (int k1 = 1; k1 < E; ++k1) {
                const Cf w = twl[t * k1];
                row[k1 * T + t] = Cf{X[k1].x * w.x - X[k1].y * w.y, X[k1].x * w.y + X[k1].y * w.x};
            }
        }
        __syncthreads();
        Cf Zs[E / T][T];
        if (act) {
#pragma unroll
            for (int i = 0; i < E / T; ++i) {
                const int k1 = t + T * i;
                Cf z[T];
#pragma unroll
                for (int s = 0; s < T; ++s) z[s] = row[k1 * T + s];
                dft<T, -1>(z, Zs[i]);
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < E / T; ++i)
#pragma unroll
                for (int k2 = 0; k2 < T; ++k2) row[t + T * i + E * k2] = Zs[i][k2];
        }
    }
    __syncthreads();
    // unpack X_a(k) = (Z_k + conj Z_-k) / 2, X_b(k) = (Z_k - conj Z_-k) / (2i)
    // into the y rows: row kz, entry y (zeros for Ny <= y < P / 2)
    {
        Cf ua[NU], ub[NU];
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const int e = tid + NT * j;
            const int p = e / HZ, k = e - p * HZ;
            ua[j] = ub[j] = Cf{0.f, 0.f};
            if (p < NZL) {
                const Cf zk = buf[p * RS + k], zm = buf[p * RS + (k == 0 ? 0 : P - k)];
                ua[j] = Cf{0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
                ub[j] = Cf{0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x)};
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const int e = tid + NT * j;
            const int p = e / HZ, k = e - p * HZ;
            if (p < NZL) {
                buf[k * RS + 2 * p] = ua[j];
                if (2 * p + 1 < Ny) buf[k * RS + 2 * p + 1] = ub[j];
            }
        }
        const int nzero = H - Ny;
        for (int e = tid; e < HZ * nzero; e += NT) {
            const int k = e / nzero;
            buf[k * RS + Ny + e - k * nzero] = Cf{0.f, 0.f};
        }
    }
    __syncthreads();
    // y transforms (input y < P / 2), stored from registers:
    // yout[x][k][kz][mu] for every k < P
    Cf *__restrict__ yo = job.yout + int64_t(x) * P * HZ * 4 + mu;
    for (int base = 0; base < HZ; base += LPI) {
        const int li = tid % LPI, t = tid / LPI, kz = base + li;
        const bool act = kz < HZ;
        Cf *row = buf + kz * RS;
        Cf X[E];
        if (act) {
            Cf v[E];
#pragma unroll
            for (int n = 0; n < E / 2; ++n) v[n] = row[t + T * n];
#pragma unroll
            for (int n = E / 2; n < E; ++n) v[n] = Cf{0.f, 0.f};
            dft_half_in<E, -1>(v, X);
        }
        __syncthreads();
        if (act) {
            row[t] = X[0];
#pragma unroll
            for (int k1 = 1; k1 < E; ++k1) {
                const Cf w = twl[t * k1];
                row[k1 * T + t] = Cf{X[k1].x * w.x - X[k1].y * w.y, X[k1].x * w.y + X[k1].y * w.x};
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < E / T; ++i) {
                const int k1 = t + T * i;
                Cf z[T], Z[T];
#pragma unroll
                for (int s = 0; s < T; ++s) z[s] = row[k1 * T + s];
                dft<T, -1>(z, Z);
#pragma unroll
                for (int k2 = 0; k2 < T; ++k2) yo[(int64_t(k1 + E * k2) * HZ + kz) * 4] = Z[k2];
            }
        }
    }
}

template <int P, int T>
__global__ __launch_bounds__(256) void k_yz_inv(PlanePass a) {
    constexpr int NT = 256, E = P / T, RS = P + 1, HZ = P / 2 + 1, LPI = NT / T, H = P / 2, ZL = 32;
    constexpr int NV = ((P / 4) * (H / 4) + NT - 1) / NT;
    constexpr int NU = ((P / 4) * HZ + NT - 1) / NT;
    static_assert(P / 4 <= ZL && ZL * T <= NT, "the z rows of a slice exceed one round of threads");
    __shared__ Cf buf[HZ * RS];
    __shared__ Cf twl[P];
    const PlaneJob &job = a.jobs[blockIdx.y];
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += NT) twl[i] = reinterpret_cast<const Cf *>(a.tw)[i];
    const int tile = xcd_tile(int(blockIdx.x), int(gridDim.x));
    const int x = tile >> 2, mu = tile & 3;
    const int Nx = a.Nx, Ny = a.Ny, Nz = a.Nz, NZL = (Ny + 1) / 2;
    __syncthreads();
    // y transforms of rows kz < Hz (all P inputs; outputs y < P / 2 back into the rows)
    const Cf *__restrict__ yi = job.yin + int64_t(x) * P * HZ * 4 + mu;
    for (int base = 0; base < HZ; base += LPI) {
        const int li = tid % LPI, t = tid / LPI, kz = base + li;
        const bool act = kz < HZ;
        Cf *row = buf + kz * RS;
        if (act) {
            Cf v[E], X[E];
#pragma unroll
            for (int n = 0; n < E; ++n) v[n] = yi[(int64_t(t + T * n) * HZ + kz) * 4];
            dft<E, +1>(v, X);
            row[t] = X[0];
#pragma unroll
            for (int k1 = 1; k1 < E; ++k1) {
                const Cf w = twl[t * k1];
                row[k1 * T + t] = Cf{X[k1].x * w.x + X[k1].y * w.y, X[k1].y * w.x - X[k1].x * w.y};
            }
        }
        __syncthreads();
        Cf Zs[E / T][T];
        if (act) {
#pragma unroll
            for (int i = 0; i < E / T; ++i) {
                const int k1 = t + T * i;
                Cf z[T];
#pragma unroll
                for (int s = 0; s < T; ++s) z[s] = row[k1 * T + s];
                dft_half_out<T, +1>(z, Zs[i]);
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < E / T; ++i)
#pragma unroll
                for (int k2 = 0; k2 < T / 2; ++k2) row[t + T * i + E * k2] = Zs[i][k2];
        }
    }
    __syncthreads();
    // z lines: Z_k = X_a(k) + i X_b(k), Z_{P-k} = conj X_a(k) + i conj X_b(k)
    // with a = y row 2p, b = 2p + 1 (zero past Ny)
    {
        Cf ua[NU], ub[NU];
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const int e = tid + NT * j;
            const int p = e / HZ, k = e - p * HZ;
            ua[j] = ub[j] = Cf{0.f, 0.f};
            if (p < NZL) {
                ua[j] = buf[k * RS + 2 * p];
                if (2 * p + 1 < Ny) ub[j] = buf[k * RS + 2 * p + 1];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const int e = tid + NT * j;
            const int p = e / HZ, k = e - p * HZ;
            if (p < NZL) {
                const Cf xa = ua[j], xb = ub[j];
                if (k == 0 || 2 * k == P) {
                    buf[p * RS + k] = Cf{xa.x, xb.x};
                } else {
                    buf[p * RS + k] = Cf{xa.x - xb.y, xa.y + xb.x};
                    buf[p * RS + (P - k)] = Cf{xa.x + xb.y, xb.x - xa.y};
                }
            }
        }
    }
    __syncthreads();
    // z transforms, outputs z < P / 2 back into the rows
    {
        const int li = tid % ZL, t = tid / ZL;
        const bool act = t < T && li < NZL;
        Cf *row = buf + li * RS;
        Cf X[E];
        if (act) {
            Cf v[E];
#pragma unroll
            for (int n = 0; n < E; ++n) v[n] = row[t + T * n];
            dft<E, +1>(v, X);
        }
        __syncthreads();
        if (act) {
            row[t] = X[0];
#pragma unroll
            for (int k1 = 1; k1 < E; ++k1) {
                const Cf w = twl[t * k1];
                row[k1 * T + t] = Cf{X[k1].x * w.x + X[k1].y * w.y, X[k1].y * w.x - X[k1].x * w.y};
            }
        }
        __syncthreads();
        Cf Zs[E / T][T];
        if (act) {
#pragma unroll
            for (int i = 0; i < E / T; ++i) {
                const int k1 = t + T * i;
                Cf z[T];
#pragma unroll
                for (int s = 0; s < T; ++s) z[s] = row[k1 * T + s];
                dft_half_out<T, +1>(z, Zs[i]);
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < E / T; ++i)
#pragma unroll
                for (int k2 = 0; k2 < T / 2; ++k2) row[t + T * i + E * k2] = Zs[i][k2];
        }
    }
    __syncthreads();
    // rows y = 2p (real parts) and 2p + 1 (imaginary parts) of z row p into
    // out[mu][x][y][z], four z at a time (+ add)
    {
        const int64_t slab = (int64_t(mu) * Nx + x) * Ny * Nz;
        const int nzq = Nz / 4, nv = NZL * nzq;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int e = tid + NT * j;
            if (e < nv) {
                const int p = e / nzq, z = 4 * (e - p * nzq);
                const int64_t o = slab + int64_t(2 * p) * Nz + z;
                const bool hb = 2 * p + 1 < Ny;
                const Cf *r = buf + p * RS + z;
                const Cf r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
                float4 va = {r0.x, r1.x, r2.x, r3.x}, vb = {r0.y, r1.y, r2.y, r3.y};
                if (job.add) {
                    const float4 da = *reinterpret_cast<const float4 *>(job.add + o);
                    va = float4{va.x + da.x, va.y + da.y, va.z + da.z, va.w + da.w};
                    if (hb) {
                        const float4 db = *reinterpret_cast<const float4 *>(job.add + o + Nz);
                        vb = float4{vb.x + db.x, vb.y + db.y, vb.z + db.z, vb.w + db.w};
                    }
                }
                *reinterpret_cast<float4 *>(job.out + o) = va;
                if (hb) *reinterpret_cast<float4 *>(job.out + o + Nz) = vb;
            }
        }
    }
}

// Threads per line of a plane pass (T * T divides P); 0: no plane pass
int plane_threads(int P) {
    switch (P) {
    case 32: case 48: case 96: return 4;
    case 64: case 128: return 8;
    default: return 0;
    }
}

template <int P>
void launch_plane(const PlanePass &pp, bool fwd, hipStream_t st) {
    constexpr int T = (P == 64 || P == 128) ? 8 : 4;
    const dim3 grid(4 * pp.Nx, pp.n_jobs);
    if (fwd) hipLaunchKernelGGL((k_zy_fwd<P, T>), grid, dim3(256), 0, st, pp);
    else hipLaunchKernelGGL((k_yz_inv<P, T>), grid, dim3(256), 0, st, pp);
}

void launch_plane_p(int P, const PlanePass &pp, bool fwd, hipStream_t st) {
    switch (P) {
    case 32: launch_plane<32>(pp, fwd, st); break;
    case 48: launch_plane<48>(pp, fwd, st); break;
    case 64: launch_plane<64>(pp, fwd, st); break;
    case 96: launch_plane<96>(pp, fwd, st); break;
    default: launch_plane<128>(pp, fwd, st); break;
    }
}

bool aligned16(const void *q) { return reinterpret_cast<uintptr_t>(q) % 16 == 0; }

}  // namespace

bool line_reg_supported(const LinePass &a) {
    if (!(a.out_fmt == RING_F32 || a.out_fmt == RING_F16 || a.out_fmt == RING_BF16 || a.out_fmt == RING_I16))
        return false;
    bool tiled = false, all_tiled = true, scaled = true;
    for (int j = 0; j < a.n_jobs; ++j) {
        tiled = tiled || a.jobs[j].tile_stride != 0;
        all_tiled = all_tiled && a.jobs[j].tile_stride != 0;
        scaled = scaled && a.jobs[j].qscale != nullptr;
    }
    if (tiled && (a.tile_comp != 4 || a.out_j != 4)) return false;
    if (a.out_fmt != RING_F32 && !(all_tiled && scaled)) return false;
    // the fused 16-bit quantisation reduces whole tiles in a block: the x
    // pass of a spectrum, lines (x-line, component), frequencies x fastest
    if (a.out_fmt == RING_I16 &&
        !(a.n_inner == 4 && a.out_inner == 1 && a.out_outer == int64_t(a.P) * 4 && a.n_out == a.P && a.dir < 0))
        return false;
    // fused lag additions: the inverse x pass of a spectrum [C][4]
    if (a.add_fmt != 0 &&
        !(a.dir > 0 && a.out_fmt == RING_F32 && !tiled && a.n_inner == 4 && a.in_inner == 1 && a.in_j == 4 &&
          a.in_outer == int64_t(a.P) * 4 && a.n_in == a.P &&
          (a.add_fmt == RING_F32 || a.add_fmt == RING_F16 || a.add_fmt == RING_BF16 || a.add_fmt == RING_I16)))
        return false;
    for (int g : {a.in_group, a.out_group})
        if (g != 0 && g != 1 && g != 2 && g != 4) return false;
    if (a.lines < 1 || a.n_in < 1 || a.lines % a.n_inner != 0) return false;
    if (a.in_j < 0 || a.in_inner < 0 || a.in_outer < 0) return false;
    if (input_extent(a) >= (int64_t(1) << 31)) return false;   // buffer loads with 32-bit offsets
    switch (a.P) {
    case 32: case 48: case 64: case 96: case 128: case 144: case 192: case 256: return true;
    default: return false;
    }
}

// FP32 z passes in registers: lengths 32, 64, 128, 192, 256, the real data at most half the
// padded line (Nz <= P / 2), Nz a multiple of 4 T (16-byte vectors), 16-byte
// aligned arrays, sources only (mode 0) and no per-block maxima (FP16/BF16
// rings keep the staged pass).  False (nothing launched) otherwise.
bool launch_zfwd_reg(const ZFwd &a, hipStream_t st) {
    const int T = z_threads(a.Pz);
    if (a.mode != 0 || T == 0 || 2 * a.Nz > a.Pz || a.Nz % (4 * T) != 0) return false;
    for (int j = 0; j < a.n_jobs; ++j) {
        const ZFwdJob &J = a.jobs[j];
        if (J.zmax) return false;
        for (const void *q : {J.src, J.s0, static_cast<const void *>(J.store)})
            if (reinterpret_cast<uintptr_t>(q) % 16) return false;
    }
    switch (a.Pz) {
    case 32: launch_zfwd_reg_p<32, 4>(a, st); break;
    case 64: launch_zfwd_reg_p<64, 8>(a, st); break;
    case 128: launch_zfwd_reg_p<128, 8>(a, st); break;
    case 192: launch_zfwd_reg_p<192, 8>(a, st); break;
    default: launch_zfwd_reg_p<256, 16>(a, st); break;
    }
    return true;
}

bool launch_zinv_reg(const ZInv &a, hipStream_t st) {
    const int T = z_threads(a.Pz);
    if (T == 0 || 2 * a.Nz > a.Pz || a.Nz % (4 * T) != 0) return false;
    for (int j = 0; j < a.n_jobs; ++j)
        for (const void *q : {static_cast<const void *>(a.jobs[j].out), a.jobs[j].add})
            if (reinterpret_cast<uintptr_t>(q) % 16) return false;
    switch (a.Pz) {
    case 32: launch_zinv_reg_p<32, 4>(a, st); break;
    case 64: launch_zinv_reg_p<64, 8>(a, st); break;
    case 128: launch_zinv_reg_p<128, 8>(a, st); break;
    case 192: launch_zinv_reg_p<192, 8>(a, st); break;
    default: launch_zinv_reg_p<256, 16>(a, st); break;
    }
    return true;
}

// FP32 line pass in registers; false (nothing launched) when the pass is not
// one this kernel covers (other lengths, FP64 output, one-component tiles,
// inputs above 2 GiB).
bool launch_line_reg(const LinePass &a0, hipStream_t st) {
    if (!line_reg_supported(a0)) return false;
    LinePass a = a0;
    a.dinner = FastDiv(uint32_t(a.n_inner));
    RegArgs ra{};
    ra.lg_in = a.in_group > 0 ? (a.in_group >> 1) : -1;
    ra.lg_out = a.out_group > 0 ? (a.out_group >> 1) : -1;
    ra.in_bytes = int(input_extent(a));
    switch (a.P) {
    case 32: launch_reg_fmt<32, 4>(a, ra, st); break;
    case 48: launch_reg_fmt<48, 4>(a, ra, st); break;
    case 64: launch_reg_fmt<64, 8>(a, ra, st); break;
    case 96: launch_reg_fmt<96, 4>(a, ra, st); break;
    case 144: launch_reg_fmt<144, 4>(a, ra, st); break;
    case 192: launch_reg_fmt<192, 8>(a, ra, st); break;
    case 128: launch_reg_fmt<128, 8>(a, ra, st); break;
    default: launch_reg_fmt<256, 16>(a, ra, st); break;
    }
    return true;
}

bool plane_shape(int Py, int Pz, int Ny, int Nz) {
    return Py == Pz && plane_threads(Pz) != 0 && Ny >= 1 && 2 * Ny <= Pz && Nz >= 4 && 2 * Nz <= Pz && Nz % 4 == 0;
}

// Forward z and y passes of the same jobs as one plane pass.  False (nothing
// launched) where it does not apply: other lengths, unequal z and y pads, Ny
// or Nz above P / 2, Nz not a multiple of 4, Green's functions, misaligned
// arrays, or a y pass of another layout than [Nx][Ny][Hz][4] -> [Nx][P][Hz][4].
// A job's zmax (scaled 16-bit float rings) receives one maximum per
// (x, component), Nx blocks of 4: the caller sizes it and the ring scales.
bool launch_zy_fwd_plane(const ZFwd &z, const LinePass &y, hipStream_t st) {
    const int P = z.Pz;
    if (z.mode != 0 || !plane_shape(z.Py, P, z.Ny, z.Nz) || y.P != P || z.Hz != P / 2 + 1 || z.Nx < 1) return false;
    const int64_t hz4 = int64_t(z.Hz) * 4;
    if (!(y.dir < 0 && y.n_in == z.Ny && y.n_out == P && y.lines == z.Nx * hz4 && y.n_inner == hz4 &&
          y.in_j == hz4 && y.in_inner == 1 && y.in_outer == z.Ny * hz4 && y.out_j == hz4 && y.out_inner == 1 &&
          y.out_outer == P * hz4 && y.out_fmt == RING_F32 && y.add_fmt == 0 && y.n_jobs == z.n_jobs))
        return false;
    PlanePass pp{};
    pp.Nx = z.Nx;
    pp.Ny = z.Ny;
    pp.Nz = z.Nz;
    pp.tw = z.tw;
    pp.n_jobs = z.n_jobs;
    for (int j = 0; j < z.n_jobs; ++j) {
        const ZFwdJob &J = z.jobs[j];
        const LineJob &Y = y.jobs[j];
        if (Y.in != J.out || Y.tile_stride != 0 || Y.head || Y.qscale) return false;
        if (!aligned16(J.src) || !aligned16(J.s0) || !aligned16(J.store) || reinterpret_cast<uintptr_t>(Y.out) % 8)
            return false;
        PlaneJob &Q = pp.jobs[j];
        Q.src = static_cast<const float *>(J.src);
        Q.s0 = static_cast<const float *>(J.s0);
        Q.src_head = J.src_head;
        Q.src_depth = J.src_depth;
        Q.src_lag = J.src_lag;
        Q.store = static_cast<float *>(J.store);
        Q.store_head = J.store_head;
        Q.yout = static_cast<Cf *>(Y.out);
        Q.zmax = J.zmax;
    }
    launch_plane_p(P, pp, true, st);
    return true;
}

// Inverse y and z passes of the same jobs as one plane pass; false (nothing
// launched) where it does not apply (as above, for a y pass
// [Nx][P][Hz][4] -> [Nx][Ny][Hz][4]).
bool launch_yz_inv_plane(const LinePass &y, const ZInv &zi, hipStream_t st) {
    const int P = zi.Pz;
    if (!plane_shape(y.P, P, zi.Ny, zi.Nz) || zi.Hz != P / 2 + 1 || zi.Nx < 1) return false;
    const int64_t hz4 = int64_t(zi.Hz) * 4;
    if (!(y.dir > 0 && y.n_in == P && y.n_out == zi.Ny && y.lines == zi.Nx * hz4 && y.n_inner == hz4 &&
          y.in_j == hz4 && y.in_inner == 1 && y.in_outer == P * hz4 && y.out_j == hz4 && y.out_inner == 1 &&
          y.out_outer == zi.Ny * hz4 && y.out_fmt == RING_F32 && y.add_fmt == 0 && y.n_jobs == zi.n_jobs))
        return false;
    PlanePass pp{};
    pp.Nx = zi.Nx;
    pp.Ny = zi.Ny;
    pp.Nz = zi.Nz;
    pp.tw = zi.tw;
    pp.n_jobs = zi.n_jobs;
    for (int j = 0; j < zi.n_jobs; ++j) {
        const ZInvJob &J = zi.jobs[j];
        const LineJob &Y = y.jobs[j];
        if (Y.out != J.in || Y.tile_stride != 0 || Y.head || Y.qscale) return false;
        if (!aligned16(J.out) || !aligned16(J.add) || reinterpret_cast<uintptr_t>(Y.in) % 8) return false;
        PlaneJob &Q = pp.jobs[j];
        Q.yin = static_cast<const Cf *>(Y.in);
        Q.out = static_cast<float *>(J.out);
        Q.add = static_cast<const float *>(J.add);
    }
    launch_plane_p(P, pp, false, st);
    return true;
}

}  // namespace rpot
