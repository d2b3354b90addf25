// Small fully connected network for the far-pair surrogate: training and
// inference kernels and their C-ABI (rp_mlp_*).
//
//   h1 = tanh(x W1 + b1),  h2 = tanh(h1 W2 + b2),  y = h2 W3 + b3 + x Ws
//   loss = sum (y - t)^2 / (2 B n_out)
//
// The linear skip x Ws carries the part of the map that is linear in the
// inputs; the two tanh layers learn the rest.  Parameters are one flat FP32
// vector [W1 (n_in x H), b1 (H), W2 (H x H), b2 (H), W3 (H x n_out),
// b3 (n_out), Ws (n_in x n_out)], row-major, in the bound workspace.
// Matrix products run in one LDS-tiled kernel on the FP32 matrix cores
// (128 x 128 output tile, 16-deep K slices, split along K when the product has
// few output tiles) with strided operands, so the transposed products of the
// backward pass need no copies.
#include "rpot.h"
#include "rpot_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

namespace rpot {

namespace {

constexpr int kMT = 128;      // output tile (rows and columns) of a block
constexpr int kKT = 16;       // K slice staged in LDS
constexpr int kLdsRow = kMT + 4;
constexpr int kMaxSplit = 32;   // K splits of a product with few output tiles
constexpr int kMinSplitK = 64;  // K columns per split at least
constexpr int kFillBlocks = 512;   // blocks a split product aims for (two per CU)

typedef float f32x16 __attribute__((ext_vector_type(16)));

struct GemmArgs {
    const float *A;        // A(i, k) = A[i * sa0 + k * sa1]
    const float *B;        // B(k, j) = B[k * sb0 + j * sb1]
    float *C;              // C(i, j) = C[i * ldc + j]
    const float *bias;     // + bias[j] (or null)
    int64_t sa0, sa1, sb0, sb1, ldc;
    int M, N, K;
    int act;               // 0 none, 1 tanh
    float beta;            // C = beta * C + A B
    int ks;                // split-K: K columns per split (blockIdx.z), 0 = no split
    float *part;           // split-K: raw partial products [split][M][N]
};

// C tile of 128 x 128 per block on the FP32 matrix cores: four waves, each a
// 64 x 64 quarter as 2 x 2 products of v_mfma_f32_32x32x2_f32 (FP32 inputs,
// FP32 accumulation).  K goes in slices of 16 through two LDS buffers; the
// next slice's global loads are issued before the current slice's products.
// A k-slice of the instruction: lane l supplies A(i0 + l % 32, k + l / 32) and
// B(k + l / 32, j0 + l % 32); accumulator register r of lane l holds
// C(i0 + 8 (r / 4) + 4 (l / 32) + r % 4, j0 + l % 32).
// The tile loads follow whichever operand stride is 1, so the transposed
// products of the backward pass read contiguous runs without copies.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ float As[2][kKT][kLdsRow];   // As[.][k][i]
    __shared__ float Bs[2][kKT][kLdsRow];   // Bs[.][k][j]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i0 = blockIdx.y * kMT, j0 = blockIdx.x * kMT;
    const int kb = g.ks ? int(blockIdx.z) * g.ks : 0;
    const int ke = g.ks ? min(g.K, kb + g.ks) : g.K;
    // per-thread tile coordinates of the 8 A and 8 B elements of a slice
    const bool a_kfast = (g.sa1 == 1), b_jfast = (g.sb1 == 1);
    const int a_i = a_kfast ? (tid >> 4) : (tid & 127), a_k = a_kfast ? (tid & 15) : (tid >> 7);
    const int a_di = a_kfast ? 16 : 0, a_dk = a_kfast ? 0 : 2;
    const int b_j = b_jfast ? (tid & 127) : (tid >> 4), b_k = b_jfast ? (tid >> 7) : (tid & 15);
    const int b_dj = b_jfast ? 0 : 16, b_dk = b_jfast ? 2 : 0;
    float ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + a_i + u * a_di, k = k0 + a_k + u * a_dk;
            ra[u] = (i < g.M && k < ke) ? g.A[int64_t(i) * g.sa0 + int64_t(k) * g.sa1] : 0.f;
            const int j = j0 + b_j + u * b_dj, kk = k0 + b_k + u * b_dk;
            rb[u] = (j < g.N && kk < ke) ? g.B[int64_t(kk) * g.sb0 + int64_t(j) * g.sb1] : 0.f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            As[buf][a_k + u * a_dk][a_i + u * a_di] = ra[u];
            Bs[buf][b_k + u * b_dk][b_j + u * b_dj] = rb[u];
        }
    };
    const int wi = (w >> 1) * 64, wj = (w & 1) * 64;
    const int lr = lane & 31, lk = lane >> 5;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
    load(kb);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += kKT) {
        const bool more = k0 + kKT < ke;
        if (more) load(k0 + kKT);
#pragma unroll
        for (int s = 0; s < kKT; s += 2) {
            const float a0 = As[buf][s + lk][wi + lr], a1 = As[buf][s + lk][wi + 32 + lr];
            const float b0 = Bs[buf][s + lk][wj + lr], b1 = Bs[buf][s + lk][wj + 32 + lr];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            const int j = j0 + wj + tj * 32 + lr;
            if (j >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = i0 + wi + ti * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                if (i >= g.M) continue;
                const float v0 = acc[ti][tj][r];
                if (g.part) {
                    g.part[(int64_t(blockIdx.z) * g.M + i) * g.N + j] = v0;
                    continue;
                }
                float v = v0;
                if (g.bias) v += g.bias[j];
                if (g.beta != 0.f) v += g.beta * g.C[int64_t(i) * g.ldc + j];
                if (g.act == 1) v = tanhf(v);
                g.C[int64_t(i) * g.ldc + j] = v;
            }
        }
}

// C = act(beta C + sum over splits of part + bias), fixed summation order
__global__ void k_splitk_reduce(GemmArgs g, int splits) {
    const int64_t n = int64_t(g.M) * g.N;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const int i = int(e / g.N), j = int(e - int64_t(i) * g.N);
        float v = 0.f;
        for (int z = 0; z < splits; ++z) v += g.part[int64_t(z) * n + e];
        if (g.bias) v += g.bias[j];
        if (g.beta != 0.f) v += g.beta * g.C[int64_t(i) * g.ldc + j];
        if (g.act == 1) v = tanhf(v);
        g.C[int64_t(i) * g.ldc + j] = v;
    }
}

// C (M x N) = act(beta C + A B + bias).  With split_buf (room for split_cap
// floats) a product with few output tiles is split along K over blockIdx.z
// (at most kMaxSplit parts, at least kMinSplitK K columns each, the partial
// products within split_cap), then reduced in a fixed order.
void gemm(hipStream_t st, const float *A, int64_t sa0, int64_t sa1, const float *B, int64_t sb0, int64_t sb1,
          float *C, int64_t ldc, int M, int N, int K, const float *bias, int act, float beta,
          float *split_buf = nullptr, int64_t split_cap = 0) {
    GemmArgs g{A, B, C, bias, sa0, sa1, sb0, sb1, ldc, M, N, K, act, beta, 0, nullptr};
    const int gx = (N + kMT - 1) / kMT, gy = (M + kMT - 1) / kMT;
    int splits = 1;
    if (split_buf) {
        const int64_t mn = int64_t(M) * N;
        splits = std::min({kMaxSplit, std::max(1, (kFillBlocks + gx * gy - 1) / (gx * gy)), std::max(1, K / kMinSplitK),
                           int(std::min<int64_t>(split_cap / std::max<int64_t>(mn, 1), kMaxSplit))});
    }
    if (splits <= 1) {
        hipLaunchKernelGGL(k_gemm, dim3(gx, gy), dim3(256), 0, st, g);
        return;
    }
    g.ks = ((K + splits - 1) / splits + kKT - 1) / kKT * kKT;
    splits = (K + g.ks - 1) / g.ks;
    g.part = split_buf;
    hipLaunchKernelGGL(k_gemm, dim3(gx, gy, splits), dim3(256), 0, st, g);
    const int64_t n = int64_t(M) * N;
    hipLaunchKernelGGL(k_splitk_reduce, dim3(unsigned(std::min<int64_t>((n + 255) / 256, 4096))), dim3(256), 0, st, g,
                       splits);
}

// dy = (y - t) / (B n_out); loss partial sums per block
__global__ void k_mse_grad(const float *y, const float *t, float *dy, int64_t n, float inv, float *part) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const float d = y[i] - t[i];
        dy[i] = d * inv;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = sum(part) * scale (one block)
__global__ void k_sum_parts(const float *part, int n, float scale, float *loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * scale;
}

// Relative RMS of the network: per block FP64 partial sums of
// (y * scale - t)^2 and t^2 over a chunk, then one block adds them (fixed
// order) to the running totals tot[0], tot[1].
__global__ void k_rms_parts(const float *y, const float *t, const float *scale, int n_out, int64_t n, double *part) {
    __shared__ double r0[256], r1[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const double tv = t[i];
        const double d = double(y[i]) * double(scale[i % n_out]) - tv;
        a += d * d;
        b += tv * tv;
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r0[0];
        part[2 * blockIdx.x + 1] = r1[0];
    }
}

__global__ void k_rms_total(const double *part, int nb, double *tot, int first) {
    if (threadIdx.x != 0) return;
    double a = first ? 0.0 : tot[0], b = first ? 0.0 : tot[1];
    for (int i = 0; i < nb; ++i) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    tot[0] = a;
    tot[1] = b;
}

// dz = dh * (1 - h^2)  (tanh derivative), in place on dh
__global__ void k_tanh_back(float *dh, const float *h, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        dh[i] *= 1.f - h[i] * h[i];
}

// db[j] = sum_i dz[i][j] in two fixed-order steps: k_colsum_part sums a
// chunk of kColRows rows for 64 columns per block (four row groups per column,
// then the four partials), k_colsum_final adds the chunk partials in order.
constexpr int kColRows = 64;

__global__ __launch_bounds__(256) void k_colsum_part(const float *dz, int rows, int cols, float *part) {
    __shared__ float red[4][64];
    const int j = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
    const int r0 = blockIdx.y * kColRows, r1 = min(rows, r0 + kColRows);
    float s = 0.f;
    if (j < cols)
        for (int i = r0 + g; i < r1; i += 4) s += dz[int64_t(i) * cols + j];
    red[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && j < cols)
        part[int64_t(blockIdx.y) * cols + j] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                               red[3][threadIdx.x];
}

__global__ void k_colsum_final(const float *part, int chunks, int cols, float *db) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[int64_t(c) * cols + j];
    db[j] = s;
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

__global__ void k_copy_f32(float *dst, const float *src, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) dst[i] = src[i];
}

int nblocks(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 4096)); }

// db = column sums of dz (rows x cols); part holds ceil(rows / kColRows) x cols
// floats (the split-K buffer, free between products)
void colsum(hipStream_t st, const float *dz, int rows, int cols, float *db, float *part) {
    const int chunks = (rows + kColRows - 1) / kColRows;
    hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, chunks), dim3(256), 0, st, dz, rows, cols, part);
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, st, part, chunks, cols, db);
}

}  // namespace
}  // namespace rpot

using namespace rpot;

struct rp_mlp_s {
    int n_in = 0, H = 0, n_out = 0, max_batch = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t n_params = 0;
    size_t off_w = 0, off_g = 0, off_m = 0, off_v = 0, off_h1 = 0, off_h2 = 0, off_y = 0, off_dy = 0, off_d2 = 0,
           off_d1 = 0, off_part = 0, off_split = 0, off_rms = 0;
    int64_t split_cap = 0;   // floats of the split-K partial products
    int64_t step = 0;
    std::string err;
    float *W1() { return f(off_w); }
    float *b1() { return W1() + int64_t(n_in) * H; }
    float *W2() { return b1() + H; }
    float *b2() { return W2() + int64_t(H) * H; }
    float *W3() { return b2() + H; }
    float *b3() { return W3() + int64_t(H) * n_out; }
    float *Ws() { return b3() + n_out; }
    float *f(size_t off) { return reinterpret_cast<float *>(ws + off); }
};

namespace {

struct MErr {
    rp_status code;
    std::string msg;
};

[[noreturn]] void mfail(rp_status c, const std::string &m) { throw MErr{c, m}; }

thread_local std::string g_mlp_create_error;

template <typename F>
rp_status mguard(rp_mlp m, F &&fn) {
    if (!m) return RP_ERR_ARG;
    try {
        m->err.clear();
        fn();
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) mfail(RP_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        return RP_OK;
    } catch (const MErr &e) {
        m->err = e.msg;
        return e.code;
    } catch (...) {
        m->err = "unknown error";
        return RP_ERR_ARG;
    }
}

void need_bound(rp_mlp m) {
    if (!m->ws) mfail(RP_ERR_STATE, "workspace not bound");
}

void check_batch(rp_mlp m, int batch) {
    if (batch < 1 || batch > m->max_batch) mfail(RP_ERR_ARG, "batch outside [1, max_batch]");
}

void forward(rp_mlp m, const float *x, int B, float *y, hipStream_t st) {
    const int H = m->H;
    float *sp = m->f(m->off_split);
    const int64_t cap = m->split_cap;
    gemm(st, x, m->n_in, 1, m->W1(), H, 1, m->f(m->off_h1), H, B, H, m->n_in, m->b1(), 1, 0.f, sp, cap);
    gemm(st, m->f(m->off_h1), H, 1, m->W2(), H, 1, m->f(m->off_h2), H, B, H, H, m->b2(), 1, 0.f, sp, cap);
    gemm(st, m->f(m->off_h2), H, 1, m->W3(), m->n_out, 1, y, m->n_out, B, m->n_out, H, m->b3(), 0, 0.f, sp, cap);
    gemm(st, x, m->n_in, 1, m->Ws(), m->n_out, 1, y, m->n_out, B, m->n_out, m->n_in, nullptr, 0, 1.f, sp, cap);
}

// Loss into *loss_dev and the gradient of every parameter into grad (flat).
void loss_grad(rp_mlp m, const float *x, const float *t, int B, float *loss_dev, float *grad) {
    hipStream_t st = m->stream;
    const int H = m->H, no = m->n_out, ni = m->n_in;
    float *y = m->f(m->off_y), *dy = m->f(m->off_dy), *h1 = m->f(m->off_h1), *h2 = m->f(m->off_h2);
    float *d2 = m->f(m->off_d2), *d1 = m->f(m->off_d1);
    float *sp = m->f(m->off_split);
    const int64_t cap = m->split_cap;
    forward(m, x, B, y, st);
    const int64_t ny = int64_t(B) * no;
    const int nb = std::min(nblocks(ny), 256);
    hipLaunchKernelGGL(k_mse_grad, dim3(nb), dim3(256), 0, st, y, t, dy, ny, 1.f / float(ny), m->f(m->off_part));
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, m->f(m->off_part), nb, 0.5f / float(ny), loss_dev);
    float *gW1 = grad, *gb1 = gW1 + int64_t(ni) * H, *gW2 = gb1 + H, *gb2 = gW2 + int64_t(H) * H;
    float *gW3 = gb2 + H, *gb3 = gW3 + int64_t(H) * no, *gWs = gb3 + no;
    // skip: gWs = x^T dy
    gemm(st, x, 1, ni, dy, no, 1, gWs, no, ni, no, B, nullptr, 0, 0.f, sp, cap);
    // layer 3: gW3 = h2^T dy, gb3 = colsum dy, d2 = dy W3^T
    gemm(st, h2, 1, H, dy, no, 1, gW3, no, H, no, B, nullptr, 0, 0.f, sp, cap);
    colsum(st, dy, B, no, gb3, sp);
    gemm(st, dy, no, 1, m->W3(), 1, no, d2, H, B, H, no, nullptr, 0, 0.f, sp, cap);
    hipLaunchKernelGGL(k_tanh_back, dim3(nblocks(int64_t(B) * H)), dim3(256), 0, st, d2, h2, int64_t(B) * H);
    // layer 2
    gemm(st, h1, 1, H, d2, H, 1, gW2, H, H, H, B, nullptr, 0, 0.f, sp, cap);
    colsum(st, d2, B, H, gb2, sp);
    gemm(st, d2, H, 1, m->W2(), 1, H, d1, H, B, H, H, nullptr, 0, 0.f, sp, cap);
    hipLaunchKernelGGL(k_tanh_back, dim3(nblocks(int64_t(B) * H)), dim3(256), 0, st, d1, h1, int64_t(B) * H);
    // layer 1
    gemm(st, x, 1, ni, d1, H, 1, gW1, H, ni, H, B, nullptr, 0, 0.f, sp, cap);
    colsum(st, d1, B, H, gb1, sp);
}

}  // namespace

namespace rpot {

bool mlp_dims(rp_mlp m, int *n_in, int *n_out, int *max_batch) {
    if (!m || !m->ws) return false;
    *n_in = m->n_in;
    *n_out = m->n_out;
    *max_batch = m->max_batch;
    return true;
}

void mlp_forward_on(rp_mlp m, const float *x, int batch, float *y, hipStream_t st) { forward(m, x, batch, y, st); }

}  // namespace rpot

extern "C" {

rp_status rp_mlp_create(rp_mlp *out, int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch,
                        void *hip_stream) {
    if (!out) {
        g_mlp_create_error = "out is null";
        return RP_ERR_ARG;
    }
    *out = nullptr;
    if (n_in < 1 || n_hidden < 1 || n_out < 1 || max_batch < 1) {
        g_mlp_create_error = "sizes must be >= 1";
        return RP_ERR_ARG;
    }
    rp_mlp m = new (std::nothrow) rp_mlp_s();
    if (!m) return RP_ERR_NOMEM;
    m->n_in = n_in;
    m->H = n_hidden;
    m->n_out = n_out;
    m->max_batch = max_batch;
    m->stream = static_cast<hipStream_t>(hip_stream);
    m->n_params = int64_t(n_in) * n_hidden + n_hidden + int64_t(n_hidden) * n_hidden + n_hidden +
                  int64_t(n_hidden) * n_out + n_out + int64_t(n_in) * n_out;
    size_t off = 0;
    auto alloc = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t P = size_t(m->n_params) * 4, BH = size_t(max_batch) * n_hidden * 4, BO = size_t(max_batch) * n_out * 4;
    m->off_w = alloc(P);
    m->off_g = alloc(P);
    m->off_m = alloc(P);
    m->off_v = alloc(P);
    m->off_h1 = alloc(BH);
    m->off_h2 = alloc(BH);
    m->off_y = alloc(BO);
    m->off_dy = alloc(BO);
    m->off_d2 = alloc(BH);
    m->off_d1 = alloc(BH);
    m->off_part = alloc(256 * 4 + 16);
    m->off_rms = alloc((2 * 256 + 2) * 8);
    m->split_cap = int64_t(kMaxSplit) * max_batch * std::max(n_hidden, n_out);
    m->off_split = alloc(size_t(m->split_cap) * 4);
    m->ws_bytes = off;
    *out = m;
    return RP_OK;
}

rp_status rp_mlp_workspace_bytes(rp_mlp m, size_t *bytes) {
    return mguard(m, [&] {
        if (!bytes) mfail(RP_ERR_ARG, "bytes is null");
        *bytes = m->ws_bytes;
    });
}

rp_status rp_mlp_n_params(rp_mlp m, int64_t *n) {
    return mguard(m, [&] {
        if (!n) mfail(RP_ERR_ARG, "n is null");
        *n = m->n_params;
    });
}

rp_status rp_mlp_bind(rp_mlp m, void *dev, size_t bytes) {
    return mguard(m, [&] {
        if (!dev || reinterpret_cast<uintptr_t>(dev) % 256) mfail(RP_ERR_ARG, "workspace must be 256-byte aligned");
        if (bytes < m->ws_bytes) mfail(RP_ERR_NOMEM, "workspace smaller than rp_mlp_workspace_bytes");
        m->ws = static_cast<char *>(dev);
        // every region is 256-byte aligned and padded, so whole 16-byte words fit
        launch_fill_zero(m->ws + m->off_m, (size_t(m->n_params) * 4 + 15) / 16 * 16, m->stream);
        launch_fill_zero(m->ws + m->off_v, (size_t(m->n_params) * 4 + 15) / 16 * 16, m->stream);
        m->step = 0;
    });
}

rp_status rp_mlp_set_params(rp_mlp m, const float *params) {
    return mguard(m, [&] {
        need_bound(m);
        if (!params) mfail(RP_ERR_ARG, "params is null");
        hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(m->n_params)), dim3(256), 0, m->stream, m->f(m->off_w), params,
                           m->n_params);
        // restart the optimiser moments with new parameters
        launch_fill_zero(m->ws + m->off_m, (size_t(m->n_params) * 4 + 15) / 16 * 16, m->stream);
        launch_fill_zero(m->ws + m->off_v, (size_t(m->n_params) * 4 + 15) / 16 * 16, m->stream);
        m->step = 0;
    });
}

rp_status rp_mlp_get_params(rp_mlp m, float *params) {
    return mguard(m, [&] {
        need_bound(m);
        if (!params) mfail(RP_ERR_ARG, "params is null");
        hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(m->n_params)), dim3(256), 0, m->stream, params, m->f(m->off_w),
                           m->n_params);
    });
}

rp_status rp_mlp_forward(rp_mlp m, const float *x, int32_t batch, float *y) {
    return mguard(m, [&] {
        need_bound(m);
        check_batch(m, batch);
        if (!x || !y) mfail(RP_ERR_ARG, "null pointer");
        forward(m, x, batch, y, m->stream);
    });
}

rp_status rp_mlp_relative_rms(rp_mlp m, const float *x, const float *t, int64_t n, const float *out_scale,
                              double *rel) {
    return mguard(m, [&] {
        need_bound(m);
        if (!x || !t || !out_scale || !rel) mfail(RP_ERR_ARG, "null pointer");
        if (n < 1) mfail(RP_ERR_ARG, "n must be >= 1");
        hipStream_t st = m->stream;
        double *part = reinterpret_cast<double *>(m->ws + m->off_rms);
        double *tot = part + 2 * 256;
        float *y = m->f(m->off_y);
        for (int64_t i0 = 0; i0 < n; i0 += m->max_batch) {
            const int B = int(std::min<int64_t>(m->max_batch, n - i0));
            forward(m, x + i0 * m->n_in, B, y, st);
            const int64_t ny = int64_t(B) * m->n_out;
            const int nb = std::min(nblocks(ny), 256);
            hipLaunchKernelGGL(k_rms_parts, dim3(nb), dim3(256), 0, st, y, t + i0 * m->n_out, out_scale, m->n_out,
                               ny, part);
            hipLaunchKernelGGL(k_rms_total, dim3(1), dim3(64), 0, st, part, nb, tot, i0 == 0 ? 1 : 0);
        }
        double h[2] = {0.0, 0.0};
        if (hipMemcpyAsync(h, tot, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            mfail(RP_ERR_DEVICE, "reading the relative RMS back failed");
        *rel = std::sqrt(h[0] / std::max(h[1], 1e-300));
    });
}

rp_status rp_mlp_loss_grad(rp_mlp m, const float *x, const float *t, int32_t batch, float *loss, float *grad) {
    return mguard(m, [&] {
        need_bound(m);
        check_batch(m, batch);
        if (!x || !t || !loss || !grad) mfail(RP_ERR_ARG, "null pointer");
        loss_grad(m, x, t, batch, loss, grad);
    });
}

rp_status rp_mlp_train_step(rp_mlp m, const float *x, const float *t, int32_t batch, float lr, float *loss) {
    return mguard(m, [&] {
        need_bound(m);
        check_batch(m, batch);
        if (!x || !t || !loss) mfail(RP_ERR_ARG, "null pointer");
        if (!(lr > 0.f)) mfail(RP_ERR_ARG, "lr must be positive");
        loss_grad(m, x, t, batch, loss, m->f(m->off_g));
        m->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f / (1.f - std::pow(b1, float(m->step)));
        const float c2 = 1.f / (1.f - std::pow(b2, float(m->step)));
        hipLaunchKernelGGL(k_adam, dim3(nblocks(m->n_params)), dim3(256), 0, m->stream, m->f(m->off_w),
                           m->f(m->off_g), m->f(m->off_m), m->f(m->off_v), m->n_params, lr, b1, b2, 1e-8f, c1, c2);
    });
}

rp_status rp_mlp_destroy(rp_mlp m) {
    if (!m) return RP_ERR_ARG;
    delete m;
    return RP_OK;
}

const char *rp_mlp_last_error(rp_mlp m) {
    if (!m) return g_mlp_create_error.c_str();
    return m->err.c_str();
}

}  // extern "C"
