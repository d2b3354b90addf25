// Kernels of the learned far-pair surrogate.
//
// The paper closes by pointing at a multipole approximation of the retarded
// potentials of far sub-domains as a further speed-up (Sec. V).  Here that far
// coupling is learned: for a far pair (target s <- source n) a small network
// maps the recent history of the source's low-order moments, rotated into a
// frame aligned with the pair, to the coefficients of the pair's potential in
// a cubic polynomial basis on the target box.  The kernels below compute the
// moments, gather the network inputs, map the outputs back to the box basis,
// add the synthesised field to the targets, and judge the surrogate against
// the plain pair sum (least-squares fit, residuals, correction).
//
// Box basis: B_b(x, y, z) = P_i(x) P_j(y) P_k(z), i + j + k <= 3 (20 functions,
// Legendre polynomials P, box coordinates mapped to [-1, 1]).
#include "rpot_internal.hpp"

#include <algorithm>

namespace rpot {

__device__ __forceinline__ void legendre4(float x, float (&p)[4]) {
    p[0] = 1.f;
    p[1] = x;
    p[2] = 0.5f * (3.f * x * x - 1.f);
    p[3] = 0.5f * x * (5.f * x * x - 3.f);
}

// basis index -> degrees along x, y, z (lexicographic, total degree <= 3); a
// compile-time table, so the unrolled basis products index registers by
// constants
struct BasisDeg {
    int8_t d[kNBasis][3];
};
constexpr BasisDeg kBasisDeg = {{{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 0, 3}, {0, 1, 0}, {0, 1, 1}, {0, 1, 2},
                                 {0, 2, 0}, {0, 2, 1}, {0, 3, 0}, {1, 0, 0}, {1, 0, 1}, {1, 0, 2}, {1, 1, 0},
                                 {1, 1, 1}, {1, 2, 0}, {2, 0, 0}, {2, 0, 1}, {2, 1, 0}, {3, 0, 0}}};

__device__ __forceinline__ float box_coord(int i, int n) { return n > 1 ? float(i) * (2.f / float(n - 1)) - 1.f : 0.f; }

// (ix, iy, iz) of linear grid index i (z fastest); grids stay below 2^31
// points, so the index arithmetic is 32-bit
__device__ __forceinline__ void grid_xyz(int64_t i, const int (&N)[3], int &ix, int &iy, int &iz) {
    const uint32_t u = uint32_t(i), nz = uint32_t(N[2]), ny = uint32_t(N[1]);
    const uint32_t r = u / nz;
    iz = int(u - r * nz);
    ix = int(r / ny);
    iy = int(r - uint32_t(ix) * ny);
}

// The 20 basis values at grid point i of an N[0] x N[1] x N[2] box.
__device__ __forceinline__ void basis_at(int64_t i, const int (&N)[3], float (&B)[kNBasis]) {
    int ix, iy, iz;
    grid_xyz(i, N, ix, iy, iz);
    float px[4], py[4], pz[4];
    legendre4(box_coord(ix, N[0]), px);
    legendre4(box_coord(iy, N[1]), py);
    legendre4(box_coord(iz, N[2]), pz);
#pragma unroll
    for (int b = 0; b < kNBasis; ++b) B[b] = px[kBasisDeg.d[b][0]] * py[kBasisDeg.d[b][1]] * pz[kBasisDeg.d[b][2]];
}

template <int NT>
__device__ __forceinline__ float block_sum(float v, float *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

template <int NT>
__device__ __forceinline__ float block_max(float v, float *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Moments.  Grid (kMomChunks, jobs): each block reduces a strided share of the
// points into partial[chunk][kNFeat]; a second launch sums the chunks in a
// fixed order (deterministic) into the ring slot of the current step.
// The moments of one grid point (position r, source differences d) added to acc.
__device__ __forceinline__ void point_moments(float (&acc)[kNMom], const float (&d)[4], const float (&r)[3]) {
    // second-moment products x_a x_b (xx yy zz xy xz yz)
    const float rr[6] = {r[0] * r[0], r[1] * r[1], r[2] * r[2], r[0] * r[1], r[0] * r[2], r[1] * r[2]};
    acc[0] += d[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[1 + c] = fmaf(d[0], r[c], acc[1 + c]);
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[4 + k] = fmaf(d[0], rr[k], acc[4 + k]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[10 + c] += d[1 + c];
#pragma unroll
        for (int e = 0; e < 3; ++e) acc[13 + 3 * c + e] = fmaf(d[1 + c], r[e], acc[13 + 3 * c + e]);
    }
    // third moments of the charge: xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz
    const float dr0 = d[0] * r[0], dr1 = d[0] * r[1], dr2 = d[0] * r[2];
    acc[22] = fmaf(dr0, rr[0], acc[22]);
    acc[23] = fmaf(dr1, rr[1], acc[23]);
    acc[24] = fmaf(dr2, rr[2], acc[24]);
    acc[25] = fmaf(dr1, rr[0], acc[25]);
    acc[26] = fmaf(dr2, rr[0], acc[26]);
    acc[27] = fmaf(dr0, rr[1], acc[27]);
    acc[28] = fmaf(dr2, rr[1], acc[28]);
    acc[29] = fmaf(dr0, rr[2], acc[29]);
    acc[30] = fmaf(dr1, rr[2], acc[30]);
    acc[31] = fmaf(dr0, rr[5], acc[31]);
    // second moments of the current: N_i,ab
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[32 + 6 * c + k] = fmaf(d[1 + c], rr[k], acc[32 + 6 * c + k]);
}

__global__ __launch_bounds__(256) void k_moments_partial(MomentArgs a) {
    const MomentJob &j = a.jobs[blockIdx.y];
    const int64_t npts = int64_t(j.N[0]) * j.N[1] * j.N[2];
    float acc[kNMom];
#pragma unroll
    for (int q = 0; q < kNMom; ++q) acc[q] = 0.f;
    const int64_t stride = int64_t(gridDim.x) * 256;
    if ((j.N[2] & 3) == 0 && ((reinterpret_cast<uintptr_t>(j.src) | reinterpret_cast<uintptr_t>(j.s0)) & 15) == 0) {
        // four consecutive z of one (x, y) per thread: 16-byte loads, all
        // eight issued before the products
        for (int64_t i = (int64_t(blockIdx.x) * 256 + threadIdx.x) * 4; i < npts; i += stride * 4) {
            float4 sv[4], qv[4];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                sv[mu] = *reinterpret_cast<const float4 *>(j.src + mu * npts + i);
                qv[mu] = *reinterpret_cast<const float4 *>(j.s0 + mu * npts + i);
            }
            int ix, iy, iz;
            grid_xyz(i, j.N, ix, iy, iz);
            const float dd[4][4] = {{sv[0].x - qv[0].x, sv[1].x - qv[1].x, sv[2].x - qv[2].x, sv[3].x - qv[3].x},
                                    {sv[0].y - qv[0].y, sv[1].y - qv[1].y, sv[2].y - qv[2].y, sv[3].y - qv[3].y},
                                    {sv[0].z - qv[0].z, sv[1].z - qv[1].z, sv[2].z - qv[2].z, sv[3].z - qv[3].z},
                                    {sv[0].w - qv[0].w, sv[1].w - qv[1].w, sv[2].w - qv[2].w, sv[3].w - qv[3].w}};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float r[3] = {j.o[0] + a.h * float(ix), j.o[1] + a.h * float(iy), j.o[2] + a.h * float(iz + e)};
                point_moments(acc, dd[e], r);
            }
        }
    } else {
        for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < npts; i += stride) {
            int ix, iy, iz;
            grid_xyz(i, j.N, ix, iy, iz);
            const float r[3] = {j.o[0] + a.h * float(ix), j.o[1] + a.h * float(iy), j.o[2] + a.h * float(iz)};
            float d[4];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) d[mu] = j.src[mu * npts + i] - j.s0[mu * npts + i];
            point_moments(acc, d, r);
        }
    }
    // Wave sums by recursive halving: at the step with lane mask m a lane
    // keeps half of its values (the upper half when its bit m is set), sends
    // the other half to lane ^ m and adds what that lane sent; after the six
    // steps lane q holds the wave's sum of moment q (63 exchanges instead of
    // 6 per moment).  Then the four waves in a fixed order.
    static_assert(kNMom <= 64, "one moment per lane");
    __shared__ float red[4][kNMom];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float v[64];
#pragma unroll
    for (int q = 0; q < 64; ++q) v[q] = q < kNMom ? acc[q] : 0.f;
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int m = 32 >> st, h = 32 >> st;   // lane mask, values kept after the step
        const bool up = (lane & m) != 0;
#pragma unroll
        for (int q = 0; q < h; ++q) {
            const float send = up ? v[q] : v[q + h];
            const float keep = up ? v[q + h] : v[q];
            v[q] = keep + __shfl_xor(send, m, 64);
        }
    }
    if (lane < kNMom) red[wave][lane] = v[0];
    __syncthreads();
    if (threadIdx.x < kNMom) {
        const int q = threadIdx.x;
        j.partial[blockIdx.x * kNMom + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

__global__ void k_moments_final(MomentArgs a) {
    const MomentJob &j = a.jobs[blockIdx.x];
    const int q = threadIdx.x;
    if (q >= kNMom) return;
    double s = 0.0;
    for (int c = 0; c < kMomChunks; ++c) s += double(j.partial[c * kNMom + q]);
    const int64_t slot = (*a.step) % a.depth;
    j.ring[slot * kFeatStride + q] = float(s * a.h3);
}

// ---------------------------------------------------------------------------
// Network inputs of every far pair: the source's moments at lags
// m = m_c - n_lags/2 + j (j < n_lags), i.e. of steps t = l - m, rotated into
// the pair's frame and scaled (H), written as the six blocks H, g H, f H,
// g f H, g^2 H, f^2 H with the pair's geometry g, f, then g and f.  Steps
// t <= 0 have dS = 0.  Block: one pair; thread: one lag.
__global__ __launch_bounds__(128) void k_features(FeatArgs a) {
    const FarPair &fp = a.pairs[blockIdx.x];
    const int64_t l = *a.step + a.step_adj;
    float *x = a.x + int64_t(blockIdx.x) * a.n_in;
    const float *ring = a.moments + int64_t(fp.src_slot) * a.depth * kFeatStride;
    float R[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = fp.rot[i];
    const float g = fp.geo[0], fr = fp.geo[1];
    const float mult[kNBlocks] = {1.f, g, fr, g * fr, g * g, fr * fr};
    const int64_t nh = int64_t(a.n_lags) * kNFeat;
    for (int jl = threadIdx.x; jl < a.n_lags; jl += blockDim.x) {
        const int64_t m = int64_t(fp.m_c) - a.n_lags / 2 + jl;
        const int64_t t = l - m;
        float f[kNFeat];
        if (t > 0 && m >= 0) {
            const float *v = ring + (t % a.depth) * kFeatStride;
#pragma unroll
            for (int q = 0; q < kNFeat; ++q) f[q] = v[q];
        } else {
#pragma unroll
            for (int q = 0; q < kNFeat; ++q) f[q] = 0.f;
        }
        const float Q[3][3] = {{f[4], f[7], f[8]}, {f[7], f[5], f[9]}, {f[8], f[9], f[6]}};
        float gq[kNFeat];
        gq[0] = f[0];
#pragma unroll
        for (int A = 0; A < 3; ++A) {
            gq[1 + A] = R[3 * A] * f[1] + R[3 * A + 1] * f[2] + R[3 * A + 2] * f[3];
            gq[10 + A] = R[3 * A] * f[10] + R[3 * A + 1] * f[11] + R[3 * A + 2] * f[12];
        }
        // rank-2 tensors: T' = R T R^T
        float RQ[3][3], RK[3][3];
#pragma unroll
        for (int A = 0; A < 3; ++A)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                RQ[A][c] = R[3 * A] * Q[0][c] + R[3 * A + 1] * Q[1][c] + R[3 * A + 2] * Q[2][c];
                RK[A][c] = R[3 * A] * f[13 + c] + R[3 * A + 1] * f[16 + c] + R[3 * A + 2] * f[19 + c];
            }
        float Qp[3][3];
#pragma unroll
        for (int A = 0; A < 3; ++A)
#pragma unroll
            for (int B = 0; B < 3; ++B) {
                Qp[A][B] = RQ[A][0] * R[3 * B] + RQ[A][1] * R[3 * B + 1] + RQ[A][2] * R[3 * B + 2];
                gq[13 + 3 * A + B] = RK[A][0] * R[3 * B] + RK[A][1] * R[3 * B + 1] + RK[A][2] * R[3 * B + 2];
            }
        gq[4] = Qp[0][0];
        gq[5] = Qp[1][1];
        gq[6] = Qp[2][2];
        gq[7] = Qp[0][1];
        gq[8] = Qp[0][2];
        gq[9] = Qp[1][2];
#pragma unroll
        for (int q = 0; q < kNFeat; ++q) {
            const float v = gq[q] * a.in_scale[q];
#pragma unroll
            for (int b = 0; b < kNBlocks; ++b) x[b * nh + jl * kNFeat + q] = mult[b] * v;
        }
    }
    if (threadIdx.x < kNGeo) x[kNBlocks * nh + threadIdx.x] = fp.geo[threadIdx.x];
}

// Coefficient maps (see XformArgs).  Block: one row; thread: one output.
__global__ __launch_bounds__(128) void k_xform(XformArgs a) {
    const int row = blockIdx.x;
    const int f = a.index ? a.index[row] : row;
    const FarPair &fp = a.pairs[f];
    const float *M = a.mats + (int64_t(f) * 2 + a.dir) * kNBasis * kNBasis;
    __shared__ float v[kNOut], w[kNOut];
    const int t = threadIdx.x;
    if (t < kNOut) {
        const float x = a.in[int64_t(row) * kNOut + t];
        v[t] = (a.dir == 0) ? x * a.scale[t] * fp.inv_d : x;
    }
    __syncthreads();
    const int mu = t / kNBasis, b = t - (t / kNBasis) * kNBasis;
    if (a.dir == 0) {
        // vector part back to the global axes: A_i = sum_j R[j][i] A'_j
        if (t < kNOut) {
            float y = v[t];
            if (mu > 0) {
                const int i = mu - 1;
                y = fp.rot[i] * v[kNBasis + b] + fp.rot[3 + i] * v[2 * kNBasis + b] + fp.rot[6 + i] * v[3 * kNBasis + b];
            }
            w[t] = y;
        }
        __syncthreads();
        if (t < kNOut) {
            float y = 0.f;
            for (int c = 0; c < kNBasis; ++c) y = fmaf(M[b * kNBasis + c], w[mu * kNBasis + c], y);
            float *o = a.out + int64_t(row) * kNOut + t;
            *o = a.accumulate ? *o + y : y;
        }
    } else {
        if (t < kNOut) {
            float y = 0.f;
            for (int c = 0; c < kNBasis; ++c) y = fmaf(M[b * kNBasis + c], v[mu * kNBasis + c], y);
            w[t] = y;
        }
        __syncthreads();
        if (t < kNOut) {
            float y = w[t];
            if (mu > 0) {
                const int j = mu - 1;
                y = fp.rot[3 * j] * w[kNBasis + b] + fp.rot[3 * j + 1] * w[2 * kNBasis + b] +
                    fp.rot[3 * j + 2] * w[3 * kNBasis + b];
            }
            a.out[int64_t(row) * kNOut + t] = y;
        }
    }
}

// Per target: the sum of its active far pairs' box coefficients (fixed order).
__global__ void k_coef_sum(CoefArgs a) {
    const int s = blockIdx.x;
    const int k = threadIdx.x;
    if (k >= kNOut) return;
    float acc = 0.f;
    for (int i = a.tgt_begin[s]; i < a.tgt_begin[s + 1]; ++i) acc += a.pc[int64_t(a.order[i]) * kNOut + k];
    a.coef[int64_t(s) * kNOut + k] = acc;
}

__global__ __launch_bounds__(256) void k_synthesize(SynthArgs a) {
    const SynthJob &j = a.jobs[blockIdx.y];
    const int64_t npts = int64_t(j.N[0]) * j.N[1] * j.N[2];
    __shared__ float c[kNOut];
    if (threadIdx.x < kNOut) c[threadIdx.x] = j.coef[threadIdx.x];
    __syncthreads();
    if ((j.N[2] & 3) == 0 && (reinterpret_cast<uintptr_t>(j.out) & 15) == 0) {
        // four consecutive z of one (x, y) per thread: 16-byte loads and
        // stores.  The four points share x and y, so the x-y factors of the
        // basis fold into W[mu][dz] = sum over b with z degree dz of
        // c[mu][b] P_dx(x) P_dy(y), and each point takes sum_dz P_dz(z) W[mu][dz].
        // One quad per thread (the grid covers the largest job): a loop here
        // would hold all 80 coefficients in registers.
        const int64_t i = (int64_t(blockIdx.x) * 256 + threadIdx.x) * 4;
        if (i < npts) {
            float4 o[4];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) o[mu] = *reinterpret_cast<const float4 *>(j.out + mu * npts + i);
            int ix, iy, iz;
            grid_xyz(i, j.N, ix, iy, iz);
            float px[4], py[4];
            legendre4(box_coord(ix, j.N[0]), px);
            legendre4(box_coord(iy, j.N[1]), py);
            float W[4][4];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
#pragma unroll
                for (int dz = 0; dz < 4; ++dz) W[mu][dz] = 0.f;
#pragma unroll
            for (int b = 0; b < kNBasis; ++b) {
                const float xy = px[kBasisDeg.d[b][0]] * py[kBasisDeg.d[b][1]];
#pragma unroll
                for (int mu = 0; mu < 4; ++mu)
                    W[mu][kBasisDeg.d[b][2]] = fmaf(c[mu * kNBasis + b], xy, W[mu][kBasisDeg.d[b][2]]);
            }
            float v[4][4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float pz[4];
                legendre4(box_coord(iz + e, j.N[2]), pz);
#pragma unroll
                for (int mu = 0; mu < 4; ++mu)
                    v[mu][e] = fmaf(pz[3], W[mu][3], fmaf(pz[2], W[mu][2], fmaf(pz[1], W[mu][1], pz[0] * W[mu][0])));
            }
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
                *reinterpret_cast<float4 *>(j.out + mu * npts + i) =
                    float4{o[mu].x + v[mu][0], o[mu].y + v[mu][1], o[mu].z + v[mu][2], o[mu].w + v[mu][3]};
        }
        return;
    }
    // one point per thread
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < npts) {
        float B[kNBasis];
        basis_at(i, j.N, B);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            float v = 0.f;
#pragma unroll
            for (int b = 0; b < kNBasis; ++b) v = fmaf(c[mu * kNBasis + b], B[b], v);
            j.out[mu * npts + i] += v;
        }
    }
}

// ---------------------------------------------------------------------------
// Judge: least-squares projection (block per (basis function, job)).
__global__ __launch_bounds__(256) void k_project(ProjArgs a) {
    const ProjJob &j = a.jobs[blockIdx.y];
    const int b = blockIdx.x;
    const float *q = j.Q + int64_t(b) * j.npts;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int64_t i = threadIdx.x; i < j.npts; i += 256) {
        const float w = q[i];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) acc[mu] = fmaf(w, j.F[mu * j.npts + i], acc[mu]);
    }
    __shared__ float red[256];
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        const float v = block_sum<256>(acc[mu], red);
        if (threadIdx.x == 0) j.coef[mu * kNBasis + b] = v;
    }
}

// Residual of F against the basis expansion with coefficients c (block per job).
__global__ __launch_bounds__(256) void k_residual(ProjArgs a) {
    const ProjJob &j = a.jobs[blockIdx.x];
    const float *cin = j.coef_in ? j.coef_in : j.coef;
    __shared__ float c[kNOut];
    if (threadIdx.x < kNOut) c[threadIdx.x] = cin[threadIdx.x];
    __syncthreads();
    float r[4] = {0.f, 0.f, 0.f, 0.f}, fm[4] = {0.f, 0.f, 0.f, 0.f};
    for (int64_t i = threadIdx.x; i < j.npts; i += 256) {
        float B[kNBasis];
        basis_at(i, j.N, B);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            float v = 0.f;
#pragma unroll
            for (int b = 0; b < kNBasis; ++b) v = fmaf(c[mu * kNBasis + b], B[b], v);
            const float F = j.F[mu * j.npts + i];
            r[mu] = fmaxf(r[mu], fabsf(F - v));
            fm[mu] = fmaxf(fm[mu], fabsf(F));
        }
    }
    __shared__ float red[256];
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        const float x = block_max<256>(r[mu], red);
        const float y = block_max<256>(fm[mu], red);
        if (threadIdx.x == 0) {
            j.resid[mu] = x;
            j.resid[4 + mu] = y;
        }
    }
}

__global__ __launch_bounds__(256) void k_budget(BudgetArgs a) {
    const BudgetJob &j = a.jobs[blockIdx.x];
    __shared__ float red[256];
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        float m = 0.f;
        for (int64_t i = threadIdx.x; i < j.npts; i += 256) m = fmaxf(m, fabsf(j.out[mu * j.npts + i]));
        m = block_max<256>(m, red);
        if (threadIdx.x == 0) j.budget[mu] = j.scale * m;
    }
}

// Grid over points; every thread walks the jobs in order, so jobs that share
// a target never write the same element concurrently.
__global__ __launch_bounds__(256) void k_correct(CorrArgs a) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    for (int jj = 0; jj < a.n_jobs; ++jj) {
        const CorrJob &j = a.jobs[jj];
        bool bad = false;
        if (j.active)
            for (int mu = 0; mu < 4; ++mu) bad |= j.resid[mu] > j.budget[mu];
        if (i == 0) j.fail[0] = bad ? 1 : 0;
        const int64_t npts = int64_t(j.N[0]) * j.N[1] * j.N[2];
        if (!bad || i >= npts) continue;
        float B[kNBasis];
        basis_at(i, j.N, B);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            float v = 0.f;
#pragma unroll
            for (int b = 0; b < kNBasis; ++b) v = fmaf(j.pc[mu * kNBasis + b], B[b], v);
            j.out[mu * npts + i] += j.F[mu * npts + i] - v;
        }
    }
}

// ---------------------------------------------------------------------------
// Analytic multipole far-pair terms (see MultipoleArgs).  With R from the
// source centre to a node, u = R/|R|, tau the retarded step l - |R|/(c dt)
// and the moments f of dS at tau (cubic Lagrange interpolation of the four
// ring samples around tau, which also gives the time derivatives f^(k)):
//   v   = q/R + u.p/R^2 + u.p^(1)/(cR) + (3 u.Q.u - tr Q)/(2R^3)
//         + (3 u.Q^(1).u - tr Q^(1))/(2cR^2) + u.Q^(2).u/(2c^2 R)
//         + (15 O_uuu - 9 u.trO)/(6R^4) + (15 O^(1)_uuu - 9 u.trO^(1))/(6cR^3)
//         + (6 O^(2)_uuu - 3 u.trO^(2))/(6c^2 R^2) + O^(3)_uuu/(6c^3 R)
//   A_i = J_i/R + (K u)_i/R^2 + (K^(1) u)_i/(cR) + (3 u.N_i.u - tr N_i)/(2R^3)
//         + (3 u.N_i^(1).u - tr N_i^(1))/(2cR^2) + u.N_i^(2).u/(2c^2 R)
// (the retarded Taylor expansion of the pair's lag sum to third order in the
// source coordinates for the charge, second order for the current; O the
// charge's third moments, N_i the current's second moments).  The value and
// first derivative carry + dt^2/12 times the next derivative: the lag sum
// reads the sources through their linear interpolant in time, whose mean over
// the spread of retarded times across a source lies that much above them.
__global__ __launch_bounds__(64) void k_multipole(MultipoleArgs a) {
    const FarPair &fp = a.pairs[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t l = *a.step + a.step_off;
    const float nodes[4] = {-1.f, -1.f / 3.f, 1.f / 3.f, 1.f};
    const float Rv[3] = {fp.d[0] + nodes[t >> 4] * fp.hw[0], fp.d[1] + nodes[(t >> 2) & 3] * fp.hw[1],
                         fp.d[2] + nodes[t & 3] * fp.hw[2]};
    const float R = sqrtf(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
    const float u[3] = {Rv[0] / R, Rv[1] / R, Rv[2] / R};
    const double tau = double(l) - double(R) * a.inv_cdt;
    const int64_t a0 = int64_t(floor(tau));
    const float x = float(tau - double(a0));
    // cubic Lagrange weights for samples at -1, 0, 1, 2 (value, d/dx, d2/dx2, d3/dx3)
    const float w[4] = {-x * (x - 1.f) * (x - 2.f) / 6.f, (x + 1.f) * (x - 1.f) * (x - 2.f) / 2.f,
                        -(x + 1.f) * x * (x - 2.f) / 2.f, (x + 1.f) * x * (x - 1.f) / 6.f};
    const float d1[4] = {-(3.f * x * x - 6.f * x + 2.f) / 6.f, (3.f * x * x - 4.f * x - 1.f) / 2.f,
                         -(3.f * x * x - 2.f * x - 2.f) / 2.f, (3.f * x * x - 1.f) / 6.f};
    const float d2[4] = {-(6.f * x - 6.f) / 6.f, (6.f * x - 4.f) / 2.f, -(6.f * x - 2.f) / 2.f, (6.f * x) / 6.f};
    const float d3[4] = {-1.f, 3.f, -3.f, 1.f};
    const float *ring = a.moments + int64_t(fp.src_slot) * a.depth * kFeatStride;
    float f0[kNMom], f1[kNMom], f2[kNMom], f3[kNMom];
#pragma unroll
    for (int q = 0; q < kNMom; ++q) f0[q] = f1[q] = f2[q] = f3[q] = 0.f;
    for (int k = 0; k < 4; ++k) {
        int64_t ts = a0 - 1 + k;
        if (ts > l) ts = l;   // never for a far pair; keeps the read inside the held history
        if (ts <= 0) continue;
        const float *v = ring + (ts % a.depth) * kFeatStride;
#pragma unroll
        for (int q = 0; q < kNMom; ++q) {
            f0[q] = fmaf(w[k], v[q], f0[q]);
            f1[q] = fmaf(d1[k], v[q], f1[q]);
            f2[q] = fmaf(d2[k], v[q], f2[q]);
            f3[q] = fmaf(d3[k], v[q], f3[q]);
        }
    }
    // per-step derivatives to per-time ones; the lag sum reads sources on the
    // chords between samples, whose mean over a source is S + dt^2/12 S''
    const float idt = 1.f / a.dt, ic = 1.f / a.c, iR = 1.f / R;
#pragma unroll
    for (int q = 0; q < kNMom; ++q) {
        f1[q] *= idt;
        f2[q] *= idt * idt;
        f3[q] *= idt * idt * idt;
        f0[q] = fmaf(a.dt * a.dt * (1.f / 12.f), f2[q], f0[q]);
        f1[q] = fmaf(a.dt * a.dt * (1.f / 12.f), f3[q], f1[q]);
    }
    auto uMu = [&](const float *m) {   // u.M.u from (xx yy zz xy xz yz)
        return m[0] * u[0] * u[0] + m[1] * u[1] * u[1] + m[2] * u[2] * u[2] +
               2.f * (m[3] * u[0] * u[1] + m[4] * u[0] * u[2] + m[5] * u[1] * u[2]);
    };
    auto octu = [&](const float *o) {  // O_uuu and u.trO from (xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz)
        const float uuu = o[0] * u[0] * u[0] * u[0] + o[1] * u[1] * u[1] * u[1] + o[2] * u[2] * u[2] * u[2] +
                          3.f * (o[3] * u[0] * u[0] * u[1] + o[4] * u[0] * u[0] * u[2] + o[5] * u[0] * u[1] * u[1] +
                                 o[6] * u[1] * u[1] * u[2] + o[7] * u[0] * u[2] * u[2] + o[8] * u[1] * u[2] * u[2]) +
                          6.f * o[9] * u[0] * u[1] * u[2];
        const float tr = u[0] * (o[0] + o[5] + o[7]) + u[1] * (o[3] + o[1] + o[8]) + u[2] * (o[4] + o[6] + o[2]);
        return make_float2(uuu, tr);
    };
    const float iR2 = iR * iR, iR3 = iR2 * iR, iR4 = iR2 * iR2;
    float v = f0[0] * iR;
    v += (u[0] * f0[1] + u[1] * f0[2] + u[2] * f0[3]) * iR2 + (u[0] * f1[1] + u[1] * f1[2] + u[2] * f1[3]) * ic * iR;
    v += (3.f * uMu(f0 + 4) - (f0[4] + f0[5] + f0[6])) * 0.5f * iR3;
    v += (3.f * uMu(f1 + 4) - (f1[4] + f1[5] + f1[6])) * 0.5f * ic * iR2;
    v += uMu(f2 + 4) * 0.5f * ic * ic * iR;
    const float2 O0 = octu(f0 + 22), O1 = octu(f1 + 22), O2 = octu(f2 + 22), O3 = octu(f3 + 22);
    v += (15.f * O0.x - 9.f * O0.y) * (1.f / 6.f) * iR4;
    v += (15.f * O1.x - 9.f * O1.y) * (1.f / 6.f) * ic * iR3;
    v += (6.f * O2.x - 3.f * O2.y) * (1.f / 6.f) * ic * ic * iR2;
    v += O3.x * (1.f / 6.f) * ic * ic * ic * iR;
    __shared__ float F[4][64];
    F[0][t] = v;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float Ku0 = f0[13 + 3 * i] * u[0] + f0[14 + 3 * i] * u[1] + f0[15 + 3 * i] * u[2];
        const float Ku1 = f1[13 + 3 * i] * u[0] + f1[14 + 3 * i] * u[1] + f1[15 + 3 * i] * u[2];
        const float *N0 = f0 + 32 + 6 * i, *N1 = f1 + 32 + 6 * i, *N2 = f2 + 32 + 6 * i;
        float A = f0[10 + i] * iR + Ku0 * iR2 + Ku1 * ic * iR;
        A += (3.f * uMu(N0) - (N0[0] + N0[1] + N0[2])) * 0.5f * iR3;
        A += (3.f * uMu(N1) - (N1[0] + N1[1] + N1[2])) * 0.5f * ic * iR2;
        A += uMu(N2) * 0.5f * ic * ic * iR;
        F[1 + i][t] = A;
    }
    __syncthreads();
    for (int o = t; o < kNOut; o += 64) {
        const int mu = o / kNBasis, b = o - mu * kNBasis;
        float acc = 0.f;
        for (int j = 0; j < 64; ++j) acc = fmaf(a.pinv[b * 64 + j], F[mu][j], acc);
        a.pc[int64_t(blockIdx.x) * kNOut + o] = acc;
    }
}

void launch_multipole(const MultipoleArgs &a, hipStream_t st) {
    if (a.n_pairs == 0) return;
    hipLaunchKernelGGL(k_multipole, dim3(a.n_pairs), dim3(64), 0, st, a);
}

// ---------------------------------------------------------------------------
void launch_moments(const MomentArgs &a, hipStream_t st) {
    if (a.n_jobs == 0) return;
    hipLaunchKernelGGL(k_moments_partial, dim3(kMomChunks, a.n_jobs), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_moments_final, dim3(a.n_jobs), dim3(64), 0, st, a);
}

void launch_features(const FeatArgs &a, hipStream_t st) {
    if (a.n_pairs == 0) return;
    hipLaunchKernelGGL(k_features, dim3(a.n_pairs), dim3(128), 0, st, a);
}

void launch_xform(const XformArgs &a, hipStream_t st) {
    if (a.n == 0) return;
    hipLaunchKernelGGL(k_xform, dim3(a.n), dim3(128), 0, st, a);
}

void launch_coef_sum(const CoefArgs &a, hipStream_t st) {
    if (a.n_targets == 0) return;
    hipLaunchKernelGGL(k_coef_sum, dim3(a.n_targets), dim3(128), 0, st, a);
}

void launch_synthesize(const SynthArgs &a, hipStream_t st) {
    if (a.n_jobs == 0) return;
    // one quad of points per thread on the 16-byte path, else one point
    int64_t blocks = 1;
    for (int q = 0; q < a.n_jobs; ++q) {
        const SynthJob &J = a.jobs[q];
        const int64_t n = int64_t(J.N[0]) * J.N[1] * J.N[2];
        const bool quad = (J.N[2] & 3) == 0 && (reinterpret_cast<uintptr_t>(J.out) & 15) == 0;
        blocks = std::max(blocks, quad ? (n + 1023) / 1024 : (n + 255) / 256);
    }
    hipLaunchKernelGGL(k_synthesize, dim3(uint32_t(blocks), a.n_jobs), dim3(256), 0, st, a);
}

void launch_project(const ProjArgs &a, bool fit, hipStream_t st) {
    if (a.n_jobs == 0) return;
    if (fit) hipLaunchKernelGGL(k_project, dim3(kNBasis, a.n_jobs), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_residual, dim3(a.n_jobs), dim3(256), 0, st, a);
}

void launch_budget(const BudgetArgs &a, hipStream_t st) {
    if (a.n_jobs == 0) return;
    hipLaunchKernelGGL(k_budget, dim3(a.n_jobs), dim3(256), 0, st, a);
}

void launch_correct(const CorrArgs &a, hipStream_t st) {
    if (a.n_jobs == 0 || a.max_pts == 0) return;
    hipLaunchKernelGGL(k_correct, dim3(unsigned((a.max_pts + 255) / 256)), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
// Judge by sample (see SampleJob): the plain pair field at 64 target points by
// the direct sum over the source's real-space history, and its comparison
// with the surrogate terms.

__device__ __forceinline__ int sample_index(int a, int n) { return (a * (n - 1) + 1) / 3; }

// Grid (64 / kSampleGroup, jobs): each block sums kSampleGroup target points
// over every source point (a strided share per thread, FP32 partial sums,
// FP64 across the block); geometry in FP64.
__global__ __launch_bounds__(256) void k_pair_sample(SampleArgs a) {
    const SampleJob &j = a.jobs[blockIdx.y];
    const int p0 = blockIdx.x * kSampleGroup;
    const int Ny = j.Nn[1], Nz = j.Nn[2];
    const int64_t npts = int64_t(j.Nn[0]) * Ny * Nz;
    double tx[kSampleGroup], ty[kSampleGroup], tz[kSampleGroup];
#pragma unroll
    for (int q = 0; q < kSampleGroup; ++q) {
        const int p = p0 + q;
        tx[q] = j.t0[0] + sample_index(p >> 4, j.Ns[0]);
        ty[q] = j.t0[1] + sample_index((p >> 2) & 3, j.Ns[1]);
        tz[q] = j.t0[2] + sample_index(p & 3, j.Ns[2]);
    }
    const int head = *j.head;
    const int depth = j.depth;
    const double lag_per_cell = a.h * a.inv_cdt;   // R / (c dt) per grid unit of distance
    float acc[kSampleGroup][4] = {};
    for (int64_t i = threadIdx.x; i < npts; i += 256) {
        const int iz = int(i % Nz);
        const int64_t r = i / Nz;
        const int iy = int(r % Ny);
        const int ix = int(r / Ny);
        float s0[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) s0[mu] = j.s0[mu * npts + i];
#pragma unroll
        for (int q = 0; q < kSampleGroup; ++q) {
            const double dx = tx[q] - ix, dy = ty[q] - iy, dz = tz[q] - iz;
            const double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (!(d > 0.0)) continue;
            const double tau = d * lag_per_cell;
            int m = int(floor(tau));
            const float f = float(tau - double(m));
            m = min(m, depth - 2);          // stays in the ring (the windows keep m + 1 < depth)
            int sa = head - m;
            if (sa < 0) sa += depth;
            const int sb = sa == 0 ? depth - 1 : sa - 1;
            const float *A = j.hist + int64_t(sa) * 4 * npts + i;
            const float *B = j.hist + int64_t(sb) * 4 * npts + i;
            const float w = a.h3 / float(d * a.h);
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
                acc[q][mu] = fmaf(w, fmaf(1.f - f, A[mu * npts], fmaf(f, B[mu * npts], -s0[mu])), acc[q][mu]);
        }
    }
    __shared__ double red[4][kSampleGroup * 4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kSampleGroup; ++q)
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            double v = acc[q][mu];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) red[wv][q * 4 + mu] = v;
        }
    __syncthreads();
    if (threadIdx.x < kSampleGroup * 4) {
        const int t = threadIdx.x;
        j.out[int64_t(p0) * 4 + t] = float(red[0][t] + red[1][t] + red[2][t] + red[3][t]);
    }
}

// Block per sampled pair, one thread per sample point.
__global__ __launch_bounds__(64) void k_sample_judge(SampleJudgeArgs a) {
    const SampleJudgeJob &j = a.jobs[blockIdx.x];
    const int p = threadIdx.x;
    const int ix = sample_index(p >> 4, j.N[0]), iy = sample_index((p >> 2) & 3, j.N[1]),
              iz = sample_index(p & 3, j.N[2]);
    float B[kNBasis];
    basis_at((int64_t(ix) * j.N[1] + iy) * j.N[2] + iz, j.N, B);
    __shared__ float red[64];
    bool bad = false;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        float v = 0.f;
#pragma unroll
        for (int b = 0; b < kNBasis; ++b) v = fmaf(j.pc[mu * kNBasis + b], B[b], v);
        const float F = j.F[p * 4 + mu];
        const float x = block_max<64>(fabsf(F - v), red);
        const float y = block_max<64>(fabsf(F), red);
        if (p == 0) {
            j.resid[mu] = x;
            j.resid[4 + mu] = y;
        }
        bad |= x > j.budget[mu];
    }
    if (p == 0) *j.fail = (j.active && bad) ? 1 : 0;
}

void launch_pair_sample(const SampleArgs &a, hipStream_t st) {
    for (int j0 = 0; j0 < a.n_jobs; j0 += 65535) {
        SampleArgs c = a;
        c.jobs = a.jobs + j0;
        c.n_jobs = std::min(65535, a.n_jobs - j0);
        hipLaunchKernelGGL(k_pair_sample, dim3(kSamplePts / kSampleGroup, c.n_jobs), dim3(256), 0, st, c);
    }
}

void launch_sample_judge(const SampleJudgeArgs &a, hipStream_t st) {
    if (a.n_jobs == 0) return;
    hipLaunchKernelGGL(k_sample_judge, dim3(a.n_jobs), dim3(64), 0, st, a);
}

// ---------------------------------------------------------------------------
// Training data of the network (teacher rows, scales, scaling).

// Row r of the audited far pairs: inputs x_out[r] = x_all[far index of r],
// targets t[r] = (t[r] - sub[r]) * |c_s - c_n| (sub: the multipole terms, or null).
__global__ void k_teacher(TeacherArgs a) {
    const int r = blockIdx.x;
    const int f = a.row_far[r];
    const float *src = a.x_all + int64_t(f) * a.n_in;
    float *dst = a.x_out + int64_t(r) * a.n_in;
    for (int j = threadIdx.x; j < a.n_in; j += blockDim.x) dst[j] = src[j];
    if (threadIdx.x < kNOut) {
        float *t = a.t + int64_t(r) * kNOut + threadIdx.x;
        float v = *t;
        if (a.sub) v -= a.sub[int64_t(r) * kNOut + threadIdx.x];
        *t = v / a.pairs[f].inv_d;
    }
}

void launch_teacher(const TeacherArgs &a, hipStream_t st) {
    if (a.n_rows == 0) return;
    hipLaunchKernelGGL(k_teacher, dim3(a.n_rows), dim3(256), 0, st, a);
}

// Scales of the training data.  Block 0: moment k of the unmodulated block H
// (columns lag * kNFeat + k, lag < n_lags), 1 / RMS over rows and lags; block
// 1: component c of the targets (columns c * kNBasis + b), RMS over rows and
// the kNBasis coefficients, repeated over the component's columns.  Each
// thread keeps one column class; the sums are FP64 in a fixed order
// (threads stride rows, then a fixed tree over the threads of a class).
constexpr int kScaleLanesIn = 32;    // threads per moment class (block 0: 22 x 32)
constexpr int kScaleLanesOut = 8;    // threads per target column (block 1: 80 x 8)
__global__ __launch_bounds__(704) void k_data_scales(ScaleDataArgs a) {
    __shared__ double part[kNFeat * kScaleLanesIn];
    const int t = threadIdx.x;
    double s = 0.0;
    if (blockIdx.x == 0) {
        // thread t reads columns t, t + 704, ... of the block H: all of moment t % 22
        const int cols = a.n_lags * kNFeat;
        for (int64_t i = 0; i < a.n; ++i) {
            const float *row = a.x + i * a.n_in;
            for (int j = t; j < cols; j += kNFeat * kScaleLanesIn) {
                const double v = row[j];
                s += v * v;
            }
        }
    } else if (t < kNOut * kScaleLanesOut) {
        // thread t: column t % 80, rows t / 80, t / 80 + 8, ...
        const int col = t % kNOut, lane = t / kNOut;
        for (int64_t i = lane; i < a.n; i += kScaleLanesOut) {
            const double v = a.t[i * kNOut + col];
            s += v * v;
        }
    }
    part[t] = s;
    __syncthreads();
    if (blockIdx.x == 0 && t < kNFeat) {
        double tot = 0.0;
        for (int l = 0; l < kScaleLanesIn; ++l) tot += part[t + l * kNFeat];
        const double rms = sqrt(tot / (double(a.n) * double(a.n_lags)));
        a.in_scale[t] = rms > 0.0 ? float(1.0 / rms) : 1.0f;
    }
    if (blockIdx.x == 1 && t < 4) {
        double tot = 0.0;
        for (int l = 0; l < kScaleLanesOut; ++l)
            for (int b = 0; b < kNBasis; ++b) tot += part[l * kNOut + t * kNBasis + b];
        const double rms = sqrt(tot / (double(a.n) * kNBasis));
        const float v = rms > 0.0 ? float(rms) : 1.0f;
        for (int b = 0; b < kNBasis; ++b) a.out_scale[t * kNBasis + b] = v;
    }
}

void launch_data_scales(const ScaleDataArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_data_scales, dim3(2), dim3(kNFeat * kScaleLanesIn), 0, st, a);
}

// In place: the six moment blocks of every input row times in_scale (per
// moment), every target row over out_scale (per column).
__global__ void k_scale_data(ScaleDataArgs a) {
    const int64_t i = blockIdx.y;
    const int blocks = 6 * a.n_lags * kNFeat;
    if (a.x_rw) {
        float *x = a.x_rw + i * a.n_in;
        for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < blocks; j += gridDim.x * blockDim.x)
            x[j] *= a.in_scale_c[j % kNFeat];
    }
    if (a.t_rw && blockIdx.x == 0 && threadIdx.x < kNOut)
        a.t_rw[i * kNOut + threadIdx.x] /= a.out_scale_c[threadIdx.x];
}

void launch_scale_data(const ScaleDataArgs &a, hipStream_t st) {
    if (a.n == 0) return;
    const int blocks = 6 * a.n_lags * kNFeat;
    hipLaunchKernelGGL(k_scale_data, dim3(unsigned(std::max(1, std::min(8, (blocks + 255) / 256))), unsigned(a.n)),
                       dim3(256), 0, st, a);
}

}  // namespace rpot
