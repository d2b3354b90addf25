// Model response of the sources: the steps either side of the potential
// evaluation in the propagation loop (Fig. 4), with Lorentz oscillators in
// place of the Kohn-Sham dynamics.
//
// Oscillator k of a domain has a fixed shape B_k [4][N] (component 0: charge
// per unit q, components 1-3: current / c per unit dq/dt) and the amplitude q_k.
// Per step, from the potentials P of step l:
//   phi_k = h^3 sum_r B_k[0] v,  psi_k = h^3 sum_r sum_a B_k[1+a] A_a   (k_osc_project, k_osc_advance)
//   F_k   = -phi_k - (psi_k - psi_k(l-1)) / dt + drive_k e_ext
//   qdot += dt (kappa F - gamma qdot - omega^2 q);  q += dt qdot        (k_osc_advance)
//   S(l+1) = (sum_k q_k B_k[0], sum_k qdot_k B_k[1..3])                 (k_osc_synth)
// The generalised force of the potentials on the shape comes from the
// interaction Lagrangian -int rho v + int (J/c).A; the current of step l thus
// drives the vector potential of step l + 1, as in the paper's loop (Sec. II).
//
// Both passes stream the shapes once: they are HBM-bound matrix-vector
// products (K x 4N), coalesced along the points, with a fixed-order FP64
// reduction of the block partials.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "plan_internal.hpp"
#include "rpot.h"

namespace {

constexpr int kOscJobs = 16;      // domains per launch
constexpr int kOscMaxK = 256;     // oscillators per domain
constexpr int kOscThreads = 256;  // 4 waves
constexpr int kOscPerThread = 4;  // points per thread
constexpr int kOscPts = kOscThreads * kOscPerThread;

template <typename T>
struct OscJob {
    const T *basis;  // [K][4][N]
    const T *pot;    // [4][N]
    T *src;          // [4][N]
    int64_t npts;
    int K;
    int osc_base;    // global index of the domain's first oscillator
    int blk_base;    // first block of this job in the launch
    int nblk;        // blocks of this domain
    int64_t part_base;  // partials of oscillator k: part_base + k * nblk + b
};

template <typename T>
struct OscArgs {
    OscJob<T> jobs[kOscJobs];
    int n_jobs;
    double *part;           // [..][2] (phi, psi) partials
    const double *state;    // q [n_osc], qdot [n_osc]
    int n_osc;
};

struct OscMeta {
    int64_t part;  // first partial of this oscillator
    int nblk;
};

template <typename T>
__device__ __forceinline__ int find_job(const OscArgs<T> &a, int b) {
    int j = 0;
    while (j + 1 < a.n_jobs && b >= a.jobs[j + 1].blk_base) ++j;
    return j;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block partials of phi_k and psi_k over kOscPts points of one domain.
template <typename T>
__global__ void __launch_bounds__(kOscThreads) k_osc_project(OscArgs<T> a) {
    __shared__ double red[kOscThreads / 64][kOscMaxK][2];
    const int j = find_job(a, blockIdx.x);
    const OscJob<T> &J = a.jobs[j];
    const int b = blockIdx.x - J.blk_base;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t N = J.npts;
    const int64_t p0 = int64_t(b) * kOscPts + t;
    T v[kOscPerThread], A[3][kOscPerThread];
#pragma unroll
    for (int i = 0; i < kOscPerThread; ++i) {
        const int64_t p = p0 + int64_t(i) * kOscThreads;
        const bool in = p < N;
        v[i] = in ? J.pot[p] : T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) A[c][i] = in ? J.pot[(1 + c) * N + p] : T(0);
    }
    for (int k = 0; k < J.K; ++k) {
        const T *B = J.basis + int64_t(k) * 4 * N;
        T sphi = T(0), spsi = T(0);
#pragma unroll
        for (int i = 0; i < kOscPerThread; ++i) {
            const int64_t p = p0 + int64_t(i) * kOscThreads;
            if (p < N) {
                sphi += B[p] * v[i];
                spsi += B[N + p] * A[0][i] + B[2 * N + p] * A[1][i] + B[3 * N + p] * A[2][i];
            }
        }
        const double wphi = wave_sum(double(sphi));
        const double wpsi = wave_sum(double(spsi));
        if (lane == 0) {
            red[wave][k][0] = wphi;
            red[wave][k][1] = wpsi;
        }
    }
    __syncthreads();
    for (int k = t; k < J.K; k += kOscThreads) {
        double sphi = 0.0, spsi = 0.0;
#pragma unroll
        for (int w = 0; w < kOscThreads / 64; ++w) {
            sphi += red[w][k][0];
            spsi += red[w][k][1];
        }
        double *out = a.part + 2 * (J.part_base + int64_t(k) * J.nblk + b);
        out[0] = sphi;
        out[1] = spsi;
    }
}

// One wave per oscillator: its partials summed in a fixed order (lane-strided
// then the wave tree), then the force and the update by lane 0.
// state: q [n], qdot [n], psi_prev [n], phi [n], psi [n].
__global__ void __launch_bounds__(64) k_osc_advance(const OscMeta *meta, const double *params, const double *part,
                                                    double *state, int n, double w, double dt, double e_ext,
                                                    int first) {
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    const OscMeta m = meta[i];
    double phi = 0.0, psi = 0.0;
    for (int b = lane; b < m.nblk; b += 64) {
        phi += part[2 * (m.part + b)];
        psi += part[2 * (m.part + b) + 1];
    }
    phi = wave_sum(phi) * w;
    psi = wave_sum(psi) * w;
    if (lane != 0) return;
    const double psi_prev = first ? psi : state[2 * n + i];
    const double omega = params[4 * i], gamma = params[4 * i + 1], kappa = params[4 * i + 2],
                 drive = params[4 * i + 3];
    const double q = state[i], qd = state[n + i];
    const double F = -phi - (psi - psi_prev) / dt + drive * e_ext;
    const double qd1 = qd + dt * (kappa * F - gamma * qd - omega * omega * q);
    state[i] = q + dt * qd1;
    state[n + i] = qd1;
    state[2 * n + i] = psi;
    state[3 * n + i] = phi;
    state[4 * n + i] = psi;
}

// Sources from the amplitudes: S[0] = sum_k q_k B_k[0], S[1+a] = sum_k qdot_k B_k[1+a].
template <typename T>
__global__ void __launch_bounds__(kOscThreads) k_osc_synth(OscArgs<T> a) {
    __shared__ T amp[kOscMaxK][2];
    const int j = find_job(a, blockIdx.x);
    const OscJob<T> &J = a.jobs[j];
    const int b = blockIdx.x - J.blk_base;
    const int t = threadIdx.x;
    for (int k = t; k < J.K; k += kOscThreads) {
        amp[k][0] = T(a.state[J.osc_base + k]);
        amp[k][1] = T(a.state[a.n_osc + J.osc_base + k]);
    }
    __syncthreads();
    const int64_t N = J.npts;
    const int64_t p0 = int64_t(b) * kOscPts + t;
    T s[4][kOscPerThread];
#pragma unroll
    for (int i = 0; i < kOscPerThread; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c][i] = T(0);
    for (int k = 0; k < J.K; ++k) {
        const T *B = J.basis + int64_t(k) * 4 * N;
        const T q = amp[k][0], qd = amp[k][1];
#pragma unroll
        for (int i = 0; i < kOscPerThread; ++i) {
            const int64_t p = p0 + int64_t(i) * kOscThreads;
            if (p < N) {
                s[0][i] += q * B[p];
                s[1][i] += qd * B[N + p];
                s[2][i] += qd * B[2 * N + p];
                s[3][i] += qd * B[3 * N + p];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kOscPerThread; ++i) {
        const int64_t p = p0 + int64_t(i) * kOscThreads;
        if (p < N)
#pragma unroll
            for (int c = 0; c < 4; ++c) J.src[c * N + p] = s[c][i];
    }
}

struct OErr {
    rp_status code;
    std::string msg;
};

[[noreturn]] void ofail(rp_status c, const std::string &m) { throw OErr{c, m}; }

thread_local std::string g_osc_create_error;

}  // namespace

struct rp_osc_s {
    int n_dom = 0, n_osc = 0;
    bool p64 = false;
    double h = 0, dt = 0;
    hipStream_t stream = nullptr;
    std::vector<int> K, osc_base, nblk;
    std::vector<int64_t> npts, part_base;
    std::vector<double> params;  // [n_osc][4]
    std::vector<const void *> basis;
    size_t off_state = 0, off_part = 0, off_meta = 0, off_params = 0, ws_bytes = 0;
    char *ws = nullptr;
    bool first = true;
    std::string err;
    double *state() { return reinterpret_cast<double *>(ws + off_state); }
};

namespace {

template <typename F>
rp_status oguard(rp_osc o, F &&fn) {
    if (!o) return RP_ERR_ARG;
    try {
        o->err.clear();
        fn();
        return RP_OK;
    } catch (const OErr &e) {
        o->err = e.msg;
        return e.code;
    } catch (...) {
        o->err = "unknown error";
        return RP_ERR_ARG;
    }
}

void ohip(hipError_t e, const char *what) {
    if (e != hipSuccess) ofail(RP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void check_launch() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) ofail(RP_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

void need_bound(rp_osc o) {
    if (!o->ws) ofail(RP_ERR_STATE, "workspace not bound");
}

// Jobs of domains [d0, d0 + cnt) with the given per-domain arrays; returns blocks.
template <typename T>
int fill_jobs(rp_osc o, OscArgs<T> &a, int d0, int cnt, const void *const *pot, void *const *src) {
    int blocks = 0;
    a.n_jobs = cnt;
    a.part = reinterpret_cast<double *>(o->ws + o->off_part);
    a.state = o->state();
    a.n_osc = o->n_osc;
    for (int j = 0; j < cnt; ++j) {
        const int n = d0 + j;
        OscJob<T> &J = a.jobs[j];
        J.basis = static_cast<const T *>(o->basis[n]);
        J.pot = pot ? static_cast<const T *>(pot[n]) : nullptr;
        J.src = src ? static_cast<T *>(src[n]) : nullptr;
        J.npts = o->npts[n];
        J.K = o->K[n];
        J.osc_base = o->osc_base[n];
        J.blk_base = blocks;
        J.nblk = o->nblk[n];
        J.part_base = o->part_base[n];
        blocks += o->nblk[n];
    }
    return blocks;
}

template <typename T>
void enqueue_project(rp_osc o, const void *const *pot) {
    for (int d0 = 0; d0 < o->n_dom; d0 += kOscJobs) {
        OscArgs<T> a{};
        const int blocks = fill_jobs<T>(o, a, d0, std::min(kOscJobs, o->n_dom - d0), pot, nullptr);
        hipLaunchKernelGGL(k_osc_project<T>, dim3(blocks), dim3(kOscThreads), 0, o->stream, a);
    }
}

template <typename T>
void enqueue_synth(rp_osc o, void *const *src) {
    for (int d0 = 0; d0 < o->n_dom; d0 += kOscJobs) {
        OscArgs<T> a{};
        const int blocks = fill_jobs<T>(o, a, d0, std::min(kOscJobs, o->n_dom - d0), nullptr, src);
        hipLaunchKernelGGL(k_osc_synth<T>, dim3(blocks), dim3(kOscThreads), 0, o->stream, a);
    }
}

void check_ptrs(rp_osc o, const void *const *arr, const char *what) {
    if (!arr) ofail(RP_ERR_ARG, std::string(what) + " is null");
    for (int n = 0; n < o->n_dom; ++n)
        if (!arr[n]) ofail(RP_ERR_ARG, std::string(what) + " has a null entry");
}

}  // namespace

extern "C" {

rp_status rp_osc_create(rp_osc *out, rp_plan plan, const int32_t *n_osc, const double *params) {
    if (!out) {
        g_osc_create_error = "out is null";
        return RP_ERR_ARG;
    }
    *out = nullptr;
    if (!plan || !n_osc) {
        g_osc_create_error = "plan or n_osc is null";
        return RP_ERR_ARG;
    }
    rp_osc o = new (std::nothrow) rp_osc_s();
    if (!o) return RP_ERR_NOMEM;
    o->n_dom = plan->n_dom;
    o->p64 = plan->p64;
    o->h = plan->h;
    o->dt = plan->dt;
    o->stream = plan->stream;
    int64_t parts = 0;
    for (int n = 0; n < o->n_dom; ++n) {
        if (n_osc[n] < 0 || n_osc[n] > kOscMaxK) {
            g_osc_create_error = "oscillators per domain must be in [0, 256]";
            delete o;
            return RP_ERR_ARG;
        }
        const int64_t N = plan->dom[n].npts;
        o->K.push_back(n_osc[n]);
        o->npts.push_back(N);
        o->osc_base.push_back(o->n_osc);
        o->nblk.push_back(int((N + kOscPts - 1) / kOscPts));
        o->part_base.push_back(parts);
        parts += int64_t(n_osc[n]) * o->nblk.back();
        o->n_osc += n_osc[n];
    }
    if (o->n_osc > 0 && !params) {
        g_osc_create_error = "params is null";
        delete o;
        return RP_ERR_ARG;
    }
    o->params.assign(params, params + 4 * size_t(o->n_osc));
    for (int i = 0; i < o->n_osc; ++i) {
        const double *p = &o->params[4 * size_t(i)];
        bool ok = std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]) && std::isfinite(p[3]) &&
                  p[0] >= 0 && p[1] >= 0;
        // semi-implicit Euler is stable for omega dt < 2
        if (ok && !(p[0] * o->dt < 2.0)) ok = false;
        if (!ok) {
            g_osc_create_error = "oscillator " + std::to_string(i) +
                                 ": params must be finite, omega and gamma >= 0, omega dt < 2";
            delete o;
            return RP_ERR_ARG;
        }
    }
    size_t off = 0;
    auto alloc = [&](size_t bytes) {
        const size_t r = off;
        off += (bytes + 255) / 256 * 256;
        return r;
    };
    o->off_state = alloc(5 * sizeof(double) * size_t(std::max(o->n_osc, 1)));
    o->off_part = alloc(2 * sizeof(double) * size_t(std::max<int64_t>(parts, 1)));
    o->off_meta = alloc(sizeof(OscMeta) * size_t(std::max(o->n_osc, 1)));
    o->off_params = alloc(4 * sizeof(double) * size_t(std::max(o->n_osc, 1)));
    o->ws_bytes = off;
    *out = o;
    return RP_OK;
}

rp_status rp_osc_workspace_bytes(rp_osc o, size_t *bytes) {
    return oguard(o, [&] {
        if (!bytes) ofail(RP_ERR_ARG, "bytes is null");
        *bytes = o->ws_bytes;
    });
}

rp_status rp_osc_bind(rp_osc o, void *dev, size_t bytes, const void *const *basis) {
    return oguard(o, [&] {
        if (!dev || reinterpret_cast<uintptr_t>(dev) % 256) ofail(RP_ERR_ARG, "workspace must be 256-byte aligned");
        if (bytes < o->ws_bytes) ofail(RP_ERR_NOMEM, "workspace smaller than rp_osc_workspace_bytes");
        if (!basis) ofail(RP_ERR_ARG, "basis is null");
        for (int n = 0; n < o->n_dom; ++n)
            if (o->K[n] > 0 && !basis[n]) ofail(RP_ERR_ARG, "basis of a domain with oscillators is null");
        o->basis.assign(basis, basis + o->n_dom);
        o->ws = static_cast<char *>(dev);
        std::vector<OscMeta> meta(size_t(o->n_osc));
        for (int n = 0; n < o->n_dom; ++n)
            for (int k = 0; k < o->K[n]; ++k)
                meta[size_t(o->osc_base[n] + k)] = OscMeta{o->part_base[n] + int64_t(k) * o->nblk[n], o->nblk[n]};
        std::vector<double> zero(5 * size_t(o->n_osc), 0.0);
        if (o->n_osc > 0) {
            ohip(hipMemcpyAsync(o->ws + o->off_meta, meta.data(), meta.size() * sizeof(OscMeta), hipMemcpyHostToDevice,
                                o->stream), "upload");
            ohip(hipMemcpyAsync(o->ws + o->off_params, o->params.data(), o->params.size() * sizeof(double),
                                hipMemcpyHostToDevice, o->stream), "upload");
            ohip(hipMemcpyAsync(o->state(), zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice, o->stream),
                 "upload");
        }
        ohip(hipStreamSynchronize(o->stream), "synchronize");
        o->first = true;
    });
}

rp_status rp_osc_set_state(rp_osc o, const double *q, const double *qdot) {
    return oguard(o, [&] {
        need_bound(o);
        if (!q || !qdot) ofail(RP_ERR_ARG, "q or qdot is null");
        if (o->n_osc > 0) {
            ohip(hipMemcpyAsync(o->state(), q, sizeof(double) * o->n_osc, hipMemcpyHostToDevice, o->stream), "upload");
            ohip(hipMemcpyAsync(o->state() + o->n_osc, qdot, sizeof(double) * o->n_osc, hipMemcpyHostToDevice,
                                o->stream), "upload");
        }
        ohip(hipStreamSynchronize(o->stream), "synchronize");
        o->first = true;
    });
}

rp_status rp_osc_sources(rp_osc o, void *const *src) {
    return oguard(o, [&] {
        need_bound(o);
        check_ptrs(o, src, "src");
        if (o->p64)
            enqueue_synth<double>(o, src);
        else
            enqueue_synth<float>(o, src);
        check_launch();
    });
}

rp_status rp_osc_step(rp_osc o, const void *const *pot, double e_ext, void *const *src_next) {
    return oguard(o, [&] {
        need_bound(o);
        check_ptrs(o, pot, "pot");
        check_ptrs(o, src_next, "src_next");
        if (!std::isfinite(e_ext)) ofail(RP_ERR_ARG, "e_ext must be finite");
        if (o->p64)
            enqueue_project<double>(o, pot);
        else
            enqueue_project<float>(o, pot);
        if (o->n_osc > 0)
            hipLaunchKernelGGL(k_osc_advance, dim3(o->n_osc), dim3(64), 0, o->stream,
                               reinterpret_cast<const OscMeta *>(o->ws + o->off_meta),
                               reinterpret_cast<const double *>(o->ws + o->off_params),
                               reinterpret_cast<const double *>(o->ws + o->off_part), o->state(), o->n_osc,
                               o->h * o->h * o->h, o->dt, e_ext, o->first ? 1 : 0);
        if (o->p64)
            enqueue_synth<double>(o, src_next);
        else
            enqueue_synth<float>(o, src_next);
        check_launch();
        o->first = false;
    });
}

rp_status rp_osc_state(rp_osc o, double *q, double *qdot, double *phi, double *psi) {
    return oguard(o, [&] {
        need_bound(o);
        double *dst[4] = {q, qdot, phi, psi};
        const int slot[4] = {0, 1, 3, 4};
        for (int i = 0; i < 4; ++i)
            if (dst[i] && o->n_osc > 0)
                ohip(hipMemcpyAsync(dst[i], o->state() + size_t(slot[i]) * o->n_osc, sizeof(double) * o->n_osc,
                                    hipMemcpyDeviceToHost, o->stream), "download");
        ohip(hipStreamSynchronize(o->stream), "synchronize");
    });
}

rp_status rp_osc_destroy(rp_osc o) {
    if (!o) return RP_ERR_ARG;
    delete o;
    return RP_OK;
}

const char *rp_osc_last_error(rp_osc o) {
    if (!o) return g_osc_create_error.c_str();
    return o->err.c_str();
}

}  // extern "C"
