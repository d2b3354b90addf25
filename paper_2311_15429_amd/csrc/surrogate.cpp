// Host side of the learned far-pair surrogate: pair classification, frames
// and basis maps, workspace, the per-step moment and inference launches, the
// plain pair responses that train and judge the network, and the fallback.
//
// A pair (s <- n) is far when its centre distance exceeds far_factor times
// the larger of the two box diagonals.  Far pairs leave the plain lag sum;
// their sources keep only a ring of moments, not of spectra, unless they are
// audit sources: those keep the plain history of all their pairs, so their
// far pairs can be judged against the plain sum and can fall back to it.
#include "plan_internal.hpp"

#include <algorithm>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstring>

using namespace rpot;

namespace rpot_host {

namespace {

const int kDeg[kNBasis][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 0, 3}, {0, 1, 0}, {0, 1, 1}, {0, 1, 2},
                              {0, 2, 0}, {0, 2, 1}, {0, 3, 0}, {1, 0, 0}, {1, 0, 1}, {1, 0, 2}, {1, 1, 0},
                              {1, 1, 1}, {1, 2, 0}, {2, 0, 0}, {2, 0, 1}, {2, 1, 0}, {3, 0, 0}};

void legendre(double x, double (&p)[4]) {
    p[0] = 1.0;
    p[1] = x;
    p[2] = 0.5 * (3.0 * x * x - 1.0);
    p[3] = 0.5 * x * (5.0 * x * x - 3.0);
}

void basis_row(const double (&x)[3], double *B) {
    double px[4], py[4], pz[4];
    legendre(x[0], px);
    legendre(x[1], py);
    legendre(x[2], pz);
    for (int b = 0; b < kNBasis; ++b) B[b] = px[kDeg[b][0]] * py[kDeg[b][1]] * pz[kDeg[b][2]];
}

// Inverse of the symmetric positive definite n x n matrix G (Cholesky).
std::vector<double> spd_inverse(std::vector<double> G, int n) {
    std::vector<double> L(size_t(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = G[size_t(j) * n + j];
        for (int k = 0; k < j; ++k) d -= L[size_t(j) * n + k] * L[size_t(j) * n + k];
        if (!(d > 0)) fail(RP_ERR_UNSUPPORTED, "surrogate basis is singular on this grid");
        L[size_t(j) * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double v = G[size_t(i) * n + j];
            for (int k = 0; k < j; ++k) v -= L[size_t(i) * n + k] * L[size_t(j) * n + k];
            L[size_t(i) * n + j] = v / L[size_t(j) * n + j];
        }
    }
    std::vector<double> inv(size_t(n) * n, 0.0);
    for (int c = 0; c < n; ++c) {
        std::vector<double> y(n, 0.0);
        for (int i = 0; i < n; ++i) {   // L y = e_c
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[size_t(i) * n + k] * y[k];
            y[i] = v / L[size_t(i) * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {   // L^T x = y
            double v = y[i];
            for (int k = i + 1; k < n; ++k) v -= L[size_t(k) * n + i] * inv[size_t(k) * n + c];
            inv[size_t(i) * n + c] = v / L[size_t(i) * n + i];
        }
    }
    return inv;
}

// X = argmin |A X - Y| for A [m][kNBasis], Y [m][kNBasis] (normal equations).
std::vector<double> lsq20(const std::vector<double> &A, const std::vector<double> &Y, int m) {
    const int n = kNBasis;
    std::vector<double> G(size_t(n) * n, 0.0), R(size_t(n) * n, 0.0);
    for (int r = 0; r < m; ++r)
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                G[size_t(i) * n + j] += A[size_t(r) * n + i] * A[size_t(r) * n + j];
                R[size_t(i) * n + j] += A[size_t(r) * n + i] * Y[size_t(r) * n + j];
            }
        }
    const std::vector<double> Gi = spd_inverse(G, n);
    std::vector<double> X(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) X[size_t(i) * n + j] += Gi[size_t(i) * n + k] * R[size_t(k) * n + j];
    return X;
}

double centre(rp_plan p, int i, int a) { return p->dom[i].o[a] + 0.5 * p->h * (p->dom[i].N[a] - 1); }

double diagonal(rp_plan p, int i) {
    double d2 = 0;
    for (int a = 0; a < 3; ++a) {
        const double e = p->h * (p->dom[i].N[a] - 1);
        d2 += e * e;
    }
    return std::sqrt(d2);
}

// Right-handed frame with e1 along d (rows of R).
void make_frame(const double (&d)[3], double (&R)[9]) {
    const double L = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double e1[3] = {d[0] / L, d[1] / L, d[2] / L};
    double a[3] = {0, 0, 1};
    if (std::fabs(e1[2]) > 0.9) a[0] = 1, a[2] = 0;
    const double ad = a[0] * e1[0] + a[1] * e1[1] + a[2] * e1[2];
    double e2[3] = {a[0] - ad * e1[0], a[1] - ad * e1[1], a[2] - ad * e1[2]};
    const double n2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    for (double &v : e2) v /= n2;
    const double e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    for (int i = 0; i < 3; ++i) {
        R[i] = e1[i];
        R[3 + i] = e2[i];
        R[6 + i] = e3[i];
    }
}

// Basis maps of a far pair.  The network's frame basis is the same
// tensor-Legendre set in u = R (r - c_s) / ell (ell = the target's largest
// half side); both sets span the polynomials of total degree <= 3, so the
// maps are exact: M takes frame coefficients to box coefficients, Minv back.
void pair_maps(rp_plan p, const FarPairH &F, float *M, float *Minv) {
    const DomainP &t = p->dom[F.s];
    double hw[3], ell = 0;
    for (int a = 0; a < 3; ++a) {
        hw[a] = 0.5 * p->h * (t.N[a] - 1);
        ell = std::max(ell, hw[a]);
    }
    const double nodes[4] = {-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0};
    const int m = 64;
    std::vector<double> Bb(size_t(m) * kNBasis), Bf(size_t(m) * kNBasis);
    int r = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k, ++r) {
                const double xi[3] = {nodes[i], nodes[j], nodes[k]};
                basis_row(xi, &Bb[size_t(r) * kNBasis]);
                const double d[3] = {xi[0] * hw[0], xi[1] * hw[1], xi[2] * hw[2]};
                double u[3];
                for (int a = 0; a < 3; ++a)
                    u[a] = (F.rot[3 * a] * d[0] + F.rot[3 * a + 1] * d[1] + F.rot[3 * a + 2] * d[2]) / ell;
                basis_row(u, &Bf[size_t(r) * kNBasis]);
            }
    const std::vector<double> X = lsq20(Bb, Bf, m), Xi = lsq20(Bf, Bb, m);
    for (int i = 0; i < kNBasis * kNBasis; ++i) {
        M[i] = float(X[i]);
        Minv[i] = float(Xi[i]);
    }
}

// LS dual basis of an N-grid box: Q = (B^T B)^-1 B^T, [kNBasis][npts].
std::vector<float> dual_basis(const int (&N)[3]) {
    const int64_t npts = int64_t(N[0]) * N[1] * N[2];
    std::vector<double> B(size_t(npts) * kNBasis);
    std::vector<double> G(kNBasis * kNBasis, 0.0);
    for (int64_t i = 0; i < npts; ++i) {
        const int iz = int(i % N[2]), iy = int((i / N[2]) % N[1]), ix = int(i / (int64_t(N[2]) * N[1]));
        const double x[3] = {2.0 * ix / (N[0] - 1) - 1.0, 2.0 * iy / (N[1] - 1) - 1.0, 2.0 * iz / (N[2] - 1) - 1.0};
        double *row = &B[size_t(i) * kNBasis];
        basis_row(x, row);
        for (int a = 0; a < kNBasis; ++a)
            for (int b = 0; b < kNBasis; ++b) G[a * kNBasis + b] += row[a] * row[b];
    }
    const std::vector<double> Gi = spd_inverse(G, kNBasis);
    std::vector<float> Q(size_t(kNBasis) * npts);
    for (int64_t i = 0; i < npts; ++i)
        for (int a = 0; a < kNBasis; ++a) {
            double v = 0;
            for (int b = 0; b < kNBasis; ++b) v += Gi[a * kNBasis + b] * B[size_t(i) * kNBasis + b];
            Q[size_t(a) * npts + i] = float(v);
        }
    return Q;
}

void upload_csr(rp_plan p, hipStream_t st) {
    SurrogateH &U = p->sur;
    const int nd = p->n_dom;
    U.h_order.clear();
    U.h_tbeg.assign(nd + 1, 0);
    std::vector<std::vector<int32_t>> by_t(nd);
    for (size_t f = 0; f < U.pairs.size(); ++f)
        if (!U.pairs[f].plain) by_t[U.pairs[f].s].push_back(int32_t(f));
    for (int s = 0; s < nd; ++s) {
        U.h_tbeg[s] = int32_t(U.h_order.size());
        U.h_order.insert(U.h_order.end(), by_t[s].begin(), by_t[s].end());
    }
    U.h_tbeg[nd] = int32_t(U.h_order.size());
    if (!U.h_order.empty())
        HIP_OK(hipMemcpyAsync(p->ws + U.off_order, U.h_order.data(), U.h_order.size() * 4, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(p->ws + U.off_tbeg, U.h_tbeg.data(), U.h_tbeg.size() * 4, hipMemcpyHostToDevice, st));
}

int active_far(rp_plan p, int s) {
    int n = 0;
    for (const FarPairH &F : p->sur.pairs) n += (F.s == s && !F.plain);
    return n;
}

// Plain pair fields of the audited far pairs at the last completed step: the
// judge lag sum (ring heads of that step), then per batch of up to kMaxJobs
// pairs with one target shape the inverse transform and crop into the judge
// field buffers; fn(batch, count) is called after each batch is enqueued.
template <typename Fn>
void judge_fields(rp_plan p, hipStream_t st, Fn &&fn) {
    SurrogateH &U = p->sur;
    enqueue_k2(p, k2_args(p, U.judge, U.judge_dev, p->at<int32_t>(p->off_prev_head)), U.judge.tg, st, p->k2_unroll,
               0);
    for (int c : U.far_cls) {
        const ClassP &K = p->cls[c];
        std::vector<int> vs;
        for (size_t v = 0; v < U.aud.size(); ++v)
            if (p->dom[U.pairs[U.aud[v]].s].cls == c) vs.push_back(int(v));
        for (size_t j0 = 0; j0 < vs.size(); j0 += kMaxJobs) {
            const int cnt = int(std::min<size_t>(kMaxJobs, vs.size() - j0));
            LinePass x = inv_x(p, K.N, K.P, K.Hz, false);
            LinePass y = inv_y(p, K.N, K.P, K.Hz, false);
            ZInv zi{};
            zi.reg = p->fft_reg;
            zi.Nx = K.N[0];
            zi.Ny = K.N[1];
            zi.Nz = K.N[2];
            zi.Pz = K.P[2];
            zi.Hz = K.Hz;
            zi.tw = tw_ptr(p, K.P[2], false);
            zi.rp = make_radix(K.P[2]);
            x.n_jobs = y.n_jobs = zi.n_jobs = cnt;
            for (int j = 0; j < cnt; ++j) {
                const int v = vs[j0 + j];
                char *t1 = p->ws + U.off_jt1 + size_t(j) * U.jt1_elems * p->csz;
                char *t2 = p->ws + U.off_jt2 + size_t(j) * U.jt2_elems * p->csz;
                x.jobs[j].in = p->ws + U.jacc_off[v];
                x.jobs[j].out = t2;
                y.jobs[j].in = t2;
                y.jobs[j].out = t1;
                zi.jobs[j].in = t1;
                zi.jobs[j].out = p->ws + U.off_jF + size_t(j) * U.jF_elems * 4;
                zi.jobs[j].add = nullptr;
            }
            launch_line_pass(x, 0, st);
            if (!(plane_ok(p) && launch_yz_inv_plane(y, zi, st))) {
                launch_line_pass(y, 0, st);
                launch_zinv(zi, 0, st);
            }
            check_launch();
            fn(&vs[j0], cnt);
        }
    }
}

float *jfield(rp_plan p, int j) { return p->at<float>(p->sur.off_jF + size_t(j) * p->sur.jF_elems * 4); }

void need_ready(rp_plan p) {
    if (!p->sur.on) fail(RP_ERR_STATE, "surrogate not configured (rp_surrogate_configure)");
    need_ws(p);
    if (p->next_step < 1 || p->pushed) fail(RP_ERR_STATE, "no completed step to evaluate");
}

}  // namespace

void sur_classify(rp_plan p) {
    SurrogateH &U = p->sur;
    const int nd = p->n_dom;
    U.pairs.clear();
    U.far_index.assign(size_t(nd) * nd, -1);
    U.src_slot.assign(nd, -1);
    U.src_doms.clear();
    U.aud.clear();
    U.aud_row.clear();
    U.mats.clear();
    U.far_cls.clear();
    U.synth_targets.clear();
    if (!U.on) return;
    const double cdt = p->c * p->dt;
    for (const SystemP &S : p->sys) {
        for (int s : S.doms) {
            for (int n : S.doms) {
                if (s == n) continue;
                double d[3], d2 = 0;
                for (int a = 0; a < 3; ++a) {
                    d[a] = centre(p, s, a) - centre(p, n, a);
                    d2 += d[a] * d[a];
                }
                const double dist = std::sqrt(d2);
                if (!(dist > U.far_factor * std::max(diagonal(p, s), diagonal(p, n)))) continue;
                for (int a = 0; a < 3; ++a)
                    if (p->dom[s].N[a] < 4)
                        fail(RP_ERR_UNSUPPORTED, "a far-pair target needs at least 4 points per axis");
                FarPairH F;
                F.s = s;
                F.n = n;
                F.dist = dist;
                F.m_c = int(std::lround(dist / cdt));
                F.frac = dist / cdt - F.m_c;
                F.audited = U.audit[n] != 0;
                make_frame(d, F.rot);
                U.far_index[size_t(s) * nd + n] = int(U.pairs.size());
                U.pairs.push_back(F);
            }
        }
    }
    U.mom_depth = 1;
    for (const FarPairH &F : U.pairs) {
        if (U.src_slot[F.n] < 0) {
            U.src_slot[F.n] = int(U.src_doms.size());
            U.src_doms.push_back(F.n);
        }
        U.mom_depth = std::max(U.mom_depth, F.m_c - U.n_lags / 2 + U.n_lags);
        // the multipole path reads up to the farthest node's retarded step plus
        // the interpolation stencil
        U.mom_depth = std::max(U.mom_depth, int(std::ceil((F.dist + 0.5 * diagonal(p, F.s)) / cdt)) + 4);
        if (F.audited) U.aud.push_back(int(&F - U.pairs.data()));
        const int c = p->dom[F.s].cls;
        if (std::find(U.far_cls.begin(), U.far_cls.end(), c) == U.far_cls.end()) U.far_cls.push_back(c);
        if (std::find(U.synth_targets.begin(), U.synth_targets.end(), F.s) == U.synth_targets.end())
            U.synth_targets.push_back(F.s);
    }
    // judge order: by system, then source (shared ring reads), then target
    std::stable_sort(U.aud.begin(), U.aud.end(), [&](int a, int b) {
        const FarPairH &A = U.pairs[a], &B = U.pairs[b];
        const int sa = p->dom[A.s].sys, sb = p->dom[B.s].sys;
        if (sa != sb) return sa < sb;
        if (A.n != B.n) return A.n < B.n;
        return A.s < B.s;
    });
    U.aud_row.assign(U.aud.size(), 0);
    for (size_t v = 0; v < U.aud.size(); ++v)
        for (int f = 0; f < U.aud[v]; ++f) U.aud_row[v] += U.pairs[f].audited ? 1 : 0;
    U.mats.resize(U.pairs.size() * 2 * kNBasis * kNBasis);
    for (size_t f = 0; f < U.pairs.size(); ++f)
        pair_maps(p, U.pairs[f], &U.mats[f * 2 * kNBasis * kNBasis], &U.mats[(f * 2 + 1) * kNBasis * kNBasis]);
}

void sur_layout(rp_plan p, size_t &off) {
    auto alloc = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
        return o;
    };
    SurrogateH &U = p->sur;
    const size_t nf = U.pairs.size(), na = U.aud.size(), ns = U.src_doms.size(), nd = p->dom.size();
    U.off_mom = alloc(ns * U.mom_depth * kFeatStride * 4);
    U.off_mpart = alloc(ns * kMomChunks * kNMom * 4);
    U.off_fpairs = alloc(nf * sizeof(FarPair));
    U.off_x = alloc(nf * U.n_in * 4);
    U.off_y = alloc(nf * kNOut * 4);
    U.off_pc = alloc(nf * kNOut * 4);
    U.off_coef = alloc(nd * kNOut * 4);
    U.off_order = alloc(nf * 4);
    U.off_tbeg = alloc((nd + 1) * 4);
    U.off_mats = alloc(nf * 2 * kNBasis * kNBasis * 4);
    U.off_inscale = alloc(kNFeat * 4);
    U.off_outscale = alloc(kNOut * 4);
    U.off_pinv = alloc(kNBasis * 64 * 4);
    U.off_Q.clear();
    U.jt1_elems = U.jt2_elems = U.jF_elems = 0;
    for (int c : U.far_cls) {
        const ClassP &K = p->cls[c];
        const size_t npts = size_t(K.N[0]) * K.N[1] * K.N[2];
        U.off_Q[c] = alloc(kNBasis * npts * 4);
        U.jt1_elems = std::max(U.jt1_elems, size_t(K.N[0]) * K.N[1] * K.Hz * 4);
        U.jt2_elems = std::max(U.jt2_elems, size_t(K.N[0]) * K.P[1] * K.Hz * 4);
        U.jF_elems = std::max(U.jF_elems, 4 * npts);
    }
    size_t jacc = 0;
    U.jacc_off.assign(na, 0);
    for (size_t v = 0; v < na; ++v) jacc += size_t(p->sys[p->dom[U.pairs[U.aud[v]].s].sys].C) * 4 * p->csz;
    U.off_jacc = alloc(jacc);
    size_t o = U.off_jacc;
    for (size_t v = 0; v < na; ++v) {
        U.jacc_off[v] = o;
        o += size_t(p->sys[p->dom[U.pairs[U.aud[v]].s].sys].C) * 4 * p->csz;
    }
    const size_t nj = std::min<size_t>(kMaxJobs, std::max<size_t>(na, 1));
    U.off_jt1 = alloc(nj * U.jt1_elems * p->csz);
    U.off_jt2 = alloc(nj * U.jt2_elems * p->csz);
    U.off_jF = alloc(nj * U.jF_elems * 4);
    U.off_jcb = alloc(kMaxJobs * kNOut * 4);
    U.off_jres = alloc(na * 8 * 4);
    U.off_budget = alloc(nd * 4 * 4);
    U.off_fail = alloc(na * 4);
    U.off_aud = alloc(na * 4);
    U.off_rowfar = alloc(na * 4);
    U.off_tcoef = alloc(na * kNOut * 4);

    // judge by sample: job tables, fields and flags of the sampled pairs, and
    // the fallback slots (rings, Green spectra, transform scratch, refill scratch)
    U.slot_W = 0;
    U.slot_Cpad = 0;
    if (U.per_judge < 0) return;
    const size_t nsp = std::max<size_t>(nf, 1);
    U.off_sjobs = alloc(nsp * sizeof(SampleJob));
    U.off_jjobs = alloc(nsp * sizeof(SampleJudgeJob));
    U.off_sfield = alloc(nsp * kSamplePts * 4 * 4);
    U.off_sres = alloc(nsp * 8 * 4);
    U.off_sfail = alloc(nsp * 4);
    if (U.slots.empty()) return;
    size_t t1 = 0, t2 = 0, zb = 0;
    for (int f : U.sampled) {
        const FarPairH &F = U.pairs[f];
        const PairP &q = p->pr(F.s, F.n);
        const DomainP &d = p->dom[F.n];
        const SystemP &S = p->sys[d.sys];
        U.slot_W = std::max(U.slot_W, q.m_hi - q.m_lo + 1);
        U.slot_Cpad = std::max(U.slot_Cpad, S.Cpad);
        t1 = std::max(t1, size_t(d.N[0]) * d.N[1] * S.Hz * 4 * p->csz);
        t2 = std::max(t2, size_t(d.N[0]) * S.P[1] * S.Hz * 4 * p->csz);
        // per-block maxima of the staged z pass, or one per x slice of the plane pass
        zb = std::max(zb, size_t(std::max(d.zblocks, d.N[0])) * 4 * sizeof(float));
    }
    if (U.slot_W == 0) return;
    const bool quant = ring_scaled(p);
    const bool zq = (p->ring_fmt == RING_F16 || p->ring_fmt == RING_BF16);
    U.fill_t1 = t1;
    U.fill_t2 = t2;
    U.fill_zmax = zq ? zb : 0;
    U.off_fillslots = alloc(U.slots.size() * size_t(U.slot_W) * 4);
    U.off_fill_t1 = alloc(kFillJobs * t1);
    U.off_fill_t2 = alloc(kFillJobs * t2);
    U.off_fill_zmax = zq ? alloc(kFillJobs * zb) : 0;
    for (SlotP &k : U.slots) {
        k.off_ring = alloc(size_t(U.slot_W) * U.slot_Cpad * 4 * p->ring_esz);
        k.off_scales = quant ? alloc(scale_bytes(p, U.slot_W, U.slot_Cpad)) : 0;
        k.off_zmax = zq ? alloc(zb) : 0;
        k.off_t1 = alloc(t1);
        k.off_t2 = alloc(t2);
    }
    // Green spectra of the slots, in the spectra's element units on whole
    // frequency tiles from the start of the spectra
    const size_t tile_bytes = size_t(kTile) * p->spec_csz;
    const size_t rem = (off - p->off_spec) % tile_bytes;
    if (rem) off += tile_bytes - rem;
    for (SlotP &k : U.slots) {
        const size_t o = alloc(size_t(U.slot_W) * U.slot_Cpad * p->spec_csz);
        k.spec_elem = int64_t((o - p->off_spec) / p->spec_csz);
    }
    // lag-sum tables of the slot pairs: one group per target, a source record
    // and W entries per slot
    const size_t nsl = U.slots.size();
    size_t tiles = 0;
    for (const SystemP &S : p->sys) tiles = std::max(tiles, size_t((S.C + kTile - 1) / kTile));
    K2Dev &D = U.k2p_dev;
    D.cap_groups = std::min(nsl, size_t(p->n_dom));
    D.cap_items = D.cap_groups * tiles;
    D.cap_srcs = nsl;
    D.cap_pairs = nsl * kGroupMax;
    D.cap_entries = D.cap_masks = nsl * size_t(U.slot_W);
    D.items = alloc(D.cap_items * sizeof(K2Item));
    D.groups = alloc(D.cap_groups * sizeof(K2Group));
    D.entries = alloc(D.cap_entries * sizeof(K2Entry));
    D.srcs = alloc(D.cap_srcs * sizeof(K2Src));
    D.pairs = alloc(D.cap_pairs * sizeof(K2Pair));
    D.masks = alloc(D.cap_masks * sizeof(uint32_t));
}

// DomDev entries of the fallback slots (ring and scale offsets; depth W while
// a pair holds the slot).
void sur_slot_tables(rp_plan p) {
    const bool quant = ring_scaled(p);
    for (const SlotP &k : p->sur.slots) {
        DomDev &D = p->domdev[size_t(k.idx)];
        D.ring_off = int64_t((k.off_ring - p->dom[0].off_ring) / (4 * p->ring_esz)) * 4;
        D.scale_off = quant ? int64_t((k.off_scales - p->dom[0].off_scales) / sizeof(float)) : 0;
        D.depth = k.f >= 0 ? k.W : 1;
    }
}

// Per step: every occupied slot whose source is in class K transforms
// S_n(l - lo) again from the real-space history into its ring.
void sur_ring_jobs(rp_plan p, const ClassP &K, std::vector<RingJob> &jobs) {
    const SurrogateH &U = p->sur;
    const int ci = int(&K - p->cls.data());
    const bool scaled = ring_scaled(p);
    const bool zq = (p->ring_fmt == RING_F16 || p->ring_fmt == RING_BF16);
    const int32_t *dhead = p->at<int32_t>(p->off_head);
    for (const SlotP &k : U.slots) {
        if (k.f < 0) continue;
        const int n = U.pairs[size_t(k.f)].n;
        const DomainP &d = p->dom[n];
        if (d.cls != ci) continue;
        RingJob J;
        J.n = n;
        J.src = p->ws + d.off_hist;
        J.src_head = dhead + d.t1_idx;
        J.src_depth = d.d1;
        J.src_lag = k.lo;
        J.t1 = p->ws + k.off_t1;
        J.t2 = p->ws + k.off_t2;
        J.ring = p->ws + k.off_ring;
        J.scales = scaled ? p->at<float>(k.off_scales) : nullptr;
        J.zmax = zq ? p->at<float>(k.off_zmax) : nullptr;
        J.head = dhead + k.idx;
        J.depth = k.W;
        jobs.push_back(J);
    }
}

// The slot pairs' lag sum, added into their targets' accumulators (set
// `phase` of a block of blocked lag-sum steps).
void sur_enqueue_slots(rp_plan p, const int32_t *head, hipStream_t st, int phase) {
    SurrogateH &U = p->sur;
    if (U.k2p.items.empty()) return;
    K2Args a = k2_args(p, U.k2p, U.k2p_dev, head);
    a.acc_set = phase;
    a.accumulate = 1;
    enqueue_k2(p, a, U.k2p.tg, st, 1, 0);
}

void sur_bind(rp_plan p) {
    SurrogateH &U = p->sur;
    hipStream_t st = p->stream;
    std::vector<FarPair> fp(U.pairs.size());
    double dbar = 0;
    for (int i = 0; i < p->n_dom; ++i) dbar += diagonal(p, i) / p->n_dom;
    for (size_t f = 0; f < U.pairs.size(); ++f) {
        const FarPairH &F = U.pairs[f];
        FarPair &D = fp[f];
        D.s = F.s;
        D.n = F.n;
        D.m_c = F.m_c;
        D.src_slot = U.src_slot[F.n];
        for (int i = 0; i < 9; ++i) D.rot[i] = float(F.rot[i]);
        D.inv_d = float(1.0 / F.dist);
        D.geo[0] = float(10.0 * dbar / F.dist);
        D.geo[1] = float(F.frac);
        for (int a = 0; a < 3; ++a) {
            D.d[a] = float(centre(p, F.s, a) - centre(p, F.n, a));
            D.hw[a] = float(0.5 * p->h * (p->dom[F.s].N[a] - 1));
        }
    }
    std::vector<int32_t> aud(U.aud.begin(), U.aud.end());
    std::vector<float> ones(kNOut, 1.0f);
    if (!fp.empty()) {
        HIP_OK(hipMemcpy(p->ws + U.off_fpairs, fp.data(), fp.size() * sizeof(FarPair), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(p->ws + U.off_mats, U.mats.data(), U.mats.size() * 4, hipMemcpyHostToDevice));
    }
    if (!aud.empty()) HIP_OK(hipMemcpy(p->ws + U.off_aud, aud.data(), aud.size() * 4, hipMemcpyHostToDevice));
    {
        // the audited far pairs in far-pair order: the rows of the teacher data
        std::vector<int32_t> rowfar;
        for (size_t f = 0; f < U.pairs.size(); ++f)
            if (U.pairs[f].audited) rowfar.push_back(int32_t(f));
        if (!rowfar.empty())
            HIP_OK(hipMemcpy(p->ws + U.off_rowfar, rowfar.data(), rowfar.size() * 4, hipMemcpyHostToDevice));
    }
    HIP_OK(hipMemcpy(p->ws + U.off_inscale, ones.data(), kNFeat * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p->ws + U.off_outscale, ones.data(), kNOut * 4, hipMemcpyHostToDevice));
    {
        // node-to-coefficient fit of the multipole path: (B^T B)^-1 B^T on the
        // 4 x 4 x 4 nodes xi in {-1, -1/3, 1/3, 1}
        const double nodes[4] = {-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0};
        std::vector<double> B(64 * kNBasis), G(kNBasis * kNBasis, 0.0);
        for (int t = 0; t < 64; ++t) {
            const double xi[3] = {nodes[t >> 4], nodes[(t >> 2) & 3], nodes[t & 3]};
            basis_row(xi, &B[size_t(t) * kNBasis]);
        }
        for (int t = 0; t < 64; ++t)
            for (int a = 0; a < kNBasis; ++a)
                for (int b = 0; b < kNBasis; ++b) G[a * kNBasis + b] += B[t * kNBasis + a] * B[t * kNBasis + b];
        const std::vector<double> Gi = spd_inverse(G, kNBasis);
        std::vector<float> pinv(kNBasis * 64);
        for (int a = 0; a < kNBasis; ++a)
            for (int t = 0; t < 64; ++t) {
                double v = 0;
                for (int b = 0; b < kNBasis; ++b) v += Gi[a * kNBasis + b] * B[t * kNBasis + b];
                pinv[a * 64 + t] = float(v);
            }
        HIP_OK(hipMemcpy(p->ws + U.off_pinv, pinv.data(), pinv.size() * 4, hipMemcpyHostToDevice));
    }
    for (const auto &kv : U.off_Q) {
        const std::vector<float> Q = dual_basis(p->cls[kv.first].N);
        HIP_OK(hipMemcpy(p->ws + kv.second, Q.data(), Q.size() * 4, hipMemcpyHostToDevice));
    }
    for (FarPairH &F : U.pairs) {
        F.plain = false;
        F.slot = -1;
    }
    // fallback slots start empty (a fresh bind)
    U.cursor = 0;
    U.k2p = K2Tables{};
    for (SlotP &k : U.slots) {
        k.f = -1;
        p->domdev[size_t(k.idx)].depth = 1;
    }
    if (!U.slots.empty())
        HIP_OK(hipMemcpyAsync(p->ws + p->off_domdev, p->domdev.data(), p->domdev.size() * sizeof(DomDev),
                              hipMemcpyHostToDevice, st));
    upload_csr(p, st);
    if (!U.src_doms.empty())   // ns * depth * 96 bytes: a multiple of 16
        launch_fill_zero(p->ws + U.off_mom, U.src_doms.size() * U.mom_depth * kFeatStride * 4, st);
    launch_fill_zero(p->ws + U.off_coef, (p->dom.size() * kNOut * 4 + 15) / 16 * 16, st);
    check_launch();
    HIP_OK(hipStreamSynchronize(st));
}

void sur_enqueue_moments(rp_plan p, const void *const *src, hipStream_t st) {
    SurrogateH &U = p->sur;
    const size_t ns = U.src_doms.size();
    for (size_t j0 = 0; j0 < ns; j0 += kMaxJobs) {
        MomentArgs a{};
        a.h = float(p->h);
        a.h3 = p->h * p->h * p->h;
        a.depth = U.mom_depth;
        a.step = p->at<int64_t>(p->off_state);
        a.n_jobs = int(std::min<size_t>(kMaxJobs, ns - j0));
        for (int j = 0; j < a.n_jobs; ++j) {
            const int slot = int(j0) + j, n = U.src_doms[slot];
            const DomainP &d = p->dom[n];
            MomentJob &J = a.jobs[j];
            J.src = static_cast<const float *>(src[n]);
            J.s0 = p->at<float>(d.off_s0);
            J.ring = p->at<float>(U.off_mom) + size_t(slot) * U.mom_depth * kFeatStride;
            J.partial = p->at<float>(U.off_mpart) + size_t(slot) * kMomChunks * kNMom;
            for (int c = 0; c < 3; ++c) {
                J.N[c] = d.N[c];
                J.o[c] = float(d.o[c] - centre(p, n, c));
            }
        }
        launch_moments(a, st);
        check_launch();
    }
}

FeatArgs feat_args(rp_plan p, float *x, int64_t adj) {
    SurrogateH &U = p->sur;
    FeatArgs f{};
    f.pairs = p->at<FarPair>(U.off_fpairs);
    f.moments = p->at<float>(U.off_mom);
    f.in_scale = p->at<float>(U.off_inscale);
    f.x = x;
    f.step = p->at<int64_t>(p->off_state);
    f.step_adj = adj;
    f.depth = U.mom_depth;
    f.n_lags = U.n_lags;
    f.n_in = U.n_in;
    f.n_pairs = int(U.pairs.size());
    return f;
}

// Inference of every far pair at the current step and the synthesis of the
// active pairs' fields into the targets' outputs.
MultipoleArgs multipole_args(rp_plan p, int step_off) {
    SurrogateH &U = p->sur;
    MultipoleArgs ma{};
    ma.pairs = p->at<FarPair>(U.off_fpairs);
    ma.moments = p->at<float>(U.off_mom);
    ma.pinv = p->at<float>(U.off_pinv);
    ma.pc = p->at<float>(U.off_pc);
    ma.step = p->at<int64_t>(p->off_state);
    ma.step_off = step_off;
    ma.depth = U.mom_depth;
    ma.n_pairs = int(U.pairs.size());
    ma.inv_cdt = float(1.0 / (p->c * p->dt));
    ma.c = float(p->c);
    ma.dt = float(p->dt);
    return ma;
}

void sur_enqueue_infer(rp_plan p, void *const *out, hipStream_t st) {
    SurrogateH &U = p->sur;
    const int nf = int(U.pairs.size());
    if ((!U.attached && !U.multipole) || nf == 0) return;
    if (U.multipole) launch_multipole(multipole_args(p, 0), st);
    if (U.attached) {
        launch_features(feat_args(p, p->at<float>(U.off_x), 0), st);
        mlp_forward_on(U.mlp, p->at<float>(U.off_x), nf, p->at<float>(U.off_y), st);
        XformArgs xa{};
        xa.pairs = p->at<FarPair>(U.off_fpairs);
        xa.mats = p->at<float>(U.off_mats);
        xa.in = p->at<float>(U.off_y);
        xa.out = p->at<float>(U.off_pc);
        xa.scale = p->at<float>(U.off_outscale);
        xa.dir = 0;
        xa.n = nf;
        xa.accumulate = U.multipole ? 1 : 0;   // a correction on top of the multipole terms
        launch_xform(xa, st);
    }
    CoefArgs ca{};
    ca.pc = p->at<float>(U.off_pc);
    ca.order = p->at<int32_t>(U.off_order);
    ca.tgt_begin = p->at<int32_t>(U.off_tbeg);
    ca.coef = p->at<float>(U.off_coef);
    ca.n_targets = p->n_dom;
    launch_coef_sum(ca, st);
    for (size_t j0 = 0; j0 < U.synth_targets.size(); j0 += kMaxJobs) {
        SynthArgs sa{};
        sa.n_jobs = int(std::min<size_t>(kMaxJobs, U.synth_targets.size() - j0));
        for (int j = 0; j < sa.n_jobs; ++j) {
            const int s = U.synth_targets[j0 + j];
            sa.jobs[j].coef = p->at<float>(U.off_coef) + size_t(s) * kNOut;
            sa.jobs[j].out = static_cast<float *>(out[s]);
            for (int c = 0; c < 3; ++c) sa.jobs[j].N[c] = p->dom[s].N[c];
        }
        launch_synthesize(sa, st);
    }
    check_launch();
}

// ---------------------------------------------------------------------------
// Fallback slots of sampled far pairs

namespace {

// Lag-sum tables of the occupied slots: per target one group (one member),
// per slot one source record over the slot's ring (lags lo .. lo + W - 1,
// newest snapshot of age lo) and its Green spectra.
void slot_k2(rp_plan p) {
    SurrogateH &U = p->sur;
    K2Tables &T = U.k2p;
    T = K2Tables{};
    std::map<int, std::vector<int>> by_target;
    for (size_t k = 0; k < U.slots.size(); ++k)
        if (U.slots[k].f >= 0) by_target[U.pairs[size_t(U.slots[k].f)].s].push_back(int(k));
    for (const auto &kv : by_target) {
        const int s = kv.first;
        const SystemP &S = p->sys[p->dom[s].sys];
        K2Group G{};
        G.C = S.C;
        G.spec_base = S.spec_base;
        G.n_members = 1;
        G.member[0] = s;
        G.entry_begin = int(T.entries.size());
        G.src_begin = int(T.srcs.size());
        for (int k : kv.second) {
            const SlotP &L = U.slots[size_t(k)];
            const int64_t spec0 = L.spec_elem - S.spec_base;   // within the system's spectra
            if (spec0 < 0 || spec0 % kTile) fail(RP_ERR_STATE, "internal: slot spectra misplaced");
            K2Src R{};
            R.n = L.idx;
            R.m_min = L.lo;
            R.m_max = L.lo + L.W - 1;
            R.m_base = L.lo;
            R.mask_off = int32_t(T.masks.size());
            for (int m = R.m_min; m <= R.m_max; ++m) T.masks.push_back(1u);
            K2Pair Qs[kGroupMax] = {};
            Qs[0].row0 = int32_t(spec0 / kTile) - L.lo;
            Qs[0].w = L.W;
            for (int t = 0; t < kGroupMax; ++t) T.pairs.push_back(Qs[t]);
            T.srcs.push_back(R);
            for (int m = R.m_min; m <= R.m_max; ++m) {
                K2Entry E{};
                E.src = L.idx;
                E.m = m;
                E.mask = 1u;
                E.spec_tile[0] = int32_t(spec0 / kTile + (m - L.lo));
                E.spec_w[0] = L.W;
                T.entries.push_back(E);
            }
        }
        G.entry_end = int(T.entries.size());
        G.src_end = int(T.srcs.size());
        const int gi = int(T.groups.size());
        T.groups.push_back(G);
        for (int64_t k0 = 0; k0 < S.C; k0 += kTile) T.items.push_back(K2Item{gi, int32_t(k0)});
    }
    finish_k2(p, T);
}

// Far pair f takes slot k after step l (the last completed step): the slot's
// ring gets depth W and, for the next step, head 1 mod W; the pair's Green
// spectra are computed into the slot; its ring is refilled with dS_n at ages
// lo .. hi of step l from the real-space history (age a at slot -(a - lo) mod
// W), so that the next step's ingest (age lo at head 1) continues it.
void slot_assign(rp_plan p, int k, int f, hipStream_t st) {
    SurrogateH &U = p->sur;
    SlotP &L = U.slots[size_t(k)];
    FarPairH &F = U.pairs[size_t(f)];
    const PairP &q = p->pr(F.s, F.n);
    const DomainP &dn = p->dom[F.n];
    const int W = q.m_hi - q.m_lo + 1;
    if (q.m_lo < 1 || q.m_hi + 1 >= dn.d1 || W > U.slot_W || dn.t1_idx < 0)
        fail(RP_ERR_STATE, "internal: a fallback window outside the slot or the history");
    L.f = f;
    L.lo = q.m_lo;
    L.W = W;
    F.slot = k;
    F.plain = true;
    DomDev &D = p->domdev[size_t(L.idx)];
    D.depth = W;
    HIP_OK(hipMemcpyAsync(p->ws + p->off_domdev + size_t(L.idx) * sizeof(DomDev), &D, sizeof(DomDev),
                          hipMemcpyHostToDevice, st));
    U.h_heads[size_t(k)] = 1 % W;
    HIP_OK(hipMemcpyAsync(p->ws + p->off_head + size_t(L.idx) * 4, &U.h_heads[size_t(k)], 4, hipMemcpyHostToDevice,
                          st));
    // Green spectra of (s <- n), lags lo .. hi, [tile][lag][kTile]
    for (int m0 = q.m_lo; m0 <= q.m_hi; m0 += kGreenChunk) {
        const int cnt = std::min(kGreenChunk, q.m_hi - m0 + 1);
        void *outs[kGreenChunk];
        for (int j = 0; j < cnt; ++j)
            outs[j] = p->ws + p->off_spec + size_t(L.spec_elem + int64_t(m0 + j - q.m_lo) * kTile) * p->spec_csz;
        green_spectra(p, F.s, F.n, 1, m0, cnt, outs, RING_F32, int64_t(W) * kTile);
    }
    // refill from the real-space history
    int32_t *slots_h = &U.h_fill[size_t(k) * U.slot_W];
    for (int i = 0; i < W; ++i) slots_h[i] = (W - i % W) % W;
    const int32_t *slots_d = p->at<int32_t>(U.off_fillslots) + size_t(k) * U.slot_W;
    HIP_OK(hipMemcpyAsync(const_cast<int32_t *>(slots_d), slots_h, size_t(W) * 4, hipMemcpyHostToDevice, st));
    const bool scaled = ring_scaled(p);
    const bool zq = (p->ring_fmt == RING_F16 || p->ring_fmt == RING_BF16);
    for (int i0 = 0; i0 < W; i0 += kFillJobs) {
        std::vector<RingJob> jobs;
        for (int i = i0; i < std::min(W, i0 + kFillJobs); ++i) {
            const int j = i - i0;
            RingJob J;
            J.n = F.n;
            J.src = p->ws + dn.off_hist;
            J.src_head = p->at<int32_t>(p->off_prev_head) + dn.t1_idx;
            J.src_depth = dn.d1;
            J.src_lag = q.m_lo + i;
            J.t1 = p->ws + U.off_fill_t1 + size_t(j) * U.fill_t1;
            J.t2 = p->ws + U.off_fill_t2 + size_t(j) * U.fill_t2;
            J.ring = p->ws + L.off_ring;
            J.scales = scaled ? p->at<float>(L.off_scales) : nullptr;
            J.zmax = zq ? p->at<float>(U.off_fill_zmax + size_t(j) * U.fill_zmax) : nullptr;
            J.head = slots_d + i;
            J.depth = W;
            jobs.push_back(J);
        }
        enqueue_ring_jobs(p, p->cls[size_t(dn.cls)], jobs, st);
    }
    check_launch();
}

void slot_release(rp_plan p, int k, hipStream_t st) {
    SurrogateH &U = p->sur;
    SlotP &L = U.slots[size_t(k)];
    if (L.f >= 0) {
        U.pairs[size_t(L.f)].slot = -1;
        U.pairs[size_t(L.f)].plain = false;
    }
    L.f = -1;
    DomDev &D = p->domdev[size_t(L.idx)];
    D.depth = 1;
    HIP_OK(hipMemcpyAsync(p->ws + p->off_domdev + size_t(L.idx) * sizeof(DomDev), &D, sizeof(DomDev),
                          hipMemcpyHostToDevice, st));
}

// Direct-sum fields of far pairs fs at their sample points into
// U.off_sfield (rows in the order of fs).
void sample_fields(rp_plan p, const std::vector<int> &fs, hipStream_t st) {
    SurrogateH &U = p->sur;
    U.h_sjobs.assign(fs.size(), SampleJob{});
    for (size_t i = 0; i < fs.size(); ++i) {
        const FarPairH &F = U.pairs[size_t(fs[i])];
        const DomainP &ds = p->dom[F.s], &dn = p->dom[F.n];
        SampleJob &J = U.h_sjobs[i];
        J.hist = p->at<float>(dn.off_hist);
        J.s0 = p->at<float>(dn.off_s0);
        J.head = p->at<int32_t>(p->off_prev_head) + dn.t1_idx;
        J.out = p->at<float>(U.off_sfield) + i * kSamplePts * 4;
        for (int a = 0; a < 3; ++a) {
            J.t0[a] = (ds.o[a] - dn.o[a]) / p->h;
            J.Ns[a] = ds.N[a];
            J.Nn[a] = dn.N[a];
        }
        J.depth = dn.d1;
    }
    if (fs.empty()) return;
    HIP_OK(hipMemcpyAsync(p->ws + U.off_sjobs, U.h_sjobs.data(), fs.size() * sizeof(SampleJob),
                          hipMemcpyHostToDevice, st));
    SampleArgs a{};
    a.jobs = p->at<SampleJob>(U.off_sjobs);
    a.n_jobs = int(fs.size());
    a.h = p->h;
    a.inv_cdt = 1.0 / (p->c * p->dt);
    a.h3 = float(p->h * p->h * p->h);
    launch_pair_sample(a, st);
    check_launch();
}

}  // namespace

void sur_sample(rp_plan p, int per_judge, int n_slots) {
    SurrogateH &U = p->sur;
    if (!U.on) fail(RP_ERR_STATE, "surrogate not configured (rp_surrogate_configure)");
    if (p->ws) fail(RP_ERR_STATE, "call rp_surrogate_sample before rp_bind_workspace");
    if (n_slots < 0 || n_slots > 4096) fail(RP_ERR_ARG, "fallback_slots must be in [0, 4096]");
    if (p->hist_host) fail(RP_ERR_UNSUPPORTED, "the judge by sample keeps its history in device memory");
    U.per_judge = per_judge < 0 ? -1 : per_judge;
    U.slots.assign(U.per_judge < 0 ? 0 : size_t(n_slots), SlotP{});
    U.n_slots = int(U.slots.size());
    U.sampled.clear();
    for (size_t f = 0; f < U.pairs.size(); ++f) {
        U.pairs[f].slot = -1;
        if (!U.pairs[f].audited) U.sampled.push_back(int(f));
    }
    U.cursor = 0;
    U.last_sampled = U.last_refused = 0;
    U.k2p = K2Tables{};
    U.k2p_dev = K2Dev{};
    plan_tables(p);
    plan_layout(p);
    U.h_fill.assign(U.slots.size() * size_t(std::max(U.slot_W, 1)), 0);
    U.h_heads.assign(U.slots.size(), 0);
    plan_stats(p);
}

void sur_sample_fields(rp_plan p, const int32_t *far_pairs, int n, float *out) {
    need_ready(p);
    SurrogateH &U = p->sur;
    if (U.per_judge < 0) fail(RP_ERR_STATE, "no judge by sample (rp_surrogate_sample)");
    if (n < 0 || (n > 0 && (!far_pairs || !out))) fail(RP_ERR_ARG, "bad pair list or output");
    if (n > int(U.pairs.size())) fail(RP_ERR_ARG, "more pairs than far pairs");
    std::vector<int> fs(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        if (far_pairs[i] < 0 || far_pairs[i] >= int(U.pairs.size())) fail(RP_ERR_ARG, "far pair index out of range");
        fs[size_t(i)] = far_pairs[i];
    }
    hipStream_t st = p->stream;
    sample_fields(p, fs, st);
    if (n > 0)
        HIP_OK(hipMemcpyAsync(out, p->ws + U.off_sfield, size_t(n) * kSamplePts * 4 * 4, hipMemcpyDeviceToDevice,
                              st));
    HIP_OK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// Entry points (called from the C ABI in plan.cpp's guard)

void sur_configure(rp_plan p, double far_factor, int n_lags, const int32_t *audit, int n_audit) {
    if (p->ws) fail(RP_ERR_STATE, "configure the surrogate before rp_bind_workspace");
    SurrogateH &U = p->sur;
    if (far_factor <= 0) {
        U = SurrogateH{};
    } else {
        if (!p->target.empty()) fail(RP_ERR_UNSUPPORTED, "the surrogate and a target subset do not combine");
        if (!std::isfinite(far_factor)) fail(RP_ERR_ARG, "far_factor must be finite");
        if (p->split_gap > 0) fail(RP_ERR_UNSUPPORTED, "the surrogate and a split history do not combine");
        if (p->p64) fail(RP_ERR_UNSUPPORTED, "the surrogate runs with FP32 outputs (not RP_FP64)");
        if (!std::isfinite(p->c)) fail(RP_ERR_UNSUPPORTED, "the surrogate needs a finite c");
        if (n_lags < 1 || n_lags > 1024) fail(RP_ERR_ARG, "n_lags must be in [1, 1024]");
        if (n_audit < 0 || (n_audit > 0 && !audit)) fail(RP_ERR_ARG, "bad audit list");
        std::vector<char> aud(p->n_dom, 0);
        for (int i = 0; i < n_audit; ++i) {
            if (audit[i] < 0 || audit[i] >= p->n_dom) fail(RP_ERR_ARG, "audit source out of range");
            aud[audit[i]] = 1;
        }
        U = SurrogateH{};
        U.on = true;
        U.far_factor = far_factor;
        U.n_lags = n_lags;
        U.n_in = kNBlocks * n_lags * kNFeat + kNGeo;
        U.audit = aud;
    }
    sur_classify(p);
    plan_tables(p);
    plan_layout(p);
    plan_stats(p);
}

void sur_attach(rp_plan p, rp_mlp mlp, const float *in_scale, const float *out_scale) {
    SurrogateH &U = p->sur;
    if (!U.on) fail(RP_ERR_STATE, "surrogate not configured (rp_surrogate_configure)");
    need_ws(p);
    release_graph(p);
    if (!mlp) {
        U.mlp = nullptr;
        U.attached = false;
        return;
    }
    if (U.multipole == 1) U.multipole = 0;   // the network replaces the multipole terms (mode 2 keeps both)
    int ni = 0, no = 0, mb = 0;
    if (!mlp_dims(mlp, &ni, &no, &mb)) fail(RP_ERR_STATE, "network workspace not bound");
    if (ni != U.n_in || no != kNOut) fail(RP_ERR_ARG, "network shape does not match the surrogate (n_in, 80)");
    if (mb < int(U.pairs.size())) fail(RP_ERR_ARG, "network max_batch below the number of far pairs");
    if (!in_scale || !out_scale) fail(RP_ERR_ARG, "scales are null");
    HIP_OK(hipStreamSynchronize(p->stream));
    HIP_OK(hipMemcpy(p->ws + U.off_inscale, in_scale, kNFeat * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p->ws + U.off_outscale, out_scale, kNOut * 4, hipMemcpyHostToDevice));
    U.mlp = mlp;
    U.attached = true;
}

void sur_multipole(rp_plan p, int enable) {
    SurrogateH &U = p->sur;
    if (!U.on) fail(RP_ERR_STATE, "surrogate not configured (rp_surrogate_configure)");
    need_ws(p);
    if (enable < 0 || enable > 2) fail(RP_ERR_ARG, "enable must be 0, 1 or 2");
    release_graph(p);
    U.multipole = enable;
    if (U.multipole == 1) {
        U.mlp = nullptr;
        U.attached = false;
    }
}

// The multipole terms of the audited far pairs at the last completed step,
// as frame coefficients (the layout of rp_surrogate_pair_response).
void sur_multipole_response(rp_plan p, float *coef) {
    need_ready(p);
    SurrogateH &U = p->sur;
    if (!coef) fail(RP_ERR_ARG, "coef is null");
    if (U.aud.empty() || U.pairs.empty()) return;
    hipStream_t st = p->stream;
    // into the network-output scratch: the step's own terms (which the judge
    // corrects with) stay intact
    MultipoleArgs ma = multipole_args(p, -1);
    ma.pc = p->at<float>(U.off_y);
    launch_multipole(ma, st);
    for (size_t v = 0; v < U.aud.size(); ++v) {
        XformArgs xa{};
        xa.pairs = p->at<FarPair>(U.off_fpairs);
        xa.mats = p->at<float>(U.off_mats);
        xa.in = p->at<float>(U.off_y) + size_t(U.aud[v]) * kNOut;
        xa.out = coef + size_t(U.aud_row[v]) * kNOut;
        xa.index = p->at<int32_t>(U.off_aud) + v;
        xa.dir = 1;
        xa.n = 1;
        launch_xform(xa, st);
    }
    check_launch();
}

void sur_teacher(rp_plan p, float *x, float *t, int residual) {
    need_ready(p);
    SurrogateH &U = p->sur;
    if (!x || !t) fail(RP_ERR_ARG, "null output");
    if (U.aud.empty()) return;
    hipStream_t st = p->stream;
    // every far pair's inputs into the inference buffer, the plain pair
    // responses (rows in far-pair order of the audited pairs) into t
    launch_features(feat_args(p, p->at<float>(U.off_x), -1), st);
    check_launch();
    sur_pair_response(p, t, p->at<float>(U.off_jres));
    if (residual) sur_multipole_response(p, p->at<float>(U.off_tcoef));
    TeacherArgs a{};
    a.pairs = p->at<FarPair>(U.off_fpairs);
    a.row_far = p->at<int32_t>(U.off_rowfar);
    a.x_all = p->at<float>(U.off_x);
    a.x_out = x;
    a.t = t;
    a.sub = residual ? p->at<float>(U.off_tcoef) : nullptr;
    a.n_rows = int(U.aud.size());
    a.n_in = U.n_in;
    launch_teacher(a, st);
    check_launch();
}

void sur_features(rp_plan p, float *x) {
    need_ready(p);
    if (!x) fail(RP_ERR_ARG, "x is null");
    launch_features(feat_args(p, x, -1), p->stream);
    check_launch();
}

void sur_pair_response(rp_plan p, float *coef, float *resid) {
    need_ready(p);
    SurrogateH &U = p->sur;
    if (!coef || !resid) fail(RP_ERR_ARG, "null output");
    if (U.aud.empty()) return;
    hipStream_t st = p->stream;
    judge_fields(p, st, [&](const int *vs, int cnt) {
        ProjArgs pa{};
        pa.n_jobs = cnt;
        for (int j = 0; j < cnt; ++j) {
            const int v = vs[j];
            const DomainP &t = p->dom[U.pairs[U.aud[v]].s];
            ProjJob &J = pa.jobs[j];
            J.F = jfield(p, j);
            J.Q = p->at<float>(U.off_Q.at(t.cls));
            J.coef_in = nullptr;
            J.coef = p->at<float>(U.off_jcb) + size_t(j) * kNOut;
            J.resid = resid + size_t(U.aud_row[v]) * 8;
            for (int c = 0; c < 3; ++c) J.N[c] = t.N[c];
            J.npts = t.npts;
        }
        launch_project(pa, true, st);
        for (int j = 0; j < cnt; ++j) {
            XformArgs xa{};
            xa.pairs = p->at<FarPair>(U.off_fpairs);
            xa.mats = p->at<float>(U.off_mats);
            xa.in = p->at<float>(U.off_jcb) + size_t(j) * kNOut;
            xa.out = coef + size_t(U.aud_row[vs[j]]) * kNOut;
            xa.index = p->at<int32_t>(U.off_aud) + vs[j];
            xa.dir = 1;
            xa.n = 1;
            launch_xform(xa, st);
        }
        check_launch();
    });
}

void sur_judge(rp_plan p, void *const *out, double tol, int32_t *n_fallback, double *worst, int32_t *n_readmitted) {
    need_ready(p);
    SurrogateH &U = p->sur;
    if (!U.attached && !U.multipole)
        fail(RP_ERR_STATE, "no far-pair terms to judge (rp_surrogate_attach or rp_surrogate_multipole)");
    if (!out) fail(RP_ERR_ARG, "out is null");
    for (int n = 0; n < p->n_dom; ++n)
        if (!out[n]) fail(RP_ERR_ARG, "an out pointer is null");
    if (!(tol > 0)) fail(RP_ERR_ARG, "tol must be positive");
    // blocked lag-sum steps: the block's pass has summed the plain pairs of
    // all its steps, so the pairs may change only before a block starts
    if (p->kb > 1 && lag_phase(p, p->next_step) != 0)
        fail(RP_ERR_STATE, "with blocked lag-sum steps the judge runs after the last step of a block");
    hipStream_t st = p->stream;
    const int na = int(U.aud.size());
    // the far pairs of non-audit sources judged by sample in this call
    std::vector<int> samp;
    if (U.per_judge >= 0 && !U.sampled.empty()) {
        const int ns = int(U.sampled.size());
        const int take = U.per_judge == 0 ? ns : std::min(U.per_judge, ns);
        for (int i = 0; i < take; ++i) samp.push_back(U.sampled[size_t((U.cursor + i) % ns)]);
        U.cursor = (U.cursor + take) % ns;
    }
    U.last_sampled = int(samp.size());
    U.last_refused = 0;
    int fell = 0, back = 0;
    double w = 0.0;
    if (na > 0 || !samp.empty()) {
        // per-pair budget: tol * (max |P_mu| over the target's system) / (active far pairs of the target),
        // so that by the triangle inequality the system's error stays within tol per component
        std::vector<int> all(p->n_dom);
        for (int i = 0; i < p->n_dom; ++i) all[i] = i;
        for (size_t j0 = 0; j0 < all.size(); j0 += kMaxJobs) {
            BudgetArgs ba{};
            ba.n_jobs = int(std::min<size_t>(kMaxJobs, all.size() - j0));
            for (int j = 0; j < ba.n_jobs; ++j) {
                const int s = all[j0 + j];
                ba.jobs[j].out = static_cast<const float *>(out[s]);
                ba.jobs[j].budget = p->at<float>(U.off_budget) + size_t(s) * 4;
                ba.jobs[j].npts = p->dom[s].npts;
                ba.jobs[j].scale = 1.0f;
            }
            launch_budget(ba, st);
        }
        check_launch();
        std::vector<float> amax(size_t(p->n_dom) * 4), bud(size_t(p->n_dom) * 4, 0.f);
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(hipMemcpy(amax.data(), p->ws + U.off_budget, amax.size() * 4, hipMemcpyDeviceToHost));
        std::vector<float> smax(p->sys.size() * 4, 0.f);
        for (int i = 0; i < p->n_dom; ++i)
            for (int mu = 0; mu < 4; ++mu)
                smax[size_t(p->dom[i].sys) * 4 + mu] = std::max(smax[size_t(p->dom[i].sys) * 4 + mu], amax[size_t(i) * 4 + mu]);
        // active far pairs per target before this judgement (the budgets' count)
        std::vector<int> n_act(p->n_dom, 0);
        for (int s : U.synth_targets) n_act[s] = active_far(p, s);
        for (int s : U.synth_targets) {
            if (n_act[s] == 0) continue;
            for (int mu = 0; mu < 4; ++mu)
                bud[size_t(s) * 4 + mu] = float(tol * smax[size_t(p->dom[s].sys) * 4 + mu] / n_act[s]);
        }
        HIP_OK(hipMemcpy(p->ws + U.off_budget, bud.data(), bud.size() * 4, hipMemcpyHostToDevice));
        // a fallen-back pair returns within readmit x the budget it would have
        // as one more active far pair of its target, in every component
        auto readmit_ok = [&](const FarPairH &F, const float *r) {
            if (U.readmit <= 0) return false;
            bool ok = true;
            for (int mu = 0; mu < 4; ++mu) {
                const double b = tol * smax[size_t(p->dom[F.s].sys) * 4 + mu] / (n_act[F.s] + 1);
                ok = ok && r[mu] <= U.readmit * b;
            }
            return ok;
        };
        auto ratio = [&](const FarPairH &F, const float *r) {
            for (int mu = 0; mu < 4; ++mu) {
                const double b = bud[size_t(F.s) * 4 + mu];
                w = std::max(w, b > 0 ? r[mu] / b : (r[mu] > 0 ? INFINITY : 0.0));
            }
        };
        if (na > 0) {
            launch_fill_zero(p->ws + U.off_fail, (size_t(na) * 4 + 15) / 16 * 16, st);
            judge_fields(p, st, [&](const int *vs, int cnt) {
                ProjArgs pa{};
                CorrArgs ca{};
                pa.n_jobs = ca.n_jobs = cnt;
                for (int j = 0; j < cnt; ++j) {
                    const int v = vs[j], f = U.aud[v];
                    const FarPairH &F = U.pairs[f];
                    const DomainP &t = p->dom[F.s];
                    ProjJob &J = pa.jobs[j];
                    J.F = jfield(p, j);
                    J.Q = nullptr;
                    J.coef_in = p->at<float>(U.off_pc) + size_t(f) * kNOut;
                    J.coef = p->at<float>(U.off_jcb) + size_t(j) * kNOut;
                    J.resid = p->at<float>(U.off_jres) + size_t(v) * 8;
                    for (int c = 0; c < 3; ++c) J.N[c] = t.N[c];
                    J.npts = t.npts;
                    CorrJob &C = ca.jobs[j];
                    C.F = J.F;
                    C.pc = J.coef_in;
                    C.resid = J.resid;
                    C.budget = p->at<float>(U.off_budget) + size_t(F.s) * 4;
                    C.out = static_cast<float *>(out[F.s]);
                    C.fail = p->at<int32_t>(U.off_fail) + v;
                    for (int c = 0; c < 3; ++c) C.N[c] = t.N[c];
                    C.active = F.plain ? 0 : 1;
                    ca.max_pts = std::max<int64_t>(ca.max_pts, t.npts);
                }
                launch_project(pa, false, st);
                launch_correct(ca, st);
                check_launch();
            });
            std::vector<int32_t> flags(na);
            std::vector<float> res(size_t(na) * 8);
            HIP_OK(hipStreamSynchronize(st));
            HIP_OK(hipMemcpy(flags.data(), p->ws + U.off_fail, size_t(na) * 4, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(res.data(), p->ws + U.off_jres, res.size() * 4, hipMemcpyDeviceToHost));
            for (int v = 0; v < na; ++v) {
                FarPairH &F = U.pairs[U.aud[v]];
                if (F.plain) {
                    if (readmit_ok(F, &res[size_t(v) * 8])) {
                        F.plain = false;
                        ++back;
                    }
                    continue;
                }
                ratio(F, &res[size_t(v) * 8]);
                if (flags[v]) {
                    F.plain = true;
                    ++fell;
                }
            }
        }
        if (!samp.empty()) {
            // plain fields at the sample points, compared with the surrogate terms
            const int ns = int(samp.size());
            sample_fields(p, samp, st);
            U.h_jjobs.assign(size_t(ns), SampleJudgeJob{});
            for (int i = 0; i < ns; ++i) {
                const FarPairH &F = U.pairs[size_t(samp[size_t(i)])];
                SampleJudgeJob &Q = U.h_jjobs[size_t(i)];
                Q.F = p->at<float>(U.off_sfield) + size_t(i) * kSamplePts * 4;
                Q.pc = p->at<float>(U.off_pc) + size_t(samp[size_t(i)]) * kNOut;
                Q.budget = p->at<float>(U.off_budget) + size_t(F.s) * 4;
                Q.resid = p->at<float>(U.off_sres) + size_t(i) * 8;
                Q.fail = p->at<int32_t>(U.off_sfail) + i;
                for (int c = 0; c < 3; ++c) Q.N[c] = p->dom[F.s].N[c];
                Q.active = F.plain ? 0 : 1;
            }
            HIP_OK(hipMemcpyAsync(p->ws + U.off_jjobs, U.h_jjobs.data(), size_t(ns) * sizeof(SampleJudgeJob),
                                  hipMemcpyHostToDevice, st));
            SampleJudgeArgs ja{};
            ja.jobs = p->at<SampleJudgeJob>(U.off_jjobs);
            ja.n_jobs = ns;
            launch_sample_judge(ja, st);
            check_launch();
            std::vector<int32_t> flags(static_cast<size_t>(ns));
            std::vector<float> res(size_t(ns) * 8);
            HIP_OK(hipStreamSynchronize(st));
            HIP_OK(hipMemcpy(flags.data(), p->ws + U.off_sfail, size_t(ns) * 4, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(res.data(), p->ws + U.off_sres, res.size() * 4, hipMemcpyDeviceToHost));
            for (int i = 0; i < ns; ++i) {
                const int f = samp[size_t(i)];
                FarPairH &F = U.pairs[size_t(f)];
                if (F.plain) {
                    if (F.slot >= 0 && readmit_ok(F, &res[size_t(i) * 8])) {
                        slot_release(p, F.slot, st);
                        ++back;
                    }
                    continue;
                }
                ratio(F, &res[size_t(i) * 8]);
                if (!flags[size_t(i)]) continue;
                int k = -1;
                for (size_t j = 0; j < U.slots.size() && k < 0; ++j)
                    if (U.slots[j].f < 0) k = int(j);
                if (k < 0) {
                    ++U.last_refused;
                    continue;
                }
                slot_assign(p, k, f, st);
                ++fell;
            }
        }
        if (fell || back) {
            // the schedules changed: a captured step no longer matches them
            release_graph(p);
            main_k2(p, p->k2, plain_pair);
            upload_k2(p, p->k2, p->k2_dev, st);
            rebuild_blocked(p, st);
            if (!U.slots.empty()) {
                slot_k2(p);
                upload_k2(p, U.k2p, U.k2p_dev, st);
            }
            upload_csr(p, st);
            HIP_OK(hipStreamSynchronize(st));
            plan_stats(p);
        }
    }
    if (n_fallback) *n_fallback = fell;
    if (worst) *worst = w;
    if (n_readmitted) *n_readmitted = back;
}

void sur_readmit(rp_plan p, double factor) {
    SurrogateH &U = p->sur;
    if (!U.on) fail(RP_ERR_STATE, "surrogate not configured (rp_surrogate_configure)");
    if (!(factor >= 0) || !std::isfinite(factor)) fail(RP_ERR_ARG, "factor must be finite and >= 0");
    U.readmit = factor;
}

}  // namespace rpot_host

extern "C" {

rp_status rp_surrogate_data_scales(const float *x, const float *t, int64_t n, int32_t n_lags, float *in_scale,
                                   float *out_scale, void *hip_stream) {
    if (!x || !t || !in_scale || !out_scale || n < 1 || n_lags < 1 || n_lags > 1024) return RP_ERR_ARG;
    ScaleDataArgs a{};
    a.x = x;
    a.t = t;
    a.in_scale = in_scale;
    a.out_scale = out_scale;
    a.n = n;
    a.n_lags = n_lags;
    a.n_in = kNBlocks * kNFeat * n_lags + kNGeo;
    launch_data_scales(a, static_cast<hipStream_t>(hip_stream));
    return hipGetLastError() == hipSuccess ? RP_OK : RP_ERR_DEVICE;
}

rp_status rp_surrogate_scale_data(float *x, float *t, int64_t n, int32_t n_lags, const float *in_scale,
                                  const float *out_scale, void *hip_stream) {
    if ((!x && !t) || (x && !in_scale) || (t && !out_scale) || n < 1 || n_lags < 1 || n_lags > 1024)
        return RP_ERR_ARG;
    if (n > int64_t(65535)) {
        // one launch row per sample: several launches of at most 65535 rows
        for (int64_t i0 = 0; i0 < n; i0 += 65535) {
            const rp_status s = rp_surrogate_scale_data(
                x ? x + i0 * (int64_t(kNBlocks) * kNFeat * n_lags + kNGeo) : nullptr, t ? t + i0 * kNOut : nullptr,
                std::min<int64_t>(65535, n - i0), n_lags, in_scale, out_scale, hip_stream);
            if (s != RP_OK) return s;
        }
        return RP_OK;
    }
    ScaleDataArgs a{};
    a.x_rw = x;
    a.t_rw = t;
    a.in_scale_c = in_scale;
    a.out_scale_c = out_scale;
    a.n = n;
    a.n_lags = n_lags;
    a.n_in = kNBlocks * kNFeat * n_lags + kNGeo;
    launch_scale_data(a, static_cast<hipStream_t>(hip_stream));
    return hipGetLastError() == hipSuccess ? RP_OK : RP_ERR_DEVICE;
}

}  // extern "C"
