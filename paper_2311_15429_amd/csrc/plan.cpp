// Host runtime: planning (lag windows, FFT pads, ring depths, Green-spectrum
// table, lag-sum schedule), workspace layout, and the C-ABI entry points.
//
// The plan follows the paper's multi-domain scheme (Secs. II-IV): every
// ordered pair (target s <- source n) of one system couples through the lags
// its point distances allow; each source keeps the spectra of its past
// source differences in a ring as deep as its longest lag; a step is the
// forward transform of the new sources, the lag sum in the frequency domain,
// and the inverse transform cropped to each target.
#include "plan_internal.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>

using namespace rpot;

namespace rpot_host {

namespace {
thread_local std::string g_create_error;

// Smallest even 2^a 3^b >= n.
int smooth_even(int n) {
    for (int m = std::max(n, 2);; ++m) {
        if (m & 1) continue;
        int r = m;
        while (r % 2 == 0) r /= 2;
        while (r % 3 == 0) r /= 3;
        if (r == 1) return m;
    }
}
}  // namespace

RadixPlan make_radix(int P) {
    RadixPlan rp{};
    int n = P;
    while (n % 4 == 0) { rp.r[rp.n++] = 4; n /= 4; }
    while (n % 2 == 0) { rp.r[rp.n++] = 2; n /= 2; }
    while (n % 3 == 0) { rp.r[rp.n++] = 3; n /= 3; }
    if (n != 1) fail(RP_ERR_UNSUPPORTED, "FFT length is not 2^a 3^b");
    return rp;
}

// ---------------------------------------------------------------------------
// Planning

// Smallest and largest |r - r'| between the grid points of target s and source
// n: per axis the displacement takes the values o_s - o_n + h d,
// d = -(N_n - 1) .. N_s - 1, and the axes are independent.
void pair_distance(const DomainP &s, const DomainP &n, double h, double &rmin, double &rmax) {
    double mn2 = 0, mx2 = 0;
    for (int a = 0; a < 3; ++a) {
        const double base = s.o[a] - n.o[a];
        const double lo = base - h * (n.N[a] - 1), hi = base + h * (s.N[a] - 1);
        double mn;
        if (lo <= 0 && hi >= 0) {
            // closest attainable value to zero
            const double d0 = std::floor(-base / h);
            mn = std::fabs(base + h * d0);
            for (double d = d0 - 1; d <= d0 + 2; d += 1) {
                if (d < -(n.N[a] - 1) || d > s.N[a] - 1) continue;
                mn = std::min(mn, std::fabs(base + h * d));
            }
        } else {
            mn = std::min(std::fabs(lo), std::fabs(hi));
        }
        const double mx = std::max(std::fabs(lo), std::fabs(hi));
        mn2 += mn * mn;
        mx2 += mx * mx;
    }
    rmin = std::sqrt(mn2);
    rmax = std::sqrt(mx2);
}

// FFT pads of every system and the shape classes.  A pair (target s <- source
// n) is a linear convolution of length N_s + N_n - 1 per axis, and only the
// targets take sources: the pad covers the largest target plus the largest
// source of the system.
void plan_pads(rp_plan p) {
    for (SystemP &S : p->sys) {
        for (int a = 0; a < 3; ++a) {
            int mt = 1, mn = 1;
            for (int i : S.doms) {
                mn = std::max(mn, p->dom[i].N[a]);
                if (is_target(p, i)) mt = std::max(mt, p->dom[i].N[a]);
            }
            S.P[a] = smooth_even(mt + mn - 1);
            if (S.P[a] > kMaxPad) fail(RP_ERR_UNSUPPORTED, "FFT pad above 512 points");
        }
        S.Hz = S.P[2] / 2 + 1;
        S.C = int64_t(S.P[0]) * S.P[1] * S.Hz;
        S.Cpad = (S.C + kTile - 1) / kTile * kTile;
    }

    // shape classes (same dims and pads) for batched FFT launches
    p->cls.clear();
    for (int i = 0; i < p->n_dom; ++i) {
        const DomainP &d = p->dom[i];
        const SystemP &S = p->sys[d.sys];
        int found = -1;
        for (size_t c = 0; c < p->cls.size(); ++c) {
            const ClassP &K = p->cls[c];
            if (std::equal(K.N, K.N + 3, d.N) && std::equal(K.P, K.P + 3, S.P)) found = int(c);
        }
        if (found < 0) {
            ClassP K{};
            std::copy(d.N, d.N + 3, K.N);
            std::copy(S.P, S.P + 3, K.P);
            K.Hz = S.Hz;
            K.C = S.C;
            p->cls.push_back(K);
            found = int(p->cls.size()) - 1;
        }
        p->cls[found].doms.push_back(i);
        if (is_target(p, i)) p->cls[found].tdoms.push_back(i);
        p->dom[i].cls = found;
        const int lpb = zfwd_lines_per_block(S.P[2], p->p64);
        p->dom[i].zblocks = (4 * ((d.N[0] * d.N[1] + 1) / 2) + lpb - 1) / lpb;
    }
}

// Domains, systems, lag windows, FFT pads and shape classes.
void plan_geometry(rp_plan p, const int32_t *dims, const double *origins, const int32_t *system_id) {
    const int nd = p->n_dom;
    p->dom.resize(nd);
    std::map<int32_t, int> sys_index;
    for (int i = 0; i < nd; ++i) {
        DomainP &d = p->dom[i];
        for (int a = 0; a < 3; ++a) {
            d.N[a] = dims[3 * i + a];
            d.o[a] = origins[3 * i + a];
            if (d.N[a] < 1) fail(RP_ERR_ARG, "dims must be >= 1");
            if (!std::isfinite(d.o[a])) fail(RP_ERR_ARG, "origins must be finite");
        }
        d.npts = int64_t(d.N[0]) * d.N[1] * d.N[2];
        const int32_t id = system_id ? system_id[i] : 0;
        auto it = sys_index.find(id);
        if (it == sys_index.end()) {
            it = sys_index.emplace(id, int(p->sys.size())).first;
            p->sys.emplace_back();
        }
        d.sys = it->second;
        p->sys[d.sys].doms.push_back(i);
    }

    // windows
    const double cdt = p->c * p->dt;
    const bool finite_c = std::isfinite(p->c);
    p->pair.assign(size_t(nd) * nd, PairP{});
    for (const SystemP &S : p->sys) {
        for (int s : S.doms) {
            for (int n : S.doms) {
                PairP &q = p->pr(s, n);
                pair_distance(p->dom[s], p->dom[n], p->h, q.rmin, q.rmax);
                if (s != n && q.rmin < p->h * (1.0 - 1e-12)) {
                    char buf[160];
                    std::snprintf(buf, sizeof buf,
                                  "sub-domains %d and %d are closer than one grid step (%.6g < h)", s, n, q.rmin);
                    fail(RP_ERR_GEOMETRY, buf);
                }
                if (finite_c) {
                    const double x = q.rmin / cdt, y = q.rmax / cdt;
                    // guard that only widens the window under rounding
                    q.m_lo = int(std::max(0.0, std::floor(x - 1e-9 * std::max(1.0, x))));
                    q.m_hi = int(std::ceil(y + 1e-9 * std::max(1.0, y)));
                    if (s == n) q.m_hi = std::max(q.m_hi, 1);   // the self cell reaches lag 1
                } else {
                    q.m_lo = q.m_hi = 0;
                }
            }
        }
    }

    plan_pads(p);
}

// A pair whose plain lag sum may run: every near pair, and a far pair whose
// source keeps its history (it can be judged and can fall back).
bool keeps_history(rp_plan p, int s, int n) {
    if (!is_target(p, s)) return false;
    const SurrogateH &S = p->sur;
    if (!S.on) return true;
    const int f = S.far_index[size_t(s) * p->n_dom + n];
    return f < 0 || S.pairs[f].audited;
}

// A pair summed by the plain lag sum of every step (a fallen-back far pair of
// a non-audit source is summed from its fallback slot instead).
bool plain_pair(rp_plan p, int s, int n) {
    if (!is_target(p, s)) return false;
    const SurrogateH &S = p->sur;
    if (!S.on) return true;
    const int f = S.far_index[size_t(s) * p->n_dom + n];
    return f < 0 || (S.pairs[f].plain && S.pairs[f].audited);
}

// Lag-sum schedule of the members (accumulator slots of system si): groups of
// up to 8 members, and per group the sources any member takes with the union
// of their windows.
void build_k2(rp_plan p, int si, const std::vector<K2Member> &members, K2Tables &T, int gmax, int m_cap) {
    const SystemP &S = p->sys[si];
    // every pair's window clipped to lags <= m_cap
    auto lo_of = [&](const PairP &q) { return q.m_lo; };
    auto hi_of = [&](const PairP &q) { return std::min(q.m_hi, m_cap); };
    for (size_t g0 = 0; g0 < members.size(); g0 += size_t(gmax)) {
        K2Group G{};
        G.C = S.C;
        G.spec_base = S.spec_base;
        G.n_members = int(std::min<size_t>(size_t(gmax), members.size() - g0));
        const K2Member *mb = members.data() + g0;
        for (int t = 0; t < G.n_members; ++t) G.member[t] = mb[t].slot;
        G.entry_begin = int(T.entries.size());
        G.src_begin = int(T.srcs.size());
        for (int n : S.doms) {
            uint32_t takes = 0;
            for (int t = 0; t < G.n_members; ++t)
                if (std::find(mb[t].srcs.begin(), mb[t].srcs.end(), n) != mb[t].srcs.end() &&
                    lo_of(p->pr(mb[t].s, n)) <= hi_of(p->pr(mb[t].s, n)))
                    takes |= 1u << t;
            if (!takes) continue;
            K2Src R{};
            R.n = n;
            R.m_min = INT32_MAX;
            R.m_max = -1;
            K2Pair Qs[kGroupMax] = {};
            for (int t = 0; t < kGroupMax; ++t) {
                if ((takes >> t) & 1u) {
                    const PairP &q = p->pr(mb[t].s, n);
                    if (q.spec0 < 0) fail(RP_ERR_STATE, "internal: lag sum over a pair without spectra");
                    Qs[t].row0 = int32_t(q.spec0 / kTile) - q.m_lo;
                    Qs[t].w = q.m_hi - q.m_lo + 1;
                    if (q.conj) R.conj |= 1u << t;
                    if (real_spec(p, mb[t].s, n)) R.real |= 1u << t;
                    R.m_min = std::min(R.m_min, lo_of(q));
                    R.m_max = std::max(R.m_max, hi_of(q));
                }
            }
            R.mask_off = int32_t(T.masks.size());
            for (int m = R.m_min; m <= R.m_max; ++m) {
                uint32_t mk = 0;
                for (int t = 0; t < G.n_members; ++t) {
                    if (!((takes >> t) & 1u)) continue;
                    const PairP &q = p->pr(mb[t].s, n);
                    if (m >= lo_of(q) && m <= hi_of(q)) mk |= 1u << t;
                }
                T.masks.push_back(mk);
            }
            // one record per ring that holds part of the window: the source's
            // ring (lags from 0) and its split rings (lags from their start)
            const DomainP &dn = p->dom[n];
            // (ring, first lag summed from it, last lag, age of its newest snapshot)
            std::vector<std::array<int, 4>> rings{{n, 0, dn.depth - 1, 0}};
            for (int v : dn.vr)
                rings.push_back({p->vring[v].idx, p->vring[v].lag_lo, p->vring[v].hi, p->vring[v].lo});
            for (const auto &rg : rings) {
                const int a = std::max(R.m_min, rg[1]), b = std::min(R.m_max, rg[2]);
                if (a > b) continue;
                K2Src Rs = R;
                Rs.n = rg[0];
                Rs.m_min = a;
                Rs.m_max = b;
                Rs.m_base = rg[3];
                Rs.mask_off = R.mask_off + (a - R.m_min);
                for (int t = 0; t < kGroupMax; ++t) T.pairs.push_back(Qs[t]);
                T.srcs.push_back(Rs);
            }
            for (int m = R.m_min; m <= R.m_max; ++m) {
                K2Entry E{};
                E.src = n;
                E.m = m;
                for (int t = 0; t < G.n_members; ++t) {
                    if (!((takes >> t) & 1u)) continue;
                    const PairP &q = p->pr(mb[t].s, n);
                    if (m < lo_of(q) || m > hi_of(q)) continue;
                    E.mask |= 1u << t;
                    if (q.conj) E.conj |= 1u << t;
                    if (real_spec(p, mb[t].s, n)) E.real |= 1u << t;
                    E.spec_tile[t] = int32_t(q.spec0 / kTile + (m - q.m_lo));
                    E.spec_w[t] = q.m_hi - q.m_lo + 1;
                }
                if (E.mask) T.entries.push_back(E);
            }
        }
        G.entry_end = int(T.entries.size());
        G.src_end = int(T.srcs.size());
        const int gi = int(T.groups.size());
        T.groups.push_back(G);
        for (int64_t k0 = 0; k0 < S.C; k0 += kTile) T.items.push_back(K2Item{gi, int32_t(k0)});
    }
}

// Template width of the schedule, work order and size checks.
void finish_k2(rp_plan p, K2Tables &T) {
    int max_members = 1;
    for (const K2Group &G : T.groups) max_members = std::max(max_members, G.n_members);
    T.tg = max_members <= 1 ? 1 : (max_members <= 2 ? 2 : (max_members <= 4 ? 4 : 8));
    // longest work first (for the persistent launch): a group's tile costs its
    // ring reads plus its spectrum reads
    std::vector<double> gcost(T.groups.size(), 0.0);
    for (size_t gi = 0; gi < T.groups.size(); ++gi) {
        const K2Group &G = T.groups[gi];
        for (int e = G.entry_begin; e < G.entry_end; ++e)
            gcost[gi] += 4.0 + double(__builtin_popcount(T.entries[e].mask));
    }
    std::stable_sort(T.items.begin(), T.items.end(),
                     [&](const K2Item &x, const K2Item &y) { return gcost[x.group] > gcost[y.group]; });
    if (T.entries.size() > size_t(INT32_MAX) || T.items.size() > size_t(INT32_MAX) ||
        T.masks.size() > size_t(INT32_MAX))
        fail(RP_ERR_UNSUPPORTED, "schedule too large");
    // ring offsets and depths (known once the layout exists)
    if (!p->domdev.empty()) {
        for (K2Entry &E : T.entries) {
            E.ring_off = p->domdev[E.src].ring_off;
            E.depth = p->domdev[E.src].depth;
        }
        for (K2Src &R : T.srcs) {
            R.ring_off = p->domdev[R.n].ring_off;
            R.depth = p->domdev[R.n].depth;
        }
    }
}

// The plain lag sum of every domain over its plain pairs (groups of up to
// gmax targets, windows clipped to lags <= m_cap).
void main_k2(rp_plan p, K2Tables &T, bool (*pred)(rp_plan, int, int), int gmax, int m_cap) {
    T = K2Tables{};
    for (size_t si = 0; si < p->sys.size(); ++si) {
        std::vector<K2Member> members;
        for (int s : p->sys[si].doms) {
            if (!is_target(p, s)) continue;
            K2Member M{s, s, {}};
            for (int n : p->sys[si].doms)
                if (pred(p, s, n)) M.srcs.push_back(n);
            members.push_back(std::move(M));
        }
        build_k2(p, int(si), members, T, gmax, m_cap);
    }
    finish_k2(p, T);
}

void order_k2b(rp_plan p) {
    K2Tables &T = p->k2b;
    std::vector<double> gcost(T.groups.size(), 0.0);
    for (size_t gi = 0; gi < T.groups.size(); ++gi)
        for (int e = T.groups[gi].entry_begin; e < T.groups[gi].entry_end; ++e) gcost[gi] += 1.0;
    if (p->k2b_tile_major)
        std::stable_sort(T.items.begin(), T.items.end(), [&](const K2Item &x, const K2Item &y) {
            return x.k0 != y.k0 ? x.k0 < y.k0 : gcost[x.group] > gcost[y.group];
        });
    else
        std::stable_sort(T.items.begin(), T.items.end(), [&](const K2Item &x, const K2Item &y) {
            return gcost[x.group] != gcost[y.group] ? gcost[x.group] > gcost[y.group] : x.k0 < y.k0;
        });
    if (p->ws && !T.items.empty())
        HIP_OK(hipMemcpyAsync(p->ws + p->k2b_dev.items, T.items.data(), T.items.size() * sizeof(K2Item),
                              hipMemcpyHostToDevice, p->stream));
}

// Targets per group of the additions of a blocked step (its lags m < i): one.
// Those lags are the self pairs' (a target's own sources), so targets share no
// source row and larger groups only raise the registers per thread.
constexpr int kAddGroup = 1;

// Device-table capacities of a schedule (its own sizes).
void size_k2(K2Dev &D, const K2Tables &T) {
    D.cap_items = T.items.size();
    D.cap_groups = T.groups.size();
    D.cap_entries = T.entries.size();
    D.cap_srcs = T.srcs.size();
    D.cap_pairs = T.pairs.size();
    D.cap_masks = T.masks.size();
}

// Capacities raised to hold schedule T as well.
void grow_k2(K2Dev &D, const K2Tables &T) {
    D.cap_items = std::max(D.cap_items, T.items.size());
    D.cap_groups = std::max(D.cap_groups, T.groups.size());
    D.cap_entries = std::max(D.cap_entries, T.entries.size());
    D.cap_srcs = std::max(D.cap_srcs, T.srcs.size());
    D.cap_pairs = std::max(D.cap_pairs, T.pairs.size());
    D.cap_masks = std::max(D.cap_masks, T.masks.size());
}

// The blocked schedules rebuilt for the current plain pairs (after the
// surrogate's judge moved pairs between the network and the plain sum) and
// copied into their device tables.
void rebuild_blocked(rp_plan p, hipStream_t st) {
    if (p->kb <= 1) return;
    main_k2(p, p->k2b, plain_pair, 1);
    order_k2b(p);
    upload_k2(p, p->k2b, p->k2b_dev, st);
    for (int i = 1; i < p->kb; ++i) {
        main_k2(p, p->k2c[size_t(i - 1)], plain_pair, kAddGroup, i - 1);
        upload_k2(p, p->k2c[size_t(i - 1)], p->k2c_dev[size_t(i - 1)], st);
    }
    update_fused_additions(p);
}

// Ring depths, stored Green spectra and the lag-sum schedules.
void plan_tables(rp_plan p) {
    const int nd = p->n_dom;
    p->vring.clear();
    p->domdev.clear();   // rebuilt by plan_layout for the new ring indices
    for (int n = 0; n < nd; ++n) {
        DomainP &d = p->dom[n];
        std::vector<std::pair<int, int>> iv;
        for (int s : p->sys[d.sys].doms)
            if (keeps_history(p, s, n)) iv.push_back({p->pr(s, n).m_lo, p->pr(s, n).m_hi});
        int mh = 0;
        for (const auto &w : iv) mh = std::max(mh, w.second);
        d.span = mh + 1;
        d.depth = mh + 1;
        d.vr.clear();
        d.d1 = 0;
        d.t1_idx = -1;
        if (p->split_gap <= 0 || iv.empty()) continue;
        // merge the pairs' windows; a gap of split_gap lags or more starts a new
        // ring.  The main ring holds lag 0 (the ingest writes there); when the
        // first window starts split_gap or more lags later (a source that is
        // not a target reaches only other domains), it keeps lag 0 alone
        // With kb lag-sum steps per pass a ring also stores the kb - 1 ages
        // below its first lag (the blocked pass reads them); gaps are counted
        // to that widened start, which stays at lag 2 or later.
        std::sort(iv.begin(), iv.end());
        const int wid = p->kb - 1;
        struct Win {
            int lo, hi, lag_lo;   // stored ages lo .. hi; lags summed from lag_lo
        };
        std::vector<Win> win{{0, iv[0].second, 0}};
        if (iv[0].first - wid - 1 >= p->split_gap) win = {{0, 0, 0}, {iv[0].first - wid, iv[0].second, iv[0].first}};
        for (size_t i = 1; i < iv.size(); ++i) {
            if (iv[i].first - wid - win.back().hi - 1 >= p->split_gap)
                win.push_back({iv[i].first - wid, iv[i].second, iv[i].first});
            else
                win.back().hi = std::max(win.back().hi, iv[i].second);
        }
        if (win.size() < 2) continue;
        // split only where the spectra saved outweigh the real-space ring (in
        // device memory; with the host tier only its staging snapshots) and
        // the transform scratch of the extra rings
        const SystemP &S = p->sys[d.sys];
        const double spec_slot = double(S.Cpad) * 4 * p->ring_esz;
        int kept = 0;
        for (const auto &w : win) kept += w.hi - w.lo + 1;
        const double saved = double(d.span - kept) * spec_slot;
        const double scratch = double(d.N[0]) * (d.N[1] + S.P[1]) * S.Hz * 4 * p->csz;
        const double real_slots = p->hist_host ? double(win.size()) : double(win.back().lo + 1);
        const double cost = real_slots * 4 * double(d.npts) * p->tsz + double(win.size() - 1) * scratch;
        if (saved <= cost) continue;
        d.depth = win[0].hi + 1;
        d.d1 = win.back().lo + 1;
        for (size_t w = 1; w < win.size(); ++w) {
            VRingP v;
            v.n = n;
            v.lo = win[w].lo;
            v.hi = win[w].hi;
            v.lag_lo = win[w].lag_lo;
            v.W = v.hi - v.lo + 1;
            d.vr.push_back(int(p->vring.size()));
            p->vring.push_back(v);
        }
    }
    // judge by sample: every far source keeps a real-space history deep enough
    // for the direct sum over its pairs' windows (retarded samples l - m and
    // l - m - 1 with m <= m_hi)
    if (p->sur.on && p->sur.per_judge >= 0)
        for (const FarPairH &F : p->sur.pairs) p->dom[F.n].d1 = std::max(p->dom[F.n].d1, p->pr(F.s, F.n).m_hi + 2);
    // head slots: domains, judge accumulators, split rings, real-space rings,
    // fallback slots
    {
        int idx = nd + int(p->sur.on ? p->sur.aud.size() : 0);
        for (VRingP &v : p->vring) v.idx = idx++;
        for (DomainP &d : p->dom)
            if (d.d1 > 0) d.t1_idx = idx++;
        for (SlotP &k : p->sur.slots) k.idx = idx++;
        p->n_heads = idx;
    }

    // Green spectra: one set per unordered pair; the reversed pair uses the
    // complex conjugate (its real-space kernel is the mirror image).  Pairs
    // that never run the plain lag sum in either direction store none.
    int64_t spec_base = 0;
    for (SystemP &S : p->sys) {
        S.spec_base = spec_base;
        int64_t cnt = 0, nsp = 0;
        for (size_t a = 0; a < S.doms.size(); ++a) {
            for (size_t b = a; b < S.doms.size(); ++b) {
                const int s = S.doms[a], n = S.doms[b];
                PairP &q = p->pr(s, n);
                PairP &r = p->pr(n, s);
                q.spec0 = r.spec0 = -1;
                if (!keeps_history(p, s, n) && !keeps_history(p, n, s)) continue;
                q.spec0 = cnt;
                q.conj = false;
                cnt += int64_t(q.m_hi - q.m_lo + 1) * S.Cpad;
                nsp += q.m_hi - q.m_lo + 1;
                if (s != n) {
                    r.spec0 = q.spec0;
                    r.conj = true;
                }
            }
        }
        S.n_spec = nsp;
        S.spec_elems = cnt;
        spec_base += cnt;
        if (cnt / kTile > int64_t(INT32_MAX)) fail(RP_ERR_UNSUPPORTED, "Green spectra table too large");
    }

    main_k2(p, p->k2, plain_pair);
    // temporal blocking: the pass of a block's first step and the lags m < i
    // of its steps i = 1 .. kb-1
    p->k2b = K2Tables{};
    p->k2c.assign(size_t(std::max(0, p->kb - 1)), K2Tables{});
    p->k2c_dev.assign(p->k2c.size(), K2Dev{});
    if (p->kb > 1) {
        main_k2(p, p->k2b, plain_pair, 1);
        order_k2b(p);
        size_k2(p->k2b_dev, p->k2b);
        for (int i = 1; i < p->kb; ++i) {
            main_k2(p, p->k2c[size_t(i - 1)], plain_pair, kAddGroup, i - 1);
            size_k2(p->k2c_dev[size_t(i - 1)], p->k2c[size_t(i - 1)]);
        }
        if (p->sur.on) {
            // room for the largest blocked schedules a fallback can reach
            K2Tables cb;
            main_k2(p, cb, keeps_history, 1);
            grow_k2(p->k2b_dev, cb);
            for (int i = 1; i < p->kb; ++i) {
                K2Tables cc;
                main_k2(p, cc, keeps_history, kAddGroup, i - 1);
                grow_k2(p->k2c_dev[size_t(i - 1)], cc);
            }
        }
    }
    update_fused_additions(p);
    // room for the largest schedule a fallback can reach
    K2Tables cap;
    main_k2(p, cap, keeps_history);
    K2Dev &D = p->k2_dev;
    D.cap_items = std::max(cap.items.size(), p->k2.items.size());
    D.cap_groups = std::max(cap.groups.size(), p->k2.groups.size());
    D.cap_entries = std::max(cap.entries.size(), p->k2.entries.size());
    D.cap_srcs = std::max(cap.srcs.size(), p->k2.srcs.size());
    D.cap_pairs = std::max(cap.pairs.size(), p->k2.pairs.size());
    D.cap_masks = std::max(cap.masks.size(), p->k2.masks.size());

    // judge schedule of the surrogate: one slot per audited far pair
    SurrogateH &U = p->sur;
    U.judge = K2Tables{};
    if (U.on && !U.aud.empty()) {
        for (size_t si = 0; si < p->sys.size(); ++si) {
            std::vector<K2Member> members;
            for (size_t v = 0; v < U.aud.size(); ++v) {
                const FarPairH &F = U.pairs[U.aud[v]];
                if (p->dom[F.s].sys != int(si)) continue;
                members.push_back(K2Member{nd + int(v), F.s, {F.n}});
            }
            build_k2(p, int(si), members, U.judge, kGroupMax, INT32_MAX);
        }
        finish_k2(p, U.judge);
        K2Dev &J = U.judge_dev;
        J.cap_items = U.judge.items.size();
        J.cap_groups = U.judge.groups.size();
        J.cap_entries = U.judge.entries.size();
        J.cap_srcs = U.judge.srcs.size();
        J.cap_pairs = U.judge.pairs.size();
        J.cap_masks = U.judge.masks.size();
    }
}

// Ring formats with per-snapshot scales (FP16/BF16: [depth][4] floats) or
// per-snapshot-and-tile scales (I16: [tile][depth][4] floats).
bool ring_scaled(rp_plan p) {
    return p->ring_fmt == RING_F16 || p->ring_fmt == RING_BF16 || p->ring_fmt == RING_I16;
}
size_t scale_bytes(rp_plan p, int depth, int64_t Cpad) {
    const size_t rows = p->ring_fmt == RING_I16 ? size_t(depth) * size_t(Cpad / kTile) : size_t(depth);
    return (rows * 4 * sizeof(float) + 15) / 16 * 16;
}

void plan_layout(rp_plan p) {
    size_t off = 0;
    auto alloc = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + kAlign - 1) / kAlign * kAlign;
        return o;
    };
    auto alloc_k2 = [&](K2Dev &D) {
        D.items = alloc(std::max<size_t>(1, D.cap_items) * sizeof(K2Item));
        D.groups = alloc(std::max<size_t>(1, D.cap_groups) * sizeof(K2Group));
        D.entries = alloc(std::max<size_t>(1, D.cap_entries) * sizeof(K2Entry));
        D.srcs = alloc(std::max<size_t>(1, D.cap_srcs) * sizeof(K2Src));
        D.pairs = alloc(std::max<size_t>(1, D.cap_pairs) * sizeof(K2Pair));
        D.masks = alloc(std::max<size_t>(1, D.cap_masks) * sizeof(uint32_t));
    };
    const size_t n_slots = size_t(p->n_heads);
    p->tw64.clear();
    p->tw32.clear();
    p->off_state = alloc(64);
    p->off_head = alloc(n_slots * sizeof(int32_t));
    p->off_prev_head = alloc(n_slots * sizeof(int32_t));
    p->off_counter = alloc(16);
    alloc_k2(p->k2_dev);
    if (p->sur.on) alloc_k2(p->sur.judge_dev);
    if (p->kb > 1) {
        alloc_k2(p->k2b_dev);
        for (K2Dev &D : p->k2c_dev) alloc_k2(D);
    }
    p->off_domdev = alloc(n_slots * sizeof(DomDev));
    for (const SystemP &S : p->sys) {
        for (int a = 0; a < 3; ++a) {
            if (!p->tw64.count(S.P[a])) {
                p->tw64[S.P[a]] = alloc(size_t(S.P[a]) * 16);
                p->tw32[S.P[a]] = alloc(size_t(S.P[a]) * 8);
            }
        }
    }
    int64_t spec_elems = 0;
    for (const SystemP &S : p->sys) spec_elems += S.spec_elems;
    p->off_spec = alloc(size_t(spec_elems) * p->spec_csz);

    const bool quant = ring_scaled(p);
    const bool zq = (p->ring_fmt == RING_F16 || p->ring_fmt == RING_BF16);
    size_t max_gtmp = 0, max_C = 0, max_t1 = 0, max_t2 = 0, max_pts = 0;
    for (DomainP &d : p->dom) {
        const SystemP &S = p->sys[d.sys];
        const size_t t1 = size_t(d.N[0]) * d.N[1] * S.Hz * 4;
        const size_t t2 = size_t(d.N[0]) * S.P[1] * S.Hz * 4;
        d.off_ring = alloc(size_t(d.depth) * S.Cpad * 4 * p->ring_esz);
        d.off_scales = quant ? alloc(scale_bytes(p, d.depth, S.Cpad)) : 0;
        // per-block maxima of the staged z pass, or one per x slice of the plane pass
        d.off_zmax = zq ? alloc(size_t(std::max(d.zblocks, d.N[0])) * 4 * sizeof(float)) : 0;
        d.off_s0 = alloc(size_t(4) * d.npts * p->tsz);
        d.off_p0 = alloc(size_t(4) * d.npts * p->tsz);
        d.off_acc = alloc(size_t(p->kb) * size_t(S.C) * 4 * p->csz);   // kb accumulator sets
        d.off_t1 = alloc(t1 * p->csz);
        d.off_t2 = alloc(t2 * p->csz);
        d.off_s0hat = alloc(size_t(S.C) * 4 * 16);
        max_gtmp = std::max(max_gtmp, size_t(S.P[0]) * S.P[1] * S.Hz);
        max_C = std::max(max_C, size_t(S.C));
        max_t1 = std::max(max_t1, t1);
        max_t2 = std::max(max_t2, t2);
        max_pts = std::max(max_pts, size_t(d.npts));
    }
    for (VRingP &v : p->vring) {
        const DomainP &d = p->dom[v.n];
        const SystemP &S = p->sys[d.sys];
        v.off_ring = alloc(size_t(v.W) * S.Cpad * 4 * p->ring_esz);
        v.off_scales = quant ? alloc(scale_bytes(p, v.W, S.Cpad)) : 0;
        v.off_zmax = zq ? alloc(size_t(std::max(d.zblocks, d.N[0])) * 4 * sizeof(float)) : 0;
        v.off_t1 = alloc(size_t(d.N[0]) * d.N[1] * S.Hz * 4 * p->csz);
        v.off_t2 = alloc(size_t(d.N[0]) * S.P[1] * S.Hz * 4 * p->csz);
        v.off_stage = p->hist_host ? alloc(size_t(4) * d.npts * p->tsz) : 0;
    }
    p->host_bytes = 0;
    p->host_dev = nullptr;
    for (DomainP &d : p->dom) {
        const size_t snap = size_t(4) * d.npts * p->tsz;
        d.off_hist = d.off_stage = d.host_off = 0;
        if (d.d1 == 0) continue;
        if (p->hist_host) {
            d.off_stage = alloc(snap);
            d.host_off = p->host_bytes;
            p->host_bytes += size_t(d.d1) * snap;
        } else {
            d.off_hist = alloc(size_t(d.d1) * snap);
        }
    }
    // I16 ring: FP32 staging of the forward transforms of one ingest launch
    // (one row per frequency tile), quantised from there into the rings
    p->off_qstage = 0;
    if (p->ring_fmt == RING_I16) {
        size_t q = 0;
        for (const ClassP &K : p->cls) {
            size_t jobs = K.doms.size();
            for (int n : K.doms) jobs += p->dom[n].vr.size();
            if (!p->sur.slots.empty()) jobs = kMaxJobs;   // slot transforms and refills
            q = std::max(q, std::min<size_t>(kMaxJobs, jobs) * size_t(p->sys[p->dom[K.doms[0]].sys].Cpad) * 4 * 8);
        }
        p->off_qstage = alloc(q);
    }
    p->off_gtmp = alloc(size_t(kGreenChunk) * max_gtmp * 16);
    p->off_accd = alloc(max_C * 4 * 16);
    p->off_gstat = alloc(max_C * 16);
    p->off_t1d = alloc(max_t1 * 16);
    p->off_t2d = alloc(max_t2 * 16);
    p->off_s0d = alloc(4 * max_pts * 8);
    p->off_p0d = alloc(4 * max_pts * 8);
    if (p->sur.on) sur_layout(p, off);
    p->ws_bytes = off;

    // device-side tables
    p->domdev.assign(n_slots, DomDev{});
    for (size_t i = 0; i < p->dom.size(); ++i) {
        const DomainP &d = p->dom[i];
        DomDev &D = p->domdev[i];
        // offsets in elements relative to the first ring / accumulator / scale
        D.ring_off = int64_t((d.off_ring - p->dom[0].off_ring) / (4 * p->ring_esz)) * 4;
        D.acc_off = int64_t((d.off_acc - p->dom[0].off_acc) / p->csz);
        D.acc_set_stride = p->sys[d.sys].C * 4;
        D.scale_off = quant ? int64_t((d.off_scales - p->dom[0].off_scales) / sizeof(float)) : 0;
        D.depth = d.depth;
        D.pad = 0;
    }
    for (const VRingP &v : p->vring) {
        DomDev &D = p->domdev[v.idx];
        D.ring_off = int64_t((v.off_ring - p->dom[0].off_ring) / (4 * p->ring_esz)) * 4;
        D.scale_off = quant ? int64_t((v.off_scales - p->dom[0].off_scales) / sizeof(float)) : 0;
        D.depth = v.W;
    }
    for (const DomainP &d : p->dom)
        if (d.t1_idx >= 0) p->domdev[d.t1_idx].depth = d.d1;
    if (p->sur.on) sur_slot_tables(p);
    if (p->sur.on) {
        // judge slots: accumulators of the audited far pairs, [slot][C][4]
        for (size_t v = 0; v < p->sur.aud.size(); ++v) {
            DomDev &D = p->domdev[p->dom.size() + v];
            D.acc_off = int64_t((p->sur.jacc_off[v] - p->dom[0].off_acc) / p->csz);
            D.depth = 1;
        }
    }
    finish_k2(p, p->k2);
    if (p->sur.on) finish_k2(p, p->sur.judge);
    if (p->kb > 1) {
        finish_k2(p, p->k2b);
        for (K2Tables &T : p->k2c) finish_k2(p, T);
    }
}

double k2_bytes(rp_plan p, const K2Tables &T) {
    double bytes = 0;
    for (const K2Group &G : T.groups) {
        double per_k = 0;
        for (int e = G.entry_begin; e < G.entry_end; ++e) {
            const K2Entry &E = T.entries[e];
            per_k += 4.0 * p->ring_esz + double(__builtin_popcount(E.mask & ~E.real)) * p->spec_csz +
                     double(__builtin_popcount(E.mask & E.real)) * 0.5 * p->spec_csz;
        }
        per_k += double(G.n_members) * 4 * p->csz;   // accumulator write
        bytes += per_k * double(G.C);
    }
    return bytes;
}

// Minimal bytes of the blocked pass of a block's first step: per target,
// source and frequency, the ring rows of the ages the walk reads
// (max(0, m_lo - kb + 1) .. m_hi) and the spectrum rows of the window, and
// the kb accumulator sets written.
double k2b_bytes(rp_plan p) {
    double bytes = 0;
    for (const K2Group &G : p->k2b.groups) {
        double per_k = 0;
        for (int si = G.src_begin; si < G.src_end; ++si) {
            const K2Src &R = p->k2b.srcs[size_t(si)];
            if (R.m_max < R.m_min) continue;
            const int d0 = std::max(R.m_base, R.m_min - (p->kb - 1));
            per_k += double(R.m_max - d0 + 1) * 4.0 * p->ring_esz +
                     double(R.m_max - R.m_min + 1) * p->spec_csz * ((R.real & 1u) ? 0.5 : 1.0);
        }
        per_k += double(G.n_members) * p->kb * 4 * p->csz;
        bytes += per_k * double(G.C);
    }
    return bytes;
}

void plan_stats(rp_plan p) {
    rp_stats &st = p->stats;
    st = rp_stats{};
    for (const SystemP &S : p->sys)
        for (int s : S.doms)
            for (int n : S.doms)
                if (plain_pair(p, s, n)) st.n_triples += p->pr(s, n).m_hi - p->pr(s, n).m_lo + 1;
    for (const SystemP &S : p->sys) st.n_spectra += S.n_spec;
    st.n_entries = int64_t(p->k2.entries.size());
    for (int n = 0; n < p->n_dom; ++n)
        if (is_target(p, n)) st.points += p->dom[n].npts;
    st.lagsum_bytes = p->kb > 1 ? k2b_bytes(p) : k2_bytes(p, p->k2);
    for (const DomainP &d : p->dom) st.ring_bytes += double(d.depth) * p->sys[d.sys].Cpad * 4 * p->ring_esz;
    for (const VRingP &v : p->vring) st.ring_bytes += double(v.W) * p->sys[p->dom[v.n].sys].Cpad * 4 * p->ring_esz;
    for (const DomainP &d : p->dom)
        if (d.d1 > 0) st.history_bytes += double(p->hist_host ? 1 + d.vr.size() : d.d1) * 4 * double(d.npts) * p->tsz;
    if (p->sur.on) {
        // fallback slots of sampled far pairs: their windows, ring rows and lag-sum bytes
        for (const SlotP &k : p->sur.slots) {
            if (k.f < 0) continue;
            st.n_triples += k.W;
            st.ring_bytes += double(k.W) * p->sur.slot_Cpad * 4 * p->ring_esz;
        }
        if (p->kb == 1) st.lagsum_bytes += k2_bytes(p, p->sur.k2p);
    }
    st.split_rings = int64_t(p->vring.size());
    st.n_classes = int64_t(p->cls.size());
    st.fused_additions = p->fuse_add ? 1 : 0;
    for (const SystemP &S : p->sys) st.spectra_bytes += double(S.spec_elems) * p->spec_csz;
    for (const DomainP &d : p->dom) {
        const SystemP &S = p->sys[d.sys];
        const double t1 = double(d.N[0]) * d.N[1] * S.Hz * 4 * p->csz;
        const double t2 = double(d.N[0]) * S.P[1] * S.Hz * 4 * p->csz;
        const double ring = double(S.C) * 4 * p->ring_esz;
        const double acc = double(S.C) * 4 * p->csz;
        const double real = double(d.npts) * 4 * p->tsz;
        // plane passes keep the z-transformed array (t1) in LDS
        const bool pl = plane_ok(p) && plane_shape(S.P[1], S.P[2], d.N[1], d.N[2]);
        const double fwd = 2 * real + (pl ? 0.0 : t1 + t1) + t2 + t2 + ring;
        st.fft_bytes_fwd += fwd;
        st.fft_bytes_inv += acc + t2 + t2 + (pl ? 0.0 : t1 + t1) + 2 * real;
        // a split history also stores the sources, and transforms them again per extra ring
        if (d.d1 > 0) st.fft_bytes_fwd += real + double(d.vr.size()) * fwd;
    }
}

// ---------------------------------------------------------------------------
// Launch helpers

void check_launch() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(RP_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

// (null before the bind: pass descriptors are also built to plan, unlaunched)
const void *tw_ptr(rp_plan p, int P, bool dbl) {
    return p->ws ? p->ws + (dbl ? p->tw64.at(P) : p->tw32.at(P)) : nullptr;
}

// whether the FP32 plane passes (z and y in one launch) may replace the
// separate passes; each launch still checks its own shapes
bool plane_ok(rp_plan p) { return !p->p64 && p->fft_reg && p->fft_plane; }

// Self pairs of FP32 plans keep their (real) spectra as rows of floats.
bool real_spec(rp_plan p, int s, int n) { return s == n && !p->p64; }

LinePass line_pass(rp_plan p, int P, bool dbl, int dir) {
    LinePass a{};
    a.P = P;
    a.lds_elems = p->fft_lds;
    a.reg = p->fft_reg;
    a.dir = dir;
    a.tw = tw_ptr(p, P, dbl);
    a.rp = make_radix(P);
    a.out_fmt = dbl ? RING_F64 : RING_F32;
    return a;
}

// Forward y pass [Nx][Ny][Hz][4] -> [Nx][Py][Hz][4].
LinePass fwd_y(rp_plan p, const int N[3], const int P[3], int Hz, bool dbl) {
    LinePass a = line_pass(p, P[1], dbl, -1);
    a.n_in = N[1];
    a.n_out = P[1];
    a.lines = N[0] * Hz * 4;
    a.n_inner = Hz * 4;
    a.in_j = Hz * 4;
    a.in_inner = 1;
    a.in_outer = int64_t(N[1]) * Hz * 4;
    a.out_j = Hz * 4;
    a.out_inner = 1;
    a.out_outer = int64_t(P[1]) * Hz * 4;
    return a;
}

// Spectra are indexed k = (y Hz + z) Px + x (x fastest): the lag sum is
// pointwise in k, and this order lets the x passes, the only ones that touch
// spectra, move whole lines of P x frequencies as contiguous runs.

// Forward x pass [Nx][Py][Hz][4] -> spectrum [C][4], C = Py Hz Px in the order
// above.  Line (yz, c) = yz * 4 + c; the linear output is written with the
// four components of a frequency fastest (out_group 4); ring outputs set their
// own group.
LinePass fwd_x(rp_plan p, const int N[3], const int P[3], int Hz, bool dbl) {
    LinePass a = line_pass(p, P[0], dbl, -1);
    a.n_in = N[0];
    a.n_out = P[0];
    a.lines = P[1] * Hz * 4;
    a.n_inner = 4;
    a.in_j = int64_t(P[1]) * Hz * 4;
    a.in_outer = 4;
    a.in_inner = 1;
    a.out_j = 4;
    a.out_outer = int64_t(P[0]) * 4;
    a.out_inner = 1;
    a.out_group = 4;
    return a;
}

// Inverse x pass spectrum [C][4] -> [Nx][Py][Hz][4] (crop).
LinePass inv_x(rp_plan p, const int N[3], const int P[3], int Hz, bool dbl) {
    LinePass a = line_pass(p, P[0], dbl, +1);
    a.n_in = P[0];
    a.n_out = N[0];
    a.lines = P[1] * Hz * 4;
    a.n_inner = 4;
    a.in_j = 4;
    a.in_outer = int64_t(P[0]) * 4;
    a.in_inner = 1;
    a.in_group = 4;
    a.out_j = int64_t(P[1]) * Hz * 4;
    a.out_outer = 4;
    a.out_inner = 1;
    return a;
}

// Inverse y pass [Nx][Py][Hz][4] -> [Nx][Ny][Hz][4] (crop).
LinePass inv_y(rp_plan p, const int N[3], const int P[3], int Hz, bool dbl) {
    LinePass a = line_pass(p, P[1], dbl, +1);
    a.n_in = P[1];
    a.n_out = N[1];
    a.lines = N[0] * Hz * 4;
    a.n_inner = Hz * 4;
    a.in_j = Hz * 4;
    a.in_inner = 1;
    a.in_outer = int64_t(P[1]) * Hz * 4;
    a.out_j = Hz * 4;
    a.out_inner = 1;
    a.out_outer = int64_t(N[1]) * Hz * 4;
    return a;
}

// Whether a blocked step's additions (its lags m < phase) can be left to the
// inverse x pass (add_own_lags): they must be the self pairs' alone, every
// other plain pair starting at lag kb - 1 or later, and every class's inverse
// x pass must be one the register kernel covers.
static bool fused_additions_allowed(rp_plan p) {
    if (p->kb <= 1 || p->p64 || !p->fft_reg) return false;
    for (const SystemP &S : p->sys)
        for (int s : S.doms)
            for (int n : S.doms)
                if (s != n && is_target(p, s) && plain_pair(p, s, n) && p->pr(s, n).m_lo <= p->kb - 2) return false;
    for (const ClassP &K : p->cls) {
        if (K.tdoms.empty()) continue;
        LinePass x = inv_x(p, K.N, K.P, K.Hz, false);
        x.add_fmt = p->ring_fmt;
        x.n_jobs = 1;
        if (!line_reg_supported(x)) return false;
    }
    return true;
}

void update_fused_additions(rp_plan p) {
    p->fuse_add = fused_additions_allowed(p);
    p->stats.fused_additions = p->fuse_add ? 1 : 0;
}

ZFwd zfwd_common(rp_plan p, int mode, const int N[3], const int P[3], int Hz, bool dbl) {
    ZFwd a{};
    a.mode = mode;
    a.reg = p->fft_reg;
    a.Nx = N[0];
    a.Ny = N[1];
    a.Nz = N[2];
    a.Px = P[0];
    a.Py = P[1];
    a.Pz = P[2];
    a.Hz = Hz;
    a.h = p->h;
    a.inv_cdt = std::isfinite(p->c) ? 1.0 / (p->c * p->dt) : 0.0;
    a.scale = 1.0 / (double(P[0]) * P[1] * P[2]);
    a.w_self0 = p->w_self0;
    a.w_self1 = p->w_self1;
    a.w_static = p->w_static;
    a.tw = tw_ptr(p, P[2], dbl);
    a.rp = make_radix(P[2]);
    return a;
}

// FP64 spectrum (one component, [Px][Py][Hz]) of the Green's function of pair
// (s <- n): lag m (mode 1) or instantaneous (mode 2), written with out_fmt.
void green_spectra(rp_plan p, int s, int n, int mode, int m0, int count, void *const *outs, int out_fmt,
                   int64_t tile_stride) {
    const DomainP &ds = p->dom[s], &dn = p->dom[n];
    const SystemP &S = p->sys[ds.sys];
    const size_t gstride = size_t(S.P[0]) * S.P[1] * S.Hz * 16;
    ZFwd z = zfwd_common(p, mode, ds.N, S.P, S.Hz, true);
    z.n_jobs = count;
    for (int j = 0; j < count; ++j) {
        ZFwdJob &J = z.jobs[j];
        J.out = p->ws + p->off_gtmp + j * gstride;
        for (int a = 0; a < 3; ++a) {
            J.off[a] = ds.o[a] - dn.o[a];
            J.Ns[a] = ds.N[a];
            J.Nn[a] = dn.N[a];
        }
        J.m = m0 + j;
        J.self = (s == n);
    }
    launch_zfwd(z, 1, p->stream);
    check_launch();

    LinePass y = line_pass(p, S.P[1], true, -1);
    y.n_in = y.n_out = S.P[1];
    y.lines = S.P[0] * S.Hz;
    y.n_inner = S.Hz;
    y.in_j = y.out_j = S.Hz;
    y.in_inner = y.out_inner = 1;
    y.in_outer = y.out_outer = int64_t(S.P[1]) * S.Hz;
    y.n_jobs = count;
    for (int j = 0; j < count; ++j) y.jobs[j].in = y.jobs[j].out = p->ws + p->off_gtmp + j * gstride;
    launch_line_pass(y, 1, p->stream);
    check_launch();

    // spectrum order k = (y Hz + z) Px + x, as for the sources
    LinePass x = line_pass(p, S.P[0], true, -1);
    x.n_in = x.n_out = S.P[0];
    x.lines = x.n_inner = S.P[1] * S.Hz;
    x.in_j = int64_t(S.P[1]) * S.Hz;
    x.in_inner = 1;
    x.out_j = 1;
    x.out_inner = S.P[0];
    x.out_fmt = out_fmt;
    x.tile_comp = 1;
    x.n_jobs = count;
    for (int j = 0; j < count; ++j) {
        x.jobs[j].in = p->ws + p->off_gtmp + j * gstride;
        x.jobs[j].out = outs[j];
        x.jobs[j].tile_stride = tile_stride;
    }
    launch_line_pass(x, 1, p->stream);
    check_launch();
}

// Copy a lag-sum schedule into its device tables (asynchronous on st; the
// host vectors must stay unchanged until the copy has completed).
void upload_k2(rp_plan p, const K2Tables &T, const K2Dev &D, hipStream_t st) {
    if (T.items.size() > D.cap_items || T.groups.size() > D.cap_groups || T.entries.size() > D.cap_entries ||
        T.srcs.size() > D.cap_srcs || T.pairs.size() > D.cap_pairs || T.masks.size() > D.cap_masks)
        fail(RP_ERR_STATE, "internal: lag-sum schedule exceeds its device tables");
    auto up = [&](size_t off, const void *src, size_t bytes) {
        if (bytes) HIP_OK(hipMemcpyAsync(p->ws + off, src, bytes, hipMemcpyHostToDevice, st));
    };
    up(D.items, T.items.data(), T.items.size() * sizeof(K2Item));
    up(D.groups, T.groups.data(), T.groups.size() * sizeof(K2Group));
    up(D.entries, T.entries.data(), T.entries.size() * sizeof(K2Entry));
    up(D.srcs, T.srcs.data(), T.srcs.size() * sizeof(K2Src));
    up(D.pairs, T.pairs.data(), T.pairs.size() * sizeof(K2Pair));
    up(D.masks, T.masks.data(), T.masks.size() * sizeof(uint32_t));
}

void release_graph(rp_plan p) {
    for (hipGraphExec_t e : p->graph_execs)
        if (e) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : p->graphs)
        if (g) (void)hipGraphDestroy(g);
    p->graph_execs.clear();
    p->graphs.clear();
}

// Phase of a step within its block of kb steps (blocks start at steps 1,
// 1 + kb, ...; step 0 runs as a block start over the empty history).
int lag_phase(rp_plan p, int64_t step) { return step <= 0 ? 0 : int((step - 1) % p->kb); }

void do_bind(rp_plan p, void *dev, size_t bytes) {
    if (!dev) fail(RP_ERR_ARG, "workspace pointer is null");
    if (reinterpret_cast<uintptr_t>(dev) % kAlign) fail(RP_ERR_ARG, "workspace must be 256-byte aligned");
    if (bytes < p->ws_bytes) fail(RP_ERR_NOMEM, "workspace smaller than rp_workspace_bytes");
    p->ws = static_cast<char *>(dev);
    hipStream_t st = p->stream;
    upload_k2(p, p->k2, p->k2_dev, st);
    if (p->sur.on) upload_k2(p, p->sur.judge, p->sur.judge_dev, st);
    if (p->kb > 1) {
        upload_k2(p, p->k2b, p->k2b_dev, st);
        for (size_t i = 0; i < p->k2c.size(); ++i) upload_k2(p, p->k2c[i], p->k2c_dev[i], st);
    }
    HIP_OK(hipMemcpyAsync(p->ws + p->off_domdev, p->domdev.data(), p->domdev.size() * sizeof(DomDev),
                          hipMemcpyHostToDevice, st));
    // twiddles exp(-2 pi i j / P), evaluated in FP64 on the host
    std::vector<Cx<double>> t64;
    std::vector<Cx<float>> t32;
    for (const auto &kv : p->tw64) {
        const int P = kv.first;
        t64.resize(P);
        t32.resize(P);
        for (int j = 0; j < P; ++j) {
            const double ang = -2.0 * M_PI * double(j) / double(P);
            t64[j] = {std::cos(ang), std::sin(ang)};
            t32[j] = {float(t64[j].x), float(t64[j].y)};
        }
        HIP_OK(hipMemcpyAsync(p->ws + kv.second, t64.data(), P * 16, hipMemcpyHostToDevice, st));
        HIP_OK(hipMemcpyAsync(p->ws + p->tw32.at(P), t32.data(), P * 8, hipMemcpyHostToDevice, st));
        HIP_OK(hipStreamSynchronize(st));   // host buffers are reused
    }
    launch_fill_zero(p->ws + p->off_state, 64, st);
    launch_fill_zero(p->ws + p->off_head, (size_t(p->n_heads) * sizeof(int32_t) + 15) / 16 * 16, st);
    launch_fill_zero(p->ws + p->off_prev_head, (size_t(p->n_heads) * sizeof(int32_t) + 15) / 16 * 16, st);
    launch_fill_zero(p->ws + p->off_counter, 16, st);
    {
        int dev = 0;
        HIP_OK(hipGetDevice(&dev));
        HIP_OK(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    for (const DomainP &d : p->dom) {
        launch_fill_zero(p->ws + d.off_ring, size_t(d.depth) * p->sys[d.sys].Cpad * 4 * p->ring_esz, st);
        if (d.off_scales) launch_fill_zero(p->ws + d.off_scales, scale_bytes(p, d.depth, p->sys[d.sys].Cpad), st);
    }
    for (const VRingP &v : p->vring) {
        launch_fill_zero(p->ws + v.off_ring, size_t(v.W) * p->sys[p->dom[v.n].sys].Cpad * 4 * p->ring_esz, st);
        if (v.off_scales)
            launch_fill_zero(p->ws + v.off_scales, scale_bytes(p, v.W, p->sys[p->dom[v.n].sys].Cpad), st);
    }
    if (p->sur.on) sur_bind(p);
    check_launch();
    HIP_OK(hipStreamSynchronize(st));
    p->green_ready = false;
    p->next_step = 0;
    p->pushed = false;
    release_graph(p);
}

// ---------------------------------------------------------------------------
// Fixed device workspace for callers that cannot allocate device memory
// (rp_bind_workspace_static).  The array exists once per device the library
// runs on and stays until the process ends.  In host code `scratch` names a
// host-side stand-in: its device address is taken once per device with
// hipGetSymbolAddress and only that address is used.
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
static_assert(kStaticWorkspaceBytes == RP_STATIC_WORKSPACE_BYTES, "rpot.h and the array disagree");
static __device__ __align__(256) char scratch[kStaticWorkspaceBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char *g_static_ptr[kMaxDevices] = {};      // device address of the array, per device
rp_plan g_static_owner[kMaxDevices] = {};  // the plan bound to it last, per device
}  // namespace

void need_ws(rp_plan p) {
    if (!p->ws) fail(RP_ERR_STATE, "workspace not bound");
    if (p->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[p->static_dev] != p)
            fail(RP_ERR_STATE, "the fixed workspace array was bound to another plan since "
                               "(rp_bind_workspace_static); bind this plan again");
    }
}

void release_static(rp_plan p) {
    if (p->static_dev < 0) return;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_owner[p->static_dev] == p) g_static_owner[p->static_dev] = nullptr;
    p->static_dev = -1;
}

void do_bind_static(rp_plan p) {
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(RP_ERR_UNSUPPORTED, "device index beyond the fixed workspace table");
    if (p->ws_bytes > kStaticWorkspaceBytes) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "the plan needs %zu bytes of workspace; the fixed array holds %zu "
                      "(use rp_bind_workspace)", p->ws_bytes, kStaticWorkspaceBytes);
        fail(RP_ERR_NOMEM, buf);
    }
    char *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!g_static_ptr[dev]) {
            void *a = nullptr;
            const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !a)
                fail(RP_ERR_DEVICE, std::string("hipGetSymbolAddress of the fixed workspace: ") + hipGetErrorString(e));
            g_static_ptr[dev] = static_cast<char *>(a);
        }
        ptr = g_static_ptr[dev];
    }
    release_static(p);
    // the bind zeroes everything that must start at zero (history, heads,
    // step counter); the rest of the array is written before it is read
    do_bind(p, ptr, kStaticWorkspaceBytes);
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_owner[dev] = p;
    p->static_dev = dev;
}

void do_green(rp_plan p) {
    need_ws(p);
    const int fmt = p->p64 ? RING_F64 : RING_F32;
    for (const SystemP &S : p->sys) {
        for (size_t a = 0; a < S.doms.size(); ++a) {
            for (size_t b = a; b < S.doms.size(); ++b) {
                const int s = S.doms[a], n = S.doms[b];
                const PairP &q = p->pr(s, n);
                if (q.spec0 < 0) continue;   // far pair without plain history
                for (int m0 = q.m_lo; m0 <= q.m_hi; m0 += kGreenChunk) {
                    const int cnt = std::min(kGreenChunk, q.m_hi - m0 + 1);
                    void *outs[kGreenChunk];
                    const int64_t W = q.m_hi - q.m_lo + 1;
                    for (int j = 0; j < cnt; ++j)
                        outs[j] = p->ws + p->off_spec +
                                  size_t(S.spec_base + q.spec0 + int64_t(m0 + j - q.m_lo) * kTile) * p->spec_csz;
                    green_spectra(p, s, n, 1, m0, cnt, outs, fmt, W * kTile);
                }
                if (real_spec(p, s, n))
                    launch_spec_real(p->ws + p->off_spec + size_t(S.spec_base + q.spec0) * p->spec_csz,
                                     int64_t(q.m_hi - q.m_lo + 1) * (S.Cpad / kTile), p->stream);
            }
        }
    }
    check_launch();
    HIP_OK(hipStreamSynchronize(p->stream));
    p->green_ready = true;
}

// Static potential P(0) of every domain in FP64: the instantaneous Coulomb
// sum of S(0) with the self-cell integral, by the same padded FFT convolution.
void do_static(rp_plan p, const void *const *src) {
    hipStream_t st = p->stream;
    for (const SystemP &S : p->sys) {
        for (int n : S.doms) {
            const DomainP &d = p->dom[n];
            const void *s64 = src[n];
            if (!p->p64) {
                launch_convert(p->ws + p->off_s0d, 1, src[n], 0, 4 * d.npts, st);
                s64 = p->ws + p->off_s0d;
            }
            ZFwd z = zfwd_common(p, 0, d.N, S.P, S.Hz, true);
            z.n_jobs = 1;
            z.jobs[0].src = s64;
            z.jobs[0].s0 = nullptr;
            z.jobs[0].out = p->ws + p->off_t1d;
            launch_zfwd(z, 1, st);
            LinePass y = fwd_y(p, d.N, S.P, S.Hz, true);
            y.n_jobs = 1;
            y.jobs[0].in = p->ws + p->off_t1d;
            y.jobs[0].out = p->ws + p->off_t2d;
            launch_line_pass(y, 1, st);
            LinePass x = fwd_x(p, d.N, S.P, S.Hz, true);
            x.n_jobs = 1;
            x.jobs[0].in = p->ws + p->off_t2d;
            x.jobs[0].out = p->ws + d.off_s0hat;
            launch_line_pass(x, 1, st);
            check_launch();
        }
        for (int s : S.doms) {
            if (!is_target(p, s)) continue;
            const DomainP &d = p->dom[s];
            launch_fill_zero(p->ws + p->off_accd, size_t(S.C) * 4 * 16, st);
            for (int n : S.doms) {
                void *outs[1] = {p->ws + p->off_gstat};
                green_spectra(p, s, n, 2, 0, 1, outs, RING_F64, 0);
                launch_static_mac(p->ws + p->off_accd, p->ws + p->off_gstat, p->ws + p->dom[n].off_s0hat, S.C, st);
            }
            LinePass x = inv_x(p, d.N, S.P, S.Hz, true);
            x.n_jobs = 1;
            x.jobs[0].in = p->ws + p->off_accd;
            x.jobs[0].out = p->ws + p->off_t2d;
            launch_line_pass(x, 1, st);
            LinePass y = inv_y(p, d.N, S.P, S.Hz, true);
            y.n_jobs = 1;
            y.jobs[0].in = p->ws + p->off_t2d;
            y.jobs[0].out = p->ws + p->off_t1d;
            launch_line_pass(y, 1, st);
            ZInv zi{};
            zi.Nx = d.N[0];
            zi.Ny = d.N[1];
            zi.Nz = d.N[2];
            zi.Pz = S.P[2];
            zi.Hz = S.Hz;
            zi.tw = tw_ptr(p, S.P[2], true);
            zi.rp = make_radix(S.P[2]);
            zi.n_jobs = 1;
            zi.jobs[0].in = p->ws + p->off_t1d;
            zi.jobs[0].out = p->ws + p->off_p0d;
            zi.jobs[0].add = nullptr;
            launch_zinv(zi, 1, st);
            launch_convert(p->ws + d.off_p0, p->p64, p->ws + p->off_p0d, 1, 4 * d.npts, st);
            check_launch();
        }
    }
}

// Forward transform of dS(l) = S(l) - S(0) of every domain into the slot of
// its ring given by the device-side head (no host-side step dependence, so
// the same launches are valid inside a captured graph).
// Line-pass tile of a shape class: its own choice, else the plan's.
int cls_lds(rp_plan p, const ClassP &K) { return K.fft_lds ? K.fft_lds : p->fft_lds; }

void enqueue_ring_jobs(rp_plan p, const ClassP &K, const std::vector<RingJob> &jobs, hipStream_t st) {
    const bool quant = (p->ring_fmt == RING_F16 || p->ring_fmt == RING_BF16);
    const bool i16 = (p->ring_fmt == RING_I16);
    const int64_t Cpad = p->sys[p->dom[K.doms[0]].sys].Cpad;
    for (size_t j0 = 0; j0 < jobs.size(); j0 += kMaxJobs) {
        const int cnt = int(std::min<size_t>(kMaxJobs, jobs.size() - j0));
        ZFwd z = zfwd_common(p, 0, K.N, K.P, K.Hz, p->p64);
        LinePass y = fwd_y(p, K.N, K.P, K.Hz, p->p64);
        LinePass x = fwd_x(p, K.N, K.P, K.Hz, p->p64);
        y.lds_elems = x.lds_elems = cls_lds(p, K);
        // I16: the x pass writes FP32 rows into the staging area, which
        // the quantiser then scales per tile into the ring
        x.out_fmt = i16 ? RING_F32 : p->ring_fmt;
        x.tile_comp = 4;
        // lanes in the order of a ring row: [c/2][k][c%2] (FP32), [c][k]
        // (FP64), [k][c] (FP16/BF16)
        x.out_group = x.out_fmt == RING_F32 ? 2 : (x.out_fmt == RING_F64 ? 1 : 4);
        // I16: the register x pass quantises in the same launch where it
        // covers the pass; else FP32 rows into the staging area and the
        // quantiser after
        bool fused_i16 = false;
        if (i16 && !p->p64 && x.reg) {
            LinePass xi = x;
            xi.out_fmt = RING_I16;
            xi.out_group = 4;
            xi.n_jobs = 1;
            xi.jobs[0].tile_stride = kTile * 4;
            xi.jobs[0].qscale = reinterpret_cast<float *>(p->ws);
            fused_i16 = line_reg_supported(xi);
        }
        if (fused_i16) {
            x.out_fmt = RING_I16;
            x.out_group = 4;
        }
        ScaleArgs sa{};
        QuantArgs qa{};
        z.n_jobs = y.n_jobs = x.n_jobs = cnt;
        sa.n_jobs = quant ? cnt : 0;
        qa.n_jobs = (i16 && !fused_i16) ? cnt : 0;
        qa.max_tiles = int(Cpad / kTile);
        for (int j = 0; j < cnt; ++j) {
            const RingJob &J = jobs[j0 + j];
            const DomainP &d = p->dom[J.n];
            z.jobs[j].src = J.src;
            z.jobs[j].src_head = J.src_head;
            z.jobs[j].src_depth = J.src_depth;
            z.jobs[j].src_lag = J.src_lag;
            z.jobs[j].store = J.store;
            z.jobs[j].store_head = J.store_head;
            z.jobs[j].s0 = p->ws + d.off_s0;
            z.jobs[j].out = J.t1;
            z.jobs[j].zmax = quant ? J.zmax : nullptr;
            y.jobs[j].in = J.t1;
            y.jobs[j].out = J.t2;
            x.jobs[j].in = J.t2;
            x.jobs[j].out = J.ring;
            x.jobs[j].head = J.head;
            x.jobs[j].slot_stride = int64_t(kTile) * 4;
            x.jobs[j].tile_stride = int64_t(J.depth) * kTile * 4;
            x.jobs[j].qscale = quant ? J.scales : nullptr;
            if (i16 && fused_i16) {
                // the x pass quantises into the ring itself
                x.jobs[j].qscale = J.scales;
            } else if (i16) {
                float *stage = p->at<float>(p->off_qstage + size_t(j) * size_t(Cpad) * 4 * 8);
                x.jobs[j].out = stage;
                x.jobs[j].head = nullptr;
                x.jobs[j].slot_stride = 0;
                x.jobs[j].tile_stride = int64_t(kTile) * 4;
                QuantJob &q = qa.jobs[j];
                q.stage = stage;
                q.ring = J.ring;
                q.scales = J.scales;
                q.head = J.head;
                q.C = p->sys[d.sys].C;
                q.depth = J.depth;
                q.n_tiles = int(Cpad / kTile);
            }
            if (quant) {
                sa.jobs[j].zmax = J.zmax;
                sa.jobs[j].scales = J.scales;
                sa.jobs[j].nblk = d.zblocks;
                sa.jobs[j].head = J.head;
                sa.jobs[j].npts = double(d.npts);
            }
        }
        if (plane_ok(p) && launch_zy_fwd_plane(z, y, st)) {
            // the plane pass wrote one maximum per x slice and component
            for (int j = 0; j < sa.n_jobs; ++j) sa.jobs[j].nblk = K.N[0];
            launch_ring_scale(sa, st);
        } else {
            launch_zfwd(z, p->p64, st);
            launch_ring_scale(sa, st);
            launch_line_pass(y, p->p64, st);
        }
        launch_line_pass(x, p->p64, st);
        launch_quant_i16(qa, st);
        check_launch();
    }
}

void enqueue_ingest(rp_plan p, const void *const *src, hipStream_t st) {
    const bool scaled = ring_scaled(p);
    const bool zq = (p->ring_fmt == RING_F16 || p->ring_fmt == RING_BF16);
    const int32_t *dhead = p->at<int32_t>(p->off_head);
    for (const ClassP &K : p->cls) {
        // jobs: every domain of the class (newest sources into its ring, and a
        // copy into its real-space ring), every split ring of those domains
        // (the sources of lo steps ago, from the real-space ring), and the
        // fallback slots of sampled far pairs with a source in the class
        std::vector<RingJob> jobs;
        for (int n : K.doms) {
            const DomainP &d = p->dom[n];
            RingJob J;
            J.n = n;
            J.src = src[n];
            if (d.d1 > 0 && p->hist_host) {
                J.store = p->ws + d.off_stage;   // written to the host ring
            } else if (d.d1 > 0) {
                J.store = p->ws + d.off_hist;
                J.store_head = dhead + d.t1_idx;
            }
            J.t1 = p->ws + d.off_t1;
            J.t2 = p->ws + d.off_t2;
            J.ring = p->ws + d.off_ring;
            J.scales = scaled ? p->at<float>(d.off_scales) : nullptr;
            J.zmax = zq ? p->at<float>(d.off_zmax) : nullptr;
            J.head = dhead + n;
            J.depth = d.depth;
            jobs.push_back(J);
        }
        for (int n : K.doms) {
            const DomainP &d = p->dom[n];
            for (int vi : d.vr) {
                const VRingP &v = p->vring[size_t(vi)];
                RingJob J;
                J.n = n;
                if (p->hist_host) {
                    J.src = p->ws + v.off_stage;   // fetched from the host ring
                } else {
                    J.src = p->ws + d.off_hist;
                    J.src_head = dhead + d.t1_idx;
                    J.src_depth = d.d1;
                    J.src_lag = v.lo;
                }
                J.t1 = p->ws + v.off_t1;
                J.t2 = p->ws + v.off_t2;
                J.ring = p->ws + v.off_ring;
                J.scales = scaled ? p->at<float>(v.off_scales) : nullptr;
                J.zmax = zq ? p->at<float>(v.off_zmax) : nullptr;
                J.head = dhead + v.idx;
                J.depth = v.W;
                jobs.push_back(J);
            }
        }
        if (p->sur.on) sur_ring_jobs(p, K, jobs);
        enqueue_ring_jobs(p, K, jobs, st);
    }
}

K2Args k2_args(rp_plan p, const K2Tables &T, const K2Dev &D, const int32_t *head) {
    K2Args k{};
    k.items = p->at<K2Item>(D.items);
    k.groups = p->at<K2Group>(D.groups);
    k.entries = p->at<K2Entry>(D.entries);
    k.srcs = p->at<K2Src>(D.srcs);
    k.pairs = p->at<K2Pair>(D.pairs);
    k.masks = p->at<uint32_t>(D.masks);
    k.doms = p->at<DomDev>(p->off_domdev);
    k.spectra = p->ws + p->off_spec;
    k.ring = p->ws + p->dom[0].off_ring;
    k.scales = ring_scaled(p) ? p->at<float>(p->dom[0].off_scales) : nullptr;
    k.acc = p->ws + p->dom[0].off_acc;
    k.head = head;
    k.counter = p->at<int>(p->off_counter);
    k.n_items = int(T.items.size());
    k.n_dom = p->n_dom;
    return k;
}

void enqueue_k2(rp_plan p, const K2Args &a, int tg, hipStream_t st, int unroll, int persist) {
    if (a.n_items == 0) return;
    const int grid = persist ? p->n_cu * lagsum_blocks_per_cu(p->p64, p->ring_fmt, tg, unroll) : 0;
    launch_lagsum(a, p->p64, p->ring_fmt, tg, unroll, grid, st);
    check_launch();
}

// The lag sum of a step of phase `phase` (0 without blocking): the plain
// pass; with kb > 1 the blocked pass at a block's first step (all kb
// accumulator sets) and the lags m < phase added to set `phase` otherwise.
void enqueue_lagsum(rp_plan p, hipStream_t st, int unroll, int persist, int phase) {
    const int32_t *head = p->at<int32_t>(p->off_head);
    if (p->kb == 1) {
        enqueue_k2(p, k2_args(p, p->k2, p->k2_dev, head), p->k2.tg, st, unroll, persist);
    } else if (phase == 0) {
        K2Args a = k2_args(p, p->k2b, p->k2b_dev, head);
        a.cached = p->k2b_cached;
        if (a.n_items > 0) {
            const int grid = persist ? p->n_cu * lagsum_block_blocks_per_cu(p->ring_fmt, p->kb, unroll) : 0;
            launch_lagsum_block(a, p->ring_fmt, p->kb, unroll, grid, st);
            check_launch();
        }
    } else if (!p->fuse_add) {
        // (with fused additions the inverse x pass adds these lags)
        const K2Tables &T = p->k2c[size_t(phase - 1)];
        K2Args a = k2_args(p, T, p->k2c_dev[size_t(phase - 1)], head);
        a.acc_set = phase;
        a.accumulate = 1;
        enqueue_k2(p, a, T.tg, st, 1, 0);
    }
    // the fallback slots' pairs, one step at a time, into this step's set
    if (p->sur.on) sur_enqueue_slots(p, head, st, phase);
}

// Inverse transform of every target's accumulated spectrum, crop to the
// domain, add P(0), write the caller's output; then advance the step.
void enqueue_inverse(rp_plan p, void *const *out, hipStream_t st, int phase) {
    for (const ClassP &K : p->cls) {
        for (size_t j0 = 0; j0 < K.tdoms.size(); j0 += kMaxJobs) {
            const int cnt = int(std::min<size_t>(kMaxJobs, K.tdoms.size() - j0));
            LinePass x = inv_x(p, K.N, K.P, K.Hz, p->p64);
            LinePass y = inv_y(p, K.N, K.P, K.Hz, p->p64);
            x.lds_elems = y.lds_elems = cls_lds(p, K);
            ZInv zi{};
            zi.reg = p->fft_reg;
            zi.Nx = K.N[0];
            zi.Ny = K.N[1];
            zi.Nz = K.N[2];
            zi.Pz = K.P[2];
            zi.Hz = K.Hz;
            zi.tw = tw_ptr(p, K.P[2], p->p64);
            zi.rp = make_radix(K.P[2]);
            x.n_jobs = y.n_jobs = zi.n_jobs = cnt;
            const bool fused = p->fuse_add && p->kb > 1 && phase > 0;
            if (fused) x.add_fmt = p->ring_fmt;
            for (int j = 0; j < cnt; ++j) {
                const int s = K.tdoms[j0 + j];
                const DomainP &d = p->dom[s];
                if (fused) {
                    // the step's lags 0 .. phase - 1 of the target's own sources
                    const PairP &q = p->pr(s, s);
                    LineJob &J = x.jobs[j];
                    J.add_ring = p->ws + d.off_ring;
                    J.add_scales = d.off_scales ? p->at<float>(d.off_scales) : nullptr;
                    J.add_head = p->at<int32_t>(p->off_head) + s;
                    J.add_spec = p->ws + p->off_spec + size_t(p->sys[d.sys].spec_base + q.spec0) * p->spec_csz;
                    J.add_depth = d.depth;
                    J.add_w = q.m_hi - q.m_lo + 1;
                    J.add_lags = std::min(phase, q.m_hi + 1);   // the self window is [0, m_hi]
                }
                x.jobs[j].in = p->ws + d.off_acc + size_t(phase) * size_t(K.C) * 4 * p->csz;
                x.jobs[j].out = p->ws + d.off_t2;
                y.jobs[j].in = p->ws + d.off_t2;
                y.jobs[j].out = p->ws + d.off_t1;
                zi.jobs[j].in = p->ws + d.off_t1;
                zi.jobs[j].out = out[s];
                zi.jobs[j].add = p->ws + d.off_p0;
            }
            launch_line_pass(x, p->p64, st);
            if (!(plane_ok(p) && launch_yz_inv_plane(y, zi, st))) {
                launch_line_pass(y, p->p64, st);
                launch_zinv(zi, p->p64, st);
            }
            check_launch();
        }
    }
}

// Surrogate far-pair terms (when a network is attached), then step += 1 and
// every ring head moves on (the previous heads are kept for the judge).
void enqueue_finish(rp_plan p, void *const *out, hipStream_t st) {
    if (p->sur.on) sur_enqueue_infer(p, out, st);
    launch_advance_step(p->at<int64_t>(p->off_state), p->at<int32_t>(p->off_head), p->at<int32_t>(p->off_prev_head),
                        p->at<DomDev>(p->off_domdev), p->n_heads, st);
    check_launch();
}

// Host tier of a split history.  After the forward transforms of step l are
// queued on st, a second stream writes S(l) from the staging buffer into its
// host slot and fetches into each split ring's staging buffer the snapshot
// that step l + 1 transforms again (S(l + 1 - lo), or S(0) before step 0);
// the copies run under the lag sum and inverse of step l and are joined
// before the step's ring heads move on (tier_join).  A split ring's window
// starts at lag 2 or later (the first window starts at 0 and a gap is at
// least one lag), so no fetch reads the slot written in the same step and
// all copies of a step go in one launch.  With write_newest false (step 0)
// only the fetches run.
bool tier_active(rp_plan p) { return p->hist_host && p->host_bytes > 0; }

void tier_fork(rp_plan p, hipStream_t st, bool write_newest) {
    if (!tier_active(p)) return;
    if (!p->host_dev) fail(RP_ERR_STATE, "the host history is not bound (rp_bind_history_host)");
    HIP_OK(hipEventRecord(p->tier_fork, st));
    HIP_OK(hipStreamWaitEvent(p->tier_stream, p->tier_fork, 0));
    p->tier_open = true;
    TierArgs a{};
    a.step = p->at<int64_t>(p->off_state);
    a.head = p->at<int32_t>(p->off_head);
    auto add = [&](const TierJob &j) {
        a.jobs[a.n_jobs++] = j;
        if (a.n_jobs == kMaxTierJobs) {
            launch_tier_copy(a, p->tier_stream);
            check_launch();
            a.n_jobs = 0;
        }
    };
    for (const DomainP &d : p->dom) {
        if (d.d1 == 0 || !write_newest) continue;
        TierJob j{};
        j.src = p->at<uint4>(d.off_stage);
        j.dst = reinterpret_cast<uint4 *>(p->host_dev + d.host_off);
        j.n16 = int64_t(4) * d.npts * int64_t(p->tsz) / 16;
        j.dst_depth = d.d1;
        j.head_idx = d.t1_idx;
        add(j);
    }
    for (const VRingP &v : p->vring) {
        const DomainP &d = p->dom[v.n];
        if (v.lo < 2) fail(RP_ERR_STATE, "internal: a split ring starts before lag 2");
        TierJob j{};
        j.src = reinterpret_cast<const uint4 *>(p->host_dev + d.host_off);
        j.dst = p->at<uint4>(v.off_stage);
        j.alt = p->at<uint4>(d.off_s0);
        j.n16 = int64_t(4) * d.npts * int64_t(p->tsz) / 16;
        j.src_depth = d.d1;
        j.shift = 1 - v.lo;
        j.head_idx = d.t1_idx;
        add(j);
    }
    if (a.n_jobs) {
        launch_tier_copy(a, p->tier_stream);
        check_launch();
    }
    HIP_OK(hipEventRecord(p->tier_join, p->tier_stream));
}

void tier_join(rp_plan p, hipStream_t st) {
    if (!p->tier_open) return;
    HIP_OK(hipStreamWaitEvent(st, p->tier_join, 0));
    p->tier_open = false;
}

// Every domain's pointer (targets_only: every target's; the others may be null).
void check_ptrs(rp_plan p, const void *const *ptrs, const char *what, bool targets_only = false) {
    if (!ptrs) fail(RP_ERR_ARG, std::string(what) + " is null");
    for (int n = 0; n < p->n_dom; ++n)
        if (!ptrs[n] && (!targets_only || is_target(p, n))) fail(RP_ERR_ARG, std::string("a ") + what + " pointer is null");
}

void do_push(rp_plan p, int64_t step, const void *const *src) {
    need_ws(p);
    if (!p->green_ready) fail(RP_ERR_STATE, "rp_set_green_kernels has not been called");
    check_ptrs(p, src, "src");
    if (tier_active(p) && !p->host_dev) fail(RP_ERR_STATE, "the host history is not bound (rp_bind_history_host)");
    if (step != p->next_step || p->pushed) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "rp_push_sources(%lld) out of order (expected step %lld%s)",
                      (long long)step, (long long)p->next_step, p->pushed ? ", already pushed" : "");
        fail(RP_ERR_STATE, buf);
    }
    hipStream_t st = p->stream;
    if (step == 0) {
        for (int n = 0; n < p->n_dom; ++n) {
            const DomainP &d = p->dom[n];
            launch_convert(p->ws + d.off_s0, p->p64, src[n], p->p64, 4 * d.npts, st);
            // the real-space ring starts with S(0) in every slot: sources before
            // step 0 are S(0) (the host tier reads S(0) itself for those)
            if (!p->hist_host && d.d1 > 0) {
                const size_t snap = size_t(4) * d.npts * p->tsz;
                launch_convert(p->ws + d.off_hist, p->p64, src[n], p->p64, 4 * d.npts, st);
                launch_broadcast(p->ws + d.off_hist + snap, p->ws + d.off_hist, int64_t(snap), d.d1 - 1, st);
            }
        }
        do_static(p, src);
        tier_fork(p, st, false);
    } else {
        enqueue_ingest(p, src, st);
        tier_fork(p, st, true);
        if (p->sur.on) sur_enqueue_moments(p, src, st);
    }
    check_launch();
    p->pushed = true;
}

void do_step(rp_plan p, int64_t step, void *const *out) {
    need_ws(p);
    check_ptrs(p, out, "out", true);
    if (step != p->next_step || !p->pushed) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "rp_retarded_step(%lld) out of order (expected step %lld%s)",
                      (long long)step, (long long)p->next_step, p->pushed ? "" : ", sources not pushed");
        fail(RP_ERR_STATE, buf);
    }
    hipStream_t st = p->stream;
    if (p->profile) {
        if (p->events.size() < 2 * (p->n_recorded + 1)) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t ev;
                HIP_OK(hipEventCreate(&ev));
                p->events.push_back(ev);
            }
        }
    }
    // with blocked steps only the pass at a block's first step is timed
    const int phase = lag_phase(p, step);
    const bool timed = p->profile && phase == 0;
    if (timed) HIP_OK(hipEventRecord(p->events[2 * p->n_recorded], st));
    enqueue_lagsum(p, st, p->k2_unroll, p->k2_persist, phase);
    if (timed) {
        HIP_OK(hipEventRecord(p->events[2 * p->n_recorded + 1], st));
        p->n_recorded += 1;
    }
    enqueue_inverse(p, out, st, phase);
    tier_join(p, st);
    enqueue_finish(p, out, st);
    p->next_step += 1;
    p->pushed = false;
}

// Record one whole step (ingest + lag sum + inverse + advance) for fixed
// source and output buffers as a HIP graph.
void do_capture(rp_plan p, const void *const *src, void *const *out) {
    need_ws(p);
    if (!p->green_ready) fail(RP_ERR_STATE, "rp_set_green_kernels has not been called");
    check_ptrs(p, src, "src");
    check_ptrs(p, out, "out", true);
    if (p->tier_open) fail(RP_ERR_STATE, "capture a step after rp_retarded_step, not between push and step");
    if (tier_active(p) && !p->host_dev) fail(RP_ERR_STATE, "the host history is not bound (rp_bind_history_host)");
    release_graph(p);
    if (!p->capture_stream) HIP_OK(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = p->capture_stream;
    // one graph per phase of a block (kb graphs; one without blocking)
    for (int phase = 0; phase < p->kb; ++phase) {
        HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_ingest(p, src, cs);
            tier_fork(p, cs, true);
            if (p->sur.on) sur_enqueue_moments(p, src, cs);
            enqueue_lagsum(p, cs, p->k2_unroll, p->k2_persist, phase);
            enqueue_inverse(p, out, cs, phase);
            tier_join(p, cs);
            enqueue_finish(p, out, cs);
        } catch (...) {
            p->tier_open = false;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            release_graph(p);
            throw;
        }
        hipGraph_t g = nullptr;
        HIP_OK(hipStreamEndCapture(cs, &g));
        p->graphs.push_back(g);
        hipGraphExec_t e = nullptr;
        HIP_OK(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
        p->graph_execs.push_back(e);
    }
}

void do_launch_graph(rp_plan p, int64_t step) {
    need_ws(p);
    if (p->graph_execs.empty()) fail(RP_ERR_STATE, "no captured step (rp_capture_step)");
    if (step < 1 || step != p->next_step || p->pushed) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "rp_launch_step(%lld) out of order (expected step %lld >= 1)",
                      (long long)step, (long long)p->next_step);
        fail(RP_ERR_STATE, buf);
    }
    HIP_OK(hipGraphLaunch(p->graph_execs[size_t(lag_phase(p, step))], p->stream));
    p->next_step += 1;
}

// The inverse x and y passes of every target (accumulator -> temporaries
// only): the autotuner's probe of the line-pass tile.
void enqueue_inverse_xy(rp_plan p, hipStream_t st, int only_cls = -1) {
    for (size_t ci = 0; ci < p->cls.size(); ++ci) {
        if (only_cls >= 0 && int(ci) != only_cls) continue;
        const ClassP &K = p->cls[ci];
        for (size_t j0 = 0; j0 < K.tdoms.size(); j0 += kMaxJobs) {
            const int cnt = int(std::min<size_t>(kMaxJobs, K.tdoms.size() - j0));
            LinePass x = inv_x(p, K.N, K.P, K.Hz, p->p64);
            LinePass y = inv_y(p, K.N, K.P, K.Hz, p->p64);
            x.lds_elems = y.lds_elems = cls_lds(p, K);
            x.n_jobs = y.n_jobs = cnt;
            for (int j = 0; j < cnt; ++j) {
                const DomainP &d = p->dom[K.tdoms[j0 + j]];
                x.jobs[j].in = p->ws + d.off_acc;
                x.jobs[j].out = p->ws + d.off_t2;
                y.jobs[j].in = p->ws + d.off_t2;
                y.jobs[j].out = p->ws + d.off_t1;
            }
            launch_line_pass(x, p->p64, st);
            launch_line_pass(y, p->p64, st);
            check_launch();
        }
    }
}

// Time every lag-sum schedule and line-pass tile on the bound plan (its
// current ring and spectra; only the accumulator and FFT temporaries are
// written) and keep the fastest.
void do_autotune(rp_plan p, int iters, int32_t *best_unroll, int32_t *best_persist, double *best_ms) {
    need_ws(p);
    if (!p->green_ready) fail(RP_ERR_STATE, "rp_set_green_kernels has not been called");
    if (iters < 1) fail(RP_ERR_ARG, "iters must be >= 1");
    hipStream_t st = p->stream;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    // the blocked pass writes every accumulator set: only between blocks
    if (p->kb > 1 && (p->pushed || lag_phase(p, p->next_step) != 0))
        fail(RP_ERR_STATE, "autotune a plan with blocked steps between blocks");
    double best = 1e300;
    int bu = p->k2_unroll, bp = p->k2_persist, bc = p->k2b_cached, bo = p->k2b_tile_major;
    try {
        // the blocked pass also chooses its cache policy and work order
        const int n_var = p->kb > 1 ? 4 : 1;
        for (int var = 0; var < n_var; ++var) {
            if (p->kb > 1) {
                p->k2b_cached = var & 1;
                if (p->k2b_tile_major != (var >> 1)) {
                    p->k2b_tile_major = var >> 1;
                    order_k2b(p);
                }
            }
            for (int persist = 0; persist <= 1; ++persist) {
                for (int unroll : {1, 2, 4}) {
                    enqueue_lagsum(p, st, unroll, persist, 0);   // warm-up
                    HIP_OK(hipEventRecord(e0, st));
                    for (int i = 0; i < iters; ++i) enqueue_lagsum(p, st, unroll, persist, 0);
                    HIP_OK(hipEventRecord(e1, st));
                    HIP_OK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
                    if (ms / iters < best) {
                        best = ms / iters;
                        bu = unroll;
                        bp = persist;
                        bc = p->k2b_cached;
                        bo = p->k2b_tile_major;
                    }
                }
            }
        }
        p->k2b_cached = bc;
        if (p->k2b_tile_major != bo) {
            p->k2b_tile_major = bo;
            order_k2b(p);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    // line-pass tile, per shape class
    try {
        for (size_t ci = 0; ci < p->cls.size(); ++ci) {
            ClassP &K = p->cls[ci];
            if (K.tdoms.empty()) continue;   // no inverse transforms to time
            double bt = 1e300;
            int bf = K.fft_lds;
            for (int e : {2048, 4096, 6144}) {
                K.fft_lds = e;
                enqueue_inverse_xy(p, st, int(ci));   // warm-up
                HIP_OK(hipEventRecord(e0, st));
                for (int i = 0; i < iters; ++i) enqueue_inverse_xy(p, st, int(ci));
                HIP_OK(hipEventRecord(e1, st));
                HIP_OK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < bt) {
                    bt = ms;
                    bf = e;
                }
            }
            K.fft_lds = bf;
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->k2_unroll = bu;
    p->k2_persist = bp;
    if (best_unroll) *best_unroll = bu;
    if (best_persist) *best_persist = bp;
    if (best_ms) *best_ms = best;
}

template <typename F>
rp_status guarded(rp_plan p, F &&f) {
    if (!p) return RP_ERR_ARG;
    try {
        p->err.clear();
        f();
        return RP_OK;
    } catch (const Error &e) {
        p->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        p->err = "host allocation failed";
        return RP_ERR_NOMEM;
    } catch (const std::exception &e) {
        p->err = e.what();
        return RP_ERR_ARG;
    } catch (...) {
        p->err = "unknown error";
        return RP_ERR_ARG;
    }
}

}  // namespace rpot_host

using namespace rpot_host;

extern "C" {

rp_status rp_plan_domains(rp_plan *out, int32_t n_dom, const int32_t *dims, const double *origins,
                          const int32_t *system_id, double h, double dt, double c, rp_precision prec,
                          void *hip_stream) {
    if (!out) {
        g_create_error = "out is null";
        return RP_ERR_ARG;
    }
    *out = nullptr;
    rp_plan p = nullptr;
    try {
        if (n_dom < 1 || !dims || !origins) fail(RP_ERR_ARG, "n_dom >= 1 and non-null dims/origins required");
        if (!(h > 0) || !std::isfinite(h)) fail(RP_ERR_ARG, "h must be positive and finite");
        if (!(dt > 0) || !std::isfinite(dt)) fail(RP_ERR_ARG, "dt must be positive and finite");
        if (!(c > 0)) fail(RP_ERR_ARG, "c must be positive (or +INFINITY)");
        if (prec < RP_FP64 || prec > RP_FP32_RING_I16) fail(RP_ERR_ARG, "unknown precision");
        p = new rp_plan_s();
        p->n_dom = n_dom;
        p->h = h;
        p->dt = dt;
        p->c = c;
        p->prec = prec;
        p->stream = static_cast<hipStream_t>(hip_stream);
        p->p64 = (prec == RP_FP64);
        p->ring_fmt = prec == RP_FP64 ? RING_F64
                      : prec == RP_FP32  ? RING_F32
                      : prec == RP_FP32_RING_FP16 ? RING_F16
                      : prec == RP_FP32_RING_BF16 ? RING_BF16 : RING_I16;
        p->tsz = p->p64 ? 8 : 4;
        p->csz = p->p64 ? 16 : 8;
        p->spec_csz = p->csz;
        p->ring_esz = p->ring_fmt == RING_F64 ? 16 : (p->ring_fmt == RING_F32 ? 8 : 4);
        // default lag-sum batching (measured on MI355X, 8 x 64^3): two lags
        // per batch for the FP32 ring, one for the narrower rings and FP64
        p->k2_unroll = (p->ring_fmt == RING_F32) ? 2 : 1;
        // self cell: the exact integral of T(m dt - |u|/c)/|u| over the cell of
        // side h around the point; C1 = int_{[-1/2,1/2]^3} d^3u/|u| = 3 ln(2 + sqrt 3) - pi/2
        const double C1 = 3.0 * std::log(2.0 + std::sqrt(3.0)) - M_PI / 2.0;
        p->w_static = h * h * C1;
        if (std::isfinite(c)) {
            if (h * std::sqrt(3.0) / 2.0 >= c * dt)
                fail(RP_ERR_UNSUPPORTED, "self cell needs h*sqrt(3)/2 < c*dt");
            p->w_self0 = h * h * C1 - h * h * h / (c * dt);
            p->w_self1 = h * h * h / (c * dt);
        } else {
            p->w_self0 = h * h * C1;
            p->w_self1 = 0.0;
        }
        plan_geometry(p, dims, origins, system_id);
        plan_tables(p);
        plan_layout(p);
        plan_stats(p);
        *out = p;
        return RP_OK;
    } catch (const Error &e) {
        g_create_error = e.msg;
        delete p;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_create_error = "host allocation failed";
        delete p;
        return RP_ERR_NOMEM;
    } catch (...) {
        g_create_error = "unknown error";
        delete p;
        return RP_ERR_ARG;
    }
}

rp_status rp_workspace_bytes(rp_plan plan, size_t *bytes) {
    return guarded(plan, [&] {
        if (!bytes) fail(RP_ERR_ARG, "bytes is null");
        *bytes = plan->ws_bytes;
    });
}

rp_status rp_bind_workspace(rp_plan plan, void *dev_ptr, size_t bytes) {
    return guarded(plan, [&] {
        release_static(plan);
        do_bind(plan, dev_ptr, bytes);
    });
}

rp_status rp_bind_workspace_static(rp_plan plan) {
    return guarded(plan, [&] { do_bind_static(plan); });
}

rp_status rp_set_green_kernels(rp_plan plan) {
    return guarded(plan, [&] { do_green(plan); });
}

rp_status rp_push_sources(rp_plan plan, int64_t step, const void *const *src) {
    return guarded(plan, [&] { do_push(plan, step, src); });
}

rp_status rp_retarded_step(rp_plan plan, int64_t step, void *const *out) {
    return guarded(plan, [&] { do_step(plan, step, out); });
}

rp_status rp_plan_info(rp_plan plan, int32_t s, int32_t n, int32_t *m_lo, int32_t *m_hi, int32_t pad[3],
                       int32_t *depth) {
    return guarded(plan, [&] {
        if (s < 0 || n < 0 || s >= plan->n_dom || n >= plan->n_dom) fail(RP_ERR_ARG, "domain index out of range");
        const PairP &q = plan->pr(s, n);
        const bool formed = is_target(plan, s);
        if (m_lo) *m_lo = formed ? q.m_lo : -1;
        if (m_hi) *m_hi = formed ? q.m_hi : -1;
        if (pad)
            for (int a = 0; a < 3; ++a) pad[a] = plan->sys[plan->dom[s].sys].P[a];
        if (depth) *depth = plan->dom[n].depth;
    });
}

rp_status rp_plan_stats(rp_plan plan, rp_stats *out) {
    return guarded(plan, [&] {
        if (!out) fail(RP_ERR_ARG, "out is null");
        *out = plan->stats;
    });
}

rp_status rp_profile_lagsum(rp_plan plan, int32_t enable) {
    return guarded(plan, [&] { plan->profile = (enable != 0); });
}

rp_status rp_lagsum_time(rp_plan plan, double *total_ms, int64_t *launches) {
    return guarded(plan, [&] {
        double tot = 0.0;
        if (plan->n_recorded) {
            HIP_OK(hipEventSynchronize(plan->events[2 * plan->n_recorded - 1]));
            for (size_t i = 0; i < plan->n_recorded; ++i) {
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, plan->events[2 * i], plan->events[2 * i + 1]));
                tot += ms;
            }
        }
        if (total_ms) *total_ms = tot;
        if (launches) *launches = int64_t(plan->n_recorded);
        plan->n_recorded = 0;
    });
}

rp_status rp_set_tuning(rp_plan plan, int32_t knob, int32_t value) {
    return guarded(plan, [&] {
        switch (knob) {
        case RP_TUNE_LAGSUM_UNROLL:
            if (value != 1 && value != 2 && value != 4) fail(RP_ERR_ARG, "lag-sum unroll must be 1, 2 or 4");
            plan->k2_unroll = value;
            break;
        case RP_TUNE_LAGSUM_PERSISTENT:
            if (value != 0 && value != 1) fail(RP_ERR_ARG, "persistent must be 0 or 1");
            plan->k2_persist = value;
            break;
        case RP_TUNE_FFT_LDS:
            if (value != 0 && value != 2048 && value != 4096 && value != 6144)
                fail(RP_ERR_ARG, "line-pass tile must be 0, 2048, 4096 or 6144");
            plan->fft_lds = value;
            for (ClassP &K : plan->cls) K.fft_lds = 0;   // the plan's value for every class
            break;
        case RP_TUNE_FFT_REG:
            if (value != 0 && value != 1) fail(RP_ERR_ARG, "register line passes must be 0 or 1");
            plan->fft_reg = value;
            update_fused_additions(plan);
            plan_stats(plan);
            break;
        case RP_TUNE_FFT_PLANE:
            if (value != 0 && value != 1) fail(RP_ERR_ARG, "plane passes must be 0 or 1");
            plan->fft_plane = value;
            plan_stats(plan);
            break;
        case RP_TUNE_LAGSUM_CACHED:
            if (value != 0 && value != 1) fail(RP_ERR_ARG, "cached must be 0 or 1");
            plan->k2b_cached = value;
            break;
        case RP_TUNE_LAGSUM_TILE_MAJOR:
            if (value != 0 && value != 1) fail(RP_ERR_ARG, "tile-major must be 0 or 1");
            plan->k2b_tile_major = value;
            if (plan->kb > 1) order_k2b(plan);
            break;
        case RP_TUNE_LAGSUM_STEPS:
            if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
                fail(RP_ERR_ARG, "lag-sum steps per pass must be 1, 2, 4, 8 or 16");
            if (plan->ws) fail(RP_ERR_STATE, "choose the lag-sum steps per pass before rp_bind_workspace");
            if (value > 1 && plan->p64) fail(RP_ERR_UNSUPPORTED, "blocked lag-sum steps need an FP32 plan");
            plan->kb = value;
            plan_tables(plan);
            plan_layout(plan);
            plan_stats(plan);
            break;
        default:
            fail(RP_ERR_ARG, "unknown tuning knob");
        }
        release_graph(plan);   // a captured step holds the old schedule
    });
}

rp_status rp_class_info(rp_plan plan, int32_t cls, int32_t dims[3], int32_t pad[3], int32_t *n_domains) {
    return guarded(plan, [&] {
        if (cls < 0 || cls >= int(plan->cls.size())) fail(RP_ERR_ARG, "shape class out of range");
        const ClassP &K = plan->cls[cls];
        for (int a = 0; a < 3; ++a) {
            if (dims) dims[a] = K.N[a];
            if (pad) pad[a] = K.P[a];
        }
        if (n_domains) *n_domains = int32_t(K.doms.size());
    });
}

rp_status rp_set_class_tuning(rp_plan plan, int32_t cls, int32_t knob, int32_t value) {
    return guarded(plan, [&] {
        if (cls < 0 || cls >= int(plan->cls.size())) fail(RP_ERR_ARG, "shape class out of range");
        if (knob != RP_TUNE_FFT_LDS) fail(RP_ERR_ARG, "only the line-pass tile is chosen per shape class");
        if (value != 0 && value != 2048 && value != 4096 && value != 6144)
            fail(RP_ERR_ARG, "line-pass tile must be 0, 2048, 4096 or 6144");
        plan->cls[cls].fft_lds = value;
        release_graph(plan);
    });
}

rp_status rp_get_class_tuning(rp_plan plan, int32_t cls, int32_t knob, int32_t *value) {
    return guarded(plan, [&] {
        if (!value) fail(RP_ERR_ARG, "value is null");
        if (cls < 0 || cls >= int(plan->cls.size())) fail(RP_ERR_ARG, "shape class out of range");
        if (knob != RP_TUNE_FFT_LDS) fail(RP_ERR_ARG, "only the line-pass tile is chosen per shape class");
        const int v = cls_lds(plan, plan->cls[cls]);
        *value = v ? v : (plan->p64 ? 4096 : 2048);
    });
}

rp_status rp_get_tuning(rp_plan plan, int32_t knob, int32_t *value) {
    return guarded(plan, [&] {
        if (!value) fail(RP_ERR_ARG, "value is null");
        switch (knob) {
        case RP_TUNE_LAGSUM_UNROLL: *value = plan->k2_unroll; break;
        case RP_TUNE_LAGSUM_PERSISTENT: *value = plan->k2_persist; break;
        case RP_TUNE_LAGSUM_STEPS: *value = plan->kb; break;
        case RP_TUNE_LAGSUM_CACHED: *value = plan->k2b_cached; break;
        case RP_TUNE_LAGSUM_TILE_MAJOR: *value = plan->k2b_tile_major; break;
        case RP_TUNE_FFT_REG: *value = plan->fft_reg; break;
        case RP_TUNE_FFT_PLANE: *value = plan->fft_plane; break;
        case RP_TUNE_FFT_LDS: *value = plan->fft_lds ? plan->fft_lds : (plan->p64 ? 4096 : 2048); break;
        default: fail(RP_ERR_ARG, "unknown tuning knob");
        }
    });
}

rp_status rp_autotune(rp_plan plan, int32_t iters, int32_t *unroll, int32_t *persistent, double *lagsum_ms) {
    return guarded(plan, [&] {
        do_autotune(plan, iters, unroll, persistent, lagsum_ms);
        release_graph(plan);
    });
}

rp_status rp_capture_step(rp_plan plan, const void *const *src, void *const *out) {
    return guarded(plan, [&] { do_capture(plan, src, out); });
}

rp_status rp_launch_step(rp_plan plan, int64_t step) {
    return guarded(plan, [&] { do_launch_graph(plan, step); });
}

rp_status rp_surrogate_configure(rp_plan plan, double far_factor, int32_t n_lags, const int32_t *audit,
                                 int32_t n_audit) {
    return guarded(plan, [&] { sur_configure(plan, far_factor, n_lags, audit, n_audit); });
}

rp_status rp_plan_targets(rp_plan plan, const int32_t *targets, int32_t n_targets) {
    return guarded(plan, [&] {
        if (plan->ws) fail(RP_ERR_STATE, "choose the targets before rp_bind_workspace");
        if (plan->sur.on) fail(RP_ERR_UNSUPPORTED, "the surrogate and a target subset do not combine");
        std::vector<char> t;
        if (targets && n_targets > 0) {
            t.assign(size_t(plan->n_dom), 0);
            for (int i = 0; i < n_targets; ++i) {
                if (targets[i] < 0 || targets[i] >= plan->n_dom) fail(RP_ERR_ARG, "target index out of range");
                t[size_t(targets[i])] = 1;
            }
            for (size_t si = 0; si < plan->sys.size(); ++si) {
                bool any = false;
                for (int n : plan->sys[si].doms) any = any || t[size_t(n)];
                if (!any) fail(RP_ERR_ARG, "every system needs at least one target");
            }
        }
        plan->target = std::move(t);
        plan_pads(plan);
        plan_tables(plan);
        plan_layout(plan);
        plan_stats(plan);
        release_graph(plan);
    });
}

rp_status rp_history_split(rp_plan plan, int32_t min_gap) {
    return guarded(plan, [&] {
        if (plan->ws) fail(RP_ERR_STATE, "split the history before rp_bind_workspace");
        if (min_gap > 0 && plan->sur.on) fail(RP_ERR_UNSUPPORTED, "the surrogate and a split history do not combine");
        plan->split_gap = std::max(0, int(min_gap));
        plan_tables(plan);
        plan_layout(plan);
        plan_stats(plan);
        release_graph(plan);
    });
}

rp_status rp_history_host(rp_plan plan, int32_t enable) {
    return guarded(plan, [&] {
        if (plan->ws) fail(RP_ERR_STATE, "choose the host tier before rp_bind_workspace");
        plan->hist_host = enable != 0;
        plan_tables(plan);
        plan_layout(plan);
        plan_stats(plan);
        release_graph(plan);
    });
}

rp_status rp_history_host_bytes(rp_plan plan, size_t *bytes) {
    return guarded(plan, [&] {
        if (!bytes) fail(RP_ERR_ARG, "bytes is null");
        *bytes = plan->host_bytes;
    });
}

rp_status rp_bind_history_host(rp_plan plan, void *host_ptr, size_t bytes) {
    return guarded(plan, [&] {
        if (!plan->hist_host) fail(RP_ERR_STATE, "the host tier is off (rp_history_host)");
        if (plan->host_bytes == 0) return;   // nothing was split: no host ring
        if (!host_ptr) fail(RP_ERR_ARG, "host buffer is null");
        if (bytes < plan->host_bytes) fail(RP_ERR_NOMEM, "host buffer smaller than rp_history_host_bytes");
        if (reinterpret_cast<uintptr_t>(host_ptr) % 16) fail(RP_ERR_ARG, "host buffer must be 16-byte aligned");
        void *dev = nullptr;
        if (hipHostGetDevicePointer(&dev, host_ptr, 0) != hipSuccess || !dev) {
            (void)hipGetLastError();
            fail(RP_ERR_ARG, "host buffer is not pinned host memory (hipHostMalloc / pin_memory)");
        }
        if (plan->tier_stream) HIP_OK(hipStreamSynchronize(plan->tier_stream));
        if (!plan->tier_stream) HIP_OK(hipStreamCreateWithFlags(&plan->tier_stream, hipStreamNonBlocking));
        if (!plan->tier_fork) HIP_OK(hipEventCreateWithFlags(&plan->tier_fork, hipEventDisableTiming));
        if (!plan->tier_join) HIP_OK(hipEventCreateWithFlags(&plan->tier_join, hipEventDisableTiming));
        plan->host_dev = static_cast<char *>(dev);
        release_graph(plan);
    });
}

rp_status rp_surrogate_info(rp_plan plan, int32_t *n_far, int32_t *n_audited, int32_t *n_in, int32_t *n_out) {
    return guarded(plan, [&] {
        const SurrogateH &U = plan->sur;
        if (n_far) *n_far = int32_t(U.pairs.size());
        if (n_audited) *n_audited = int32_t(U.aud.size());
        if (n_in) *n_in = U.on ? U.n_in : 0;
        if (n_out) *n_out = U.on ? kNOut : 0;
    });
}

rp_status rp_surrogate_pairs(rp_plan plan, int32_t *target, int32_t *source, double *dist, int32_t *audited,
                             int32_t *fallen_back) {
    return guarded(plan, [&] {
        const SurrogateH &U = plan->sur;
        for (size_t f = 0; f < U.pairs.size(); ++f) {
            const FarPairH &F = U.pairs[f];
            if (target) target[f] = F.s;
            if (source) source[f] = F.n;
            if (dist) dist[f] = F.dist;
            if (audited) audited[f] = F.audited ? 1 : 0;
            if (fallen_back) fallen_back[f] = F.plain ? 1 : 0;
        }
    });
}

rp_status rp_surrogate_attach(rp_plan plan, rp_mlp mlp, const float *in_scale, const float *out_scale) {
    return guarded(plan, [&] { sur_attach(plan, mlp, in_scale, out_scale); });
}

rp_status rp_surrogate_multipole(rp_plan plan, int32_t enable) {
    return guarded(plan, [&] { sur_multipole(plan, enable); });
}

rp_status rp_surrogate_multipole_response(rp_plan plan, float *coef) {
    return guarded(plan, [&] { sur_multipole_response(plan, coef); });
}

rp_status rp_surrogate_features(rp_plan plan, float *x) {
    return guarded(plan, [&] { sur_features(plan, x); });
}

rp_status rp_surrogate_pair_response(rp_plan plan, float *coef, float *resid) {
    return guarded(plan, [&] { sur_pair_response(plan, coef, resid); });
}

rp_status rp_surrogate_judge(rp_plan plan, void *const *out, double tol, int32_t *n_fallback, double *worst,
                             int32_t *n_readmitted) {
    return guarded(plan, [&] { sur_judge(plan, out, tol, n_fallback, worst, n_readmitted); });
}

rp_status rp_surrogate_teacher(rp_plan plan, float *x, float *t, int32_t residual) {
    return guarded(plan, [&] { sur_teacher(plan, x, t, residual); });
}

rp_status rp_surrogate_readmit(rp_plan plan, double factor) {
    return guarded(plan, [&] { sur_readmit(plan, factor); });
}

rp_status rp_surrogate_sample(rp_plan plan, int32_t pairs_per_judge, int32_t fallback_slots) {
    return guarded(plan, [&] { sur_sample(plan, pairs_per_judge, fallback_slots); });
}

rp_status rp_surrogate_sample_fields(rp_plan plan, const int32_t *far_pairs, int32_t n, float *out) {
    return guarded(plan, [&] { sur_sample_fields(plan, far_pairs, n, out); });
}

rp_status rp_surrogate_judge_stats(rp_plan plan, int32_t *sampled, int32_t *refused, int32_t *slots_used,
                                   int32_t *next_pair) {
    return guarded(plan, [&] {
        const SurrogateH &U = plan->sur;
        if (!U.on) fail(RP_ERR_STATE, "surrogate not configured (rp_surrogate_configure)");
        int used = 0;
        for (const SlotP &k : U.slots) used += k.f >= 0;
        if (sampled) *sampled = U.last_sampled;
        if (refused) *refused = U.last_refused;
        if (slots_used) *slots_used = used;
        if (next_pair) *next_pair = U.sampled.empty() ? -1 : U.sampled[size_t(U.cursor)];
    });
}

rp_status rp_plan_destroy(rp_plan plan) {
    if (!plan) return RP_ERR_ARG;
    release_static(plan);
    for (hipEvent_t ev : plan->events) (void)hipEventDestroy(ev);
    release_graph(plan);
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    if (plan->tier_stream) {
        (void)hipStreamSynchronize(plan->tier_stream);
        (void)hipStreamDestroy(plan->tier_stream);
    }
    if (plan->tier_fork) (void)hipEventDestroy(plan->tier_fork);
    if (plan->tier_join) (void)hipEventDestroy(plan->tier_join);
    delete plan;
    return RP_OK;
}

const char *rp_last_error(rp_plan plan) {
    if (!plan) return g_create_error.c_str();
    return plan->err.c_str();
}

}  // extern "C"
