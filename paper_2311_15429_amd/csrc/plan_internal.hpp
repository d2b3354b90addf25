// Host-side plan state shared by the runtime (plan.cpp) and the far-pair
// surrogate (surrogate.cpp).  Not part of the C ABI.
#pragma once

#include "rpot.h"
#include "rpot_internal.hpp"

#include <map>
#include <string>
#include <vector>

namespace rpot_host {

using namespace rpot;

struct Error {
    rp_status code;
    std::string msg;
};

[[noreturn]] inline void fail(rp_status c, const std::string &m) { throw Error{c, m}; }

#define HIP_OK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) fail(RP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kGroupMax = 8;      // targets per lag-sum thread
constexpr int kGreenChunk = kMaxJobs;
constexpr int kMaxPad = 512;      // z passes stage >= 4 lines of the pad in 32 KiB of LDS
constexpr size_t kAlign = 256;

struct DomainP {
    int N[3];
    double o[3];
    int sys;
    int64_t npts;
    int depth = 1;           // spectral ring: lags 0 .. depth - 1
    int span = 1;            // history the pairs need: max m_hi + 1
    int zblocks = 0;
    int cls = 0;
    size_t off_ring = 0, off_scales = 0, off_zmax = 0, off_s0 = 0, off_p0 = 0, off_acc = 0;
    size_t off_t1 = 0, off_t2 = 0, off_s0hat = 0;
    // split history: later lag windows in their own spectral rings, fed from
    // a real-space ring of the raw sources (d1 slots; head at slot index t1_idx)
    std::vector<int> vr;
    int d1 = 0;
    int t1_idx = -1;
    size_t off_hist = 0;
    // with the host tier: the real-space ring at byte host_off of the pinned
    // host buffer, and a one-snapshot device staging buffer for the newest sources
    size_t host_off = 0, off_stage = 0;
};

// A later lag window [lo, hi] of source n with its own spectral ring.
// It stores the snapshots of ages lo .. hi (lo below lag_lo by kb - 1 with
// blocked lag-sum steps, whose pass reads kb - 1 younger ages); the lags
// lag_lo .. hi of the source's pairs are summed from it.
struct VRingP {
    int n = 0, lo = 0, hi = 0, W = 1;
    int lag_lo = 0;
    int idx = 0;             // ring / head slot index
    size_t off_ring = 0, off_scales = 0, off_zmax = 0, off_t1 = 0, off_t2 = 0;
    size_t off_stage = 0;    // host tier: the snapshot the next step transforms again
};

struct SystemP {
    std::vector<int> doms;
    int P[3];
    int Hz;
    int64_t C;
    int64_t Cpad;            // C rounded up to whole frequency tiles
    int64_t spec_base = 0;   // complex elements
    int64_t n_spec = 0;      // stored spectra (one per lag of every unordered pair)
    int64_t spec_elems = 0;  // their storage, tile-major per pair
};

struct PairP {
    int m_lo = -1, m_hi = -1;
    double rmin = 0, rmax = 0;
    int64_t spec0 = -1;      // element offset (within the system) of the pair's spectra,
                             // stored [tile][lag][kTile]; -1 when not stored
    bool conj = false;
};

struct ClassP {
    int N[3];
    int P[3];
    int Hz;
    int64_t C;
    std::vector<int> doms;
    std::vector<int> tdoms;  // the targets among doms (potentials evaluated)
    int fft_lds = 0;         // this class's line-pass tile (0: the plan's)
};

// One lag-sum schedule: groups of up to 8 accumulator slots of one system,
// their (source, lag) walk, and the work items (group x frequency tile).
struct K2Tables {
    std::vector<K2Group> groups;
    std::vector<K2Entry> entries;
    std::vector<K2Src> srcs;
    std::vector<K2Pair> pairs;
    std::vector<uint32_t> masks;
    std::vector<K2Item> items;
    int tg = 1;
};

// Device copy of a schedule, with room for the largest schedule the plan can
// switch to (the surrogate's fallback adds pairs to the plain lag sum).
struct K2Dev {
    size_t items = 0, groups = 0, entries = 0, srcs = 0, pairs = 0, masks = 0;
    size_t cap_items = 0, cap_groups = 0, cap_entries = 0, cap_srcs = 0, cap_pairs = 0, cap_masks = 0;
};

// A lag-sum accumulator slot: slot index into the DomDev table (a domain, or
// a judge slot past the domains), the target domain whose pairs it sums, and
// the sources it takes.
struct K2Member {
    int slot;
    int s;
    std::vector<int> srcs;
};

// Far-pair surrogate state (host).
struct FarPairH {
    int s = 0, n = 0;        // target, source
    double dist = 0;         // |c_s - c_n|
    int m_c = 0;             // round(dist / (c dt))
    double frac = 0;         // dist / (c dt) - m_c
    bool audited = false;    // the source keeps the plain history of this pair
    bool plain = false;      // fallen back: summed by the plain lag sum
    int slot = -1;           // fallback slot of a sampled pair (index into SurrogateH::slots)
    double rot[9] = {};      // frame axes (rows)
};

// A fallback slot of the judge by sample: a spectral ring of one far pair's
// lag window (ages lo .. lo + W - 1 of the source), refilled from the
// source's real-space history when the pair falls back, and the pair's Green
// spectra; its lag sum is added into the target's accumulator.
struct SlotP {
    int f = -1;              // far pair in the slot, or -1
    int idx = 0;             // ring / head slot index
    int W = 1, lo = 0;
    size_t off_ring = 0, off_scales = 0, off_zmax = 0, off_t1 = 0, off_t2 = 0;
    int64_t spec_elem = 0;   // its Green spectra: element offset from the start of the spectra
};

struct SurrogateH {
    bool on = false;
    double far_factor = 0;
    int n_lags = 0;
    int n_in = 0;
    std::vector<char> audit;       // per domain
    std::vector<int> far_index;    // [s * n_dom + n] -> far pair index, or -1
    std::vector<FarPairH> pairs;
    std::vector<int> src_slot;     // per domain: moment ring index, or -1
    std::vector<int> src_doms;     // moment ring index -> domain
    int mom_depth = 1;
    std::vector<int> aud;          // far pair indices with an audited source (judge order)
    std::vector<int> aud_row;      // judge slot -> row among audited pairs in far-pair order
    std::vector<float> mats;       // [n_far][2][kNBasis^2]: frame -> box, box -> frame
    std::vector<int> far_cls;      // target shape classes of far pairs
    std::map<int, size_t> off_Q;   // class -> LS dual basis [kNBasis][npts]
    K2Tables judge;
    K2Dev judge_dev;
    int n_chunks = 1;              // moment partial sums per source
    size_t off_mom = 0, off_mpart = 0, off_fpairs = 0, off_x = 0, off_y = 0, off_pc = 0, off_coef = 0;
    size_t off_order = 0, off_tbeg = 0, off_mats = 0, off_inscale = 0, off_outscale = 0;
    size_t off_jacc = 0, off_jt1 = 0, off_jt2 = 0, off_jF = 0, off_jcoef = 0, off_jres = 0;
    size_t off_budget = 0, off_fail = 0, off_aud = 0, off_jcb = 0;
    size_t off_rowfar = 0, off_tcoef = 0;   // teacher rows: far-pair index per audited row, multipole terms
    size_t jt1_elems = 0, jt2_elems = 0, jF_elems = 0;
    std::vector<size_t> jacc_off;  // judge slot -> byte offset of its accumulator
    std::vector<int> synth_targets;  // domains that are the target of a far pair
    std::vector<int32_t> h_order, h_tbeg;   // active far pairs by target (CSR)
    rp_mlp mlp = nullptr;
    bool attached = false;
    int multipole = 0;             // analytic multipole far-pair terms: 1 alone, 2 plus the network's correction
    double readmit = 0;            // a fallen-back pair within readmit x its budget returns (0: never)
    size_t off_pinv = 0;           // [kNBasis][64] node-to-coefficient fit
    // judge by sample (rp_surrogate_sample)
    int per_judge = -1;            // far pairs of non-audit sources judged per call (0: all; < 0: off)
    int n_slots = 0;
    std::vector<int> sampled;      // far pairs of non-audit sources (far-pair order)
    int cursor = 0;                // next position in `sampled`
    int last_sampled = 0, last_refused = 0;
    std::vector<SlotP> slots;
    int slot_W = 0;                // lag window capacity of a slot
    int64_t slot_Cpad = 0;
    K2Tables k2p;                  // lag sum of the slot pairs (added into the targets)
    K2Dev k2p_dev;
    size_t off_sjobs = 0, off_jjobs = 0, off_sfield = 0, off_sres = 0, off_sfail = 0, off_fillslots = 0;
    size_t off_fill_t1 = 0, off_fill_t2 = 0, off_fill_zmax = 0;
    size_t fill_t1 = 0, fill_t2 = 0, fill_zmax = 0;   // bytes per fill job
    std::vector<SampleJob> h_sjobs;        // host copies of uploaded tables (kept until copied)
    std::vector<SampleJudgeJob> h_jjobs;
    std::vector<int32_t> h_fill, h_heads;
    std::vector<DomDev> h_dd;
};

constexpr int kFillJobs = 8;       // ring refills per launch (scratch sets)

// One forward transform into a spectral ring (ingest of a step, or a refill):
// the sources (the newest, or a snapshot of a real-space ring), the scratch of
// the passes, and the ring slot written.
struct RingJob {
    int n = 0;                         // source domain (shape, S(0), z blocks)
    const void *src = nullptr;
    const int32_t *src_head = nullptr; // src is a real-space ring: read slot (*src_head - src_lag) mod src_depth
    int src_depth = 0, src_lag = 0;
    void *store = nullptr;             // also copy the sources to slot *store_head of this ring (null: none)
    const int32_t *store_head = nullptr;
    char *t1 = nullptr, *t2 = nullptr;
    char *ring = nullptr;
    float *scales = nullptr, *zmax = nullptr;
    const int32_t *head = nullptr;     // ring slot written
    int depth = 1;
};

}  // namespace rpot_host

struct rp_plan_s {
    int n_dom = 0;
    double h = 0, dt = 0, c = 0;
    rp_precision prec = RP_FP64;
    hipStream_t stream = nullptr;
    bool p64 = true;
    int ring_fmt = rpot::RING_F64;
    size_t tsz = 8, csz = 16, ring_esz = 16, spec_csz = 16;
    double w_self0 = 0, w_self1 = 0, w_static = 0;

    std::vector<rpot_host::DomainP> dom;
    std::vector<rpot_host::SystemP> sys;
    std::vector<rpot_host::PairP> pair;   // [s * n_dom + n]
    std::vector<rpot_host::ClassP> cls;

    rpot_host::K2Tables k2;               // the plain lag sum of every step
    rpot_host::K2Dev k2_dev;
    std::vector<rpot::DomDev> domdev;     // domains, then judge slots
    int k2_unroll = 1;   // lags whose loads a lag-sum thread issues together
    int k2_persist = 0;  // persistent lag-sum launch (work counter) instead of one block per item
    int fft_lds = 0;     // line-pass tile: complex elements staged per block (0: default)
    int fft_reg = 1;     // FP32 line passes of the supported lengths in registers
    int fft_plane = 1;   // FP32 forward z+y and inverse y+z passes as plane passes where they apply
    int split_gap = 0;   // split a source's history at lag gaps of at least this many lags (0: off)
    std::vector<rpot_host::VRingP> vring;
    // host tier of a split history: real-space rings in pinned host memory
    bool hist_host = false;
    size_t host_bytes = 0;            // pinned host bytes the rings need
    char *host_dev = nullptr;         // device-visible address of the bound host buffer
    hipStream_t tier_stream = nullptr;
    hipEvent_t tier_fork = nullptr, tier_join = nullptr;
    bool tier_open = false;           // host-tier copies forked and not yet joined
    int n_heads = 0;     // ring heads: domains, judge slots, split rings, real-space rings
    int n_cu = 0;        // compute units of the bound device
    // captured steps: one graph, or one per phase of a block of kb steps
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> graph_execs;
    // temporal blocking of the lag sum: kb steps per pass (1: off).  k2b is the
    // pass of a block's first step (one target per thread), k2c[i] adds the
    // lags m < i of the block's step i (i = 1 .. kb-1)
    int kb = 1;
    bool fuse_add = false;   // blocked steps: own-source lags added by the inverse x pass (fused_additions)
    int k2b_cached = 0;      // blocked pass: cached loads (else non-temporal)
    int k2b_tile_major = 0;  // blocked pass: items of one frequency tile next to each other (else costliest first)
    rpot_host::K2Tables k2b;
    rpot_host::K2Dev k2b_dev;
    std::vector<rpot_host::K2Tables> k2c;
    std::vector<rpot_host::K2Dev> k2c_dev;
    hipStream_t capture_stream = nullptr;

    std::map<int, size_t> tw64, tw32;   // FFT length -> byte offset of its twiddles
    size_t off_state = 0, off_head = 0, off_prev_head = 0, off_domdev = 0, off_counter = 0;
    size_t off_spec = 0, off_gtmp = 0, off_accd = 0, off_gstat = 0, off_t1d = 0, off_t2d = 0;
    size_t off_qstage = 0;   // I16 ring: FP32 staging of one ingest launch
    size_t off_s0d = 0, off_p0d = 0;
    size_t ws_bytes = 0;
    char *ws = nullptr;

    bool profile = false;
    std::vector<hipEvent_t> events;   // begin/end pairs of recorded lag-sum launches
    size_t n_recorded = 0;

    int static_dev = -1;     // device whose fixed workspace array the plan is bound to (-1: none)
    std::vector<char> target;   // per domain: potentials evaluated (empty: every domain)
    bool green_ready = false;
    int64_t next_step = 0;
    bool pushed = false;
    std::string err;
    rp_stats stats{};

    rpot_host::SurrogateH sur;

    template <typename P = void>
    P *at(size_t off) const { return reinterpret_cast<P *>(ws + off); }
    const rpot_host::PairP &pr(int s, int n) const { return pair[size_t(s) * n_dom + n]; }
    rpot_host::PairP &pr(int s, int n) { return pair[size_t(s) * n_dom + n]; }
};

namespace rpot_host {

// plan.cpp
void check_launch();
RadixPlan make_radix(int P);
const void *tw_ptr(rp_plan p, int P, bool dbl);
bool plane_ok(rp_plan p);
bool real_spec(rp_plan p, int s, int n);
LinePass inv_x(rp_plan p, const int N[3], const int P[3], int Hz, bool dbl);
LinePass inv_y(rp_plan p, const int N[3], const int P[3], int Hz, bool dbl);
// gmax: targets per group; m_cap: every pair's window clipped to lags <= m_cap.
void build_k2(rp_plan p, int sys, const std::vector<K2Member> &members, K2Tables &T, int gmax, int m_cap);
void finish_k2(rp_plan p, K2Tables &T);
void plan_tables(rp_plan p);
void plan_layout(rp_plan p);
// Domain s is a target: its potential is evaluated (rp_plan_targets).
inline bool is_target(rp_plan p, int s) { return p->target.empty() || p->target[size_t(s)] != 0; }
// A bound workspace, and for a plan on the fixed array of rp_bind_workspace_static
// that no later bind on its device has taken the array over (RP_ERR_STATE otherwise).
void need_ws(rp_plan p);
void plan_stats(rp_plan p);
void release_graph(rp_plan p);
void upload_k2(rp_plan p, const K2Tables &T, const K2Dev &D, hipStream_t st);
void rebuild_blocked(rp_plan p, hipStream_t st);   // blocked schedules for the current plain pairs
void update_fused_additions(rp_plan p);            // whether the inverse x pass adds a step's own lags
int lag_phase(rp_plan p, int64_t step);            // phase of a step within its block of blocked steps
K2Args k2_args(rp_plan p, const K2Tables &T, const K2Dev &D, const int32_t *head);
void enqueue_k2(rp_plan p, const K2Args &a, int tg, hipStream_t st, int unroll, int persist);
bool keeps_history(rp_plan p, int s, int n);
bool plain_pair(rp_plan p, int s, int n);
bool ring_scaled(rp_plan p);
size_t scale_bytes(rp_plan p, int depth, int64_t Cpad);
void green_spectra(rp_plan p, int s, int n, int mode, int m0, int count, void *const *outs, int out_fmt,
                   int64_t tile_stride);
// Forward transforms of jobs of one shape class, kMaxJobs per launch.
void enqueue_ring_jobs(rp_plan p, const ClassP &K, const std::vector<RingJob> &jobs, hipStream_t st);
double k2_bytes(rp_plan p, const K2Tables &T);

// surrogate.cpp
void sur_classify(rp_plan p);                 // after the windows, before plan_tables
void sur_layout(rp_plan p, size_t &off);      // workspace for the surrogate
void sur_bind(rp_plan p);                     // uploads after bind
void sur_enqueue_moments(rp_plan p, const void *const *src, hipStream_t st);
void sur_enqueue_infer(rp_plan p, void *const *out, hipStream_t st);
void sur_configure(rp_plan p, double far_factor, int n_lags, const int32_t *audit, int n_audit);
void sur_attach(rp_plan p, rp_mlp mlp, const float *in_scale, const float *out_scale);
void sur_features(rp_plan p, float *x);
void sur_pair_response(rp_plan p, float *coef, float *resid);
void sur_judge(rp_plan p, void *const *out, double tol, int32_t *n_fallback, double *worst, int32_t *n_readmitted);
void sur_readmit(rp_plan p, double factor);
void sur_multipole(rp_plan p, int enable);
void sur_multipole_response(rp_plan p, float *coef);
void sur_teacher(rp_plan p, float *x, float *t, int residual);
void sur_sample(rp_plan p, int per_judge, int n_slots);
void sur_sample_fields(rp_plan p, const int32_t *far_pairs, int n, float *out);
void sur_slot_tables(rp_plan p);                          // after plan_layout's DomDev table
void sur_ring_jobs(rp_plan p, const ClassP &K, std::vector<RingJob> &jobs);   // the slots' per-step transforms
void sur_enqueue_slots(rp_plan p, const int32_t *head, hipStream_t st, int phase);   // the slots' lag sum
// The plain lag sum of every target over the pairs pred admits: groups of up
// to gmax targets, windows clipped to lags <= m_cap.
void main_k2(rp_plan p, K2Tables &T, bool (*pred)(rp_plan, int, int), int gmax = kGroupMax, int m_cap = INT32_MAX);

}  // namespace rpot_host
