// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

typedef struct rp_mlp_s *rp_mlp;

namespace rpot {

template <typename T>
struct Cx {
    T x, y;
};

// Division by a fixed divisor d >= 1 through a multiply-high:
// n / d = (mulhi(n, mul) + n) >> shift for every n < 2^31.
struct FastDiv {
    uint32_t mul = 1, shift = 0;
    FastDiv() = default;
    __host__ explicit FastDiv(uint32_t d) {
        while ((uint64_t(1) << shift) < d) ++shift;
        mul = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << shift) - d)) / d + 1);
    }
    __device__ __forceinline__ int div(int n) const {
        return int((uint64_t(__umulhi(uint32_t(n), mul)) + uint32_t(n)) >> shift);
    }
};

// Mixed-radix factorisation of an FFT length (radices 4, 2, 3), with the
// per-stage divisors of the Stockham index map (butterflies per line
// nq = P / r and the stride p of the radices before the stage).
constexpr int kMaxFft = 512;      // longest FFT
struct RadixPlan {
    int n;
    int r[16];
    FastDiv dq[16], dp[16];
    int tws[16];                  // twiddle stride P / (p r)
};

constexpr int kMaxJobs = 16;
constexpr int kFftThreads = 256;
// Frequencies per lag-sum block.  The history ring and the Green spectra are
// stored tile-major ([tile][slot or lag][kTile][...]) so that one block streams
// contiguous memory across consecutive lags.
constexpr int kTile = 256;

// Ring storage formats of the source-spectrum history.
// RING_I16: 16-bit integers, one scale per (slot, frequency tile, component).
enum RingFmt : int { RING_F64 = 0, RING_F32 = 1, RING_F16 = 2, RING_BF16 = 3, RING_I16 = 4 };

// ---------------------------------------------------------------------------
// Generic strided line FFT (complex to complex).  A line is addressed as
//   base + outer * s_outer + inner * s_inner + j * s_j   (element = one complex)
// with line = outer * n_inner + inner.  Only the first n_in points of a line
// are read (the rest are zero) and only the first n_out are written.
struct LineJob {
    const void *in;
    void *out;
    float *qscale;         // ring quantisation: scales [depth][4] of the domain (FP16/BF16, read), or
                           // [tile][depth][4] (16-bit integers, written by the quantising x pass); else null
    const int32_t *head;   // ring output: current slot of the domain's ring, else null
    int64_t slot_stride;   // ring output: elements per slot
    int64_t tile_stride;   // tiled output: elements per frequency tile (0: linear output)
    // Inverse x pass of a blocked lag-sum step (LinePass::add_fmt != 0): the
    // step's lags m < add_lags of the target's own sources (its self pair) are
    // added to the accumulated spectrum as it is read, instead of a separate
    // read-modify-write of the accumulator.
    const void *add_ring;      // the target's history ring (tile-major rows)
    const float *add_scales;   // its scales (FP16/BF16 [depth][4], I16 [tile][depth][4])
    const int32_t *add_head;   // its head (slot of the newest snapshot, lag 0)
    const void *add_spec;      // Green spectra of the self pair: row tile * add_w + m, real (kTile
                               // floats at the start of each row's place of kTile complex values)
    int32_t add_depth, add_w, add_lags;
};

struct LinePass {
    int P, n_in, n_out;
    int lines, n_inner;
    int L;                 // lines per block (set by the launcher)
    int lds_elems;         // complex elements staged per block: 0 (default 4096), 2048, 4096 or 6144
                           // (FP32; half of it in FP64)
    int reg;               // 1: register-resident pass where the length allows (FP32)
    int add_fmt;           // ring format of the fused lag additions (0: none; see LineJob)
    FastDiv dL, dP, dinner, dnout;   // set by the launcher
    int64_t in_j, in_inner, in_outer;
    int64_t out_j, out_inner, out_outer;
    int dir;               // -1 forward, +1 inverse
    // element order of the global reads / writes of a block's tile: 0 = the
    // block's lines fastest (j-fastest when the stride of j is 1); g > 0 =
    // groups of g consecutive lines fastest, then j, then the groups (g lines
    // interleaved at stride 1 with j at stride g: one run per group of lines)
    int in_group, out_group;
    int out_fmt;           // RingFmt of the output (F64/F32 = plain complex)
    int tile_comp;         // tiled output: components per frequency (1 or 4); the
                           // linear index e = k * tile_comp + c goes to tile
                           // k / kTile (stride tile_stride), and within it to
                           // [c/2][k%kTile][c%2] (FP32 ring), [c][k%kTile] (FP64
                           // ring) or [k%kTile][c] (FP16/BF16 ring, one component)
    const void *tw;        // twiddles exp(-2 pi i j / P), j < P
    RadixPlan rp;
    int n_jobs;
    LineJob jobs[kMaxJobs];
};

// ---------------------------------------------------------------------------
// Real-to-complex z pass.
//  mode 0: sources.  Line (x, y) of component mu is dS = S - S0 along z
//          (Nz points, zero-padded to Pz); output [Nx][Ny][Hz][4] interleaved.
//  mode 1: Green's function of lag m for the pair (s <- n) generated on the
//          fly on the full Px x Py x Pz grid; output [Px][Py][Hz].
//  mode 2: as mode 1 with the instantaneous (static) kernel h^3/R.
struct ZFwdJob {
    const void *src;       // mode 0: S  [4][Nx][Ny][Nz]; with src_head a ring of such arrays
    const void *s0;        // mode 0: S0 [4][Nx][Ny][Nz] (null: transform S itself)
    const int32_t *src_head;  // mode 0: read slot (*src_head - src_lag) mod src_depth of the src ring
    void *store;           // mode 0: also copy S into slot *store_head of this ring (or null)
    const int32_t *store_head;   // slot of the store ring (null: store is one snapshot)
    int32_t src_depth, src_lag;
    void *out;
    float *zmax;           // mode 0: per-block max |dS| per component, or null
    double off[3];         // modes 1/2: o_s - o_n
    int Ns[3], Nn[3];      // modes 1/2: target / source dims
    int m;                 // mode 1: lag
    int self;              // modes 1/2: s == n
};

struct ZFwd {
    int mode;
    int reg;               // 1: the register-resident pass where it applies (FP32 sources)
    int Nx, Ny, Nz;        // mode 0 dims (common to every job of a launch)
    int Px, Py, Pz, Hz;
    FastDiv dP, dHz, dPy2; // set by the launcher
    double h, inv_cdt, scale;      // inv_cdt = 1/(c dt) (0 for c = inf); scale = 1/(Px Py Pz)
    double w_self0, w_self1, w_static;
    const void *tw;
    RadixPlan rp;
    int n_jobs;
    ZFwdJob jobs[kMaxJobs];
};

// Complex-to-real z pass with crop: input [Nx][Ny][Hz][4], output
// out[mu][x][y][z] = IFFT(...)[z] (+ add[mu][x][y][z]) for z < Nz.
struct ZInvJob {
    const void *in;
    void *out;
    const void *add;       // static potential, or null
};

struct ZInv {
    int reg;               // 1: the register-resident pass where it applies (FP32)
    int Nx, Ny, Nz;
    int Pz, Hz;
    FastDiv dHz, dNz, dnp; // set by the launcher (dnp: position pairs per block)
    const void *tw;
    RadixPlan rp;
    int n_jobs;
    ZInvJob jobs[kMaxJobs];
};

// ---------------------------------------------------------------------------
// Lag-sum multiply-accumulate.
struct K2Entry {
    int32_t src;           // source domain (global index)
    int32_t m;             // lag
    uint32_t mask;         // group members fed by this (source, lag)
    uint32_t conj;         // members that use the conjugate of the stored spectrum
    int64_t ring_off;      // the source's ring (complex elements from the first ring)
    int32_t depth;         // the source's ring depth
    uint32_t real;         // members whose spectra are real (K2Src::real)
    int32_t spec_tile[8];  // per member: (pair base + lag * kTile) / kTile within the system
    int32_t spec_w[8];     // per member: lags of the pair (spectrum tile stride / kTile)
};

// Per (group, source): the lag range covered by any member and the ring.
struct K2Src {
    int32_t n;             // ring (and head) index: the source domain, or one of its split rings
    int32_t m_min, m_max;  // union of the members' lag windows for this source (within this ring)
    int32_t depth;         // the ring's depth
    int64_t ring_off;      // the ring (complex elements from the first ring)
    uint32_t conj;         // members that use the conjugate of the stored spectra
    int32_t mask_off;      // masks[mask_off + m - m_min]: members whose window holds lag m
    int32_t m_base;        // lag of the ring's newest snapshot (0, or a split ring's first lag)
    uint32_t real;         // members whose spectra are real: rows of kTile floats (the first
                           // half of the row's place), for the self pairs of FP32 plans
};

// Per (group, source, member): where the pair's spectra sit.  They are stored
// [tile][lag][kTile]; the row (kTile complex values) of lag m in tile `tile`
// is row0 + tile * w + m (relative to the system's spectra).
struct K2Pair {
    int32_t row0;          // (pair base) / kTile - m_lo
    int32_t w;             // lags of the pair
};

struct K2Group {
    int64_t C;             // spectrum length of the system
    int64_t spec_base;     // element offset of the system's spectra
    int32_t entry_begin, entry_end;
    int32_t src_begin, src_end;   // K2Src records; K2Pair records at [src * 8 + member]
    int32_t n_members;
    int32_t member[8];     // global target domain index per member
};

struct K2Item {
    int32_t group;
    int32_t k0;
};

struct DomDev {
    int64_t ring_off;      // element offset (complex) of the domain's ring [tile][slot][kTile][4]
    int64_t acc_off;       // element offset (complex) of the domain's accumulator (set 0)
    int64_t acc_set_stride;   // complex elements between the accumulator sets of a blocked lag sum
    int64_t scale_off;     // float offset of the ring's scales: [depth][4] (FP16/BF16),
                           // [tile][depth][4] (I16)
    int32_t depth;
    int32_t pad;
};

struct K2Args {
    const K2Item *items;
    const K2Group *groups;
    const K2Entry *entries;
    const K2Src *srcs;
    const K2Pair *pairs;
    const uint32_t *masks;
    const DomDev *doms;
    const void *spectra;
    const void *ring;
    const float *scales;
    void *acc;
    const int32_t *head;   // current slot of every ring (step mod depth)
    int *counter;          // persistent launch: next work item
    int n_items;
    int n_dom;
    int acc_set;           // accumulator set written (0 unless steps are blocked)
    int accumulate;        // 1: add to the accumulator set instead of overwriting it
    int cached;            // blocked pass: cached loads instead of non-temporal ones
};

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).
void launch_line_pass(const LinePass &a, int prec64, hipStream_t st);
// register-resident FP32 line pass (fft_reg.hip); false when it does not
// cover the pass (nothing launched)
bool launch_line_reg(const LinePass &a, hipStream_t st);
// whether launch_line_reg covers the pass (an x pass into a 16-bit integer
// ring then quantises in the same launch)
bool line_reg_supported(const LinePass &a);
// register-resident FP32 z passes (fft_reg.hip); false when they do not cover
// the launch (nothing launched)
bool launch_zfwd_reg(const ZFwd &a, hipStream_t st);
bool launch_zinv_reg(const ZInv &a, hipStream_t st);
// FP32 plane passes (fft_reg.hip): the forward z and y passes, or the inverse
// y and z passes, of the same jobs in one launch; false when they do not cover
// the pair of passes (nothing launched)
bool launch_zy_fwd_plane(const ZFwd &z, const LinePass &y, hipStream_t st);
bool launch_yz_inv_plane(const LinePass &y, const ZInv &zi, hipStream_t st);
// whether a grid of Ny x Nz (y, z) points with pads Py, Pz has plane passes
bool plane_shape(int Py, int Pz, int Ny, int Nz);
void launch_zfwd(const ZFwd &a, int prec64, hipStream_t st);
void launch_zinv(const ZInv &a, int prec64, hipStream_t st);
int zfwd_lines_per_block(int Pz, int prec64);
// grid_persist > 0: persistent launch with that many blocks (capped at the
// item count); 0: one block per item.
void launch_lagsum(const K2Args &a, int prec64, int ring_fmt, int tg, int unroll, int grid_persist,
                   hipStream_t st);
int lagsum_blocks_per_cu(int prec64, int ring_fmt, int tg, int unroll);
// Lag sum of kb steps in one pass (FP32 paths, one target per thread, kb = 2,
// 4 or 8): every item writes the kb accumulator sets of its target.  unroll:
// snapshots whose loads are issued before their products (1, 2 or 4).
void launch_lagsum_block(const K2Args &a, int ring_fmt, int kb, int unroll, int grid_persist, hipStream_t st);
// Self-pair spectra to real rows: each of n_rows rows of kTile complex FP32
// values becomes kTile floats (the real parts) in the first half of its place.
void launch_spec_real(void *rows, int64_t n_rows, hipStream_t st);
int lagsum_block_blocks_per_cu(int ring_fmt, int kb, int unroll);
// Per-snapshot ring scales: for each job, scales[head*4 + mu] =
// 2^(e-15) with npts * max_blocks zmax[b][mu] <= 2^e (1 when the max is 0).
struct ScaleJob {
    const float *zmax;
    float *scales;
    const int32_t *head;   // current ring slot of the domain
    int32_t nblk;
    int32_t pad_;
    double npts;
};
struct ScaleArgs {
    int n_jobs;
    ScaleJob jobs[kMaxJobs];
};
void launch_ring_scale(const ScaleArgs &a, hipStream_t st);
// Block-floating-point quantisation of freshly transformed source spectra
// into a 16-bit integer ring (RING_I16).  stage holds the spectrum as FP32
// rows [tile][c/2][kTile][c%2] (the FP32 ring row order, one row per tile);
// frequencies k >= C are ignored.  Per tile and component the largest |Re|,
// |Im| M gives the scale M / 32767; the row [kTile][c] of int16 (re, im)
// pairs goes to slot *head of the ring [tile][depth][kTile][4], the scales to
// scales[(tile * depth + slot) * 4 + c].
struct QuantJob {
    const float *stage;
    void *ring;
    float *scales;
    const int32_t *head;
    int64_t C;
    int32_t depth;
    int32_t n_tiles;
};
struct QuantArgs {
    int n_jobs;
    int max_tiles;
    QuantJob jobs[kMaxJobs];
};
void launch_quant_i16(const QuantArgs &a, hipStream_t st);
void launch_static_mac(void *acc, const void *g, const void *s, int64_t C, hipStream_t st);
void launch_convert(void *dst, int dst64, const void *src, int src64, int64_t n, hipStream_t st);
void launch_fill_zero(void *dst, size_t bytes, hipStream_t st);
// step += 1 and every domain's ring head moves one slot (mod its depth); the
// heads before the move are kept in prev.
void launch_advance_step(int64_t *step, int32_t *head, int32_t *prev, const DomDev *doms, int n_dom, hipStream_t st);

// Host tier of a split history: copies of one real-space snapshot between a
// device staging buffer and a ring in pinned host memory.  Slots are taken
// from the device-side step counter and ring head, so a captured step replays
// correctly at every step.  Ring slot: (head[head_idx] + shift) mod depth; a
// copy with alt reads alt instead while step + shift <= 0 (a snapshot from
// before step 0, which is S(0)).
struct TierJob {
    const uint4 *src;
    uint4 *dst;
    const uint4 *alt;
    int64_t n16;          // 16-byte words per snapshot
    int32_t src_depth;    // > 0: src is a ring of that many snapshots
    int32_t dst_depth;    // > 0: dst is a ring of that many snapshots
    int32_t shift;
    int32_t head_idx;
};
constexpr int kMaxTierJobs = 16;
struct TierArgs {
    const int64_t *step;
    const int32_t *head;
    int n_jobs;
    TierJob jobs[kMaxTierJobs];
};
void launch_tier_copy(const TierArgs &a, hipStream_t st);

// ---------------------------------------------------------------------------
// Far-pair surrogate.
//
// Moments of dS = S(l) - S(0) of a source about its centre (weight h^3), in
// ring order:
//   0 q = sum dS_0;  1..3 p_i = sum dS_0 x_i;  4..9 Q = sum dS_0 x_i x_j for
//   (xx, yy, zz, xy, xz, yz);  10..12 J_i = sum dS_{1+i};
//   13..21 K_ij = sum dS_{1+i} x_j (row-major i, j).
constexpr int kNFeat = 22;        // moments the network reads (q, p, Q, J, K)
constexpr int kNMom = 50;         // plus the charge's third and the current's second moments
constexpr int kFeatStride = 56;   // floats per moment-ring slot
constexpr int kNBasis = 20;       // tensor-Legendre functions of total degree <= 3
constexpr int kNOut = 4 * kNBasis;
constexpr int kNGeo = 2;          // geometry features of a pair
constexpr int kNBlocks = 6;       // history blocks H, gH, fH, gfH, g^2 H, f^2 H
constexpr int kMomChunks = 64;    // partial sums per source

struct MomentJob {
    const float *src;      // S(l) [4][Nx][Ny][Nz]
    const float *s0;       // S(0)
    float *ring;           // the source's moment ring [depth][kFeatStride]
    float *partial;        // the source's partial sums [kMomChunks][kNMom]
    int N[3];
    float o[3];            // position of point (0,0,0) relative to the domain centre
};
struct MomentArgs {
    float h;
    double h3;
    int depth;
    const int64_t *step;
    int n_jobs;
    MomentJob jobs[kMaxJobs];
};

// A far pair (target s <- source n) on the device.  rot holds the frame axes
// as rows: e1 along c_s - c_n, e2 and e3 completing a right-handed frame.
struct FarPair {
    int32_t s, n;
    int32_t m_c;           // centre lag round(|c_s - c_n| / (c dt))
    int32_t src_slot;      // moment ring of the source
    float rot[9];
    float inv_d;           // 1 / |c_s - c_n|
    float geo[kNGeo];      // (r_ref / |c_s - c_n|, |c_s - c_n| / (c dt) - m_c)
    float d[3];            // c_s - c_n
    float hw[3];           // half side of the target box per axis
};
struct FeatArgs {
    const FarPair *pairs;
    const float *moments;  // [n_src][depth][kFeatStride]
    const float *in_scale; // [kNFeat]
    float *x;              // [n_pairs][n_in]
    const int64_t *step;
    int64_t step_adj;      // the features are those of step *step + step_adj
    int depth;
    int n_lags;
    int n_in;
    int n_pairs;
};
// Coefficient maps between the network's frame basis and the target box basis:
//  dir 0: out = M (R^T-mixed (in * scale * inv_d))   (frame -> box)
//  dir 1: out = R-mixed (Minv in)                    (box -> frame)
// mats = [n_far][2][kNBasis * kNBasis] (M, Minv), row r uses pair index[r]
// (or r when index is null).
struct XformArgs {
    const FarPair *pairs;
    const float *mats;
    const float *in;
    float *out;
    const float *scale;    // [kNOut], dir 0 only
    const int32_t *index;
    int dir;
    int n;
    int accumulate;        // dir 0: add to out instead of writing it
};
// coef[s] = sum of pc[order[i]] over i in [tgt_begin[s], tgt_begin[s + 1])
struct CoefArgs {
    const float *pc;
    const int32_t *order;
    const int32_t *tgt_begin;
    float *coef;
    int n_targets;
};
struct SynthJob {
    const float *coef;     // [4][kNBasis]
    float *out;            // [4][Nx][Ny][Nz], += sum_b coef[mu][b] B_b
    int N[3];
};
struct SynthArgs {
    int n_jobs;
    SynthJob jobs[kMaxJobs];
};
// Least-squares coefficients coef = Q F (Q: [kNBasis][npts]) and residuals
// resid[mu] = max |F_mu - sum_b c[mu][b] B_b|, resid[4 + mu] = max |F_mu|
// with c = coef_in (or the fitted coef when coef_in is null).
struct ProjJob {
    const float *F;        // [4][npts]
    const float *Q;
    const float *coef_in;
    float *coef;
    float *resid;
    int N[3];
    int64_t npts;
};
struct ProjArgs {
    int n_jobs;
    ProjJob jobs[kMaxJobs];
};
// budget[mu] = scale * max |out_mu|
struct BudgetJob {
    const float *out;
    float *budget;
    int64_t npts;
    float scale;
};
struct BudgetArgs {
    int n_jobs;
    BudgetJob jobs[kMaxJobs];
};
// Judge correction: a pair that is active and whose residual exceeds the
// budget in any component has out += F - sum_b pc B_b and fail = 1.
struct CorrJob {
    const float *F;
    const float *pc;
    const float *resid;
    const float *budget;
    float *out;
    int32_t *fail;
    int N[3];
    int active;
};
struct CorrArgs {
    int n_jobs;
    int64_t max_pts;
    CorrJob jobs[kMaxJobs];
};
void launch_moments(const MomentArgs &a, hipStream_t st);
void launch_features(const FeatArgs &a, hipStream_t st);
struct TeacherArgs {
    const FarPair *pairs;
    const int32_t *row_far;    // [n_rows]: far-pair index of each audited row
    const float *x_all;        // [n_far][n_in] network inputs of every far pair
    float *x_out;              // [n_rows][n_in]
    float *t;                  // [n_rows][kNOut] pair coefficients in, targets out
    const float *sub;          // [n_rows][kNOut] subtracted first, or null
    int n_rows, n_in;
};
void launch_teacher(const TeacherArgs &a, hipStream_t st);
struct ScaleDataArgs {
    const float *x, *t;        // scales: x [n][n_in], t [n][kNOut]
    float *in_scale, *out_scale;
    float *x_rw, *t_rw;        // scaling in place
    const float *in_scale_c, *out_scale_c;
    int64_t n;
    int n_in, n_lags;
};
void launch_data_scales(const ScaleDataArgs &a, hipStream_t st);
void launch_scale_data(const ScaleDataArgs &a, hipStream_t st);
void launch_xform(const XformArgs &a, hipStream_t st);
void launch_coef_sum(const CoefArgs &a, hipStream_t st);
void launch_synthesize(const SynthArgs &a, hipStream_t st);
void launch_project(const ProjArgs &a, bool fit, hipStream_t st);
void launch_budget(const BudgetArgs &a, hipStream_t st);
// Analytic multipole far-pair terms: the retarded multipole field of every
// far pair's source at a 4 x 4 x 4 node grid on the target box
// (xi in {-1, -1/3, 1/3, 1} per axis), fitted to the box basis by pinv
// ([kNBasis][64]), into pc ([n_pairs][kNOut]).
struct MultipoleArgs {
    const FarPair *pairs;
    const float *moments;  // [n_src][depth][kFeatStride]
    const float *pinv;
    float *pc;
    const int64_t *step;
    int step_off;          // evaluate at step *step + step_off
    int depth;
    int n_pairs;
    float inv_cdt, c, dt;
};
void launch_multipole(const MultipoleArgs &a, hipStream_t st);
void launch_correct(const CorrArgs &a, hipStream_t st);

// Judge by sample.  The plain field of a far pair (target s <- source n) at
// 64 sample points of the target at the last completed step l, by the direct
// sum of the sampled scheme over the source's real-space history:
//   P(r_k) = sum_k' h^3 / R [(1 - f) dS(r_k', l - m) + f dS(r_k', l - m - 1)],
//   R = |r_k - r_k'|, R / (c dt) = m + f, dS = S - S(0).
// Sample point p = 16 a_x + 4 a_y + a_z sits at grid index
// floor((a (N - 1) + 1) / 3) along each axis.
constexpr int kSamplePts = 64;
constexpr int kSampleGroup = 8;       // sample points per block
struct SampleJob {
    const float *hist;     // real-space ring of S_n [depth][4][npts_n]
    const float *s0;       // S_n(0) [4][npts_n]
    const int32_t *head;   // slot of S_n(l) in hist
    float *out;            // [64][4]
    double t0[3];          // (o_s - o_n) / h: the target origin in source grid units
    int32_t Ns[3], Nn[3];
    int32_t depth;
    int32_t pad_;
};
struct SampleArgs {
    const SampleJob *jobs;
    int n_jobs;
    double h;
    double inv_cdt;        // 1 / (c dt)
    float h3;
};
void launch_pair_sample(const SampleArgs &a, hipStream_t st);
// Per sampled pair: max over the points of |F - surrogate| and of |F| per
// component (resid[0..3], resid[4..7]); fail = active and any
// resid[mu] > budget[mu].
struct SampleJudgeJob {
    const float *F;        // [64][4]
    const float *pc;       // the pair's box coefficients [4][20]
    const float *budget;   // [4] of the target
    float *resid;          // [8]
    int32_t *fail;
    int32_t N[3];
    int32_t active;
};
struct SampleJudgeArgs {
    const SampleJudgeJob *jobs;
    int n_jobs;
};
void launch_sample_judge(const SampleJudgeArgs &a, hipStream_t st);
// count copies of the bytes at src (a multiple of 16) after one another at dst
void launch_broadcast(void *dst, const void *src, int64_t bytes, int32_t count, hipStream_t st);

// Network forward pass of the surrogate on a given stream (mlp.hip).
bool mlp_dims(rp_mlp m, int *n_in, int *n_out, int *max_batch);
void mlp_forward_on(rp_mlp m, const float *x, int batch, float *y, hipStream_t st);

}  // namespace rpot
