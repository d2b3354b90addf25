/*
 * rpot -- retarded Lorenz-gauge potentials of many sub-domains on MI355X (gfx950).
 *
 * The library evaluates, at every time step l, the induced 4-potential
 * P = (v, Ax, Ay, Az) on every grid point of every sub-domain from the stored
 * history of the 4-vector sources S = (q rho, q Jx/c, q Jy/c, q Jz/c) of every
 * sub-domain (Eq. "4v potential" and its multi-domain sum, Sec. II), as the
 * discrete lag sum of Eq. "retardation space-time sampled lorentz four vector
 * potential" (Sec. III):
 *
 *   P(r_k, l dt) = sum_n [ P_n(r_k, 0) + sum_{k' in d_n} sum_{m} G_m[k,k'] dS(r_k', (l-m) dt) ]
 *
 * with the sampled Green's function G_m[k,k'] = h^3 T(m dt - R/c)/R of Eq.
 * "retardation space-time sampled green interpolation", T the triangle basis
 * T(x) = max(0, 1 - |x|/dt), dS = S - S(0), and the lag m restricted to the
 * window the sub-domain sizes and distances allow (Sec. IV, "Computational
 * Complexity Analysis").  The spatial sums are zero-padded FFT convolutions,
 * one per lag and (target, source) pair; the source spectra are kept in a ring
 * buffer in device memory (the retained history of Sec. IV).
 *
 * The component index is opaque to the library: every component of P is the
 * same functional of the same component of S.
 *
 * Conventions shared by every entry point:
 *  - Every entry point returns rp_status (RP_OK = 0) and never throws.  On
 *    failure rp_last_error(plan) describes the error (rp_last_error(NULL) for a
 *    failed rp_plan_domains).
 *  - Grids: sub-domain n has dims[n] = (Nx, Ny, Nz) points, spacing h shared by
 *    all sub-domains, and origins[n] = the position (bohr) of its point (0,0,0);
 *    point (i,j,k) sits at origin + h (i,j,k).  Arrays are [4][Nx][Ny][Nz],
 *    z fastest, component-major.
 *  - Sub-domains must not overlap: two sub-domains of one system closer than one
 *    grid cell (minimal point distance < h) give RP_ERR_GEOMETRY (Sec. III:
 *    the method assumes non-overlapping sub-domains).
 *  - Steps are 0, 1, 2, ... consecutively.  rp_push_sources(l) must precede
 *    rp_retarded_step(l); anything else gives RP_ERR_STATE.
 *  - All device work is enqueued asynchronously on the plan's HIP stream; the
 *    step path makes no host synchronisation.
 *  - Ownership: the caller owns every device buffer it passes (sources,
 *    outputs, the bound workspace) and keeps the workspace alive until
 *    rp_plan_destroy.  The library owns only its small host-side plan and never
 *    frees caller memory.  Sources are read before the enqueued work of the
 *    call completes; the caller may reuse them once that work has completed.
 *  - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef RPOT_H
#define RPOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rp_plan_s *rp_plan;

typedef enum {
    RP_OK = 0,
    RP_ERR_ARG = 1,         /* bad argument (null pointer, size, enum)            */
    RP_ERR_GEOMETRY = 2,    /* overlapping or touching sub-domains                */
    RP_ERR_NOMEM = 3,       /* workspace too small / host allocation failed       */
    RP_ERR_STATE = 4,       /* call out of order (step sequence, unbound plan)    */
    RP_ERR_DEVICE = 5,      /* a HIP call failed                                  */
    RP_ERR_UNSUPPORTED = 6  /* valid request outside what this build supports     */
} rp_status;

typedef enum {
    RP_FP64 = 0,            /* FP64 sources, FFTs, history and accumulation        */
    RP_FP32 = 1,            /* FP32 sources, FFTs, history and accumulation        */
    RP_FP32_RING_FP16 = 2,  /* FP32, history spectra stored as scaled FP16          */
    RP_FP32_RING_BF16 = 3,  /* FP32, history spectra stored as scaled BF16          */
    RP_FP32_RING_I16 = 4    /* FP32, history spectra stored as 16-bit integers with
                               one FP32 scale per (snapshot, tile of 256
                               frequencies, component): block floating point     */
} rp_precision;

/*
 * Reduced-precision history (the ring formats 2-4) keeps FP32 FFTs and FP32
 * accumulation; only the stored source spectra dS^(k) of the lag sum are
 * rounded, to 16 bits per real number (half the bytes of the FP32 ring).
 *   FP16/BF16: each value rounded to FP16 (11 significant bits) or BF16 (8)
 *     after division by one power-of-two scale per (snapshot, component).
 *   I16: the ring of every source is cut into tiles of 256 consecutive
 *     frequencies; per (snapshot, tile, component) the largest |Re|, |Im|
 *     M maps to 32767 and every value is rounded to the nearest integer
 *     multiple of M / 32767.  The rounding error of a value is at most
 *     M / 65534, an absolute bound shared by the tile, so the large,
 *     low-frequency values that carry the potential keep about 15
 *     significant bits, where FP16 keeps 11.
 */

/*
 * Plan the multi-domain evaluation (host only; makes no HIP call).
 *
 * n_dom      number of sub-domains (>= 1).
 * dims       [n_dom][3] grid points per axis (each >= 1).
 * origins    [n_dom][3] position of grid point (0,0,0), bohr.
 * system_id  [n_dom] or NULL.  Sub-domains with different ids are independent
 *            systems batched in one plan: no pair across systems is formed.
 *            NULL puts every sub-domain in one system.
 * h, dt, c   grid step, time step and speed of light (atomic units); c may be
 *            +INFINITY (instantaneous Coulomb coupling, the Hartree limit).
 * prec       arithmetic and history storage (rp_precision).
 * hip_stream hipStream_t on which every device call of this plan is enqueued;
 *            NULL is the null stream.
 *
 * For every ordered pair (s <- n) of one system the lag window is
 * [floor(Rmin/(c dt)), ceil(Rmax/(c dt))] with Rmin/Rmax the smallest/largest
 * distance between their grid points (Sec. IV: only lags allowed by the
 * sub-domain sizes and distances contribute); the ring of source n keeps
 * max_s ceil(Rmax(s,n)/(c dt)) + 1 past spectra.
 * The self cell needs h sqrt(3)/2 < c dt (RP_ERR_UNSUPPORTED otherwise).
 */
rp_status rp_plan_domains(rp_plan *out, int32_t n_dom, const int32_t *dims,
                          const double *origins, const int32_t *system_id,
                          double h, double dt, double c, rp_precision prec,
                          void *hip_stream);

/*
 * Evaluate the potentials of a subset of the sub-domains only (host only):
 * targets [n_targets] are domain indices; every sub-domain stays a source of
 * the targets of its system, and only the pairs (target <- source) are formed
 * (windows, Green spectra, history and lag sum).  A system's FFT pad then
 * covers its largest target plus its largest source, and with a split history
 * each source keeps only the windows of the pairs into the targets.  This is
 * how a workload too large for one device runs in pieces (waves of target
 * groups, each its own plan): the sum over sources of Eq. "multi domain ...
 * convolution" is per target, so the targets' results do not depend on which
 * other targets share the plan.  rp_retarded_step (and rp_capture_step) then
 * write only the targets' outputs; out[n] of a non-target may be NULL.
 * Before rp_workspace_bytes / rp_bind_workspace (RP_ERR_STATE after).
 * n_targets <= 0 or targets NULL: every sub-domain is a target (the default).
 * RP_ERR_ARG on an index out of range or a system left without a target;
 * RP_ERR_UNSUPPORTED together with the far-pair surrogate.  Re-plans pads,
 * ring depths, spectra, schedules, shape classes (their tuning is reset) and
 * the workspace size.
 */
rp_status rp_plan_targets(rp_plan plan, const int32_t *targets, int32_t n_targets);

/* Device workspace the plan needs, in bytes (host only). */
rp_status rp_workspace_bytes(rp_plan plan, size_t *bytes);

/*
 * Bind caller-allocated device memory of at least rp_workspace_bytes bytes
 * (256-byte aligned).  Uploads the plan's tables, zeroes the history and
 * resets the step sequence to 0.  May synchronise the stream.
 */
rp_status rp_bind_workspace(rp_plan plan, void *dev_ptr, size_t bytes);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: bind the plan
 * to a fixed array of RP_STATIC_WORKSPACE_BYTES (64 MiB) that the library holds
 * in device memory, once per device it runs on, until the process ends,
 * instead of to a caller-allocated workspace.  Otherwise the same as
 * rp_bind_workspace (uploads the tables, zeroes the history, resets the step
 * sequence; may synchronise the stream), on the current device.  Allocates
 * nothing: no hipMalloc, hipFree or other allocating call.
 * RP_ERR_NOMEM (nothing changed) if rp_workspace_bytes exceeds the array; the
 * FP64 plan of two 16^3 sub-domains needs 52 MiB.
 * The array is shared by every plan on its device and keeps the contents the
 * last plan left: the bind clears what must start at zero.  Binding a plan
 * takes the array over; from then on the calls that use the workspace of a
 * plan bound to it before on the same device fail with RP_ERR_STATE until that
 * plan is bound again (its step sequence then restarts).  Work of two plans on
 * the array that overlaps in time races.  rp_bind_workspace or
 * rp_plan_destroy releases the array.
 */
#define RP_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
rp_status rp_bind_workspace_static(rp_plan plan);

/*
 * Generate the sampled Green's-function spectra of every (target, source, lag)
 * triple in FP64 (Eq. "retardation space-time sampled green interpolation",
 * with h^3 as the quadrature weight and the exact self-cell integral for the
 * singular point, whose treatment the paper delegates to a smoothed Green's
 * function) and store them in the plan's precision.  Synchronises the stream.
 */
rp_status rp_set_green_kernels(rp_plan plan);

/*
 * Ingest the sources of step `step` for every sub-domain.
 * src[n] is a device pointer to [4][Nx][Ny][Nz] values, double for RP_FP64 and
 * float otherwise.  Step 0 is the ground state S(0): it is kept, and the static
 * potential P(0) (the ground-state term of Eq. "multi domain TDCDFT lorenz
 * space-time sampled simplify 1") is computed from it in FP64.  A step l >= 1
 * stores the spectrum of dS(l) = S(l) - S(0) in the history ring.
 */
rp_status rp_push_sources(rp_plan plan, int64_t step, const void *const *src);

/*
 * Evaluate P at step `step` on every sub-domain.  out[n] is a device pointer to
 * [4][Nx][Ny][Nz] values (same type as the sources) that receives
 * (v, Ax, Ay, Az) = P(0) + the lag sum over every source sub-domain.
 */
rp_status rp_retarded_step(rp_plan plan, int64_t step, void *const *out);

/*
 * Planned window of the ordered pair (target s <- source n): lags [m_lo, m_hi]
 * (-1, -1 if the pair is not formed), the FFT pad of their system, and the
 * depth of source n's spectral ring (the lags it holds from 0; with a split
 * history the later windows sit in rings of their own).  Any output pointer
 * may be NULL.
 */
rp_status rp_plan_info(rp_plan plan, int32_t s, int32_t n, int32_t *m_lo,
                       int32_t *m_hi, int32_t pad[3], int32_t *depth);

/* Counts and per-step byte figures of a plan (for reporting). */
typedef struct {
    int64_t n_triples;        /* (target, source, lag) triples per step            */
    int64_t n_spectra;        /* stored Green spectra (reversed pairs share one)   */
    int64_t n_entries;        /* (source, lag) ring reads per step                 */
    int64_t points;           /* target grid points (updates per step)             */
    double lagsum_bytes;      /* minimal HBM bytes of one lag-sum launch           */
    double ring_bytes;        /* history ring                                      */
    double spectra_bytes;     /* Green spectra                                     */
    double fft_bytes_fwd;     /* minimal bytes of the forward FFT passes per step  */
    double fft_bytes_inv;     /* minimal bytes of the inverse FFT passes per step  */
    double history_bytes;     /* real-space source rings of a split history, device
                                 part (with the host tier: its staging snapshots)  */
    int64_t split_rings;      /* extra spectral rings of a split history           */
    int64_t n_classes;        /* shape classes (same grid and FFT pad)             */
    int64_t fused_additions;  /* 1: with blocked lag-sum steps (RP_TUNE_LAGSUM_STEPS)
                                 a step's own lags m < i, which only the self pairs
                                 reach, are added by the inverse transform as it
                                 reads the accumulated spectrum (no separate pass
                                 over the accumulators); 0: a separate pass     */
} rp_stats;

rp_status rp_plan_stats(rp_plan plan, rp_stats *out);

/*
 * Profiling of the lag-sum launch (reporting only).  While enabled, every
 * rp_retarded_step brackets its lag-sum kernel with HIP events recorded on the
 * plan's stream.  rp_lagsum_time waits for the last recorded event, returns the
 * summed kernel time (ms) and the number of launches recorded since the last
 * query, and starts a new count.
 */
rp_status rp_profile_lagsum(rp_plan plan, int32_t enable);
rp_status rp_lagsum_time(rp_plan plan, double *total_ms, int64_t *launches);

/*
 * Tuning knobs (schedule choices that never change results beyond rounding
 * order; every value is valid for every plan).
 *   RP_TUNE_LAGSUM_UNROLL      lags whose loads one lag-sum thread issues
 *                              before accumulating: 1, 2 or 4.
 *   RP_TUNE_LAGSUM_PERSISTENT  1: one persistent lag-sum launch sized to the
 *                              device drains the work list (system group x
 *                              frequency tile, longest first) through a device
 *                              counter; 0: one block per work item.
 *   RP_TUNE_FFT_LDS            complex values an FFT line-pass block stages in
 *                              LDS (whole lines): 2048, 4096 or 6144 in FP32
 *                              (half as many in FP64); 0 = default (2048 for
 *                              FP32 plans, 4096 for FP64 plans).  Also per
 *                              shape class (below).
 *   RP_TUNE_LAGSUM_STEPS       steps of the lag sum per pass over the history:
 *                              1 (default), 2, 4, 8 or 16.  The potential of step
 *                              l + i depends on the sources of steps after l
 *                              only through its lags m < i (Eq. "retardation
 *                              space-time sampled lorentz four vector
 *                              potential": lag m reads the sources of step
 *                              l + i - m).  With kb steps per pass, steps are
 *                              grouped into blocks starting at steps 1, 1 + kb,
 *                              ...: the block's first step reads every
 *                              snapshot and Green spectrum of the windows once
 *                              and sums the lags m >= i of each of its kb steps
 *                              i = 0 .. kb-1; step i of the block adds its lags
 *                              m < i once its own sources are pushed.  Each
 *                              step returns exactly its own potential from the
 *                              sources pushed so far (a coupled loop may
 *                              compute step l + 1's sources from step l's
 *                              output); only the order of the sums changes.
 *                              The history is read about 1/kb as often.  FP32
 *                              plans only (RP_ERR_UNSUPPORTED for RP_FP64);
 *                              set before rp_bind_workspace (RP_ERR_STATE
 *                              after): it re-plans the workspace (kb
 *                              accumulators per target).  rp_capture_step then
 *                              records one graph per step of a block, and
 *                              rp_launch_step replays the one of its step;
 *                              rp_profile_lagsum times the passes of the
 *                              blocks' first steps; rp_plan_stats gives the
 *                              bytes of that pass as lagsum_bytes.
 *   RP_TUNE_LAGSUM_CACHED      blocked pass: 1 loads through the caches, 0
 *                              (default) non-temporal loads.  Its items (one
 *                              target and frequency tile each) of one tile read
 *                              the same source rows for different targets.
 *   RP_TUNE_LAGSUM_TILE_MAJOR  blocked pass work order: 1 the items of one
 *                              frequency tile next to each other, 0 (default)
 *                              the costliest target first.
 *   RP_TUNE_FFT_REG            1 (default): FP32 line passes of length 32, 48,
 *                              64, 96, 128, 192 or 256 run register-resident (each
 *                              line split over T threads, one LDS exchange);
 *                              0: every line pass stages whole lines in LDS
 *                              (RP_TUNE_FFT_LDS).  FP64 passes always stage.
 *   RP_TUNE_FFT_PLANE          1 (default): with RP_TUNE_FFT_REG, the FP32
 *                              forward z and y passes (and the inverse y and z
 *                              passes) of pads 32, 48, 64, 96 and 128 run as
 *                              one launch per x slice and component, the z
 *                              transform kept in LDS between them, where the
 *                              grid is at most half the pad in y and z and Nz
 *                              is a multiple of 4; 0: separate passes.
 * Setting a knob discards a captured step (rp_capture_step).
 */
enum { RP_TUNE_LAGSUM_UNROLL = 1, RP_TUNE_LAGSUM_PERSISTENT = 2, RP_TUNE_FFT_LDS = 4, RP_TUNE_LAGSUM_STEPS = 8,
       RP_TUNE_LAGSUM_CACHED = 16, RP_TUNE_LAGSUM_TILE_MAJOR = 32, RP_TUNE_FFT_REG = 64,
       RP_TUNE_FFT_PLANE = 128 };
rp_status rp_set_tuning(rp_plan plan, int32_t knob, int32_t value);
/*
 * Shape classes: sub-domains with the same grid and FFT pad share their
 * transform launches.  rp_class_info gives class cls (0 <= cls < n_classes of
 * rp_plan_stats): its grid, pad and number of sub-domains.  The line-pass tile
 * (RP_TUNE_FFT_LDS, the only per-class knob) may be chosen per class:
 * rp_set_class_tuning (0: the plan's value), rp_get_class_tuning (the value in
 * effect).  rp_set_tuning(RP_TUNE_FFT_LDS) resets every class to the plan's
 * value; rp_autotune chooses a tile per class.
 */
rp_status rp_class_info(rp_plan plan, int32_t cls, int32_t dims[3], int32_t pad[3], int32_t *n_domains);
rp_status rp_set_class_tuning(rp_plan plan, int32_t cls, int32_t knob, int32_t value);
rp_status rp_get_class_tuning(rp_plan plan, int32_t cls, int32_t knob, int32_t *value);
rp_status rp_get_tuning(rp_plan plan, int32_t knob, int32_t *value);

/*
 * Autotuner: times every lag-sum schedule (unroll x persistent; with blocked
 * steps the blocked pass, between blocks only) `iters` times
 * on the bound plan (after rp_set_green_kernels; only accumulator and FFT
 * scratch are written, the step sequence is untouched), keeps the fastest and
 * returns it with its mean kernel time; then times the inverse line passes at
 * every line-pass tile and keeps the fastest (read it with rp_get_tuning).  Synchronises the stream.  Output pointers may be
 * NULL.  Discards a captured step.
 */
rp_status rp_autotune(rp_plan plan, int32_t iters, int32_t *unroll, int32_t *persistent,
                      double *lagsum_ms);

/*
 * Graph-captured step (batched systems are one graph launch per step).
 * rp_capture_step records one whole step -- ingest of src, lag sum, inverse
 * and crop into out, advance of the step -- for these fixed device buffers
 * (same layout as rp_push_sources / rp_retarded_step) into a HIP graph owned
 * by the plan; it enqueues no work.  rp_launch_step(plan, step) replays it on
 * the plan's stream as step `step` (>= 1, in sequence; step 0 must have been
 * done by rp_push_sources / rp_retarded_step): the caller writes the step's
 * sources into the captured src buffers before the launch.  Replays and the
 * eager calls may be interleaved as long as the steps stay in sequence.
 */
rp_status rp_capture_step(rp_plan plan, const void *const *src, void *const *out);
rp_status rp_launch_step(rp_plan plan, int64_t step);

/*
 * Small fully connected network of the far-pair surrogate (training and
 * inference run in this library's kernels), two tanh layers and a linear skip:
 *   h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3 + x Ws,
 *   loss = sum (y - t)^2 / (2 batch n_out).
 * Parameters: one flat FP32 vector [W1 (n_in x H), b1 (H), W2 (H x H), b2 (H),
 * W3 (H x n_out), b3 (n_out), Ws (n_in x n_out)], row-major.  x, t, y are row-major
 * [batch][n_in] / [batch][n_out] FP32 device arrays; batch <= max_batch.
 * All calls are asynchronous on the stream given at creation; loss and grad
 * outputs are device pointers.  The caller initialises the parameters
 * (rp_mlp_set_params, which also restarts the optimiser).
 */
typedef struct rp_mlp_s *rp_mlp;
rp_status rp_mlp_create(rp_mlp *out, int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch,
                        void *hip_stream);
rp_status rp_mlp_workspace_bytes(rp_mlp mlp, size_t *bytes);
rp_status rp_mlp_bind(rp_mlp mlp, void *dev_ptr, size_t bytes);
rp_status rp_mlp_n_params(rp_mlp mlp, int64_t *n);
rp_status rp_mlp_set_params(rp_mlp mlp, const float *params);
rp_status rp_mlp_get_params(rp_mlp mlp, float *params);
rp_status rp_mlp_forward(rp_mlp mlp, const float *x, int32_t batch, float *y);
/* loss (1 float) and the gradient of every parameter (flat, as the parameters) */
rp_status rp_mlp_loss_grad(rp_mlp mlp, const float *x, const float *t, int32_t batch, float *loss, float *grad);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch; loss of the batch before the step */
rp_status rp_mlp_train_step(rp_mlp mlp, const float *x, const float *t, int32_t batch, float lr, float *loss);
/* Relative RMS of the network on n rows (device x [n][n_in] as the network
 * reads them, t [n][n_out] unscaled targets, out_scale [n_out] device):
 * sqrt(sum (y * out_scale - t)^2 / sum t^2), FP64 sums, in chunks of
 * max_batch.  Synchronises the stream; *rel is a host value. */
rp_status rp_mlp_relative_rms(rp_mlp mlp, const float *x, const float *t, int64_t n, const float *out_scale,
                              double *rel);
rp_status rp_mlp_destroy(rp_mlp mlp);
const char *rp_mlp_last_error(rp_mlp mlp);

/*
 * Split history (the retained history of Sec. IV, kept compact).  A source's
 * spectral ring holds every lag from 0 to the largest m_hi of its pairs, but
 * far pairs read only narrow windows of it.  With min_gap > 0 the windows of
 * a source's pairs are merged where they are less than min_gap lags apart;
 * every window after the first then gets a spectral ring of its own width
 * (and so does the first when it starts min_gap or more lags after lag 0, as
 * for a source that is not a target, rp_plan_targets: the source's own ring
 * then keeps lag 0 alone),
 * fed each step by transforming again the sources of `window start` steps
 * ago, which the source keeps in a real-space ring (source precision,
 * window start + 1 slots).  A source is split only where the spectra saved
 * exceed the real-space ring and the extra transform scratch.  Results are
 * identical to the unsplit plan (the same transforms of the same data).
 * Before rp_workspace_bytes / rp_bind_workspace (RP_ERR_STATE after);
 * min_gap <= 0 switches it off.  Not combined with the far-pair surrogate
 * (RP_ERR_UNSUPPORTED).  Re-plans ring depths, schedules and the workspace.
 */
rp_status rp_history_split(rp_plan plan, int32_t min_gap);

/*
 * Host tier of a split history (Sec. IV keeps the retained history on disk;
 * here the real-space rings move to pinned host memory and stream back one
 * snapshot per split ring and step).  With enable != 0 the real-space ring of
 * every split source lives in a caller-owned pinned host buffer
 * (rp_history_host_bytes; hipHostMalloc or a pinned torch tensor), and the
 * device keeps only staging snapshots: the newest sources of each split
 * source and, per split ring, the snapshot the next step transforms again.
 * The split rule then counts only the staging against the spectra saved.
 * Each step, after the forward transforms, a second stream of the plan
 * writes the newest sources to their host slot and fetches the next step's
 * snapshots (PCIe, about 2 x 4 N x sizeof(source) bytes per split source per
 * step); the copies overlap the lag sum and the inverse and are joined before
 * the step ends.  Slots follow the device-side step counter, so captured
 * steps work.  Results are bitwise identical to the device-resident tier.
 *   rp_history_host: before rp_workspace_bytes / rp_bind_workspace
 *     (RP_ERR_STATE after); re-plans like rp_history_split.
 *   rp_history_host_bytes: host bytes needed (0 when nothing is split).
 *   rp_bind_history_host: host_ptr 16-byte aligned pinned host memory of at
 *     least that many bytes (RP_ERR_ARG if it is not pinned, RP_ERR_NOMEM if
 *     too small); the caller owns it and keeps it alive while the plan runs.
 *     A no-op when rp_history_host_bytes is 0.  rp_push_sources and
 *     rp_capture_step fail with RP_ERR_STATE while a needed host buffer is
 *     unbound.
 */
rp_status rp_history_host(rp_plan plan, int32_t enable);
rp_status rp_history_host_bytes(rp_plan plan, size_t *bytes);
rp_status rp_bind_history_host(rp_plan plan, void *host_ptr, size_t bytes);

/*
 * Learned far-pair surrogate (an extension: the paper's closing section points
 * at a multipole approximation of the retarded potentials of far sub-domains
 * as a further speed-up; here the far coupling is learned from the plain
 * method's pair responses).
 *
 * A pair (target s <- source n, s != n, one system) is far when the distance
 * of the box centres |c_s - c_n| exceeds far_factor times the larger of the
 * two box diagonals.  Far pairs leave the plain lag sum.  Every source of a far
 * pair keeps a ring of 22 moments of dS = S - S(0) about its centre, weight h^3:
 *   q = sum dS_0, p_i = sum dS_0 x_i, Q_ij = sum dS_0 x_i x_j (xx yy zz xy xz yz),
 *   J_i = sum dS_{1+i}, K_ij = sum dS_{1+i} x_j.
 * The network input of a far pair at step l is built from H[j][k], the
 * moments of step l - m for the n_lags lags m = m_c - n_lags/2 + j
 * (m_c = round(|c_s - c_n| / (c dt)); zero for l - m <= 0) rotated into the
 * pair frame (rows e1 along c_s - c_n, e2, e3) and multiplied by in_scale[k],
 * and the pair's geometry g = 10 dbar / |c_s - c_n| (dbar the mean box
 * diagonal of the plan) and f = |c_s - c_n| / (c dt) - m_c: six blocks
 * H, g H, f H, g f H, g^2 H, f^2 H (each [n_lags][22]), then g and f:
 * n_in = 132 n_lags + 2.  (The far coupling is linear in the history with
 * weights that vary smoothly with g and f; the blocks let the network's
 * linear skip carry it.)  Its 80 outputs y,
 * times out_scale[80] / |c_s - c_n|, are the coefficients a[mu][b] of the pair's
 * potential component mu (frame components for A) in the tensor-Legendre basis
 * P_i P_j P_k (i + j + k <= 3, lexicographic (i, j, k)) of
 * u = R (r - c_s) / ell, ell = the target's largest half side.  The library maps
 * them to the target box basis (box coordinates in [-1, 1]) and adds the field
 * of the target's active far pairs to its output in rp_retarded_step (and in a
 * captured step).
 *
 * Audit sources keep the plain history of all their pairs (ring and spectra):
 * their far pairs are judged against the plain pair sum, may fall back to it,
 * and give the plain pair responses that train the network.
 *
 * rp_surrogate_configure  before rp_workspace_bytes / rp_bind_workspace
 *     (RP_ERR_STATE after).  far_factor <= 0 switches the surrogate off.
 *     Needs a finite c, a precision other than RP_FP64, 1 <= n_lags <= 1024, and
 *     at least 4 points per axis on every far-pair target (RP_ERR_UNSUPPORTED).
 *     audit: n_audit source domains (host array, may be NULL when n_audit = 0).
 *     Re-plans ring depths, spectra, schedules and the workspace size.
 * rp_surrogate_info   counts: far pairs, audited far pairs, n_in, n_out (80).
 * rp_surrogate_pairs  host arrays [n_far] (any may be NULL): target, source,
 *     centre distance, audited flag, fallen-back flag, in far-pair order.
 * rp_surrogate_attach the network used by every later step (NULL detaches:
 *     far pairs then contribute nothing).  in_scale [22], out_scale [80] are host
 *     arrays.  The network must have n_in inputs, 80 outputs and max_batch >= the
 *     far-pair count, stay alive while attached, and not run on another stream
 *     during a step.  Discards a captured step.
 * rp_surrogate_features  device [n_far][n_in] FP32: the network inputs of the
 *     last completed step.
 * rp_surrogate_pair_response  for the audited far pairs (in the order of
 *     rp_surrogate_pairs restricted to audited pairs) at the last completed step:
 *     the plain pair field F (the lag sum over that pair alone, inverse
 *     transformed and cropped), its least-squares coefficients a[mu][b] in the
 *     network's frame basis (device [n_aud][80]) and resid (device [n_aud][8]):
 *     max |F_mu - fit_mu| for mu < 4, then max |F_mu|.
 * rp_surrogate_judge  judges every active audited far pair of the last
 *     completed step: a pair whose error max_r |F_mu - surrogate_mu| exceeds
 *     tol * M_mu / (active far pairs of s), M_mu = max |out_mu| over every point
 *     of the target's system (the norm of the relative error per component),
 *     in any component falls
 *     back to the plain lag sum from the next step on, and its term in out (the
 *     outputs of that step, corrected in place) is replaced by F.  Returns the
 *     number of pairs that fell back and the largest error/budget ratio over the
 *     judged pairs.  With a re-admission factor (rp_surrogate_readmit) a
 *     fallen-back audited pair whose far-pair terms are within factor x
 *     tol * M_mu / (active far pairs of s + 1) in every component returns to
 *     them from the next step on (n_readmitted, may be NULL).  Synchronises the
 *     stream.  A call in which a pair falls back or returns discards a
 *     captured step (the lag-sum schedule changed); otherwise it stays valid.
 *     With rp_surrogate_sample the same call also judges far pairs of the
 *     other sources by sample (below).
 * rp_surrogate_readmit  the re-admission factor (>= 0; 0, the default: a pair
 *     that falls back stays with the plain lag sum).  A transient, such as the
 *     light-cone front of a source's switch-on crossing the target box, then
 *     costs only the judge intervals it spans.
 */
rp_status rp_surrogate_configure(rp_plan plan, double far_factor, int32_t n_lags, const int32_t *audit,
                                 int32_t n_audit);
rp_status rp_surrogate_info(rp_plan plan, int32_t *n_far, int32_t *n_audited, int32_t *n_in, int32_t *n_out);
rp_status rp_surrogate_pairs(rp_plan plan, int32_t *target, int32_t *source, double *dist, int32_t *audited,
                             int32_t *fallen_back);
rp_status rp_surrogate_attach(rp_plan plan, rp_mlp mlp, const float *in_scale, const float *out_scale);
/*
 * Analytic multipole far-pair terms instead of a network (enable != 0; it
 * detaches any network; 0 switches them off).  For every far pair the
 * retarded multipole field of the source is evaluated at a 4 x 4 x 4 node grid
 * of the target box (box coordinates -1, -1/3, 1/3, 1) and fitted to the box
 * basis.  With R from the source centre, u = R/|R|, the moments at the retarded
 * time (cubic interpolation in time, which also gives the time derivatives
 * f^(k)), O the charge's third moments and N_i the current's second moments:
 *   v   = q/R + u.p/R^2 + u.p^(1)/(cR) + (3 u.Q.u - tr Q)/(2R^3)
 *         + (3 u.Q^(1).u - tr Q^(1))/(2cR^2) + u.Q^(2).u/(2c^2 R)
 *         + (15 O_uuu - 9 u.trO)/(6R^4) + (15 O^(1)_uuu - 9 u.trO^(1))/(6cR^3)
 *         + (6 O^(2)_uuu - 3 u.trO^(2))/(6c^2 R^2) + O^(3)_uuu/(6c^3 R),
 *   A_i = J_i/R + (K u)_i/R^2 + (K^(1) u)_i/(cR) + (3 u.N_i.u - tr N_i)/(2R^3)
 *         + (3 u.N_i^(1).u - tr N_i^(1))/(2cR^2) + u.N_i^(2).u/(2c^2 R),
 * each moment and first derivative plus dt^2/12 times its next derivative
 * (the lag sum reads the sources on the chords between samples).
 * The multipole approximation of far sub-domains named in Sec. V; it needs no
 * training.  The judge and fallback work as with a network.  Discards a
 * captured step.
 * enable = 2 keeps the attached network (and a network attached later) and
 * adds its output to the multipole terms: the network then models what the
 * expansion leaves out, trained on the plain pair responses minus
 * rp_surrogate_multipole_response.
 */
rp_status rp_surrogate_multipole(rp_plan plan, int32_t enable);
/*
 * The multipole terms of the audited far pairs at the last completed step, as
 * frame coefficients a[mu][b] (device [n_aud][80], the rows and basis of
 * rp_surrogate_pair_response).  Works in every surrogate mode.
 */
rp_status rp_surrogate_multipole_response(rp_plan plan, float *coef);
rp_status rp_surrogate_features(rp_plan plan, float *x);
rp_status rp_surrogate_pair_response(rp_plan plan, float *coef, float *resid);
rp_status rp_surrogate_judge(rp_plan plan, void *const *out, double tol, int32_t *n_fallback, double *worst,
                             int32_t *n_readmitted);
rp_status rp_surrogate_readmit(rp_plan plan, double factor);

/*
 * Judging every far pair by sample.  Only the far pairs of audit sources keep
 * their spectral history; rp_surrogate_sample (after rp_surrogate_configure,
 * before the bind) lets rp_surrogate_judge check the others too:
 * - every far source keeps a real-space history of its sources S_n in FP32,
 *   (largest far lag m_hi of its pairs) + 2 snapshots deep, written by the
 *   ingest of every step (4 x 4 bytes per source point and snapshot: far
 *   sources ~1900 lags deep at 48^3 points hold 3.4 GB each);
 * - each judge call takes the next pairs_per_judge far pairs whose source is
 *   not an audit source (far-pair order, wrapping; 0: all of them) and
 *   evaluates their plain pair field at the last completed step l by the
 *   direct sum of Sec. III's sampled scheme, P(r_k) = sum_k' h^3 / R *
 *   [(1 - f) dS_n(r_k', l - m) + f dS_n(r_k', l - m - 1)] with
 *   R = |r_k - r_k'|, R / (c dt) = m + f (0 <= f < 1), dS = S - S(0) (zero
 *   before step 0): the same sum as the pair's lag sum over its window, here
 *   at 64 sample points of the target, the grid points (i_x, i_y, i_z) with
 *   i = floor((a (N - 1) + 1) / 3), a = 0 .. 3 along each axis (corners,
 *   edge and face thirds, the multipole path's nodes on the grid);
 * - a sampled pair whose largest difference to its surrogate terms at those
 *   points exceeds the budget of the audited pairs (the same tol * M_mu /
 *   active far pairs of s) falls back: it takes one of fallback_slots
 *   slots (each a spectral ring of its lag window, refilled from the real-space
 *   history, and its Green spectra, computed then), and from the next step on
 *   its lag sum runs plainly: the ingest transforms S_n(l - m_lo) again into
 *   the slot's ring and a second lag-sum launch adds the slot pairs into their
 *   targets.  The judge call's own outputs keep the pair's surrogate terms.
 *   With every slot in use the pair stays on its surrogate terms (counted as
 *   refused).  With a re-admission factor a sampled pair in a slot returns to
 *   its far-pair terms under the audited pairs' rule and frees its slot.
 * pairs_per_judge < 0 switches sampling off (the default).  fallback_slots in
 * 0 .. 4096.  RP_ERR_STATE after the bind or without a configured surrogate.
 *
 * rp_surrogate_sample_fields: the plain pair fields of far pairs
 *   far_pairs[0 .. n) (indices into rp_surrogate_pairs, host array) at their
 *   64 sample points at the last completed step, out device [n][64][4]
 *   (point p = 16 a_x + 4 a_y + a_z; component v, Ax, Ay, Az).  Any far
 *   pair, audited or not.  Synchronises the stream.
 * rp_surrogate_judge_stats: of the last rp_surrogate_judge call, the far pairs
 *   judged by sample and the fallbacks refused for want of a free slot; the
 *   slots in use now; the next pair of the rotation.  Any pointer may be NULL.
 */
rp_status rp_surrogate_sample(rp_plan plan, int32_t pairs_per_judge, int32_t fallback_slots);
rp_status rp_surrogate_sample_fields(rp_plan plan, const int32_t *far_pairs, int32_t n, float *out);
rp_status rp_surrogate_judge_stats(rp_plan plan, int32_t *sampled, int32_t *refused, int32_t *slots_used,
                                   int32_t *next_pair);

/*
 * Training data of the network, from the plain method (the teacher).
 * rp_surrogate_teacher: for the audited far pairs of the last completed step
 *   (rows in far-pair order, as rp_surrogate_pair_response): x [n_aud][n_in]
 *   the network inputs (as rp_surrogate_features gives them: times the
 *   attached network's in_scale, 1 without a network), t [n_aud][80] the
 *   targets: the least-squares frame coefficients of the plain pair field
 *   times the centre distance |c_s - c_n| (the network's output times
 *   out_scale reproduces them); residual != 0 subtracts the multipole terms
 *   (rp_surrogate_multipole_response) first.  Device arrays, asynchronous.
 * rp_surrogate_data_scales: scales of n training rows (device x [n][n_in],
 *   t [n][80], n_in = 132 n_lags + 2): in_scale[k] = 1 / RMS of moment k over
 *   the rows and lags of the unmodulated block H (the first 22 n_lags
 *   inputs), out_scale[c * 20 + b] = RMS of component c's 20 coefficients over
 *   the rows; an all-zero column gets 1.  FP64 sums in a fixed order.
 *   in_scale [22], out_scale [80]: device arrays.  Asynchronous on hip_stream.
 * rp_surrogate_scale_data: in place, every moment of the six input blocks
 *   times in_scale (the two geometry inputs unchanged) and every target over
 *   out_scale: the rows the network trains on.  x or t may be NULL (with its
 *   scale): only the other is scaled.
 * Both return RP_ERR_ARG on a null pointer, n < 1 or n_lags outside
 * 1 .. 1024, RP_ERR_DEVICE if a launch fails.
 */
rp_status rp_surrogate_teacher(rp_plan plan, float *x, float *t, int32_t residual);
rp_status rp_surrogate_data_scales(const float *x, const float *t, int64_t n, int32_t n_lags, float *in_scale,
                                   float *out_scale, void *hip_stream);
rp_status rp_surrogate_scale_data(float *x, float *t, int64_t n, int32_t n_lags, const float *in_scale,
                                  const float *out_scale, void *hip_stream);

/*
 * Model response of the sources: the steps either side of the potential
 * evaluation in the propagation loop of Fig. 4, with Lorentz oscillators in
 * place of the Kohn-Sham dynamics (the current of step l drives the vector
 * potential of step l + 1, Sec. II).  Oscillator k of domain n has a fixed
 * shape B [4][N_n] (component 0: charge per unit q; components 1-3: current / c
 * per unit dq/dt) and the amplitude q.  Sources S = (sum_k q_k B_k[0],
 * sum_k qdot_k B_k[1..3]).  One rp_osc_step, from the potentials P of step l:
 *   phi_k = h^3 sum_r B_k[0] v,   psi_k = h^3 sum_r sum_a B_k[1+a] A_a,
 *   F_k   = -phi_k - (psi_k - psi_k(l-1)) / dt + drive_k e_ext
 *           (the generalised force of the potentials on the shape; psi(l-1) =
 *           psi(l) on the first step after bind or rp_osc_set_state),
 *   qdot  = qdot + dt (kappa F - gamma qdot - omega^2 q),  q = q + dt qdot,
 * then writes S(l + 1) of the new state.  The state is FP64 on the device.
 *
 * rp_osc_create  n_osc [n_dom] oscillators per domain (0..256), params
 *     [total][4] = omega, gamma, kappa, drive (host, copied; finite, omega and
 *     gamma >= 0, omega dt < 2 for a stable step; else RP_ERR_ARG).  Takes the
 *     plan's grids, h, dt and stream; the plan may be destroyed afterwards.
 * rp_osc_bind  device workspace (256-byte aligned, >= rp_osc_workspace_bytes)
 *     and basis [n_dom] device pointers to [K_n][4][N_n] shapes in the plan's
 *     source type (FP64 for RP_FP64, else FP32; NULL where K_n = 0), which the
 *     caller keeps alive.  Sets q = qdot = 0.  Synchronises the stream.
 * rp_osc_set_state  host q, qdot [total].  Synchronises the stream.
 * rp_osc_sources  writes S of the current state into src [n_dom] ([4][N_n]).
 * rp_osc_step  pot [n_dom]: outputs of rp_retarded_step of step l; e_ext: the
 *     external field amplitude at l dt; src_next [n_dom]: S(l + 1).
 *     Asynchronous on the stream, no allocation.
 * rp_osc_state  host copies [total] of q, qdot and the last phi, psi (any may
 *     be NULL).  Synchronises the stream.
 */
typedef struct rp_osc_s *rp_osc;
rp_status rp_osc_create(rp_osc *out, rp_plan plan, const int32_t *n_osc, const double *params);
rp_status rp_osc_workspace_bytes(rp_osc osc, size_t *bytes);
rp_status rp_osc_bind(rp_osc osc, void *dev_ptr, size_t bytes, const void *const *basis);
rp_status rp_osc_set_state(rp_osc osc, const double *q, const double *qdot);
rp_status rp_osc_sources(rp_osc osc, void *const *src);
rp_status rp_osc_step(rp_osc osc, const void *const *pot, double e_ext, void *const *src_next);
rp_status rp_osc_state(rp_osc osc, double *q, double *qdot, double *phi, double *psi);
rp_status rp_osc_destroy(rp_osc osc);
const char *rp_osc_last_error(rp_osc osc);

/* HBM read-stream calibration (no plan): reads `bytes` of device memory at
 * `buf` once, 16-byte non-temporal loads as in the lag sum, on `grid` blocks
 * of 256 threads with `unroll` (1, 2, 4 or 8) loads in flight per thread.
 * Timing it gives the practical read bandwidth that the lag sum's roofline
 * fraction is set against (Sec. IV names the retarded potential and the
 * memory it needs as the main cost of a step).  buf: device, 16-byte aligned, bytes a
 * multiple of 16.  sink: device, grid * 256 uint32 (one folded word per
 * thread, written; the caller owns both).  Asynchronous on hip_stream (NULL:
 * the null stream); no allocation.  RP_ERR_ARG on a null pointer, a bad size,
 * alignment, grid (1 .. 2^20) or unroll; RP_ERR_DEVICE if the launch fails. */
rp_status rp_read_stream(const void *buf, size_t bytes, uint32_t *sink, int32_t grid, int32_t unroll,
                         void *hip_stream);

/* Release the host plan (the workspace stays the caller's). */
rp_status rp_plan_destroy(rp_plan plan);

/* Description of the last error of `plan` (or of the last failed plan creation
 * when plan is NULL).  The string lives until the next call on the plan. */
const char *rp_last_error(rp_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* RPOT_H */
