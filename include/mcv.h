/*
 * mcv: the per-iteration sample pass of the adaptive multi-channel VEGAS
 * integrator (VAMP) on one MI355X (gfx950).
 *
 * Method: S. Brass, W. Kilian, J. Reuter, "Parallel Adaptive Monte Carlo
 * Integration with the Event Generator WHIZARD", arXiv:1811.09711.
 *   Sec. 3.2   VEGAS step map, eq. g(x); grid adaptation, eq. 30 / eq. 31
 *   Sec. 3.4   multi-channel sampling, channel weights alpha, eq. 15
 *   Sec. 3.5   VAMP: per-channel grids, eq. gc(x), eq. vamp-master, eq. g(p);
 *              the organisation of an iteration and of event generation
 *   Sec. 2     unweighting efficiency, eq. efficiency
 *
 * Conventions for every entry point:
 *  - Return an mcv_status; never throw across the ABI.  mcv_last_error()
 *    returns a thread-local message for the last failing call of the thread.
 *  - "device" pointers are HIP device (or managed) addresses; "host" pointers
 *    are ordinary CPU memory.  Arrays are dense, row-major, in the shapes given.
 *  - An integrator owns all of its device memory (taken from the allocator
 *    installed with mcv_set_allocator, else hipMalloc).  Calls on one integrator
 *    are ordered on the HIP stream bound at creation (or by mcv_set_stream);
 *    entry points documented "asynchronous" only enqueue work.  One thread at
 *    a time may use an integrator.
 *  - MCV_E_INVALID: a bad argument (the call did nothing).  MCV_E_STATE: the
 *    call is not allowed in the current state (e.g. a result before any
 *    iteration).  MCV_E_NOMEM: device allocation failed.  MCV_E_DEVICE: a HIP
 *    runtime call failed (the integrator should be destroyed).
 */
#ifndef MCV_H
#define MCV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcv_integrator mcv_integrator;
typedef struct mcv_batch mcv_batch;
typedef struct mcv_server mcv_server;

typedef enum {
  MCV_OK = 0,
  MCV_E_INVALID = -1,
  MCV_E_NOMEM = -2,
  MCV_E_DEVICE = -3,
  MCV_E_STATE = -4,
  MCV_E_NUMERIC = -5
} mcv_status;

/* Arithmetic of the sample pass.  MCV_FP64: everything in FP64.
 * MCV_FP32_MIXED: draws, maps, integrand and densities in FP32; sums of w and
 * w^2, histograms, grid refinement and the alpha update in FP64 with
 * compensated summation; grids refined in FP64 and rounded to FP32. */
enum { MCV_FP64 = 0, MCV_FP32_MIXED = 1 };

/* 1-d factor of a peak or of a channel mapping (product over dimensions).
 * FLAT: 1 on [0,1] (identity map).  GAUSS: normal, loc = centre, width =
 * sigma; as a channel, the truncated-normal inverse CDF on [0,1].  BW:
 * Breit-Wigner, loc = centre, width = full width at half maximum; as a
 * channel, the truncated arctan (Cauchy inverse CDF) map on [0,1].  These
 * play the role of the channel mappings phi_c of Sec. 3.4. */
enum { MCV_FLAT = 0, MCV_GAUSS = 1, MCV_BW = 2 };

enum { MCV_REFINE_GRID = 1, MCV_REFINE_ALPHA = 2 };

/* Random numbers of the sample pass.  MCV_RNG_PHILOX: Philox4x32-10, words
 * keyed by (seed, call, iteration).  MCV_RNG_MRG32K3A: the paper's
 * generator (Sec. 4.4, eq. mrg32k3a and eq. rngstream) with its streams and
 * substreams: channel c uses stream 1024 seed + c (2^127 outputs apart; the
 * generator starts from 12345 in all six state words), the call with index i
 * among the channel's calls uses substream i of it (2^76 apart), and
 * iteration t starts 64 t outputs into the substream; unweighting trial q
 * uses substream q of stream 1024 seed + 1023.  An output z becomes the word
 * floor(z 2^32 / (m1 + 1)).  MRG32K3A needs n_channels <= 1023 and seed <
 * 2^54, and single integrators (batches and servers use Philox). */
enum { MCV_RNG_PHILOX = 0, MCV_RNG_MRG32K3A = 1 };

/* Sampling of r space in integration passes (Sec. 3.3).  strat = 0:
 * importance sampling, r uniform in the unit cube.  strat = s >= 2
 * (at most 2^20): pseudo-stratified sampling, the cube of each channel cut
 * into nr^dim equal boxes (nr the largest with s nr^dim <= N_c, at most
 * 2^20), every box getting the same number m = floor(N_c / nr^dim) >= s of
 * calls, uniform inside it, before the VEGAS map; a channel then takes
 * m nr^dim calls (so a pass may use fewer than n_points; Sec. 3.4 lets N and
 * alpha follow whole numbers of calls) and its error comes from the spread
 * of the weights inside the boxes.  Unweighting always samples
 * importance-wise.  Single integrators only. */

/* Problem descriptor (host memory; deep-copied by mcv_create_integrator).
 *   integrand f(p) = sum_i peak_weight[i] prod_k pdf(peak_kind[i][k], p_k)
 *     (untruncated, normalised 1-d densities; FLAT = 1)
 *   channel c maps x in (0,1)^dim to p by the 1-d maps chan_kind[c][k].
 * Limits: 1 <= dim <= 32, 1 <= n_bins <= 256, 1 <= n_channels <= 1024,
 * 1 <= n_peaks <= 1024; non-FLAT loc in [0,1] and width > 0, all finite.
 * Jointly, one channel's grid and its per-bin sums must fit the 160 KiB LDS
 * of a workgroup: dim * (2 s t + 8 n_bins) + 192 <= 163840 bytes, with
 * t = n_bins + 2 rounded up to even and s = 8 (FP64) or 4 (FP32 mixed); e.g.
 * FP64 with dim 32 allows n_bins <= 211.  Larger problems are refused with
 * MCV_E_INVALID.
 * grid_power: exponent of the bin measure of eq. 30 (> = 0, default 1.5).
 * channel_power: exponent beta of eq. 15 (>= 0, default 0.5).
 * min_calls: floor on the calls N_c of a channel (>= 1, default 10).
 * max_iterations: capacity of the per-iteration history (>= 1). */
typedef struct {
  int32_t dim, n_channels, n_bins, n_peaks, precision;
  const int32_t* peak_kind;   /* host [n_peaks][dim] */
  const double* peak_loc;     /* host [n_peaks][dim] */
  const double* peak_width;   /* host [n_peaks][dim] */
  const double* peak_weight;  /* host [n_peaks] */
  const int32_t* chan_kind;   /* host [n_channels][dim] */
  const double* chan_loc;     /* host [n_channels][dim] */
  const double* chan_width;   /* host [n_channels][dim] */
  uint64_t seed;              /* Philox key */
  double grid_power;
  double channel_power;
  int64_t min_calls;
  int32_t max_iterations;
  int32_t rng;                /* MCV_RNG_PHILOX or MCV_RNG_MRG32K3A */
  int32_t strat;              /* 0: importance sampling; s >= 2: pseudo-stratified */
} mcv_problem;

/* Device-memory allocator of the library.  alloc(bytes, ctx) returns a
 * device pointer (>= 256-byte aligned) or NULL on failure; release(ptr, ctx)
 * takes back a pointer that alloc returned.  Neither may call back into the
 * library. */
typedef void* (*mcv_alloc_fn)(size_t bytes, void* ctx);
typedef void (*mcv_free_fn)(void* ptr, void* ctx);

/* Install the allocator that every later device allocation of the library
 * uses (integrators, batches, servers, work buffers), so that a framework's
 * caching allocator owns the memory; both NULL restores hipMalloc / hipFree.
 * Process-wide.  A block is always returned to the allocator that made it,
 * after the device has finished the work queued so far (release is called
 * after a device synchronisation, as hipFree would wait).  ctx is passed
 * through unchanged.  MCV_E_INVALID if exactly one function is NULL.  Not
 * for use while another thread is inside the library. */
mcv_status mcv_set_allocator(mcv_alloc_fn alloc, mcv_free_fn release, void* ctx);

/* Combined result over iterations first_iter..last (Sec. 3.5, final
 * paragraph of the iteration organisation): inverse-variance weighted mean
 * of the per-iteration estimates, its error, chi^2 per degree of freedom. */
typedef struct {
  double integral, error, chi2_ndf;
  double w_max;          /* largest weight of the last iteration */
  int32_t n_iter_used;
  int64_t n_points;      /* points summed over the iterations used */
  int64_t n_bad;         /* non-finite weights, excluded from the sums */
} mcv_summary;

/* Create an integrator: equidistant grids for every channel (Sec. 3.2,
 * Sec. 3.5) and alpha_c = 1/K (Sec. 3.4).  hip_stream: a hipStream_t, or
 * NULL for the default stream.  *out receives the handle.  Synchronous. */
mcv_status mcv_create_integrator(const mcv_problem* problem, void* hip_stream,
                                 mcv_integrator** out);

/* Rebind the integrator to another HIP stream (NULL = default stream). */
mcv_status mcv_set_stream(mcv_integrator* h, void* hip_stream);

/* One integration pass of n_points calls (Sec. 3.5: generate a sample of N
 * events; Sec. 3.4: N_c = alpha_c N made integer, at least min_calls each, so
 * the pass may use slightly more than n_points; stratified problems round
 * each channel down to whole boxes).  For every call: random words (Philox,
 * keyed by (seed, iteration, call), or MRG32k3a streams), uniform r (in the
 * call's box when stratified), the VEGAS step map of its channel
 * (eq. g(x)), the channel map, the integrand, the multi-channel density
 * (eq. g(p)), the weight w = f/g, and the sums of w, w^2 and the per-bin sums
 * of w^2 of eq. 31.  Appends (E, sigma) to the history.  Asynchronous.
 * Errors: MCV_E_INVALID if n_points < n_channels * min_calls or > 2^50;
 * MCV_E_STATE if the history is full. */
mcv_status mcv_sample_iteration(mcv_integrator* h, int64_t n_points);

/* Adapt after a pass (Sec. 3.5): what = MCV_REFINE_GRID rebins every
 * channel's grid by eq. 30 / eq. 31; MCV_REFINE_ALPHA updates the channel
 * weights by eq. 15.  Both may be or-ed.  Asynchronous.
 * MCV_E_STATE before the first pass. */
mcv_status mcv_refine(mcv_integrator* h, uint32_t what);

/* Channel equivalences (Sec. 3.5: channels that share a structure pool the
 * bin weights their grids adapt to).  eq: host [n_eq][2 + 2*dim] int32 rows
 * (c, c', perm[dim], mode[dim]): along axis k, channel c takes channel c''s
 * per-bin sums of w^2 (eq. 31) of axis perm[k] (perm a permutation of the
 * axes) mapped by mode[k]: MCV_EQ_IDENTITY (bin j), MCV_EQ_INVERT (bin
 * n_bins-1-j), MCV_EQ_SYMMETRIC (the mean of both), MCV_EQ_INVARIANT (weight
 * 1 in every bin: the axis keeps its grid).  At every MCV_REFINE_GRID, a
 * channel named on the left of any row is rebinned with the sum of its rows
 * in list order (its own sums only through a row (c, c, identity, ...));
 * other channels with their own sums.  n_eq = 0 removes the list.  The list
 * is copied; it is configuration, not part of the saved state.  Synchronous.
 * MCV_E_INVALID for a channel out of range, axes that are not a permutation
 * or an unknown mode (the previous list stays). */
enum { MCV_EQ_IDENTITY = 0, MCV_EQ_INVERT = 1, MCV_EQ_SYMMETRIC = 2, MCV_EQ_INVARIANT = 3 };
mcv_status mcv_set_equivalences(mcv_integrator* h, int32_t n_eq, const int32_t* eq);

/* Combine iterations first_iter.. (0-based) into *out (host)./* Combine iterations first_iter.. (0-based) into *out (host).  Synchronises
 * the stream.  MCV_E_STATE if first_iter is not a completed iteration. */
mcv_status mcv_result(mcv_integrator* h, int32_t first_iter, mcv_summary* out);

/* Per-iteration history, host [n][5]: E, sigma, N_tot, w_max, n_bad, for the
 * min(cap, done) first iterations; *n_iter receives the number done.
 * Synchronises the stream. */
mcv_status mcv_get_history(mcv_integrator* h, double* host_out, int32_t cap, int32_t* n_iter);

/* Rejection unweighting with the current (fixed) grids and weights (Sec. 2,
 * eq. efficiency; Sec. 3.5, last paragraph): trials draw a channel with
 * probability N_c/N_tot, follow the same map and weight chain, and are kept
 * with probability |w| / w_max (weights are negative where the integrand is:
 * Sec. 3.1 allows integrands that are not positive semidefinite; see
 * mcv_unweight_signed for the signs).  w_max starts at the largest |w| of the
 * last pass and is raised, between batches of `batch` trials, to the largest
 * |w| seen.  Accepted points are written in trial order to d_events
 * (device, [dim][n_events]; double in MCV_FP64 mode, float in
 * MCV_FP32_MIXED mode; caller-owned).  host_stats (may be NULL) receives
 * trials, n_overweight, final w_max, efficiency.  Successive calls continue
 * the trial sequence.  Synchronous (the host reads the accepted count).
 * MCV_E_STATE before the first pass; MCV_E_INVALID for n_events < 1 or
 * batch < 1. */
mcv_status mcv_unweight(mcv_integrator* h, int64_t n_events, int64_t batch, void* d_events,
                        double* host_stats);

/* mcv_unweight for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same trials, decisions and events as mcv_unweight, with the batch's
 * work buffers (accept flags, weights, points, compaction records) taken
 * from a static per-device work area of 8 MiB instead of the allocator.  No
 * device memory is allocated or freed.  The area is shared by every call on
 * a device: calls that overlap on one device race (serialise them).
 * MCV_E_INVALID if a batch's buffers do not fit the area (about
 * 8 MiB / (9 + dim * s) trials with s = 8 (FP64) or 4 (FP32 mixed)) or if
 * the integrator's device is not the current device.  Synchronous. */
mcv_status mcv_unweight_noalloc(mcv_integrator* h, int64_t n_events, int64_t batch,
                                void* d_events, double* host_stats);

/* mcv_unweight for integrands of either sign (Sec. 3.1: an NLO integrand
 * need not be positive semidefinite): the same trials and events, and the
 * sign of each kept event's weight, +1 or -1, in trial order to d_signs
 * (device int8 [n_events], caller-owned; NULL: not written).  An event
 * sample with signs estimates the integrand through sum(sign) w_max-scaled
 * counts: I ~ (n_plus - n_minus) / n_trials * w_max. */
mcv_status mcv_unweight_signed(mcv_integrator* h, int64_t n_events, int64_t batch,
                               void* d_events, int8_t* d_signs, double* host_stats);

/* Host copies of the state: edges [K][dim][n_bins+1] (FP64 master grid),
 * alpha [K], alloc [K+1] = N_c of the last allocation and N_tot.  Any pointer
 * may be NULL.  Synchronises the stream. */
mcv_status mcv_get_state(mcv_integrator* h, double* edges, double* alpha, int64_t* alloc);

/* Overwrite grids and/or channel weights from host arrays (either may be
 * NULL); edges must be strictly increasing from 0 to 1 on every axis, alpha
 * non-negative with a positive sum (it is used as given, not normalised).
 * For tests that need both implementations in an identical state.
 * Synchronous. */
mcv_status mcv_set_state_for_test(mcv_integrator* h, const double* edges, const double* alpha);

/* Host copies of the last pass: per-bin sums of w^2, [K][dim][n_bins]; and
 * per channel [K][7]: S1, S2, w_max, n_bad, E_c, W_c, V_c.  Either may be
 * NULL.  Synchronises the stream. */
mcv_status mcv_get_pass_stats(mcv_integrator* h, double* hist, double* channel_stats);

/* Per-call trace of a pass of n_points at iteration index `iteration`, for
 * calls [first, first+count), without changing the state.  Host outputs:
 * words [count][n_words] (Philox words 0..n_words-1, n_words <= 4*ceil((dim+3)/4)),
 * chan [count], bins [count][K][dim] (own channel: the drawn bins; other
 * channels: the bin that holds the point's inverse map), p [count][dim],
 * fgw [count][3] = f, g, w.  Any output may be NULL.  Synchronous. */
mcv_status mcv_debug_trace(mcv_integrator* h, int64_t n_points, int64_t iteration, int64_t first,
                           int64_t count, int32_t n_words, uint32_t* words, int32_t* chan,
                           int32_t* bins, double* p, double* fgw);

/* Per-call values of a pass computed by the sample-pass kernel itself: the
 * instantiation mcv_sample_iteration launches (same lookups, the same
 * skipping of channel terms that cannot change g, the same grid of
 * workgroups), run over a pass of n_points at iteration index `iteration`
 * with the current grids and weights (allocated as mcv_debug_trace does),
 * writing for calls [first, first+count) host fgw [count][3] = f, g (eq.
 * g(p)) and w = f/g (eq. vamp-master) in the pass precision, widened to
 * double.  The state (grids, weights, history, sums) is unchanged.
 * Synchronous.  MCV_E_INVALID for a range beyond the pass or count > 2^24. */
mcv_status mcv_debug_sample_trace(mcv_integrator* h, int64_t n_points, int64_t iteration,
                                  int64_t first, int64_t count, double* fgw);

/* Serialise the adaptive state/* Serialise the adaptive state (grids, alpha, allocation, iteration count,
 * history, unweighting w_max and trial count) into host_buf.  With host_buf
 * NULL, *inout_size receives the size needed.  Synchronises the stream. */
mcv_status mcv_save_state(mcv_integrator* h, void* host_buf, size_t* inout_size);
/* Restore a state saved from an integrator with the same problem.
 * MCV_E_INVALID if the size or the problem shape does not match. */
mcv_status mcv_load_state(mcv_integrator* h, const void* host_buf, size_t size);

/* Duration of the sample kernel of pass `iteration` (0-based), measured with
 * HIP events recorded on the integrator's stream immediately around that
 * kernel's launch, and the number of workgroups it ran with (either pointer
 * may be NULL).  Synchronises on that pass's end event.  MCV_E_STATE if the
 * pass has not been issued (or was restored by mcv_load_state). */
mcv_status mcv_pass_timing(mcv_integrator* h, int32_t iteration, double* sample_ms,
                           int32_t* workgroups);

/* Release all device memory of the integrator (synchronises its stream). */
void mcv_destroy(mcv_integrator* h);

/* ------------------------------------------------------------------------
 * Batched integration: many independent jobs (each an integrator of its
 * own, Sec. 3.5) advance one iteration together.  Per iteration: one
 * allocation kernel, one persistent sample launch over a queue of work units
 * (a unit = a contiguous range of one job's calls) spanning every job, then
 * the per-job reduction, rebinning (eq. 30) and channel-weight update
 * (eq. 15) as batched kernels.  A job's pass is split into
 * ceil(n_points / unit_calls) units, so its results depend on its own
 * problem, calls and the tuning only -- not on the other jobs of the batch.
 * ------------------------------------------------------------------------ */

/* Launch shape of the batched sample kernel.  block: workgroup size
 * (multiple of 64, <= 1024; one call per lane and round).  unit_calls: calls
 * per work unit (>= block, <= 2^26).  launch_bound: the kernel variant
 * compiled for at most this many threads per workgroup, 256, 512 or 1024
 * (>= block; 0 = 1024): the 512 variant may use twice the registers per
 * lane, at half the resident waves; the 256 variant caps the registers for
 * at least 6 (FP32) or 4 (FP64) resident waves per SIMD.  term_bound: 1 = a
 * channel's grid lookups run only where its term of g(p) can change the sum
 * (a per-channel bound proves the others below half an ulp: the same
 * result, less work where channel densities fall off fast); 0 = wherever
 * the term is not exactly zero (no bound test: fewer registers, faster where
 * terms rarely fall that low).  Both give identical results. */
typedef struct {
  int32_t block, unit_calls, launch_bound, term_bound;
} mcv_tuning;

/* Create a batch of n_jobs (1..65535) problems, all of the same precision,
 * with n_points[i] calls per pass of job i (>= n_channels * min_calls,
 * <= 2^40).  tuning NULL: block 1024, unit_calls 16384, launch bound 1024, term bound 1.  Every
 * job starts as mcv_create_integrator would.  Synchronous.  MCV_E_INVALID
 * names the offending job in mcv_last_error(). */
mcv_status mcv_batch_create(const mcv_problem* problems, const int64_t* n_points, int32_t n_jobs,
                            const mcv_tuning* tuning, void* hip_stream, mcv_batch** out);

/* One iteration of every job: allocation, sample pass, reduction into each
 * job's history, then the adaptation `what` (MCV_REFINE_* flags, may be 0).
 * use_graph != 0: the sequence is captured once per `what` as a HIP graph
 * and replayed on the batch's stream; otherwise the kernels are launched
 * directly.  Asynchronous.  MCV_E_STATE if a job's history is full. */
mcv_status mcv_batch_iterate(mcv_batch* b, uint32_t what, int32_t use_graph);

/* History, combined result and state of job `job` (0-based), as
 * mcv_get_history / mcv_result / mcv_get_state.  Synchronise the stream. */
mcv_status mcv_batch_get_history(mcv_batch* b, int32_t job, double* host_out, int32_t cap,
                                 int32_t* n_iter);
mcv_status mcv_batch_result(mcv_batch* b, int32_t job, int32_t first_iter, mcv_summary* out);
mcv_status mcv_batch_get_state(mcv_batch* b, int32_t job, double* edges, double* alpha,
                               int64_t* alloc);

/* Work units per pass, persistent workgroups, LDS bytes per workgroup and
 * the tuning in use (any pointer may be NULL). */
mcv_status mcv_batch_info(mcv_batch* b, int32_t* n_units, int32_t* workgroups,
                          int32_t* lds_bytes, mcv_tuning* tuning);

/* Durations of iteration `iteration` (0-based, in issue order) from HIP
 * events on the batch's stream: the whole iteration, and (direct launches
 * only, else -1) the sample kernel.  Synchronises on that iteration. */
mcv_status mcv_batch_timing(mcv_batch* b, int32_t iteration, double* iteration_ms,
                            double* sample_ms);

/* Release the batch (synchronises its stream). */
void mcv_batch_destroy(mcv_batch* b);

/* Autotuner: times one sample pass of a scratch batch of these jobs for each
 * candidate launch shape and returns the fastest in *out (and its time in
 * *best_ms, may be NULL).  cache_path (may be NULL): a JSON file mapping a
 * workload key (precision, dimension bucket, channel bucket, bins, total
 * calls and jobs rounded to powers of two) to a tuning; a hit returns the
 * cached entry without timing, a miss adds the result.  Synchronous.
 * MCV_E_INVALID for a malformed cache. */
mcv_status mcv_autotune(const mcv_problem* problems, const int64_t* n_points, int32_t n_jobs,
                        void* hip_stream, const char* cache_path, mcv_tuning* out,
                        double* best_ms);

/* The autotuner's workload key of a batch, NUL-terminated into buf. */
mcv_status mcv_tuning_key(const mcv_problem* problems, const int64_t* n_points, int32_t n_jobs,
                          char* buf, size_t cap);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching step loop over integration requests.  A
 * request is a problem, the calls per pass, a number of iterations and a
 * number of unweighted events (Sec. 3.5: integrate, then generate events
 * with the adapted grids).  Requests are admitted in arrival order while the
 * device-memory budget and the slot limit allow.  Every mcv_server_step
 * advances each admitted job by one unit: jobs still integrating run one
 * iteration together (one batched pass, as mcv_batch_iterate; grids and
 * alpha adapt after every pass but the last); the others run one
 * unweighting batch of unweight_batch trials each (as one batch of
 * mcv_unweight, with the last pass's grids, allocation and w_max).  A job's results depend only on its own request and the server's
 * tuning and unweight_batch, not on the other jobs.  One thread at a time
 * may use a server.
 * ------------------------------------------------------------------------ */
enum { MCV_JOB_QUEUED = 0, MCV_JOB_INTEGRATING = 1, MCV_JOB_GENERATING = 2, MCV_JOB_DONE = 3 };

/* precision: of every request.  max_active: admitted jobs at most
 * (1..65535).  hbm_budget: device bytes that admitted jobs may hold (job
 * state, pass buffers, events); 0 = 90 % of the free device memory at
 * creation.  unweight_batch: trials per unweighting step (1..2^24).
 * tuning: batched sample kernel shape (block 0 = the default shape).
 * keep_events: keep each finished job's events for mcv_server_events. */
typedef struct {
  int32_t precision;
  int32_t max_active;
  int64_t hbm_budget;
  int64_t unweight_batch;
  mcv_tuning tuning;
  int32_t keep_events;
} mcv_server_config;

/* Per-request report.  Times are mcv_server_clock seconds: submit, admit and
 * completion (the end of the step in which the job's last event was
 * accepted).  result combines all iterations (valid once generating). */
typedef struct {
  int32_t state;
  int32_t iterations_done;
  mcv_summary result;
  int64_t n_events, trials, n_overweight;
  double w_max, efficiency;
  double submit_time, admit_time, finish_time;
  int64_t device_bytes;  /* device memory the job holds while admitted */
} mcv_job_report;

/* What one step did, and the server's occupancy after it. */
typedef struct {
  int32_t n_integrating, n_generating, n_admitted, n_finished, n_queued, n_active;
  int64_t bytes_in_use;
} mcv_step_info;

/* Create a server on hip_stream (a second, internal stream runs job
 * set-up).  Synchronous. */
mcv_status mcv_server_create(const mcv_server_config* cfg, void* hip_stream, mcv_server** out);

/* Seconds since the server was created (monotonic host clock). */
mcv_status mcv_server_clock(mcv_server* s, double* seconds);

/* Queue a request (the problem is deep-copied); *ticket identifies it.
 * n_iterations in [1, 1000]; n_points >= n_channels * min_calls; n_events
 * >= 0.  MCV_E_INVALID also if the request alone exceeds the budget.  Does
 * not touch the device. */
mcv_status mcv_server_submit(mcv_server* s, const mcv_problem* problem, int64_t n_points,
                             int32_t n_iterations, int64_t n_events, int64_t* ticket);

/* One step: admit, launch the step's kernels, admit more while they run,
 * wait for them, then retire finished jobs.  info may be NULL.  Synchronous. */
mcv_status mcv_server_step(mcv_server* s, mcv_step_info* info);

/* Tickets finished since the last call (at most cap into host tickets[]). */
mcv_status mcv_server_finished(mcv_server* s, int64_t* tickets, int32_t cap, int32_t* n);

/* Report of a ticket (queued, active or finished).  MCV_E_INVALID if unknown. */
mcv_status mcv_server_report(mcv_server* s, int64_t ticket, mcv_job_report* out);

/* Copy a finished job's events (kept with keep_events) to d_out (device,
 * [dim][n_events], the server's precision) and release them.  Synchronous.
 * MCV_E_STATE if the job is not finished or its events are gone. */
mcv_status mcv_server_events(mcv_server* s, int64_t ticket, void* d_out);

/* Release the server and every job's device memory (synchronises). */
void mcv_server_destroy(mcv_server* s);

/* Message of the last failing call on this thread ("" if none). */
const char* mcv_last_error(void);

/* Library version string. */
const char* mcv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MCV_H */
