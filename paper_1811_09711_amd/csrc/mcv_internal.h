// Internal host-side view of one integration job's device buffers and the
// launch functions of every kernel of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcv_device.h"

namespace mcv {

// Number of FP64 values in one per-segment partial record:
// S1 (sum, compensation), S2 (sum, compensation), w_max, n_bad, SSW (stratified
// passes: the sum over boxes of the squared deviations of w from the box
// mean), 1 spare.
constexpr int kPartStride = 8;
// Per-channel statistics record: S1, S2, w_max, n_bad, E_c, W_c, V_c, N_c.
constexpr int kStatStride = 8;
// History record per iteration: E, sigma, N_tot, w_max, n_bad.
constexpr int kHistStride = 5;

struct JobDev {
  int d = 0, K = 0, n = 0, P = 0, prec = 0, npow2 = 1;
  int sT = 2;          // per-axis stride of the (edge, density) tables: n+1 rounded up to even
  int M = 512;         // cells of the per-axis hint maps (hint_cells_for_bins(n))
  int mshift = 18;     // the log map's shift (hint_cell_shift(M))
  int n_cu = 256;      // compute units of the device
  uint64_t seed = 0;
  double grid_power = 1.5, channel_power = 0.5;
  int64_t min_calls = 10;
  int max_iter = 0;
  int gmax = 0;  // most sample-pass work units the partial buffers are sized for
  int64_t n_points = 0;          // calls per pass when a job table supplies them
  int32_t adapt_passes = 1 << 30;  // grids and alpha adapt only after passes 1..adapt_passes-1
  int rng = 0;                   // 0 Philox4x32-10, 1 MRG32k3a streams
  int strat = 0;                 // 0 uniform r; s >= 2: pseudo-stratified, >= s calls per box
  // stratified layout of the allocation [K]: boxes per axis, calls per box;
  // box prefix [K+1] (the pass's work is split over boxes); the same two for
  // the trace allocation
  int64_t* nr = nullptr;
  int64_t* spb = nullptr;
  int64_t* bstart = nullptr;
  int64_t* t_nr = nullptr;
  int64_t* t_spb = nullptr;
  // MRG32k3a: jump entries [kMrgTables][kMrgEntry] (entry b < 64: 2^b steps,
  // entry 64 + b: 2^(76+b) steps; each the 3x3 matrix of component 1, then
  // of component 2), then the stream starts [K+1][6] (channel c: stream
  // 1024 seed + c; entry K: the unweighting stream 1024 seed + 1023)
  uint32_t* mrg = nullptr;
  int32_t* iter_dev = nullptr;   // completed passes = iteration tag of the next pass
  JobDev* self = nullptr;        // device copy of this record (a job table of one)

  // problem description
  int32_t* ckind = nullptr;
  double* cloc = nullptr;
  double* cwidth = nullptr;
  int32_t* pkind = nullptr;
  double* ploc = nullptr;
  double* pwidth = nullptr;
  double* pweight = nullptr;
  // derived constants
  DimMap<double>* cmap64 = nullptr;
  DimMap<float>* cmap32 = nullptr;
  double* cnorm64 = nullptr;
  float* cnorm32 = nullptr;
  PeakDim<double>* pmap64 = nullptr;
  PeakDim<float>* pmap32 = nullptr;
  double* pnorm64 = nullptr;
  float* pnorm32 = nullptr;
  // channel c's density shares its exponential with the peak of identical
  // shape, if any (twin_peak[c], -1 if none): f picks up twin_pn[c] * r_c
  int32_t* twin_peak = nullptr;  // [K]
  ChanType* ctype = nullptr;     // [K]: axis kinds of each channel
  double* twin_pn64 = nullptr;   // [K]
  float* twin_pn32 = nullptr;    // [K]
  int32_t* orphans = nullptr;    // [P]: peaks no channel shares
  int n_orphan = 0;
  // grids: FP64 master edges; FP32 copy; p-space edges and bin densities in
  // the pass precision
  double* edges = nullptr;   // [K][d][n+1]
  // Pair<T> [K][d][sT]: (x-space edge X_j, bin density 1/(n (X_{j+1}-X_j)));
  // X_0 = 0, X_n = 1, density 0 from j = n on
  void* xtab = nullptr;
  // Pair<T> [K][d][sT]: (p-space edge P_j = phi(X_j), same density);
  // P_0 = -inf, P_j = +inf from j = n on
  void* ptab = nullptr;
  // Cell<T> [K][d][M]: per hint cell, its start bin and its single edge (if
  // any) with the densities on either side
  void* ctab = nullptr;
  // T [K]: per channel, an upper bound of 2^s cnorm_c prod_k max_j dens_kj
  // (s = 25 in FP32, 54 in FP64), so that alpha_c gbound_c r_c(p) bounds
  // 2^s times the channel's term of g(p) before its lookups
  void* gbound = nullptr;
  // T [3][K]: per channel, (T)alpha_c gbound_c (the term bound's factor),
  // (T)alpha_c cnorm_c (the factor of the channel's term) and alpha_c cnorm_c
  // 2^s (1 + m) rounded up (the factor of the bound from looked-up densities),
  // in the pass precision, for the pass's alpha (written with the
  // allocation); t_aterm the same for the trace allocation's t_alpha
  void* aterm = nullptr;
  void* t_aterm = nullptr;
  // T [K][d][2]: the density-kernel constants of every axis in the pass
  // precision, contiguous per channel: (ga, gb) on a Gaussian axis, (m, h^2)
  // on a Breit-Wigner one, 0 on a flat one
  void* gab = nullptr;
  // float [K][d][2]: the hint-map constants (a, b) of every axis, contiguous
  // per channel: (hs, hb) on channels Gaussian on every axis, (ls, lb) on the
  // others (the map of x starts from a x + b)
  float* hab = nullptr;
  // int32 [K][2]: per channel, the exponent offsets (EA, EB) of the skip test
  // of an all-Gaussian channel from a partial exponent (written with the
  // allocation, as they depend on alpha): the channel's terms of f and g are
  // below half an ulp of f and g when the partial exponent sum is at least
  // max(EA - ex(f), EB - ex(g))
  int32_t* skx = nullptr;
  // channel weights and allocation
  double* alpha = nullptr;   // [K]
  int64_t* nc = nullptr;     // [K]
  int64_t* start = nullptr;  // [K+1]
  // scratch allocation for traces
  double* t_alpha = nullptr;
  int64_t* t_nc = nullptr;
  int64_t* t_start = nullptr;
  // pass accumulators
  double* part = nullptr;    // [(gmax+K)][kPartStride]
  double* hpart = nullptr;   // [(gmax+K)][d][n]
  double* hist = nullptr;    // [K][d][n]
  // channel equivalences: [n_eq][2 + 2d] = c, c', perm[d], mode[d] (device),
  // and the bin weights the grids are rebinned with when n_eq > 0
  const int32_t* eq = nullptr;
  int n_eq = 0;
  double* hist_eq = nullptr; // [K][d][n]
  double* chstats = nullptr; // [K][kStatStride]
  double* history = nullptr; // [max_iter][kHistStride]
};

// A set of jobs whose per-iteration kernels are launched together: every
// kernel reads its job from the device table `dev` (one job per grid row).
// A single integrator is a set of one.
struct JobSet {
  int n = 0;                    // jobs
  const JobDev* host = nullptr; // host copies [n]
  const JobDev* dev = nullptr;  // device table [n]
  int prec = 0;                 // precision of every job of the set
  int maxK = 0, maxKd = 0, maxd = 0;
  bool has_eq = false;          // some job has channel equivalences
  int64_t maxTab = 0, maxCells = 0;
  // sample pass work units: unit u belongs to job j when
  // unit_prefix[j] <= u < unit_prefix[j+1]; nullptr for a set of one job
  const int* unit_prefix = nullptr;
  int n_units = 0;
  int* counter = nullptr;       // device work-queue counters [8] (reset by allocate)
  const void* sargs = nullptr;  // device sample-kernel arguments [n] (job precision)
  int block = 1024;             // sample-kernel workgroup size
  int bound = 1024;             // its launch bound (kernel variant)
  int term_bound = 1;           // lookups guarded by the channel term bound (kernel variant)
  int lds = 0;                  // sample-kernel dynamic LDS (max over jobs)
  int grid = 0;                 // persistent sample-kernel workgroups
};

// Fills the maxima of a set from its host copies.
void set_extents(JobSet& js);

// The set of one job, whose device table is the job's own device record.
inline JobSet single_set(const JobDev& j) {
  JobSet js;
  js.n = 1;
  js.host = &j;
  js.dev = j.self;
  js.prec = j.prec;
  set_extents(js);
  return js;
}

// Set-up of one job: derived map constants, equidistant grids (FP32-snapped
// in the mixed mode), alpha = 1/K.
void launch_setup(const JobDev& j, hipStream_t s);
// Edge/density tables in the pass precision and the hint-cell records, from
// the master grids.
void launch_tables(const JobSet& js, hipStream_t s);
// Integer allocation N_c from alpha and the calls per pass (n_override > 0,
// or each job's n_points); alpha = N_c / N_tot.  to_trace: write the trace
// allocation (t_nc, t_start, t_alpha) instead and leave alpha alone.
// Resets the set's 8 work-queue counters.
void launch_allocate(const JobSet& js, int64_t n_override, bool to_trace, hipStream_t s);
// Stratified pass (jobs with strat > 0): G work units over the boxes;
// returns G, or -1.
int launch_sample_strat(const JobDev& j, int64_t n_points, hipStream_t s);
// LDS bytes of the single-job sample kernel's layout.
int sample_lds_bytes(const JobDev& j);
// The single-job sample pass (a set of one, G workgroups chosen here for
// n_points calls); returns G, or -1 if the kernel cannot get its LDS.
int launch_sample(const JobSet& js, int64_t n_points, hipStream_t s);
// Batched sample pass: argument record of one job for a workgroup size,
// written to args_host (sample_args_bytes(prec) bytes); returns the LDS bytes
// the job's layout uses.
size_t sample_args_bytes(int prec);
int sample_queue_layout(const JobDev& j, int block, void* args_host);
// Single-job sample kernels of each precision (n_points calls; returns the
// workgroups, or -1 if the kernel cannot get its LDS).
int launch_sample_f32(const JobDev& j, int64_t n_points, hipStream_t s);
int launch_sample_f64(const JobDev& j, int64_t n_points, hipStream_t s);
// Workgroups the single-job sample kernel of each precision runs a pass of
// n_points with (-1 if it cannot get its LDS).
int sample_grid_f32(const JobDev& j, int64_t n_points);
int sample_grid_f64(const JobDev& j, int64_t n_points);
// The sample kernel's trace instantiation: a pass over the trace allocation
// with G workgroups at iteration tag `tag`, writing f, g, w (double) of calls
// [first, first+count) to out[count][3]; nothing else of the state changes
// except the per-unit partial buffers.  Returns G, or -1.
int launch_sample_trace_f32(const JobDev& j, int G, uint32_t tag, int64_t first, int64_t count,
                            double* out, hipStream_t s);
int launch_sample_trace_f64(const JobDev& j, int G, uint32_t tag, int64_t first, int64_t count,
                            double* out, hipStream_t s);
// The same three for jobs drawing from MRG32k3a streams (mrg_f32.hip,
// mrg_f64.hip); the functions above hand such jobs to these.
int launch_sample_mrg_f32(const JobDev& j, int64_t n_points, hipStream_t s);
int launch_sample_mrg_f64(const JobDev& j, int64_t n_points, hipStream_t s);
int sample_grid_mrg_f32(const JobDev& j, int64_t n_points);
int sample_grid_mrg_f64(const JobDev& j, int64_t n_points);
int launch_sample_trace_mrg_f32(const JobDev& j, int G, uint32_t tag, int64_t first,
                                int64_t count, double* out, hipStream_t s);
int launch_sample_trace_mrg_f64(const JobDev& j, int G, uint32_t tag, int64_t first,
                                int64_t count, double* out, hipStream_t s);
// Batched sample kernels (queue.hip, one object per precision P (1: FP32),
// launch bound LB and term-bound option TB): the kernel for a set whose
// largest dimension is maxd.
#define MCV_QUEUE_NAME(P, LB, TB) MCV_QUEUE_NAME_(P, LB, TB)
#define MCV_QUEUE_NAME_(P, LB, TB) queue_kernel_##P##_##LB##_##TB
const void* MCV_QUEUE_NAME(1, 256, 1)(int maxd);
const void* MCV_QUEUE_NAME(1, 256, 0)(int maxd);
const void* MCV_QUEUE_NAME(1, 512, 1)(int maxd);
const void* MCV_QUEUE_NAME(1, 512, 0)(int maxd);
const void* MCV_QUEUE_NAME(1, 1024, 1)(int maxd);
const void* MCV_QUEUE_NAME(1, 1024, 0)(int maxd);
const void* MCV_QUEUE_NAME(0, 256, 1)(int maxd);
const void* MCV_QUEUE_NAME(0, 256, 0)(int maxd);
const void* MCV_QUEUE_NAME(0, 512, 1)(int maxd);
const void* MCV_QUEUE_NAME(0, 512, 0)(int maxd);
const void* MCV_QUEUE_NAME(0, 1024, 1)(int maxd);
const void* MCV_QUEUE_NAME(0, 1024, 0)(int maxd);
// Largest co-resident workgroups per CU of the batched kernel for a set.
int sample_queue_occupancy(const JobSet& js);
// One persistent launch over the set's work-unit queue.
int launch_sample_queue(const JobSet& js, hipStream_t s);
// Per-channel and total reduction of the pass into each job's history row
// *iter_dev, which is then incremented; G for a set of one.
void launch_finalize(const JobSet& js, int G, hipStream_t s);
void launch_refine_grid(const JobSet& js, hipStream_t s);
void launch_update_alpha(const JobSet& js, hipStream_t s);
// Trace of calls [first, first+count) with the trace allocation.
void launch_trace(const JobDev& j, uint32_t tag, int64_t first, int64_t count, int n_words,
                  uint32_t* words, int32_t* chan, int32_t* bins, double* p, double* fgw,
                  hipStream_t s);

// Unweighting: one batch of trials [q0, q0 + count).  Writes the accept flag
// (0/1) and the weight of every trial; points of accepted trials go to
// pts[count][d] (pass precision).
void launch_unweight_batch(const JobDev& j, uint64_t q0, int64_t count, const double* wmax,
                           uint8_t* accept, double* wts, void* pts, hipStream_t s);
// Ordered compaction of one batch: accepted points, in trial order, to
// out[k * out_stride + out_base + r] for the first `need` of them, and their
// weights' signs to signs[out_base + r] (+1 / -1; signs may be null).  res
// (device, 6 doubles): used, accepted in batch, last used index (-1: none),
// n_overweight among used, batch max |w|, spare.
// Bytes of the accept-flag buffer of an unweighting batch of `count` trials:
// the flags, then the compaction's per-tile scratch.
size_t compact_accept_bytes(int64_t count);
void launch_compact(const JobDev& j, const uint8_t* accept, const double* wts, const void* pts,
                    int64_t count, const double* wmax, int64_t need, void* out,
                    int64_t out_stride, int64_t out_base, int8_t* signs, double* res,
                    hipStream_t s);

}  // namespace mcv
