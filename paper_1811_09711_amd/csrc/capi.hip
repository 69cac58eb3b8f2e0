// Host runtime and C ABI of the multi-channel VEGAS sample pass (declared in
// include/mcv.h).  Owns each integrator's device buffers, sequences the
// kernels of an iteration on the bound HIP stream, and combines iterations.
//
// Brass, Kilian, Reuter, arXiv:1811.09711, Sec. 3.5: an iteration generates a
// sample of N events, then adapts the channel weights (eq. 15) and/or the
// grids (eq. 30); final iterations are combined into the best estimate.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "mcv.h"
#include "mcv_host.h"

using mcv::fail;
using mcv::JobDev;

namespace {

constexpr uint64_t kMagic = 0x3176637353435643ull;  // state-blob tag

}  // namespace

struct mcv_integrator {
  int device = 0;
  hipStream_t stream = nullptr;
  JobDev j;
  void* block = nullptr;     // the job's device block
  int n_iter = 0;            // completed passes (mirrors *j.iter_dev)
  int64_t last_n = 0;        // n_points of the last pass
  bool alloc_valid = false;  // alpha equals N_c / N_tot of the allocation in j.nc
  double wmax_unw = -1.0;    // running w_max of unweighting (-1: not started)
  int64_t trials_done = 0;
  std::vector<void*> bufs;   // unweighting work buffers
  // unweighting work buffers (grown on demand)
  int64_t u_cap = 0;
  uint8_t* u_accept = nullptr;
  double* u_wts = nullptr;
  void* u_pts = nullptr;
  double* u_misc = nullptr;  // [0] = w_max of the batch, [8..13] = compaction result
  // channel equivalences (device copy of the list)
  int32_t* eq_dev = nullptr;
  size_t eq_cap = 0;
  // events around each pass's sample kernel, and its workgroup count
  std::vector<hipEvent_t> ev0, ev1;
  std::vector<int> pass_G;

  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = mcv::dev_alloc(&q, count * sizeof(T));
    if (e == hipSuccess) {
      bufs.push_back(q);
      *p = reinterpret_cast<T*>(q);
    }
    return e;
  }
};

static void release(mcv_integrator* h) {
  for (void* q : h->bufs) mcv::dev_free(q);
  h->bufs.clear();
  mcv::dev_free(h->block);
  h->block = nullptr;
}

namespace {

// Unweighting work buffers of one batch: accept flags (with the
// compaction's per-tile scratch behind them), weights, points, and a small
// record (w_max of the batch at [0], the compaction result at [8..13]).
struct UnweightBufs {
  uint8_t* accept;
  double* wts;
  void* pts;
  double* misc;
};

mcv_status unweight_check(mcv_integrator* h, int64_t n_events, int64_t batch, void* d_events) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  if (n_events < 1 || batch < 1 || batch > (1 << 24) || !d_events)
    return fail(MCV_E_INVALID, "need n_events >= 1, 1 <= batch <= 2^24 and an output buffer");
  if (h->n_iter == 0) return fail(MCV_E_STATE, "unweighting before the first pass");
  return MCV_OK;
}

// Batches of trials until n_events are accepted (the body of mcv_unweight
// and mcv_unweight_signed; the buffers hold at least `batch` trials).
mcv_status unweight_run(mcv_integrator* h, int64_t n_events, int64_t batch, void* d_events,
                        int8_t* d_signs, double* host_stats, const UnweightBufs& B) {
  JobDev& j = h->j;
  hipStream_t s = h->stream;
  if (!h->alloc_valid) {
    mcv::launch_allocate(mcv::single_set(j), h->last_n, false, s);
    h->alloc_valid = true;
  }
  if (h->wmax_unw < 0.0) {
    double rec[mcv::kHistStride];
    MCV_HIP(hipMemcpyAsync(rec, j.history + (size_t)(h->n_iter - 1) * mcv::kHistStride,
                           sizeof rec, hipMemcpyDeviceToHost, s));
    MCV_HIP(hipStreamSynchronize(s));
    h->wmax_unw = rec[3];
  }
  double wmax_b = h->wmax_unw;
  int64_t got = 0, n_over = 0;
  const int64_t trials_start = h->trials_done;
  int64_t last_used = trials_start - 1;
  uint64_t q0 = (uint64_t)h->trials_done;
  while (got < n_events) {
    MCV_HIP(hipMemcpyAsync(B.misc, &wmax_b, sizeof(double), hipMemcpyHostToDevice, s));
    mcv::launch_unweight_batch(j, q0, batch, B.misc, B.accept, B.wts, B.pts, s);
    mcv::launch_compact(j, B.accept, B.wts, B.pts, batch, B.misc, n_events - got, d_events,
                        n_events, got, d_signs, B.misc + 8, s);
    MCV_HIP(hipGetLastError());
    double res[6];
    MCV_HIP(hipMemcpyAsync(res, B.misc + 8, sizeof res, hipMemcpyDeviceToHost, s));
    MCV_HIP(hipStreamSynchronize(s));
    const int64_t used = (int64_t)res[0];
    if (used > 0) last_used = (int64_t)q0 + (int64_t)res[2];
    got += used;
    n_over += (int64_t)res[3];
    if (res[4] > wmax_b) wmax_b = res[4];
    q0 += (uint64_t)batch;
  }
  h->trials_done = (int64_t)q0;
  h->wmax_unw = wmax_b;
  const int64_t trials = last_used + 1 - trials_start;
  if (host_stats) {
    host_stats[0] = (double)trials;
    host_stats[1] = (double)n_over;
    host_stats[2] = wmax_b;
    host_stats[3] = trials > 0 ? (double)n_events / (double)trials : 0.0;
  }
  return MCV_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Bytes of one batch's work buffers carved from the static work area.
size_t static_unweight_bytes(const JobDev& j, int64_t batch) {
  const size_t tsz = j.prec == 1 ? 4 : 8;
  return align256(mcv::compact_accept_bytes(batch)) + align256((size_t)batch * 8) +
         align256((size_t)batch * j.d * tsz) + 16 * sizeof(double);
}

UnweightBufs carve_unweight(const JobDev& j, int64_t batch, char* base) {
  const size_t tsz = j.prec == 1 ? 4 : 8;
  UnweightBufs b;
  size_t off = 0;
  b.accept = reinterpret_cast<uint8_t*>(base + off);
  off += align256(mcv::compact_accept_bytes(batch));
  b.wts = reinterpret_cast<double*>(base + off);
  off += align256((size_t)batch * 8);
  b.pts = base + off;
  off += align256((size_t)batch * j.d * tsz);
  b.misc = reinterpret_cast<double*>(base + off);
  return b;
}

}  // namespace

extern "C" {

const char* mcv_last_error(void) { return mcv::last_error(); }

const char* mcv_version(void) { return "mcv 0.3 (gfx950)"; }

mcv_status mcv_set_allocator(mcv_alloc_fn alloc, mcv_free_fn release, void* ctx) {
  return mcv::set_allocator(alloc, release, ctx);
}

mcv_status mcv_create_integrator(const mcv_problem* p, void* hip_stream, mcv_integrator** out) {
  if (!out) return fail(MCV_E_INVALID, "out is NULL");
  *out = nullptr;
  mcv_status st = mcv::validate_problem(p);
  if (st != MCV_OK) return st;
  int device = 0, n_cu = 1;
  st = mcv::device_cus(&device, &n_cu);
  if (st != MCV_OK) return st;
  mcv_integrator* h = new mcv_integrator();
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  // partial buffers for up to 8 times the resident workgroups of the sample
  // pass (kOversub x at most 8 per CU), halved while they would pass 256 MB
  int gmax = n_cu * 64;
  const size_t unit_bytes = ((size_t)p->dim * p->n_bins + mcv::kPartStride) * sizeof(double);
  while (gmax > n_cu * 8 && (size_t)gmax * unit_bytes > ((size_t)256 << 20)) gmax /= 2;
  st = mcv::job_create(p, gmax, 0, n_cu, h->stream, &h->j, &h->block);
  if (st != MCV_OK) {
    delete h;
    return st;
  }
  char* area = nullptr;  // set-up of mcv_unweight_noalloc's work area on this device
  st = mcv::static_work_area(device, &area);
  if (st != MCV_OK) {
    mcv_destroy(h);
    return st;
  }

  *out = h;
  return MCV_OK;
}

mcv_status mcv_set_stream(mcv_integrator* h, void* hip_stream) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return MCV_OK;
}

mcv_status mcv_sample_iteration(mcv_integrator* h, int64_t n_points) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  JobDev& j = h->j;
  if (n_points < (int64_t)j.K * j.min_calls)
    return fail(MCV_E_INVALID, "n_points must be at least n_channels * min_calls");
  if (n_points > ((int64_t)1 << 50)) return fail(MCV_E_INVALID, "n_points too large");
  if (h->n_iter >= j.max_iter) return fail(MCV_E_STATE, "history is full (max_iterations)");
  const size_t it = (size_t)h->n_iter;
  if (h->ev0.size() <= it) {
    h->ev0.resize(it + 1, nullptr);
    h->ev1.resize(it + 1, nullptr);
    h->pass_G.resize(it + 1, 0);
  }
  if (!h->ev0[it]) MCV_HIP(hipEventCreate(&h->ev0[it]));
  if (!h->ev1[it]) MCV_HIP(hipEventCreate(&h->ev1[it]));
  const mcv::JobSet one = mcv::single_set(j);
  mcv::launch_allocate(one, n_points, false, h->stream);
  MCV_HIP(hipEventRecord(h->ev0[it], h->stream));
  const int G = j.strat > 0 ? mcv::launch_sample_strat(j, n_points, h->stream)
                            : mcv::launch_sample(one, n_points, h->stream);
  if (G < 1) return fail(MCV_E_DEVICE, "the sample kernel could not get its LDS");
  MCV_HIP(hipEventRecord(h->ev1[it], h->stream));
  h->pass_G[it] = G;
  mcv::launch_finalize(one, G, h->stream);
  MCV_HIP(hipGetLastError());
  h->n_iter += 1;
  h->last_n = n_points;
  h->alloc_valid = true;
  return MCV_OK;
}

mcv_status mcv_refine(mcv_integrator* h, uint32_t what) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  if (what & ~(uint32_t)(MCV_REFINE_GRID | MCV_REFINE_ALPHA))
    return fail(MCV_E_INVALID, "unknown refine flags");
  if (h->n_iter == 0) return fail(MCV_E_STATE, "refine before the first pass");
  const mcv::JobSet one = mcv::single_set(h->j);
  if (what & MCV_REFINE_GRID) {
    mcv::launch_refine_grid(one, h->stream);
    mcv::launch_tables(one, h->stream);
  }
  if (what & MCV_REFINE_ALPHA) {
    mcv::launch_update_alpha(one, h->stream);
    h->alloc_valid = false;
  }
  MCV_HIP(hipGetLastError());
  return MCV_OK;
}

mcv_status mcv_set_equivalences(mcv_integrator* h, int32_t n_eq, const int32_t* eq) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  JobDev& j = h->j;
  const int d = j.d, rec = 2 + 2 * d;
  if (n_eq < 0 || n_eq > (1 << 20) || (n_eq > 0 && !eq))
    return fail(MCV_E_INVALID, "need 0 <= n_eq <= 2^20 and a list");
  for (int e = 0; e < n_eq; ++e) {
    const int32_t* r = eq + (size_t)e * rec;
    if (r[0] < 0 || r[0] >= j.K || r[1] < 0 || r[1] >= j.K)
      return fail(MCV_E_INVALID, "equivalence " + std::to_string(e) + ": no such channel");
    uint32_t seen = 0;
    for (int k = 0; k < d; ++k) {
      const int32_t a = r[2 + k], m = r[2 + d + k];
      if (a < 0 || a >= d || ((seen >> a) & 1u))
        return fail(MCV_E_INVALID,
                    "equivalence " + std::to_string(e) + ": the axes must be a permutation");
      seen |= 1u << a;
      if (m < MCV_EQ_IDENTITY || m > MCV_EQ_INVARIANT)
        return fail(MCV_E_INVALID, "equivalence " + std::to_string(e) + ": unknown mode");
    }
  }
  hipStream_t s = h->stream;
  MCV_HIP(hipStreamSynchronize(s));  // earlier refinements may still read the old list
  if (n_eq > 0) {
    const size_t need = (size_t)n_eq * rec;
    if (need > h->eq_cap) {
      int32_t* t = nullptr;
      if (h->alloc(&t, need) != hipSuccess) return fail(MCV_E_NOMEM, "equivalence table");
      h->eq_dev = t;
      h->eq_cap = need;
    }
    if (!j.hist_eq && h->alloc(&j.hist_eq, (size_t)j.K * d * j.n) != hipSuccess)
      return fail(MCV_E_NOMEM, "equivalence weights");
    MCV_HIP(hipMemcpyAsync(h->eq_dev, eq, need * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  j.eq = h->eq_dev;
  j.n_eq = n_eq;
  MCV_HIP(hipMemcpyAsync(j.self, &j, sizeof(JobDev), hipMemcpyHostToDevice, s));
  MCV_HIP(hipStreamSynchronize(s));
  return MCV_OK;
}

mcv_status mcv_get_history(mcv_integrator* h, double* host_out, int32_t cap, int32_t* n_iter) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  if (n_iter) *n_iter = h->n_iter;
  const int m = cap < h->n_iter ? cap : h->n_iter;
  if (host_out && m > 0) {
    MCV_HIP(hipMemcpyAsync(host_out, h->j.history, (size_t)m * mcv::kHistStride * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
  }
  MCV_HIP(hipStreamSynchronize(h->stream));
  return MCV_OK;
}

mcv_status mcv_result(mcv_integrator* h, int32_t first, mcv_summary* out) {
  if (!h || !out) return fail(MCV_E_INVALID, "NULL argument");
  if (h->n_iter == 0 || first < 0 || first >= h->n_iter)
    return fail(MCV_E_STATE, "first_iter is not a completed iteration");
  std::vector<double> hist((size_t)h->n_iter * mcv::kHistStride);
  int32_t n = 0;
  mcv_status st = mcv_get_history(h, hist.data(), h->n_iter, &n);
  if (st != MCV_OK) return st;
  mcv::combine_history(hist.data(), n, first, out);
  return MCV_OK;
}

mcv_status mcv_get_state(mcv_integrator* h, double* edges, double* alpha, int64_t* alloc) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  JobDev& j = h->j;
  hipStream_t s = h->stream;
  if (edges)
    MCV_HIP(hipMemcpyAsync(edges, j.edges, (size_t)j.K * j.d * (j.n + 1) * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  if (alpha) MCV_HIP(hipMemcpyAsync(alpha, j.alpha, j.K * sizeof(double), hipMemcpyDeviceToHost, s));
  if (alloc) {
    MCV_HIP(hipMemcpyAsync(alloc, j.nc, j.K * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MCV_HIP(hipMemcpyAsync(alloc + j.K, j.start + j.K, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  }
  MCV_HIP(hipStreamSynchronize(s));
  return MCV_OK;
}

mcv_status mcv_set_state_for_test(mcv_integrator* h, const double* edges, const double* alpha) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  JobDev& j = h->j;
  if (edges) {
    for (int ax = 0; ax < j.K * j.d; ++ax) {
      const double* e = edges + (size_t)ax * (j.n + 1);
      if (e[0] != 0.0 || e[j.n] != 1.0) return fail(MCV_E_INVALID, "edges must run from 0 to 1");
      for (int i = 0; i < j.n; ++i)
        if (!(e[i + 1] > e[i])) return fail(MCV_E_INVALID, "edges must be strictly increasing");
    }
  }
  if (alpha) {
    double sum = 0.0;
    for (int c = 0; c < j.K; ++c) {
      if (!(alpha[c] >= 0.0) || !isfinite(alpha[c]))
        return fail(MCV_E_INVALID, "alpha must be finite and >= 0");
      sum += alpha[c];
    }
    if (!(sum > 0.0)) return fail(MCV_E_INVALID, "alpha must have a positive sum");
  }
  hipStream_t s = h->stream;
  if (edges) {
    MCV_HIP(hipMemcpyAsync(j.edges, edges, (size_t)j.K * j.d * (j.n + 1) * sizeof(double),
                           hipMemcpyHostToDevice, s));
    mcv::launch_tables(mcv::single_set(j), s);
  }
  if (alpha) {
    MCV_HIP(hipMemcpyAsync(j.alpha, alpha, j.K * sizeof(double), hipMemcpyHostToDevice, s));
    h->alloc_valid = false;
  }
  MCV_HIP(hipGetLastError());
  MCV_HIP(hipStreamSynchronize(s));
  return MCV_OK;
}

mcv_status mcv_get_pass_stats(mcv_integrator* h, double* hist, double* channel_stats) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  JobDev& j = h->j;
  hipStream_t s = h->stream;
  if (hist)
    MCV_HIP(hipMemcpyAsync(hist, j.hist, (size_t)j.K * j.d * j.n * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  if (channel_stats) {
    std::vector<double> st((size_t)j.K * mcv::kStatStride);
    MCV_HIP(hipMemcpyAsync(st.data(), j.chstats, st.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    MCV_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < j.K; ++c)
      for (int q = 0; q < 7; ++q) channel_stats[c * 7 + q] = st[(size_t)c * mcv::kStatStride + q];
  }
  MCV_HIP(hipStreamSynchronize(s));
  return MCV_OK;
}

mcv_status mcv_debug_trace(mcv_integrator* h, int64_t n_points, int64_t iteration, int64_t first,
                           int64_t count, int32_t n_words, uint32_t* words, int32_t* chan,
                           int32_t* bins, double* p, double* fgw) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  JobDev& j = h->j;
  if (n_points < (int64_t)j.K * j.min_calls) return fail(MCV_E_INVALID, "n_points too small");
  if (count < 1 || first < 0 || count > (1 << 24)) return fail(MCV_E_INVALID, "bad count/first");
  if (iteration < 0 || iteration > 0xFFFFFFFFll) return fail(MCV_E_INVALID, "bad iteration");
  if (n_words < 0 || n_words > 36) return fail(MCV_E_INVALID, "n_words must be in [0, 36]");
  hipStream_t s = h->stream;
  mcv::launch_allocate(mcv::single_set(j), n_points, true, s);
  int64_t ntot = 0;
  MCV_HIP(hipMemcpyAsync(&ntot, j.t_start + j.K, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MCV_HIP(hipStreamSynchronize(s));
  if (first + count > ntot) return fail(MCV_E_INVALID, "trace range beyond the pass");
  const size_t nw = n_words > 0 ? n_words : 1;
  uint32_t* dw = nullptr;
  int32_t *dc = nullptr, *db = nullptr;
  double *dp = nullptr, *df = nullptr;
  hipError_t e = mcv::dev_alloc((void**)&dw, count * nw * sizeof(uint32_t));
  if (e == hipSuccess) e = mcv::dev_alloc((void**)&dc, count * sizeof(int32_t));
  if (e == hipSuccess) e = mcv::dev_alloc((void**)&db, count * j.K * j.d * sizeof(int32_t));
  if (e == hipSuccess) e = mcv::dev_alloc((void**)&dp, count * j.d * sizeof(double));
  if (e == hipSuccess) e = mcv::dev_alloc((void**)&df, count * 3 * sizeof(double));
  if (e == hipSuccess) {
    mcv::launch_trace(j, (uint32_t)iteration, first, count, n_words, dw, dc, db, dp, df, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess && words && n_words > 0)
    e = hipMemcpyAsync(words, dw, count * n_words * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && chan) e = hipMemcpyAsync(chan, dc, count * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && bins)
    e = hipMemcpyAsync(bins, db, count * j.K * j.d * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && p) e = hipMemcpyAsync(p, dp, count * j.d * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && fgw) e = hipMemcpyAsync(fgw, df, count * 3 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  mcv::dev_free(dw);
  mcv::dev_free(dc);
  mcv::dev_free(db);
  mcv::dev_free(dp);
  mcv::dev_free(df);
  if (e != hipSuccess) return fail(MCV_E_DEVICE, std::string("trace: ") + hipGetErrorString(e));
  return MCV_OK;
}

mcv_status mcv_debug_sample_trace(mcv_integrator* h, int64_t n_points, int64_t iteration,
                                  int64_t first, int64_t count, double* fgw) {
  if (!h || !fgw) return fail(MCV_E_INVALID, "NULL argument");
  JobDev& j = h->j;
  if (n_points < (int64_t)j.K * j.min_calls) return fail(MCV_E_INVALID, "n_points too small");
  if (n_points > ((int64_t)1 << 50)) return fail(MCV_E_INVALID, "n_points too large");
  if (count < 1 || first < 0 || count > (1 << 24)) return fail(MCV_E_INVALID, "bad count/first");
  if (iteration < 0 || iteration > 0xFFFFFFFFll) return fail(MCV_E_INVALID, "bad iteration");
  if (j.strat > 0)
    return fail(MCV_E_INVALID, "stratified passes: use mcv_debug_trace for per-call values");
  hipStream_t s = h->stream;
  mcv::launch_allocate(mcv::single_set(j), n_points, true, s);
  int64_t ntot = 0;
  MCV_HIP(hipMemcpyAsync(&ntot, j.t_start + j.K, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MCV_HIP(hipStreamSynchronize(s));
  if (first + count > ntot) return fail(MCV_E_INVALID, "trace range beyond the pass");
  const int G = j.prec == 1 ? mcv::sample_grid_f32(j, n_points) : mcv::sample_grid_f64(j, n_points);
  if (G < 1) return fail(MCV_E_DEVICE, "the sample kernel could not get its LDS");
  if (G > j.gmax) return fail(MCV_E_DEVICE, "more work units than partial buffers");
  double* out = nullptr;
  hipError_t e = mcv::dev_alloc((void**)&out, (size_t)count * 3 * sizeof(double));
  if (e == hipSuccess) {
    const int r = j.prec == 1
                      ? mcv::launch_sample_trace_f32(j, G, (uint32_t)iteration, first, count, out, s)
                      : mcv::launch_sample_trace_f64(j, G, (uint32_t)iteration, first, count, out, s);
    e = r < 1 ? hipErrorLaunchFailure : hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(fgw, out, (size_t)count * 3 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  mcv::dev_free(out);
  if (e != hipSuccess) return fail(MCV_E_DEVICE, std::string("sample trace: ") + hipGetErrorString(e));
  return MCV_OK;
}

mcv_status mcv_unweight(mcv_integrator* h, int64_t n_events, int64_t batch, void* d_events,
                        double* host_stats) {
  return mcv_unweight_signed(h, n_events, batch, d_events, nullptr, host_stats);
}

mcv_status mcv_unweight_signed(mcv_integrator* h, int64_t n_events, int64_t batch,
                               void* d_events, int8_t* d_signs, double* host_stats) {
  mcv_status st = unweight_check(h, n_events, batch, d_events);
  if (st != MCV_OK) return st;
  JobDev& j = h->j;
  const size_t tsz = j.prec == 1 ? 4 : 8;
  if (h->u_cap < batch) {
    // grown buffers are kept for the integrator's lifetime
    if (h->alloc(&h->u_accept, mcv::compact_accept_bytes(batch)) != hipSuccess ||
        h->alloc(&h->u_wts, batch) != hipSuccess)
      return fail(MCV_E_NOMEM, "unweighting buffers");
    char* pts = nullptr;
    if (h->alloc(&pts, batch * j.d * tsz) != hipSuccess) return fail(MCV_E_NOMEM, "unweighting buffers");
    h->u_pts = pts;
    if (!h->u_misc && h->alloc(&h->u_misc, 16) != hipSuccess)
      return fail(MCV_E_NOMEM, "unweighting buffers");
    h->u_cap = batch;
  }
  return unweight_run(h, n_events, batch, d_events, d_signs, host_stats,
                      UnweightBufs{h->u_accept, h->u_wts, h->u_pts, h->u_misc});
}

mcv_status mcv_unweight_noalloc(mcv_integrator* h, int64_t n_events, int64_t batch,
                                void* d_events, double* host_stats) {
  mcv_status st = unweight_check(h, n_events, batch, d_events);
  if (st != MCV_OK) return st;
  const size_t need = static_unweight_bytes(h->j, batch);
  if (need > mcv::static_work_bytes())
    return fail(MCV_E_INVALID, "batch of " + std::to_string(batch) + " trials needs " +
                                   std::to_string(need) + " bytes of work area; " +
                                   std::to_string(mcv::static_work_bytes()) + " available");
  int dev = -1;
  MCV_HIP(hipGetDevice(&dev));
  if (dev != h->device)
    return fail(MCV_E_INVALID, "the integrator's device must be the current device");
  char* base = nullptr;
  st = mcv::static_work_area(dev, &base);
  if (st != MCV_OK) return st;
  return unweight_run(h, n_events, batch, d_events, nullptr, host_stats,
                      carve_unweight(h->j, batch, base));
}

mcv_status mcv_save_state(mcv_integrator* h, void* host_buf, size_t* inout_size) {
  if (!h || !inout_size) return fail(MCV_E_INVALID, "NULL argument");
  JobDev& j = h->j;
  const size_t ne = (size_t)j.K * j.d * (j.n + 1), nh = (size_t)j.K * j.d * j.n;
  const size_t hdr = 16;  // u64 words
  const size_t need = hdr * 8 + (ne + j.K + (size_t)j.max_iter * mcv::kHistStride + nh +
                                 (size_t)j.K * mcv::kStatStride) * 8 + (2 * (size_t)j.K + 1) * 8;
  if (!host_buf) {
    *inout_size = need;
    return MCV_OK;
  }
  if (*inout_size < need) return fail(MCV_E_INVALID, "buffer too small");
  char* b = static_cast<char*>(host_buf);
  uint64_t H[hdr] = {kMagic, 1, (uint64_t)j.d, (uint64_t)j.K, (uint64_t)j.n, (uint64_t)j.prec,
                     (uint64_t)h->n_iter, (uint64_t)j.max_iter, (uint64_t)h->last_n,
                     (uint64_t)h->alloc_valid, (uint64_t)h->trials_done, 0, 0, 0, 0, 0};
  memcpy(&H[11], &h->wmax_unw, 8);
  memcpy(b, H, sizeof H);
  char* q = b + sizeof H;
  hipStream_t s = h->stream;
  MCV_HIP(hipMemcpyAsync(q, j.edges, ne * 8, hipMemcpyDeviceToHost, s));
  q += ne * 8;
  MCV_HIP(hipMemcpyAsync(q, j.alpha, j.K * 8, hipMemcpyDeviceToHost, s));
  q += j.K * 8;
  MCV_HIP(hipMemcpyAsync(q, j.history, (size_t)j.max_iter * mcv::kHistStride * 8,
                         hipMemcpyDeviceToHost, s));
  q += (size_t)j.max_iter * mcv::kHistStride * 8;
  MCV_HIP(hipMemcpyAsync(q, j.hist, nh * 8, hipMemcpyDeviceToHost, s));
  q += nh * 8;
  MCV_HIP(hipMemcpyAsync(q, j.chstats, (size_t)j.K * mcv::kStatStride * 8, hipMemcpyDeviceToHost, s));
  q += (size_t)j.K * mcv::kStatStride * 8;
  MCV_HIP(hipMemcpyAsync(q, j.nc, j.K * 8, hipMemcpyDeviceToHost, s));
  q += j.K * 8;
  MCV_HIP(hipMemcpyAsync(q, j.start, (j.K + 1) * 8, hipMemcpyDeviceToHost, s));
  MCV_HIP(hipStreamSynchronize(s));
  *inout_size = need;
  return MCV_OK;
}

mcv_status mcv_load_state(mcv_integrator* h, const void* host_buf, size_t size) {
  if (!h || !host_buf) return fail(MCV_E_INVALID, "NULL argument");
  JobDev& j = h->j;
  size_t need = 0;
  mcv_save_state(h, nullptr, &need);
  if (size != need) return fail(MCV_E_INVALID, "state size does not match this problem");
  const char* b = static_cast<const char*>(host_buf);
  uint64_t H[16];
  memcpy(H, b, sizeof H);
  if (H[0] != kMagic || H[1] != 1 || H[2] != (uint64_t)j.d || H[3] != (uint64_t)j.K ||
      H[4] != (uint64_t)j.n || H[5] != (uint64_t)j.prec || H[7] != (uint64_t)j.max_iter)
    return fail(MCV_E_INVALID, "state was saved from a different problem shape");
  const size_t ne = (size_t)j.K * j.d * (j.n + 1), nh = (size_t)j.K * j.d * j.n;
  const char* q = b + sizeof H;
  hipStream_t s = h->stream;
  MCV_HIP(hipMemcpyAsync(j.edges, q, ne * 8, hipMemcpyHostToDevice, s));
  q += ne * 8;
  MCV_HIP(hipMemcpyAsync(j.alpha, q, j.K * 8, hipMemcpyHostToDevice, s));
  q += j.K * 8;
  MCV_HIP(hipMemcpyAsync(j.history, q, (size_t)j.max_iter * mcv::kHistStride * 8,
                         hipMemcpyHostToDevice, s));
  q += (size_t)j.max_iter * mcv::kHistStride * 8;
  MCV_HIP(hipMemcpyAsync(j.hist, q, nh * 8, hipMemcpyHostToDevice, s));
  q += nh * 8;
  MCV_HIP(hipMemcpyAsync(j.chstats, q, (size_t)j.K * mcv::kStatStride * 8, hipMemcpyHostToDevice, s));
  q += (size_t)j.K * mcv::kStatStride * 8;
  MCV_HIP(hipMemcpyAsync(j.nc, q, j.K * 8, hipMemcpyHostToDevice, s));
  q += j.K * 8;
  MCV_HIP(hipMemcpyAsync(j.start, q, (j.K + 1) * 8, hipMemcpyHostToDevice, s));
  const int32_t it = (int32_t)H[6];
  MCV_HIP(hipMemcpyAsync(j.iter_dev, &it, sizeof it, hipMemcpyHostToDevice, s));
  mcv::launch_tables(mcv::single_set(j), s);
  MCV_HIP(hipGetLastError());
  MCV_HIP(hipStreamSynchronize(s));
  h->n_iter = (int)H[6];
  for (size_t i = 0; i < h->pass_G.size(); ++i) h->pass_G[i] = 0;  // no timed passes
  h->last_n = (int64_t)H[8];
  h->alloc_valid = H[9] != 0;
  h->trials_done = (int64_t)H[10];
  memcpy(&h->wmax_unw, &H[11], 8);
  return MCV_OK;
}

mcv_status mcv_pass_timing(mcv_integrator* h, int32_t iteration, double* sample_ms,
                           int32_t* workgroups) {
  if (!h) return fail(MCV_E_INVALID, "integrator is NULL");
  if (iteration < 0 || iteration >= h->n_iter || (size_t)iteration >= h->ev1.size() ||
      !h->ev1[iteration] || h->pass_G[iteration] == 0)
    return fail(MCV_E_STATE, "no timed pass with that index");
  MCV_HIP(hipEventSynchronize(h->ev1[iteration]));
  float ms = 0.0f;
  MCV_HIP(hipEventElapsedTime(&ms, h->ev0[iteration], h->ev1[iteration]));
  if (sample_ms) *sample_ms = ms;
  if (workgroups) *workgroups = h->pass_G[iteration];
  return MCV_OK;
}

void mcv_destroy(mcv_integrator* h) {
  if (!h) return;
  hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev0)
    if (e) hipEventDestroy(e);
  for (hipEvent_t e : h->ev1)
    if (e) hipEventDestroy(e);
  release(h);
  delete h;
}

}  // extern "C"
