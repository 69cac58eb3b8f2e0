// Serving: a continuous-batching step loop over integration requests.
//
// Every step, each admitted job advances by one unit of work: jobs still
// integrating run one adaptation iteration together (one batched pass over
// every integrating job, as in batch.hip); jobs past their last iteration
// run one unweighting batch each with their final grids.  Grids, channel
// weights, histories and the running w_max of every job stay in device
// memory for the job's lifetime.  Requests are admitted in arrival order
// while the device-memory budget and the slot limit allow; admission (job
// set-up) runs on a second stream while the step's kernels run.
//
// Brass, Kilian, Reuter, arXiv:1811.09711, Sec. 3.5: a job is an
// integration (iterations of sampling and adaptation, eq. 30 and eq. 15)
// followed by event generation with the adapted grids (Sec. 2, eq.
// efficiency: rejection against the largest weight seen).
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "mcv.h"
#include "mcv_batch.h"
#include "mcv_host.h"

using mcv::fail;
using mcv::JobDev;

namespace {

struct Request {
  int64_t ticket = 0;
  mcv_problem p{};
  std::vector<int32_t> pk, ck;
  std::vector<double> pl, pw, pwt, cl, cw;
  int64_t n_points = 0, n_events = 0;
  int32_t n_iter = 0;
  size_t bytes = 0;
  double submit = 0.0;
};

struct Served {
  int job = -1;  // index into the engine's job list
  int dim = 0;
  mcv_job_report rep{};
  int64_t n_points = 0, n_events = 0;
  int32_t n_iter = 0;
  size_t bytes = 0;
  void* events = nullptr;  // device [dim][n_events]
  // unweighting state (as mcv_unweight; the allocation of the last pass
  // stays valid since alpha does not adapt after it)
  double wmax = -1.0;
  int64_t got = 0, n_over = 0, last_used = -1;
  uint64_t q0 = 0;
  int gen_slot = -1;  // row of this step's result arrays
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct mcv_server {
  mcv::Engine e;
  mcv_server_config cfg{};
  std::chrono::steady_clock::time_point t0;
  hipStream_t admit_stream = nullptr;
  size_t budget = 0, in_use = 0;
  int64_t next_ticket = 0;
  std::deque<Request> queue;
  std::map<int64_t, Served> active;  // ticket order = arrival order
  std::map<int64_t, Served> done;
  std::vector<int64_t> finished_unread;
  bool set_dirty = true;
  // shared unweighting work area (one job's batch at a time, stream order)
  uint8_t* u_accept = nullptr;
  double* u_wts = nullptr;
  void* u_pts = nullptr;
  // per-step generation arrays: w_max in, compaction results out
  double* wm_dev = nullptr;
  double* res_dev = nullptr;
  double* wm_host = nullptr;   // pinned
  double* res_host = nullptr;  // pinned
  int gen_cap = 0;

  ~mcv_server() {
    if (e.stream) hipStreamSynchronize(e.stream);
    for (auto* m : {&active, &done})
      for (auto& kv : *m)
        mcv::dev_free(kv.second.events);
    for (auto& jb : e.jobs)
      mcv::dev_free(jb.block);
    e.jobs.clear();
    mcv::dev_free(u_accept);
    mcv::dev_free(u_wts);
    mcv::dev_free(u_pts);
    mcv::dev_free(wm_dev);
    mcv::dev_free(res_dev);
    if (wm_host) hipHostFree(wm_host);
    if (res_host) hipHostFree(res_host);
    if (admit_stream) hipStreamDestroy(admit_stream);
  }
};

namespace {

size_t tsize(int prec) { return prec == MCV_FP32_MIXED ? 4 : 8; }

// Device bytes a request holds while admitted: its job block, its share of
// the pass's partial buffers and its event buffer.
size_t request_bytes(const mcv_problem& p, int64_t n_points, int64_t n_events, int unit_calls) {
  JobDev shape;
  shape.d = p.dim;
  shape.K = p.n_channels;
  shape.n = p.n_bins;
  const int G = (int)((n_points + unit_calls - 1) / unit_calls);
  return mcv::job_block_bytes(&p, 0) + mcv::partial_bytes(shape, G > 0 ? G : 1) +
         (size_t)p.dim * (size_t)n_events * tsize(p.precision) + 4096;
}

mcv_status grow_gen_arrays(mcv_server* S, int n) {
  if (n <= S->gen_cap) return MCV_OK;
  int cap = S->gen_cap > 0 ? S->gen_cap : 64;
  while (cap < n) cap *= 2;
  mcv::dev_free(S->wm_dev);
  mcv::dev_free(S->res_dev);
  if (S->wm_host) hipHostFree(S->wm_host);
  if (S->res_host) hipHostFree(S->res_host);
  S->wm_dev = S->res_dev = S->wm_host = S->res_host = nullptr;
  S->gen_cap = 0;
  MCV_HIP(mcv::dev_alloc((void**)&S->wm_dev, cap * sizeof(double)));
  MCV_HIP(mcv::dev_alloc((void**)&S->res_dev, (size_t)cap * 8 * sizeof(double)));
  MCV_HIP(hipHostMalloc(&S->wm_host, cap * sizeof(double), 0));
  MCV_HIP(hipHostMalloc(&S->res_host, (size_t)cap * 8 * sizeof(double), 0));
  S->gen_cap = cap;
  return MCV_OK;
}

// Admits queued requests in order while the budget and the slot limit allow.
mcv_status admit(mcv_server* S, int* admitted) {
  *admitted = 0;
  while (!S->queue.empty() && (int)S->active.size() < S->cfg.max_active) {
    Request& r = S->queue.front();
    if (S->in_use + r.bytes > S->budget) break;
    Served sv;
    sv.dim = r.p.dim;
    sv.n_points = r.n_points;
    sv.n_events = r.n_events;
    sv.n_iter = r.n_iter;
    sv.bytes = r.bytes;
    sv.rep.state = MCV_JOB_INTEGRATING;
    sv.rep.submit_time = r.submit;
    sv.rep.device_bytes = (int64_t)r.bytes;
    mcv::Job jb;
    jb.n_points = r.n_points;
    mcv_status st = mcv::job_create(&r.p, 0, r.n_points, S->e.n_cu, S->admit_stream, &jb.j,
                                    &jb.block);
    if (st != MCV_OK) return st;
    jb.j.adapt_passes = r.n_iter;  // the last pass's grids are the ones used to generate
    jb.live = true;
    if (r.n_events > 0) {
      hipError_t he = mcv::dev_alloc((void**)&sv.events, (size_t)r.p.dim * r.n_events * tsize(r.p.precision));
      if (he != hipSuccess) {
        mcv::dev_free(jb.block);
        return fail(MCV_E_NOMEM, "event buffer");
      }
    }
    S->e.jobs.push_back(jb);
    sv.job = (int)S->e.jobs.size() - 1;
    sv.rep.admit_time = now_s(S->t0);
    S->in_use += r.bytes;
    S->active.emplace(r.ticket, sv);
    S->queue.pop_front();
    S->set_dirty = true;
    ++*admitted;
  }
  return MCV_OK;
}

void retire(mcv_server* S, int64_t ticket, Served& sv) {
  mcv::Job& jb = S->e.jobs[sv.job];
  mcv::dev_free(jb.block);
  jb.block = nullptr;
  jb.live = false;
  if (sv.events && !S->cfg.keep_events) {
    mcv::dev_free(sv.events);
    sv.events = nullptr;
  }
  S->in_use -= sv.bytes;
  sv.rep.state = MCV_JOB_DONE;
  sv.rep.finish_time = now_s(S->t0);
  S->done.emplace(ticket, sv);
  S->finished_unread.push_back(ticket);
}

// Reclaims engine job slots of retired jobs once none is referenced.
void compact_jobs(mcv_server* S) {
  if (S->e.jobs.size() < 4096) return;
  std::vector<mcv::Job> keep;
  keep.reserve(S->active.size());
  for (auto& kv : S->active) {
    keep.push_back(S->e.jobs[kv.second.job]);
    kv.second.job = (int)keep.size() - 1;
  }
  S->e.jobs.swap(keep);
  S->set_dirty = true;
}

}  // namespace

extern "C" {

mcv_status mcv_server_create(const mcv_server_config* cfg, void* hip_stream, mcv_server** out) {
  if (!out || !cfg) return fail(MCV_E_INVALID, "NULL argument");
  *out = nullptr;
  if (cfg->precision != MCV_FP64 && cfg->precision != MCV_FP32_MIXED)
    return fail(MCV_E_INVALID, "precision must be MCV_FP64 or MCV_FP32_MIXED");
  if (cfg->max_active < 1 || cfg->max_active > 65535)
    return fail(MCV_E_INVALID, "max_active must be in [1, 65535]");
  if (cfg->unweight_batch < 1 || cfg->unweight_batch > (1 << 24))
    return fail(MCV_E_INVALID, "unweight_batch must be in [1, 2^24]");
  if (cfg->hbm_budget < 0) return fail(MCV_E_INVALID, "hbm_budget must be >= 0");
  mcv_tuning t = cfg->tuning;
  if (t.block == 0) t = mcv::default_tuning();
  mcv_status st = mcv::check_tuning(t);
  if (st != MCV_OK) return st;
  mcv_server* S = new mcv_server();
  S->cfg = *cfg;
  S->cfg.tuning = t;
  S->e.stream = reinterpret_cast<hipStream_t>(hip_stream);
  S->e.prec = cfg->precision;
  S->e.tune = t;
  S->t0 = std::chrono::steady_clock::now();
  st = mcv::device_cus(&S->e.device, &S->e.n_cu);
  const int64_t B = cfg->unweight_batch;
  hipError_t he = hipSuccess;
  if (st == MCV_OK) {
    he = hipStreamCreateWithFlags(&S->admit_stream, hipStreamNonBlocking);
    if (he == hipSuccess) he = mcv::dev_alloc((void**)&S->u_accept, mcv::compact_accept_bytes(B));
    if (he == hipSuccess) he = mcv::dev_alloc((void**)&S->u_wts, B * sizeof(double));
    if (he == hipSuccess) he = mcv::dev_alloc((void**)&S->u_pts, B * 32 * tsize(cfg->precision));
    if (he != hipSuccess) st = fail(MCV_E_NOMEM, std::string("server buffers: ") + hipGetErrorString(he));
  }
  if (st == MCV_OK) st = grow_gen_arrays(S, 64);
  if (st == MCV_OK) {
    if (cfg->hbm_budget > 0) {
      S->budget = (size_t)cfg->hbm_budget;
    } else {
      size_t fr = 0, tot = 0;
      he = hipMemGetInfo(&fr, &tot);
      if (he != hipSuccess) st = fail(MCV_E_DEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(he));
      S->budget = (size_t)(0.9 * (double)fr);
    }
  }
  if (st != MCV_OK) {
    delete S;
    return st;
  }
  *out = S;
  return MCV_OK;
}

mcv_status mcv_server_clock(mcv_server* S, double* seconds) {
  if (!S || !seconds) return fail(MCV_E_INVALID, "NULL argument");
  *seconds = now_s(S->t0);
  return MCV_OK;
}

mcv_status mcv_server_submit(mcv_server* S, const mcv_problem* p, int64_t n_points,
                             int32_t n_iterations, int64_t n_events, int64_t* ticket) {
  if (!S || !ticket) return fail(MCV_E_INVALID, "NULL argument");
  mcv_status st = mcv::validate_problem(p);
  if (st != MCV_OK) return st;
  if (p->precision != S->cfg.precision) return fail(MCV_E_INVALID, "precision differs from the server's");
  if (p->rng != MCV_RNG_PHILOX)
    return fail(MCV_E_INVALID, "served requests draw Philox words (rng = MCV_RNG_PHILOX)");
  if (p->strat != 0) return fail(MCV_E_INVALID, "served requests sample importance-wise (strat = 0)");
  if (n_iterations < 1 || n_iterations > 1000) return fail(MCV_E_INVALID, "n_iterations must be in [1, 1000]");
  if (n_points < (int64_t)p->n_channels * p->min_calls || n_points > ((int64_t)1 << 40))
    return fail(MCV_E_INVALID, "n_points must be in [n_channels * min_calls, 2^40]");
  if (n_events < 0 || n_events > ((int64_t)1 << 32)) return fail(MCV_E_INVALID, "n_events must be in [0, 2^32]");
  Request r;
  r.ticket = S->next_ticket;
  const size_t kd = (size_t)p->n_channels * p->dim, pd = (size_t)p->n_peaks * p->dim;
  r.pk.assign(p->peak_kind, p->peak_kind + pd);
  r.pl.assign(p->peak_loc, p->peak_loc + pd);
  r.pw.assign(p->peak_width, p->peak_width + pd);
  r.pwt.assign(p->peak_weight, p->peak_weight + p->n_peaks);
  r.ck.assign(p->chan_kind, p->chan_kind + kd);
  r.cl.assign(p->chan_loc, p->chan_loc + kd);
  r.cw.assign(p->chan_width, p->chan_width + kd);
  r.p = *p;
  r.p.max_iterations = n_iterations;
  r.n_points = n_points;
  r.n_events = n_events;
  r.n_iter = n_iterations;
  r.bytes = request_bytes(r.p, n_points, n_events, S->cfg.tuning.unit_calls);
  if (r.bytes > S->budget) return fail(MCV_E_INVALID, "the job alone exceeds the memory budget");
  r.submit = now_s(S->t0);
  S->queue.push_back(std::move(r));
  Request& q = S->queue.back();  // arrays now live in the queued request
  q.p.peak_kind = q.pk.data();
  q.p.peak_loc = q.pl.data();
  q.p.peak_width = q.pw.data();
  q.p.peak_weight = q.pwt.data();
  q.p.chan_kind = q.ck.data();
  q.p.chan_loc = q.cl.data();
  q.p.chan_width = q.cw.data();
  *ticket = S->next_ticket++;
  return MCV_OK;
}

mcv_status mcv_server_step(mcv_server* S, mcv_step_info* info) {
  if (!S) return fail(MCV_E_INVALID, "server is NULL");
  mcv::Engine& e = S->e;
  hipStream_t s = e.stream;
  mcv_status st = MCV_OK;
  int admitted = 0;
  if (S->active.empty()) {  // nothing runs: admit first, synchronously
    st = admit(S, &admitted);
    if (st != MCV_OK) return st;
  }
  // the integrating set
  if (S->set_dirty) {
    compact_jobs(S);
    std::vector<int> members;
    for (auto& kv : S->active)
      if (kv.second.rep.state == MCV_JOB_INTEGRATING) members.push_back(kv.second.job);
    st = e.build_set(members);
    if (st != MCV_OK) return st;
    S->set_dirty = false;
  }
  int n_int = e.js.n;
  if (n_int > 0) {
    st = e.enqueue_iteration(MCV_REFINE_GRID | MCV_REFINE_ALPHA, s, nullptr, nullptr);
    if (st != MCV_OK) return st;
  }
  // one unweighting batch per generating job
  std::vector<std::pair<int64_t, Served*>> gen;
  for (auto& kv : S->active)
    if (kv.second.rep.state == MCV_JOB_GENERATING) gen.emplace_back(kv.first, &kv.second);
  st = grow_gen_arrays(S, (int)gen.size());
  if (st != MCV_OK) return st;
  const int64_t B = S->cfg.unweight_batch;
  if (!gen.empty()) {
    for (size_t i = 0; i < gen.size(); ++i) S->wm_host[i] = gen[i].second->wmax;
    MCV_HIP(hipMemcpyAsync(S->wm_dev, S->wm_host, gen.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
    for (size_t i = 0; i < gen.size(); ++i) {
      Served& sv = *gen[i].second;
      const JobDev& j = e.jobs[sv.job].j;
      mcv::launch_unweight_batch(j, sv.q0, B, S->wm_dev + i, S->u_accept, S->u_wts, S->u_pts, s);
      mcv::launch_compact(j, S->u_accept, S->u_wts, S->u_pts, B, S->wm_dev + i,
                          sv.n_events - sv.got, sv.events, sv.n_events, sv.got, nullptr,
                          S->res_dev + 8 * i, s);
      sv.gen_slot = (int)i;
    }
    MCV_HIP(hipMemcpyAsync(S->res_host, S->res_dev, gen.size() * 8 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  }
  MCV_HIP(hipGetLastError());
  // admission overlaps the step's kernels
  if (admitted == 0) {
    st = admit(S, &admitted);
    if (st != MCV_OK) return st;
  }
  MCV_HIP(hipStreamSynchronize(s));

  // bookkeeping
  std::vector<int64_t> finished;
  for (size_t i = 0; i < gen.size(); ++i) {
    Served& sv = *gen[i].second;
    const double* r = S->res_host + 8 * i;
    const int64_t used = (int64_t)r[0];
    if (used > 0) sv.last_used = (int64_t)sv.q0 + (int64_t)r[2];
    sv.got += used;
    sv.n_over += (int64_t)r[3];
    if (r[4] > sv.wmax) sv.wmax = r[4];
    sv.q0 += (uint64_t)B;
    if (sv.got >= sv.n_events) finished.push_back(gen[i].first);
  }
  std::map<int, std::pair<const int64_t, Served>*> by_job;
  if (n_int > 0)
    for (auto& kv : S->active)
      if (kv.second.rep.state == MCV_JOB_INTEGRATING) by_job[kv.second.job] = &kv;
  for (int m = 0; m < n_int; ++m) {
    const int idx = e.set_members[m];
    auto f = by_job.find(idx);
    if (f == by_job.end()) continue;
    {
      auto& kv = *f->second;
      Served& sv = kv.second;
      sv.rep.iterations_done += 1;
      if (sv.rep.iterations_done >= sv.n_iter) {
        std::vector<double> h((size_t)sv.n_iter * mcv::kHistStride);
        MCV_HIP(hipMemcpy(h.data(), e.jobs[idx].j.history, h.size() * sizeof(double),
                          hipMemcpyDeviceToHost));
        mcv::combine_history(h.data(), sv.n_iter, 0, &sv.rep.result);
        sv.wmax = h[(size_t)(sv.n_iter - 1) * mcv::kHistStride + 3];
        sv.rep.state = MCV_JOB_GENERATING;
        S->set_dirty = true;
        if (sv.n_events == 0) finished.push_back(kv.first);
      }
    }
  }
  for (int64_t t : finished) {
    auto it = S->active.find(t);
    Served& sv = it->second;
    sv.rep.n_events = sv.got < sv.n_events ? sv.got : sv.n_events;
    sv.rep.trials = sv.last_used + 1;
    sv.rep.n_overweight = sv.n_over;
    sv.rep.w_max = sv.wmax;
    sv.rep.efficiency = sv.rep.trials > 0 ? (double)sv.rep.n_events / (double)sv.rep.trials : 0.0;
    retire(S, t, sv);
    S->active.erase(it);
  }
  if (info) {
    info->n_integrating = n_int;
    info->n_generating = (int32_t)gen.size();
    info->n_admitted = admitted;
    info->n_finished = (int32_t)finished.size();
    info->n_queued = (int32_t)S->queue.size();
    info->n_active = (int32_t)S->active.size();
    info->bytes_in_use = (int64_t)S->in_use;
  }
  return MCV_OK;
}

mcv_status mcv_server_finished(mcv_server* S, int64_t* tickets, int32_t cap, int32_t* n) {
  if (!S || !n) return fail(MCV_E_INVALID, "NULL argument");
  const int32_t m = (int32_t)S->finished_unread.size() < cap ? (int32_t)S->finished_unread.size() : cap;
  for (int32_t i = 0; i < m; ++i) tickets[i] = S->finished_unread[i];
  S->finished_unread.erase(S->finished_unread.begin(), S->finished_unread.begin() + m);
  *n = m;
  return MCV_OK;
}

mcv_status mcv_server_report(mcv_server* S, int64_t ticket, mcv_job_report* out) {
  if (!S || !out) return fail(MCV_E_INVALID, "NULL argument");
  auto d = S->done.find(ticket);
  if (d != S->done.end()) {
    *out = d->second.rep;
    return MCV_OK;
  }
  auto a = S->active.find(ticket);
  if (a != S->active.end()) {
    *out = a->second.rep;
    return MCV_OK;
  }
  for (const Request& r : S->queue)
    if (r.ticket == ticket) {
      memset(out, 0, sizeof *out);
      out->state = MCV_JOB_QUEUED;
      out->submit_time = r.submit;
      out->device_bytes = (int64_t)r.bytes;
      return MCV_OK;
    }
  return fail(MCV_E_INVALID, "unknown ticket");
}

mcv_status mcv_server_events(mcv_server* S, int64_t ticket, void* d_out) {
  if (!S || !d_out) return fail(MCV_E_INVALID, "NULL argument");
  auto d = S->done.find(ticket);
  if (d == S->done.end()) return fail(MCV_E_STATE, "the job is not finished");
  Served& sv = d->second;
  if (!sv.events) return fail(MCV_E_STATE, "the job's events were not kept or were released");
  const size_t bytes = (size_t)sv.dim * (size_t)sv.n_events * tsize(S->cfg.precision);
  MCV_HIP(hipMemcpyAsync(d_out, sv.events, bytes, hipMemcpyDeviceToDevice, S->e.stream));
  MCV_HIP(hipStreamSynchronize(S->e.stream));
  mcv::dev_free(sv.events);
  sv.events = nullptr;
  return MCV_OK;
}

void mcv_server_destroy(mcv_server* S) { delete S; }

}  // extern "C"
