// Batched integration: many independent jobs advance one iteration together.
// Per iteration one allocation kernel, ONE persistent sample launch that
// drains a work-unit queue spanning every job, and batched reduction,
// rebinning and channel-weight kernels (one grid row per job).  The sequence
// is captured once per refine mode as a HIP graph and replayed.  An
// autotuner times the sample launch over candidate workgroup sizes, unit
// sizes and LDS budgets and keeps the winners in a JSON cache.
//
// Brass, Kilian, Reuter, arXiv:1811.09711, Sec. 3.5: every job is an
// independent VAMP integration; its iteration is the sample pass followed by
// the grid (eq. 30) and channel-weight (eq. 15) adaptation.  Sec. 4 runs
// independent work in parallel; here the unit of parallel work is a range
// of one job's calls.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "mcv.h"
#include "mcv_batch.h"
#include "mcv_host.h"

using mcv::fail;
using mcv::JobDev;

namespace mcv {

mcv_status check_tuning(const mcv_tuning& t) {
  if (t.block < 64 || t.block > 1024 || t.block % 64 != 0)
    return fail(MCV_E_INVALID, "tuning.block must be a multiple of 64 in [64, 1024]");
  if (t.unit_calls < t.block || t.unit_calls > (1 << 26))
    return fail(MCV_E_INVALID, "tuning.unit_calls must be in [block, 2^26]");
  if (t.launch_bound != 0 && t.launch_bound != 256 && t.launch_bound != 512 &&
      t.launch_bound != 1024)
    return fail(MCV_E_INVALID, "tuning.launch_bound must be 0, 256, 512 or 1024");
  if (t.launch_bound != 0 && t.launch_bound < t.block)
    return fail(MCV_E_INVALID, "tuning.launch_bound must be at least tuning.block");
  if (t.term_bound != 0 && t.term_bound != 1)
    return fail(MCV_E_INVALID, "tuning.term_bound must be 0 or 1");
  return MCV_OK;
}

mcv_tuning default_tuning() {
  mcv_tuning t;
  t.block = 1024;
  t.unit_calls = 16384;
  t.launch_bound = 1024;
  t.term_bound = 1;
  return t;
}

void Engine::free_set_buffers() {
  dev_free(table);
  dev_free(scratch);
  table = nullptr;
  scratch = nullptr;
  scratch_cap = 0;
  table_cap = 0;
  drop_graphs();
}

void Engine::drop_graphs() {
  for (auto& g : graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
}

Engine::~Engine() {
  if (stream) hipStreamSynchronize(stream);
  free_set_buffers();
  if (cap_stream) hipStreamDestroy(cap_stream);
  for (auto& e : ev)
    for (hipEvent_t x : {e.a, e.b, e.c, e.d})
      if (x) hipEventDestroy(x);
}

// Units per job, partial buffers, device job table, unit prefix, sample
// arguments and the persistent grid for the jobs listed in `listed`.  The set
// holds them ordered by dimension (stable), so that the units of one
// dimension are contiguous and the batched kernel's workgroups on one XCD
// mostly run the body compiled for one d.
mcv_status Engine::build_set(const std::vector<int>& listed) {
  MCV_HIP(hipStreamSynchronize(stream));  // earlier passes may still read the table
  drop_graphs();
  std::vector<int> members = listed;
  std::stable_sort(members.begin(), members.end(),
                   [this](int x, int y) { return jobs[x].j.d < jobs[y].j.d; });
  const int n = (int)members.size();
  set_members = members;
  set_jobs.clear();
  js = JobSet();
  if (n == 0) return MCV_OK;
  if (n > 65535) return fail(MCV_E_INVALID, "at most 65535 jobs per step");
  set_jobs.reserve(n);
  std::vector<int> prefix(n + 1, 0);
  size_t pbytes = 0;
  for (int i = 0; i < n; ++i) {
    const Job& jb = jobs[members[i]];
    const int64_t G64 = (jb.n_points + tune.unit_calls - 1) / tune.unit_calls;
    const int G = (int)std::max<int64_t>(1, G64);
    if ((int64_t)prefix[i] + G > (1ll << 30)) return fail(MCV_E_INVALID, "too many work units");
    prefix[i + 1] = prefix[i] + G;
    pbytes += (partial_bytes(jb.j, G) + 255) & ~(size_t)255;
  }
  const size_t abytes = sample_args_bytes(prec);
  const size_t off_prefix = 0;
  const size_t off_counter = (off_prefix + (size_t)(n + 1) * sizeof(int) + 255) & ~(size_t)255;
  const size_t off_table = off_counter + 256;
  const size_t off_args = (off_table + (size_t)n * sizeof(JobDev) + 255) & ~(size_t)255;
  const size_t tbytes = off_args + (size_t)n * abytes;
  if (tbytes > table_cap) {
    dev_free(table);
    table = nullptr;
    table_cap = 0;
    const size_t want = tbytes + tbytes / 2;  // headroom for sets that grow
    if (dev_alloc(&table, want) != hipSuccess) return fail(MCV_E_NOMEM, "job table");
    table_cap = want;
  }
  if (pbytes > scratch_cap) {
    dev_free(scratch);
    scratch = nullptr;
    scratch_cap = 0;
    const size_t want = pbytes + pbytes / 2;
    if (dev_alloc(&scratch, want) != hipSuccess) return fail(MCV_E_NOMEM, "partial buffers");
    scratch_cap = want;
  }
  char* tb = static_cast<char*>(table);
  std::vector<char> host(tbytes, 0);
  memcpy(host.data() + off_prefix, prefix.data(), (size_t)(n + 1) * sizeof(int));
  size_t poff = 0;
  int lds = 0;
  for (int i = 0; i < n; ++i) {
    JobDev j = jobs[members[i]].j;
    const int G = prefix[i + 1] - prefix[i];
    carve_partials(j, G, static_cast<char*>(scratch) + poff);
    poff += (partial_bytes(j, G) + 255) & ~(size_t)255;
    const int b = sample_queue_layout(j, tune.block, host.data() + off_args + (size_t)i * abytes);
    if (b > lds) lds = b;
    set_jobs.push_back(j);
  }
  memcpy(host.data() + off_table, set_jobs.data(), (size_t)n * sizeof(JobDev));
  if (lds > 160 * 1024) return fail(MCV_E_INVALID, "a job's tables do not fit the LDS");
  MCV_HIP(hipMemcpyAsync(tb, host.data(), tbytes, hipMemcpyHostToDevice, stream));
  MCV_HIP(hipStreamSynchronize(stream));
  js.n = n;
  js.host = set_jobs.data();
  js.dev = reinterpret_cast<const JobDev*>(tb + off_table);
  js.prec = prec;
  set_extents(js);
  js.unit_prefix = reinterpret_cast<const int*>(tb + off_prefix);
  js.n_units = prefix[n];
  js.counter = reinterpret_cast<int*>(tb + off_counter);
  js.sargs = tb + off_args;
  js.block = tune.block;
  js.bound = tune.launch_bound > 0 ? tune.launch_bound : 1024;
  js.term_bound = tune.term_bound;
  js.lds = lds;
  const int occ = sample_queue_occupancy(js);
  if (occ < 1) return fail(MCV_E_DEVICE, "the batched sample kernel cannot be resident");
  int grid = n_cu * occ;
  if (grid > js.n_units) grid = js.n_units;
  js.grid = grid;
  return MCV_OK;
}

// One iteration of every job of the current set on stream s.
mcv_status Engine::enqueue_iteration(uint32_t what, hipStream_t s, hipEvent_t after_alloc,
                                     hipEvent_t after_sample) {
  launch_allocate(js, 0, false, s);
  if (after_alloc) MCV_HIP(hipEventRecord(after_alloc, s));
  if (launch_sample_queue(js, s) < 1) return fail(MCV_E_DEVICE, "batched sample launch failed");
  if (after_sample) MCV_HIP(hipEventRecord(after_sample, s));
  launch_finalize(js, 0, s);
  if (what & MCV_REFINE_GRID) {
    launch_refine_grid(js, s);
    launch_tables(js, s);
  }
  if (what & MCV_REFINE_ALPHA) launch_update_alpha(js, s);
  MCV_HIP(hipGetLastError());
  return MCV_OK;
}

mcv_status Engine::iterate(uint32_t what, bool use_graph) {
  if (js.n < 1) return fail(MCV_E_STATE, "no jobs");
  const size_t it = ev.size();
  Ev e;
  MCV_HIP(hipEventCreate(&e.a));
  MCV_HIP(hipEventCreate(&e.d));
  if (!use_graph) {
    MCV_HIP(hipEventCreate(&e.b));
    MCV_HIP(hipEventCreate(&e.c));
  }
  e.graphed = use_graph;
  ev.push_back(e);
  if (use_graph) {
    Graph& g = graphs[what & 3];
    if (!g.exec) {
      if (!cap_stream) MCV_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
      MCV_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
      mcv_status st = enqueue_iteration(what, cap_stream, nullptr, nullptr);
      hipGraph_t graph = nullptr;
      hipError_t ee = hipStreamEndCapture(cap_stream, &graph);
      if (st != MCV_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
      }
      if (ee != hipSuccess) return fail(MCV_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
      ee = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (ee != hipSuccess) {
        g.exec = nullptr;
        return fail(MCV_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ee));
      }
    }
    MCV_HIP(hipEventRecord(ev[it].a, stream));
    MCV_HIP(hipGraphLaunch(g.exec, stream));
    MCV_HIP(hipEventRecord(ev[it].d, stream));
  } else {
    MCV_HIP(hipEventRecord(ev[it].a, stream));
    mcv_status st = enqueue_iteration(what, stream, ev[it].c, ev[it].b);
    if (st != MCV_OK) return st;
    MCV_HIP(hipEventRecord(ev[it].d, stream));
  }
  for (int m : set_members) jobs[m].iters += 1;
  return MCV_OK;
}

mcv_status Engine::timing(int iteration, double* iter_ms, double* sample_ms) {
  if (iteration < 0 || iteration >= (int)ev.size()) return fail(MCV_E_STATE, "no such iteration");
  const Ev& e = ev[iteration];
  MCV_HIP(hipEventSynchronize(e.d));
  float ms = 0.0f;
  MCV_HIP(hipEventElapsedTime(&ms, e.a, e.d));
  if (iter_ms) *iter_ms = ms;
  if (sample_ms) *sample_ms = -1.0;
  if (!e.graphed) {
    MCV_HIP(hipEventElapsedTime(&ms, e.c, e.b));
    if (sample_ms) *sample_ms = ms;
  }
  return MCV_OK;
}

mcv_status Engine::add_job(const mcv_problem* p, int64_t n_points, int* index) {
  if (p->precision != prec) return fail(MCV_E_INVALID, "every job of a batch has the batch's precision");
  if (p->rng != MCV_RNG_PHILOX)
    return fail(MCV_E_INVALID, "batched jobs draw Philox words (rng = MCV_RNG_PHILOX)");
  if (p->strat != 0) return fail(MCV_E_INVALID, "batched jobs sample importance-wise (strat = 0)");
  if (n_points < (int64_t)p->n_channels * p->min_calls)
    return fail(MCV_E_INVALID, "n_points must be at least n_channels * min_calls");
  if (n_points > ((int64_t)1 << 40)) return fail(MCV_E_INVALID, "n_points too large");
  Job jb;
  jb.n_points = n_points;
  mcv_status st = job_create(p, 0, n_points, n_cu, stream, &jb.j, &jb.block);
  if (st != MCV_OK) return st;
  jb.live = true;
  jobs.push_back(jb);
  *index = (int)jobs.size() - 1;
  return MCV_OK;
}

void Engine::remove_job(int index) {
  Job& jb = jobs[index];
  dev_free(jb.block);
  jb.block = nullptr;
  jb.live = false;
}

mcv_status Engine::history(int index, double* out, int cap, int* n_iter) {
  if (index < 0 || index >= (int)jobs.size() || !jobs[index].live)
    return fail(MCV_E_INVALID, "no such job");
  const Job& jb = jobs[index];
  MCV_HIP(hipStreamSynchronize(stream));
  int32_t it = 0;
  MCV_HIP(hipMemcpy(&it, jb.j.iter_dev, sizeof it, hipMemcpyDeviceToHost));
  if (n_iter) *n_iter = it;
  const int m = cap < it ? cap : it;
  if (out && m > 0)
    MCV_HIP(hipMemcpy(out, jb.j.history, (size_t)m * kHistStride * sizeof(double),
                      hipMemcpyDeviceToHost));
  return MCV_OK;
}

}  // namespace mcv

// ---------------------------------------------------------------------------
// Autotuning cache: a JSON object mapping a workload key to its tuning,
// {"<key>": {"block": B, "unit_calls": U, "launch_bound": L, "term_bound": S,
// "ms": T}, ...} (other fields are ignored; a missing term_bound is 1).
// ---------------------------------------------------------------------------
namespace {

struct CacheEntry {
  mcv_tuning t;
  double ms;
};

bool parse_number(const std::string& s, size_t& i, double* v) {
  while (i < s.size() && isspace((unsigned char)s[i])) ++i;
  const char* b = s.c_str() + i;
  char* e = nullptr;
  *v = strtod(b, &e);
  if (e == b) return false;
  i += (size_t)(e - b);
  return true;
}

bool parse_string(const std::string& s, size_t& i, std::string* out) {
  while (i < s.size() && isspace((unsigned char)s[i])) ++i;
  if (i >= s.size() || s[i] != '"') return false;
  ++i;
  out->clear();
  while (i < s.size() && s[i] != '"') {
    if (s[i] == '\\') return false;  // keys and fields never need escapes
    out->push_back(s[i++]);
  }
  if (i >= s.size()) return false;
  ++i;
  return true;
}

bool expect(const std::string& s, size_t& i, char c) {
  while (i < s.size() && isspace((unsigned char)s[i])) ++i;
  if (i >= s.size() || s[i] != c) return false;
  ++i;
  return true;
}

// Reads the cache; a missing file is an empty cache, a malformed one is an
// error.
bool read_cache(const char* path, std::map<std::string, CacheEntry>* out) {
  out->clear();
  FILE* f = fopen(path, "rb");
  if (!f) return true;
  std::string s;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
  fclose(f);
  size_t i = 0;
  if (!expect(s, i, '{')) return false;
  if (expect(s, i, '}')) return true;
  for (;;) {
    std::string key;
    if (!parse_string(s, i, &key) || !expect(s, i, ':') || !expect(s, i, '{')) return false;
    CacheEntry e{mcv::default_tuning(), 0.0};
    for (;;) {
      std::string field;
      double v = 0.0;
      if (!parse_string(s, i, &field) || !expect(s, i, ':') || !parse_number(s, i, &v)) return false;
      if (field == "block") e.t.block = (int32_t)v;
      else if (field == "unit_calls") e.t.unit_calls = (int32_t)v;
      else if (field == "launch_bound") e.t.launch_bound = (int32_t)v;
      else if (field == "term_bound") e.t.term_bound = (int32_t)v;
      else if (field == "ms") e.ms = v;
      if (expect(s, i, '}')) break;
      if (!expect(s, i, ',')) return false;
    }
    (*out)[key] = e;
    if (expect(s, i, '}')) return true;
    if (!expect(s, i, ',')) return false;
  }
}

bool write_cache(const char* path, const std::map<std::string, CacheEntry>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : m) {
    fprintf(f,
            "  \"%s\": {\"block\": %d, \"unit_calls\": %d, \"launch_bound\": %d, "
            "\"term_bound\": %d, \"ms\": %.6g}%s\n",
            kv.first.c_str(), kv.second.t.block, kv.second.t.unit_calls, kv.second.t.launch_bound,
            kv.second.t.term_bound, kv.second.ms, (++k < m.size()) ? "," : "");
  }
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path) == 0;
}

int bucket_d(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 12 ? 12 : d <= 16 ? 16 : 32; }

int ceil_log2(double x) {
  int k = 0;
  while (k < 62 && (double)(1ll << k) < x) ++k;
  return k;
}

// Workload key: precision, dimension bucket of the kernel, channel bucket,
// bins, and the totals of calls and jobs rounded to powers of two.
std::string workload_key(const mcv_problem* p, const int64_t* n_points, int n_jobs) {
  int maxd = 0, maxK = 0, maxn = 0;
  double calls = 0.0;
  for (int i = 0; i < n_jobs; ++i) {
    maxd = std::max(maxd, p[i].dim);
    maxK = std::max(maxK, p[i].n_channels);
    maxn = std::max(maxn, p[i].n_bins);
    calls += (double)n_points[i];
  }
  char buf[160];
  snprintf(buf, sizeof buf, "%s d<=%d K<=2^%d n<=%d calls~2^%d jobs~2^%d",
           p[0].precision == MCV_FP32_MIXED ? "fp32" : "fp64", bucket_d(maxd), ceil_log2(maxK),
           maxn, ceil_log2(calls), ceil_log2(n_jobs));
  return buf;
}

}  // namespace

struct mcv_batch {
  mcv::Engine e;
};

extern "C" {

mcv_status mcv_batch_create(const mcv_problem* problems, const int64_t* n_points, int32_t n_jobs,
                            const mcv_tuning* tuning, void* hip_stream, mcv_batch** out) {
  if (!out) return fail(MCV_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!problems || !n_points || n_jobs < 1 || n_jobs > 65535)
    return fail(MCV_E_INVALID, "need 1 <= n_jobs <= 65535 problems and call counts");
  const mcv_tuning t = tuning ? *tuning : mcv::default_tuning();
  mcv_status st = mcv::check_tuning(t);
  if (st != MCV_OK) return st;
  for (int i = 0; i < n_jobs; ++i) {
    st = mcv::validate_problem(&problems[i]);
    if (st != MCV_OK) return fail(st, "job " + std::to_string(i) + ": " + mcv::last_error());
    if (problems[i].precision != problems[0].precision)
      return fail(MCV_E_INVALID, "every job of a batch has the same precision");
  }
  mcv_batch* b = new mcv_batch();
  mcv::Engine& e = b->e;
  e.stream = reinterpret_cast<hipStream_t>(hip_stream);
  e.prec = problems[0].precision;
  e.tune = t;
  st = mcv::device_cus(&e.device, &e.n_cu);
  std::vector<int> members;
  for (int i = 0; i < n_jobs && st == MCV_OK; ++i) {
    int idx = 0;
    st = e.add_job(&problems[i], n_points[i], &idx);
    if (st != MCV_OK) st = fail(st, "job " + std::to_string(i) + ": " + mcv::last_error());
    members.push_back(idx);
  }
  if (st == MCV_OK) st = e.build_set(members);
  if (st != MCV_OK) {
    for (size_t i = 0; i < e.jobs.size(); ++i) e.remove_job((int)i);
    delete b;
    return st;
  }
  *out = b;
  return MCV_OK;
}

mcv_status mcv_batch_iterate(mcv_batch* b, uint32_t what, int32_t use_graph) {
  if (!b) return fail(MCV_E_INVALID, "batch is NULL");
  if (what & ~(uint32_t)(MCV_REFINE_GRID | MCV_REFINE_ALPHA))
    return fail(MCV_E_INVALID, "unknown refine flags");
  mcv::Engine& e = b->e;
  for (int m : e.set_members)
    if (e.jobs[m].iters >= e.jobs[m].j.max_iter)
      return fail(MCV_E_STATE, "a job's history is full (max_iterations)");
  return e.iterate(what, use_graph != 0);
}

mcv_status mcv_batch_get_history(mcv_batch* b, int32_t job, double* host_out, int32_t cap,
                                 int32_t* n_iter) {
  if (!b) return fail(MCV_E_INVALID, "batch is NULL");
  int n = 0;
  mcv_status st = b->e.history(job, host_out, cap, &n);
  if (n_iter) *n_iter = n;
  return st;
}

mcv_status mcv_batch_result(mcv_batch* b, int32_t job, int32_t first, mcv_summary* out) {
  if (!b || !out) return fail(MCV_E_INVALID, "NULL argument");
  int n = 0;
  mcv_status st = b->e.history(job, nullptr, 0, &n);
  if (st != MCV_OK) return st;
  if (n == 0 || first < 0 || first >= n) return fail(MCV_E_STATE, "first_iter is not a completed iteration");
  std::vector<double> h((size_t)n * mcv::kHistStride);
  st = b->e.history(job, h.data(), n, &n);
  if (st != MCV_OK) return st;
  mcv::combine_history(h.data(), n, first, out);
  return MCV_OK;
}

mcv_status mcv_batch_get_state(mcv_batch* b, int32_t job, double* edges, double* alpha,
                               int64_t* alloc) {
  if (!b) return fail(MCV_E_INVALID, "batch is NULL");
  mcv::Engine& e = b->e;
  if (job < 0 || job >= (int)e.jobs.size() || !e.jobs[job].live)
    return fail(MCV_E_INVALID, "no such job");
  const JobDev& j = e.jobs[job].j;
  MCV_HIP(hipStreamSynchronize(e.stream));
  if (edges)
    MCV_HIP(hipMemcpy(edges, j.edges, (size_t)j.K * j.d * (j.n + 1) * sizeof(double),
                      hipMemcpyDeviceToHost));
  if (alpha) MCV_HIP(hipMemcpy(alpha, j.alpha, j.K * sizeof(double), hipMemcpyDeviceToHost));
  if (alloc) {
    MCV_HIP(hipMemcpy(alloc, j.nc, j.K * sizeof(int64_t), hipMemcpyDeviceToHost));
    MCV_HIP(hipMemcpy(alloc + j.K, j.start + j.K, sizeof(int64_t), hipMemcpyDeviceToHost));
  }
  return MCV_OK;
}

mcv_status mcv_batch_info(mcv_batch* b, int32_t* n_units, int32_t* workgroups, int32_t* lds_bytes,
                          mcv_tuning* tuning) {
  if (!b) return fail(MCV_E_INVALID, "batch is NULL");
  if (n_units) *n_units = b->e.js.n_units;
  if (workgroups) *workgroups = b->e.js.grid;
  if (lds_bytes) *lds_bytes = b->e.js.lds;
  if (tuning) *tuning = b->e.tune;
  return MCV_OK;
}

mcv_status mcv_batch_timing(mcv_batch* b, int32_t iteration, double* iteration_ms,
                            double* sample_ms) {
  if (!b) return fail(MCV_E_INVALID, "batch is NULL");
  return b->e.timing(iteration, iteration_ms, sample_ms);
}

void mcv_batch_destroy(mcv_batch* b) {
  if (!b) return;
  if (b->e.stream) hipStreamSynchronize(b->e.stream);
  for (size_t i = 0; i < b->e.jobs.size(); ++i) b->e.remove_job((int)i);
  delete b;
}

mcv_status mcv_autotune(const mcv_problem* problems, const int64_t* n_points, int32_t n_jobs,
                        void* hip_stream, const char* cache_path, mcv_tuning* out,
                        double* best_ms) {
  if (!out) return fail(MCV_E_INVALID, "out is NULL");
  if (!problems || !n_points || n_jobs < 1 || n_jobs > 65535)
    return fail(MCV_E_INVALID, "need 1 <= n_jobs <= 65535 problems and call counts");
  for (int i = 0; i < n_jobs; ++i) {
    mcv_status st = mcv::validate_problem(&problems[i]);
    if (st != MCV_OK) return st;
  }
  const std::string key = workload_key(problems, n_points, n_jobs);
  std::map<std::string, CacheEntry> cache;
  if (cache_path) {
    if (!read_cache(cache_path, &cache)) return fail(MCV_E_INVALID, "malformed tuning cache");
    auto it = cache.find(key);
    if (it != cache.end() && mcv::check_tuning(it->second.t) == MCV_OK) {
      *out = it->second.t;
      if (best_ms) *best_ms = it->second.ms;
      return MCV_OK;
    }
  }
  // candidates: (workgroup size, launch bound) -- the 1024 bound keeps 16
  // waves per CU resident, the 512 bound gives more registers per lane at
  // fewer waves, the 256 bound caps registers for more waves -- times four
  // unit sizes, times with and without the term-bound test; one call per
  // lane and round
  static const int kBL[][2] = {{1024, 1024}, {512, 1024}, {256, 1024},
                               {512, 512},   {256, 512},  {256, 256}};
  static const int kUnits[] = {2048, 4096, 16384, 65536};
  constexpr int kNU = sizeof(kUnits) / sizeof(kUnits[0]);
  mcv_batch* b = nullptr;
  mcv_status st = mcv_batch_create(problems, n_points, n_jobs, nullptr, hip_stream, &b);
  if (st != MCV_OK) return st;
  mcv::Engine& e = b->e;
  std::vector<int> members = e.set_members;
  double best = INFINITY;
  mcv_tuning bt = mcv::default_tuning();
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t he = hipEventCreate(&t0);
  if (he == hipSuccess) he = hipEventCreate(&t1);
  for (const auto& bl : kBL) {
    for (int cand = 0; cand < 2 * kNU; ++cand) {
      if (st != MCV_OK || he != hipSuccess) break;
      mcv_tuning t;
      t.block = bl[0];
      t.launch_bound = bl[1];
      t.unit_calls = std::max(kUnits[cand % kNU], bl[0]);
      t.term_bound = cand < kNU ? 1 : 0;
      e.tune = t;
      st = e.build_set(members);
      if (st != MCV_OK) {
        st = MCV_OK;  // a candidate that cannot run is skipped
        continue;
      }
      float ms = 0.0f;
      for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {
        mcv::launch_allocate(e.js, 0, false, e.stream);
        he = hipEventRecord(t0, e.stream);
        if (he == hipSuccess && mcv::launch_sample_queue(e.js, e.stream) < 1) he = hipErrorLaunchFailure;
        if (he == hipSuccess) he = hipEventRecord(t1, e.stream);
        if (he == hipSuccess) he = hipEventSynchronize(t1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, t0, t1);
      }
      if (he == hipSuccess && ms < best) {
        best = ms;
        bt = t;
      }
    }
  }
  if (t0) hipEventDestroy(t0);
  if (t1) hipEventDestroy(t1);
  mcv_batch_destroy(b);
  if (he != hipSuccess) return fail(MCV_E_DEVICE, std::string("autotune: ") + hipGetErrorString(he));
  if (st != MCV_OK) return st;
  if (!isfinite(best)) return fail(MCV_E_INVALID, "no tuning candidate fits these jobs");
  *out = bt;
  if (best_ms) *best_ms = best;
  if (cache_path) {
    cache[key] = CacheEntry{bt, best};
    if (!write_cache(cache_path, cache)) return fail(MCV_E_INVALID, "cannot write the tuning cache");
  }
  return MCV_OK;
}

mcv_status mcv_tuning_key(const mcv_problem* problems, const int64_t* n_points, int32_t n_jobs,
                          char* buf, size_t cap) {
  if (!problems || !n_points || n_jobs < 1 || !buf || cap < 1)
    return fail(MCV_E_INVALID, "NULL argument");
  const std::string key = workload_key(problems, n_points, n_jobs);
  if (key.size() + 1 > cap) return fail(MCV_E_INVALID, "buffer too small");
  memcpy(buf, key.c_str(), key.size() + 1);
  return MCV_OK;
}

}  // extern "C"
